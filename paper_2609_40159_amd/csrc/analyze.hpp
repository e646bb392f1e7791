// Level-set analysis internals shared by rwt_analyze and the solve plans.
#pragma once

#include "common.hpp"

namespace rwt {

// Transposed (successor) pattern of the off-diagonal entries of L:
// successors of column j are csc_row[csc_ptr[j] .. csc_ptr[j+1]) in
// ascending row order; csc_map gives each entry's position in L's CSR.
struct Csc {
    int32_t* ptr = nullptr;   // n+1
    int32_t* row = nullptr;   // nnz - n
    int32_t* map = nullptr;   // nnz - n
};

struct LevelOut {
    int32_t* level = nullptr;      // n
    int32_t* perm = nullptr;       // n
    int32_t* level_ptr = nullptr;  // n+1
    int32_t* rows = nullptr;       // n
    int64_t* cost = nullptr;       // n
    rwt_level_stats* stats = nullptr;  // device
};

// Workspace bytes for build_csc / levelize beyond the outputs.
size_t csc_ws(int32_t n, int64_t nnz);
size_t levels_ws(int32_t n, int64_t nnz);

rwt_status build_csc(const rwt_csr& L, const Csc& out, void* ws, hipStream_t s);

// Levels, permutation, level pointers, per-level rows/cost and statistics.
// Needs the successor pattern.  ctrl: device control block (zeroed here).
rwt_status compute_levels(const rwt_csr& L, const Csc& csc, const LevelOut& out, Ctrl* ctrl,
                          void* ws, hipStream_t s, int watchdog_ms);

// Check the CSR on the device (pattern, and diagonal values when
// check_vals); 16 bytes of device workspace; synchronizes the stream.
rwt_status validate_device(const rwt_csr& L, bool check_vals, void* ws16, int32_t* bad_row,
                           hipStream_t s);

// host conversion of the 128-bit numerator (used for host-side checks)
double cv_from_sums(int32_t D, uint64_t S1, uint64_t S2_lo, uint64_t S2_hi);

}  // namespace rwt
