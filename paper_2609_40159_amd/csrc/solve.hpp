// Triangular solve kernels and their launch parameters.
#pragma once

#include "analyze.hpp"

namespace rwt {

// Everything a solve kernel needs, forward (L) or transposed (L^T).
struct SolveArgs {
    int32_t n;
    const int32_t* rowptr;     // L
    const int32_t* colidx;
    const void* vals;
    const int32_t* cptr;       // successors (transposed solve)
    const int32_t* crow;
    const int32_t* cmap;
    const int32_t* perm;       // level order
    const int32_t* level_ptr;
    int32_t nlev;              // levels
    const int4* ldesc;         // level-scheduled: per row in level order {row, first, end, diagonal}
    // level-scheduled: segments of levels (begin, end, narrow flag)
    const int32_t* seg;
    int32_t nseg;
    // sync-free: row blocks
    int32_t block_rows;
    int32_t nblocks;
    const int32_t* bperm;      // rows grouped by block, each block in (level, row) order
    const int32_t* step_pos;   // start of each step (one level of one block) in bperm
    const int32_t* blk_step;   // first step of each block
    // right-hand sides
    const void* B;
    int64_t ldb;
    void* X;
    int64_t ldx;
    int32_t k;
    int32_t kc;                // sync-free: right-hand sides per chain (1..4)
    int32_t lanes;             // lanes per row (power of two, 1..64)
    int32_t stage_x;           // sync-free: helper waves prefetch x values of earlier blocks
    const int4* desc;          // sync-free: per row in bperm order {row, first, end, diagonal}
    int32_t lds_bytes;         // sync-free: dynamic LDS per workgroup
    Ctrl* ctrl;
    int64_t ticks;
    int32_t hold_row;          // >= 0: this row's values are never published (watchdog test)
    const void* vt;            // row-order walk, transposed: values in successor-list order
};

enum class Algo { Level, SyncFree, Walk };

// Row-order walk (walk.hpp): one wave per right-hand-side column, two
// per workgroup; for the transposed walk a.vt must hold the values in
// successor-list order (walk_gather_vals).
rwt_status walk_launch(const SolveArgs& a, rwt_dtype dt, bool transposed, hipStream_t s);
rwt_status walk_gather_vals(const int32_t* map, int64_t m, const void* vals, void* out,
                            rwt_dtype dt, hipStream_t s);
// 64-row chunks of consecutive rows: the sum over chunks of the rounds the
// walk needs on the chunk (its longest chain of internal dependencies plus
// one), into *d_out (zeroed by the call); the walk suits matrices whose
// chunks need few rounds (the pattern must be valid)
rwt_status chunk_rounds(const int32_t* rowptr, const int32_t* colidx, int32_t n,
                        unsigned long long* d_out, hipStream_t s);

// Fill X with the not-ready sentinel and reset the control block.
rwt_status solve_prepare(const SolveArgs& a, rwt_dtype dt, hipStream_t s);
rwt_status solve_launch(const SolveArgs& a, rwt_dtype dt, Algo algo, bool transposed,
                        unsigned grid, hipStream_t s);
// LDS of one sync-free workgroup: the block's x values, its step starts and
// the helper waves' stage ring (lanes per row G)
int syncfree_lds_bytes(int block_rows, int k, rwt_dtype dt, int lanes);
constexpr int SF_LDS_BUDGET = 80 * 1024;   // two workgroups per compute unit
// workgroups of a persistent solve launch (all resident); k: columns per
// chain (sync-free) or per launch (level-scheduled)
unsigned solve_grid(Algo algo, rwt_dtype dt, bool transposed, int k, size_t lds, int cus);

}  // namespace rwt
