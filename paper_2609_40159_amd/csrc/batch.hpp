// Batched analysis + solve internals.
#pragma once

#include "common.hpp"

namespace rwt {

// One matrix as seen by the batched symbolic rewrite.
struct BatchRwMat {
    int32_t n;
    int32_t pad;
    const int32_t* rowptr;
    const int32_t* colidx;
    const int32_t* level;
};

// Host description of a batched symbolic pass over candidate rows.
constexpr int PATTERN_BUMPS = 64;   // one-pass patterns: parts of the overflow region

struct BatchRwArgs {
    const BatchRwMat* mats;     // device
    const int32_t* cand_ptr;    // device, C+1
    const int32_t* cand_mat;    // device, C
    int32_t C;
    int32_t qcap;               // capacity of the candidate row list
    const int32_t* rows;        // device, candidate rows (concatenated)
    const int32_t* targets;     // device or NULL (level - 1)
    int32_t* counts_q;          // device, qcap (+1)
    int32_t* pat_ptr;           // device, qcap + 1 (qmode 2 reads it, qmode 3 writes it)
    int32_t* pat;               // device, pat_cap
    int32_t pat_cap;
    int32_t slot_len;           // qmode 3: entries of each position's fixed slot
    int32_t* bump;              // qmode 3: PATTERN_BUMPS counters of the overflow region's parts
    int32_t* redo;              // qmode 3 sets it when the overflow region is full
    const int32_t* gate;        // qmodes 1, 2: run only when *gate != 0 (NULL: always)
    int32_t* ovf;               // device, qcap: positions over the small LDS tier
    int32_t* ovf2;              // device, qcap: positions over the large LDS tier
    unsigned char* ovf_mark;    // device, qcap
    int32_t* ctrl;              // device, 8 ints
    unsigned char* cand_bad;    // device, C: candidate row list rejected
    unsigned char* slab;        // device, nslab * slab_stride
    int64_t slab_stride;
    int32_t slab_cap;
    int32_t nslab;
};

size_t batch_rw_slab_stride(int32_t nmax);
// qmode 1: new row lengths; qmode 2: new patterns (needs pat_ptr); qmode 3:
// both in one pass, position q's pattern in slot [q * slot_len, ...) when it
// fits, else in the region after qcap * slot_len (bump allocation), its
// start in pat_ptr[q] and its length in counts_q[q].  When that region is
// full, qmode 3 sets *redo and the two passes (gated on it) run after it.
rwt_status batch_rewrite_pass(const BatchRwArgs& h, int qmode, hipStream_t s);

}  // namespace rwt
