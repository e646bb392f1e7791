// Solve plan internals shared by the single-matrix entry points and the
// batched launch.
#pragma once

#include "solve.hpp"

struct rwt_plan {
    rwt_csr L;
    rwt_plan_opts opts;
    rwt_level_stats stats;
    int32_t D = 0;
    rwt::Ctrl* ctrl = nullptr;
    int32_t* level = nullptr;
    int32_t* perm = nullptr;
    int32_t* level_ptr = nullptr;
    rwt::Csc csc;
    int32_t* seg = nullptr;
    int32_t nseg = 0;
    int32_t R = 0;
    int32_t nblocks = 0;
    int32_t* bperm = nullptr;
    int32_t* step_pos = nullptr;
    int32_t* blk_step = nullptr;
    int4* desc_f = nullptr;   // forward row descriptors in block order
    int4* desc_t = nullptr;   // transposed row descriptors in block order
    int4* ldesc_f = nullptr;  // forward row descriptors in level order
    int4* ldesc_t = nullptr;  // transposed row descriptors in level order
    void* xtmp = nullptr;     // n * kmax values
    void* xtmp2 = nullptr;    // n * min(kmax, 64) values (autotuning)
    int32_t kc = 1;           // sync-free right-hand sides per chain
    rwt::Algo fwd = rwt::Algo::SyncFree;
    rwt::Algo bwd = rwt::Algo::SyncFree;
    int32_t lanes = 4;
    int32_t stage_x = 1;      // sync-free: helper waves stage outside x values (1) or not (2)
    int cus = 256;
    double tuned_level = 0, tuned_sf = 0, tuned_walk = 0;
    void* vt = nullptr;                  // values in successor-list order (transposed walk)
    unsigned long long* span = nullptr;  // device word: rounds summed over 64-row chunks
    double chunk_rounds = 0;             // mean rounds the walk needs per 64-row chunk
    bool walk_ok = false;                // the row-order walk suits this matrix
};

namespace rwt {
// forward / transposed solve on a plan (dispatch on the plan's algorithm)
rwt_status plan_solve(const rwt_plan* p, bool transposed, const void* B, int32_t k, int64_t ldb,
                      void* X, int64_t ldx, hipStream_t s);
}  // namespace rwt
