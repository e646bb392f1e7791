// Level-table helpers shared by the rewrite-list generator and the
// environment step: the thin test, and the rows of a matrix in (level,
// dependencies, row) order -- the node of a source level with the fewest
// dependencies (ties to the lower row) is then the first of its unmoved
// rows in this table.
#pragma once

#include "common.hpp"

namespace rwt {

// ent[q] = (row, dependency count nnz_i - 1) of the q-th row in (level,
// dependencies, row) order, from the CSR row pointers and the level of every
// row (levels below D).  keys/vals/tkeys/tvals [n] and rws (radix_ws(n)
// bytes) are scratch; two stable radix sorts on the stream.
// A level cost c is an integer below 2^32, exact in double, so the thin
// test (double)c < thr holds exactly when c < ceil(thr): the comparison is
// done on integers against that bound.
__device__ __forceinline__ int64_t cost_bound(double thr) {
    if (!(thr > 0.0)) return 0;
    const double b = ceil(thr);
    return b >= 9.0e18 ? INT64_MAX : (int64_t)b;
}

// thin: non-empty and cost below the threshold
__device__ __forceinline__ bool thin_of(int32_t r, int64_t c, int64_t cb) {
    return r > 0 && c < cb;
}

rwt_status rows_by_level_and_deps(const int32_t* rowptr, const int32_t* level, int32_t n,
                                  int32_t D, uint32_t* keys, int32_t* vals, uint32_t* tkeys,
                                  int32_t* tvals, void* rws, int2* ent, hipStream_t s);

}  // namespace rwt
