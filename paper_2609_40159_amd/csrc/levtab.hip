// Rows in (level, dependencies, row) order (see levtab.hpp).
#include "levtab.hpp"

#include "prim.hpp"

namespace rwt {
namespace {

__global__ void k_lt_keys_deps(const int32_t* rowptr, int32_t n, uint32_t* keys, int32_t* vals) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        keys[i] = (uint32_t)(rowptr[i + 1] - rowptr[i] - 1);
        vals[i] = i;
    }
}

__global__ void k_lt_keys_level(const int32_t* level, const int32_t* vals, int32_t n,
                                uint32_t* keys) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x)
        keys[q] = (uint32_t)level[vals[q]];
}

__global__ void k_lt_ent(const int32_t* rowptr, const int32_t* vals, int32_t n, int2* ent) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < n; q += gridDim.x * blockDim.x) {
        const int32_t i = vals[q];
        ent[q] = make_int2(i, rowptr[i + 1] - rowptr[i] - 1);
    }
}

}  // namespace

rwt_status rows_by_level_and_deps(const int32_t* rowptr, const int32_t* level, int32_t n,
                                  int32_t D, uint32_t* keys, int32_t* vals, uint32_t* tkeys,
                                  int32_t* tvals, void* rws, int2* ent, hipStream_t s) {
    if (n <= 0) return RWT_OK;
    const unsigned gb = blocks_for(n, 256, 4096);
    // by dependencies (rows ascending within equal counts), then stably by level
    hipLaunchKernelGGL(k_lt_keys_deps, dim3(gb), dim3(256), 0, s, rowptr, n, keys, vals);
    RWT_LAUNCHED();
    RWT_TRY(radix_sort(keys, vals, tkeys, tvals, n, bits_for((uint64_t)n), rws, s));
    hipLaunchKernelGGL(k_lt_keys_level, dim3(gb), dim3(256), 0, s, level, vals, n, keys);
    RWT_LAUNCHED();
    RWT_TRY(radix_sort(keys, vals, tkeys, tvals, n, bits_for((uint64_t)D), rws, s));
    hipLaunchKernelGGL(k_lt_ent, dim3(gb), dim3(256), 0, s, rowptr, vals, n, ent);
    RWT_LAUNCHED();
    return RWT_OK;
}

}  // namespace rwt
