// Entry -> row map of a slice of at most 256 consecutive CSR rows, for
// workgroups that walk the slice's contiguous entries one per thread.
// s_ptr holds the slice's nr + 1 row starts (global entry positions).
#pragma once

#include "common.hpp"

namespace rwt {

constexpr int ROW_MAP = 4096;   // entries one slice's map holds (one byte each)

// When the slice's entries fit, s_row[p - s_ptr[0]] = local row of entry p
// (a byte: nr <= 256).  Every thread of the workgroup calls it (it ends
// with a barrier); returns whether the map was filled.
__device__ __forceinline__ bool map_rows(const int32_t* s_ptr, int32_t nr, unsigned char* s_row) {
    const int32_t pb = s_ptr[0];
    const bool mapped = s_ptr[nr] - pb <= ROW_MAP;
    if (mapped)
        for (int32_t t = threadIdx.x; t < nr; t += blockDim.x)
            for (int32_t p = s_ptr[t]; p < s_ptr[t + 1]; ++p) s_row[p - pb] = (unsigned char)t;
    __syncthreads();
    return mapped;
}

// local row of entry p (s_ptr[0] <= p < s_ptr[nr]): from the map, else the
// last row whose start is <= p by binary search
__device__ __forceinline__ int row_of(const int32_t* s_ptr, int32_t nr, const unsigned char* s_row,
                                      bool mapped, int32_t p) {
    if (mapped) return s_row[p - s_ptr[0]];
    int lo = 0, hi = nr - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_ptr[mid] <= p) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

}  // namespace rwt
