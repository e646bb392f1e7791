// Device-wide building blocks: prefix sums, stable radix sort, fills.
#pragma once

#include "common.hpp"

namespace rwt {

// Exclusive prefix sum of in[0..n) into out[0..n], out[n] = total.
// in may equal out.  Workspace: scan_ws(n) bytes.
size_t scan_ws(int64_t n);
rwt_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s);
rwt_status scan_exclusive(const int64_t* in, int64_t* out, int64_t n, void* ws, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs by the low key_bits bits of
// the key.  keys/vals hold the input and receive the output; tmp_keys /
// tmp_vals are scratch of the same length.  Workspace: radix_ws(n).
size_t radix_ws(int64_t n);
rwt_status radix_sort(uint32_t* keys, int32_t* vals, uint32_t* tmp_keys, int32_t* tmp_vals,
                      int64_t n, int key_bits, void* ws, hipStream_t s);

// Small fills that are safe inside graph capture (no memset nodes).
rwt_status fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
rwt_status fill_u8(void* p, int64_t bytes, hipStream_t s);   // zero bytes

// ptr[c] = first position q with keys[q] >= c, for c in [0, nseg] (keys
// ascending).  With nseg_dev != nullptr only c <= *nseg_dev is written.
rwt_status segment_starts(const uint32_t* keys, int64_t nkeys, int64_t nseg, int32_t* ptr,
                          const int32_t* nseg_dev, hipStream_t s);

// row index of every stored entry
rwt_status expand_rows(const int32_t* rowptr, int32_t n, int32_t* rowidx, hipStream_t s);

inline int bits_for(uint64_t maxval) {
    int b = 0;
    while (b < 64 && (maxval >> b) != 0) ++b;
    return b < 1 ? 1 : b;
}

}  // namespace rwt
