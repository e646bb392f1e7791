// Exact 128-bit unsigned arithmetic for the sums of squared level costs and
// the correctly rounded CV (host and device).
#pragma once

#include <cmath>
#include <cstdint>

#include <hip/hip_runtime.h>

namespace rwt {

struct U128 {
    uint64_t lo, hi;
};

__host__ __device__ inline U128 u128_add(U128 a, U128 b) {
    U128 r;
    r.lo = a.lo + b.lo;
    r.hi = a.hi + b.hi + (r.lo < a.lo ? 1u : 0u);
    return r;
}

__device__ inline U128 u128_sq(uint64_t v) {
    U128 r;
    r.lo = v * v;
    r.hi = __umul64hi(v, v);
    return r;
}

// D * S2 for D < 2^31 and S2 < 2^97 (fits 128 bits)
__host__ __device__ inline U128 u128_mul_small(U128 a, uint64_t d) {
    // split a.lo into 32-bit halves to get the carry into the high word
    uint64_t lo_lo = (a.lo & 0xffffffffull) * d;
    uint64_t lo_hi = (a.lo >> 32) * d;
    U128 r;
    r.lo = lo_lo + (lo_hi << 32);
    uint64_t carry = (lo_hi >> 32) + (r.lo < lo_lo ? 1u : 0u);
    r.hi = a.hi * d + carry;
    return r;
}

__host__ __device__ inline U128 u128_sq_host(uint64_t v) {
    uint64_t a = v & 0xffffffffull, b = v >> 32;
    uint64_t aa = a * a, ab = a * b, bb = b * b;
    U128 r;
    uint64_t mid = ab << 1;                 // 2ab may carry
    uint64_t mid_carry = ab >> 63;
    r.lo = aa + (mid << 32);
    uint64_t c0 = r.lo < aa ? 1u : 0u;
    r.hi = bb + (mid >> 32) + (mid_carry << 32) + c0;
    return r;
}

__host__ __device__ inline U128 u128_sub(U128 a, U128 b) {
    U128 r;
    r.lo = a.lo - b.lo;
    r.hi = a.hi - b.hi - (a.lo < b.lo ? 1u : 0u);
    return r;
}

// Round-to-nearest-even conversion of a 128-bit integer to double: the top
// 64 bits (with every lower bit folded into a sticky bit 0) are converted
// once, then scaled by a power of two (exact).
__host__ __device__ inline double u128_to_double(U128 v) {
    if (v.hi == 0) return (double)v.lo;
    int s = __builtin_clzll(v.hi);
    uint64_t top, rest;
    if (s == 0) {
        top = v.hi;
        rest = v.lo;
    } else {
        top = (v.hi << s) | (v.lo >> (64 - s));
        rest = v.lo << s;
    }
    if (rest) top |= 1u;
    return ldexp((double)top, 64 - s);
}

// sum over the 64 lanes of a wave
__device__ inline U128 wave_sum128(U128 s) {
    for (int o = 32; o > 0; o >>= 1) {
        U128 u;
        u.lo = __shfl_xor(s.lo, o);
        u.hi = __shfl_xor(s.hi, o);
        s = u128_add(s, u);
    }
    return s;
}

__host__ __device__ inline double cv_exact(uint64_t D, uint64_t S1, U128 S2) {
    if (D <= 1 || S1 == 0) return 0.0;
    U128 a = u128_mul_small(S2, D);
    U128 b = u128_sq_host(S1);
    U128 num = u128_sub(a, b);
    return sqrt(u128_to_double(num)) / (double)S1;
}


}  // namespace rwt
