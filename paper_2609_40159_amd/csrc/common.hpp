// Shared host and device helpers of the rwtrsv library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>

#include "../../include/rwtrsv.h"

namespace rwt {

// ---------------------------------------------------------------------------
// host-side error reporting
// ---------------------------------------------------------------------------
void set_error(const char* fmt, ...);
void set_hip_error(hipError_t e, const char* where);

#define RWT_REQUIRE(cond, code, ...)       \
    do {                                   \
        if (!(cond)) {                     \
            ::rwt::set_error(__VA_ARGS__); \
            return (code);                 \
        }                                  \
    } while (0)

#define RWT_HIP(call)                                     \
    do {                                                  \
        hipError_t e_ = (call);                           \
        if (e_ != hipSuccess) {                           \
            ::rwt::set_hip_error(e_, #call);              \
            return RWT_ERR_HIP;                           \
        }                                                 \
    } while (0)

#define RWT_TRY(call)                     \
    do {                                  \
        rwt_status s_ = (call);           \
        if (s_ != RWT_OK) return s_;      \
    } while (0)

// Launch check: a launch error is reported after the kernel call.
#define RWT_LAUNCHED() RWT_HIP(hipGetLastError())

inline hipStream_t hs(rwt_stream_t s) { return reinterpret_cast<hipStream_t>(s); }

// ---------------------------------------------------------------------------
// workspace carving: 256-byte aligned slices of one caller buffer
// ---------------------------------------------------------------------------
struct Carver {
    char* base;
    size_t off = 0;
    explicit Carver(void* b) : base(static_cast<char*>(b)) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    size_t used() const { return (off + 255) & ~size_t(255); }
};

inline size_t dtype_size(rwt_dtype dt) { return dt == RWT_F64 ? 8 : 4; }

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------
constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// number of set bits of mask below this lane
__device__ __forceinline__ int lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Value arithmetic rounded one operation at a time (no contraction into
// fused multiply-adds), so that results follow a fixed rounding order.
template <typename T>
__device__ __forceinline__ T mul_rn(T a, T b) {
#pragma clang fp contract(off)
    return a * b;
}
template <typename T>
__device__ __forceinline__ T sub_rn(T a, T b) {
#pragma clang fp contract(off)
    return a - b;
}
template <typename T>
__device__ __forceinline__ T add_rn(T a, T b) {
#pragma clang fp contract(off)
    return a + b;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const T u = __shfl_xor(v, o);
        v = u < v ? u : v;
    }
    return v;
}

// sum over an aligned group of G lanes (G a power of two <= 64)
template <typename T>
__device__ __forceinline__ T group_sum(T v, int G) {
    for (int o = G / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// agent-scope (device-wide) atomics
// A pointer read from memory (a table of matrices, say) has no known address
// space, so the compiler accesses its data with flat instructions, which
// count against the LDS wait counter too: every LDS wait then also waits
// for the global loads in flight (and the walks and row blocks keep loads in
// flight on purpose). Passed through an opaque value in the global address
// space, every access derived from it becomes a global one.
template <typename T>
__device__ __forceinline__ T* in_global(T* p) {
    __attribute__((address_space(1))) T* g = (__attribute__((address_space(1))) T*)p;
    asm("" : "+v"(g));
    return (T*)g;
}

template <typename T>
__device__ __forceinline__ T ld_relaxed(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_relaxed(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_acquire(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_release(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T fetch_add(T* p, T v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Control block of persistent kernels (device memory, zeroed before use).
struct Ctrl {
    uint32_t bar_count;   // grid barrier arrivals (cumulative)
    uint32_t bar_gen;     // grid barrier generation
    uint32_t ticket;      // work ticket for dynamically scheduled kernels
    int32_t err;          // RWT_OK or RWT_ERR_DEADLOCK
    uint32_t heartbeat;   // progress counter read by waiting workgroups
    int32_t i0, i1, i2;   // kernel-specific scalars
    int64_t l0, l1;
};

// Wait (bounded) until a grid barrier's generation passes gen.  Each poll
// loads the generation and the error flag together (one memory round
// trip: a poll that also waited for the clock and the heartbeat in turn
// took three, which is what a barrier's last waiter pays after the
// release); the clock and the heartbeat (progress elsewhere restarts the
// bound) are read every 16th poll.  False when a wait expired somewhere.
__device__ inline bool wait_generation(Ctrl* c, uint32_t gen, int64_t ticks) {
    int64_t t0 = wall_clock64();
    uint32_t hb = ld_relaxed(&c->heartbeat);
    for (uint32_t polls = 1;; ++polls) {
        const uint32_t g = ld_relaxed(&c->bar_gen);
        const int32_t e = ld_relaxed(&c->err);
        if (g > gen) return true;
        if (e != 0) return false;
        if ((polls & 15u) == 0u) {
            const int64_t now = wall_clock64();
            const uint32_t h2 = ld_relaxed(&c->heartbeat);
            if (h2 != hb) {
                hb = h2;
                t0 = now;
            }
            if (now - t0 > ticks) {
                __hip_atomic_store(&c->err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                return false;
            }
        }
    }
}

// Readiness carried by the value itself: X is pre-filled with a signalling
// NaN payload that no arithmetic result can equal (arithmetic quiets NaNs).
template <typename T> struct Sentinel;
template <> struct Sentinel<double> {
    using U = unsigned long long;
    static constexpr U bits = 0x7FF4DEADBEEF0001ull;
};
template <> struct Sentinel<float> {
    using U = unsigned int;
    static constexpr U bits = 0x7FA0BEEFu;
};

template <typename T>
__device__ __forceinline__ bool is_sentinel(T v) {
    using U = typename Sentinel<T>::U;
    U b;
    __builtin_memcpy(&b, &v, sizeof(U));
    return b == Sentinel<T>::bits;
}

template <typename T>
__device__ __forceinline__ T sentinel_value() {
    using U = typename Sentinel<T>::U;
    U b = Sentinel<T>::bits;
    T v;
    __builtin_memcpy(&v, &b, sizeof(T));
    return v;
}

// Load x[j] written by another workgroup; spin (bounded) until it is ready.
template <typename T>
__device__ __forceinline__ T wait_value(const T* p, int32_t* err, int64_t ticks) {
    using U = typename Sentinel<T>::U;
    const U* pu = reinterpret_cast<const U*>(p);
    U b = ld_relaxed(pu);
    if (b != Sentinel<T>::bits) {
        T v;
        __builtin_memcpy(&v, &b, sizeof(T));
        return v;
    }
    int64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(0);
        b = ld_relaxed(pu);
        if (b != Sentinel<T>::bits) break;
        if (ld_relaxed(err) != 0) {   // another wait already expired: stop waiting
            b = 0;
            break;
        }
        if (wall_clock64() - t0 > ticks) {
            __hip_atomic_store(err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            b = 0;
            break;
        }
    }
    T v;
    __builtin_memcpy(&v, &b, sizeof(T));
    return v;
}

// ---------------------------------------------------------------------------
// launch-shape helpers
// ---------------------------------------------------------------------------
struct DeviceInfo {
    int cus = 256;
    int device = 0;
};
rwt_status device_info(DeviceInfo* out);

inline unsigned blocks_for(size_t work, unsigned per_block, unsigned cap = 1u << 20) {
    size_t b = (work + per_block - 1) / per_block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return static_cast<unsigned>(b);
}

inline int64_t watchdog_ticks(int ms) {
    if (ms <= 0) ms = 5000;
    return static_cast<int64_t>(ms) * 100000;   // 100 MHz wall clock
}

}  // namespace rwt
