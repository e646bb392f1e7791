// Device measurement of the cross-workgroup hand-off that bounds every
// sync-free schedule from below: a value published by one workgroup with a
// relaxed device-scope store and found by another workgroup's relaxed
// device-scope load (the readiness mechanism of the solves).  Two
// workgroups play ping-pong through a slot array; the time of a round trip
// over two is the one-way hand-off.  Every wait is bounded by the wall
// clock, so the kernel always ends.
#include "common.hpp"
#include "prim.hpp"

namespace rwt {
namespace {

__global__ void __launch_bounds__(WAVE) k_handoff(double* slots, int32_t rounds, int64_t ticks,
                                                   int64_t* t_out, int32_t* err) {
    if (threadIdx.x != 0) return;
    const int me = blockIdx.x;   // 0 serves, 1 answers
    const int64_t t0 = wall_clock64();
    for (int32_t i = 0; i < rounds; ++i) {
        double* mine = &slots[2 * i + me];
        double* theirs = &slots[2 * i + 1 - me];
        if (me == 0) __hip_atomic_store(mine, (double)(i + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (__hip_atomic_load(theirs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0.0) {
            if (wall_clock64() - t0 > ticks || __hip_atomic_load(err, __ATOMIC_RELAXED,
                                                                  __HIP_MEMORY_SCOPE_AGENT) != 0) {
                __hip_atomic_store(err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
        }
        if (me == 1) __hip_atomic_store(mine, (double)(i + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (me == 0) *t_out = wall_clock64() - t0;
}

}  // namespace
}  // namespace rwt

using namespace rwt;

extern "C" size_t rwt_probe_handoff_ws(int32_t rounds) {
    return rounds < 1 ? 0 : sizeof(double) * 2 * (size_t)rounds + 256;
}

extern "C" rwt_status rwt_probe_handoff(int32_t rounds, void* d_ws, size_t ws_bytes,
                                        double* h_ns_one_way, rwt_stream_t stream) {
    RWT_REQUIRE(rounds >= 1 && rounds <= (1 << 20) && h_ns_one_way != nullptr, RWT_ERR_INVALID_ARG,
                "rounds must be 1..2^20 and the result pointer non-NULL");
    const size_t need = rwt_probe_handoff_ws(rounds);
    RWT_REQUIRE(d_ws && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "probe workspace must hold %zu bytes", need);
    hipStream_t s = hs(stream);
    char* buf = static_cast<char*>(d_ws);
    const size_t slot_bytes = sizeof(double) * 2 * (size_t)rounds;
    double* slots = reinterpret_cast<double*>(buf);
    int64_t* t_dev = reinterpret_cast<int64_t*>(buf + slot_bytes);
    int32_t* err = reinterpret_cast<int32_t*>(buf + slot_bytes + 8);
    RWT_TRY(fill_u8(buf, (int64_t)need, s));
    // at most 100 ms for the whole exchange
    hipLaunchKernelGGL(k_handoff, dim3(2), dim3(WAVE), 0, s, slots, rounds, watchdog_ticks(100),
                       t_dev, err);
    RWT_LAUNCHED();
    int64_t ticks = 0;
    int32_t herr = 0;
    RWT_HIP(hipMemcpyAsync(&ticks, t_dev, sizeof ticks, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipMemcpyAsync(&herr, err, sizeof herr, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipStreamSynchronize(s));
    RWT_REQUIRE(herr == 0, RWT_ERR_DEADLOCK, "a hand-off did not arrive within 100 ms");
    // wall clock at 100 MHz: 10 ns per tick; one round is two hand-offs
    *h_ns_one_way = (double)ticks * 10.0 / (2.0 * (double)rounds);
    return RWT_OK;
}
