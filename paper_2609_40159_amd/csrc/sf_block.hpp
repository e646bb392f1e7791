// Device building blocks of the sync-free solve, shared by the single-matrix
// and the batched persistent kernels.
#pragma once

#include "common.hpp"

namespace rwt {

// Workgroup barrier that orders LDS only: global stores stay in flight
// (other workgroups read them through the readiness wait).
__device__ __forceinline__ void lds_barrier() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}

// Row of the current level step for one lane group, with its data loaded
// ahead of time (software pipeline: descriptors two steps ahead, entries
// one step ahead), so that only the x values wait on the dependency chain.
struct SfDesc {
    int32_t i, pb, pe, dpos;
    bool act;
};
template <typename T>
struct SfEnt {
    int32_t j;   // first entry of this lane (-1: none)
    T v;
    T diag;
};

// One row block of a sync-free solve: rows [r0, r1) in (level, row) order,
// level by level inside the block, x values of the block in LDS.
struct SfBlockArgs {
    int32_t r0, r1;          // rows of the block
    int32_t sb, ns;          // first step (in step_pos) and number of steps
    int32_t k;               // right-hand sides
    int32_t lanes;           // lanes per row
    int32_t stage_x;         // staged body: helper waves prefetch x values of earlier blocks
    int64_t ldb, ldx;
    const int32_t* colidx;   // forward pattern
    const int32_t* crow;     // successor pattern (transposed solve)
    const int32_t* cmap;
    const void* vals;
    const int4* desc;        // row descriptors in block order
    const int32_t* step_pos;
    const void* B;
    void* X;
    int32_t* err;
    int64_t ticks;
    int32_t lds_rows;        // rows the LDS x area is laid out for
    int32_t hold_row;        // >= 0: never publish this row to X (forces the watchdog path)
};

__host__ __device__ inline int sf_x_bytes(int rows, int k, int s) { return (rows * k * s + 15) & ~15; }

template <typename T, bool TRANS, int KT>
__device__ __forceinline__ void sf_block(const SfBlockArgs& b, unsigned char* s_raw) {
    const int k = b.k;
    const int32_t r0 = b.r0, r1 = b.r1, sb = b.sb, ns = b.ns;
    T* xs = reinterpret_cast<T*>(s_raw);
    int32_t* sp = reinterpret_cast<int32_t*>(s_raw + sf_x_bytes(b.lds_rows, k, (int)sizeof(T)));
    const T* vals = static_cast<const T*>(b.vals);
    const T* Bg = static_cast<const T*>(b.B);
    T* X = static_cast<T*>(b.X);
    const int32_t* idx = TRANS ? b.crow : b.colidx;
    const int G = b.lanes;
    const int gl = threadIdx.x & (G - 1);
    const int lane = lane_id();
    const int groups_per_wave = WAVE / G;
    const int wave_in_block = threadIdx.x / WAVE;
    const int waves_per_block = blockDim.x / WAVE;
    const int32_t ngroups = waves_per_block * groups_per_wave;
    const int32_t gi = wave_in_block * groups_per_wave + lane / G;
    int32_t* err = b.err;
    auto value_at = [&](int32_t p) -> T { return TRANS ? vals[b.cmap[p]] : vals[p]; };

    for (int32_t u = threadIdx.x; u <= ns; u += blockDim.x) sp[u] = b.step_pos[sb + u] - r0;
    // the block's right-hand sides, coalesced, into the LDS x area: a row
    // reads b_i there and overwrites it with x_i (rows of one step never
    // read each other), so no step waits on a global load of B
    {
        const int32_t nr = r1 - r0;
        for (int32_t e = threadIdx.x; e < nr * k; e += blockDim.x) {
            const int32_t q = e / nr, i = e - q * nr;
            xs[i * k + q] = Bg[r0 + i + (int64_t)q * b.ldb];
        }
    }
    __syncthreads();

    // Loads of future steps are issued by every lane unconditionally (an
    // inactive lane reads a valid element and discards it): a load under a
    // branch would let the compiler's wait counting assume nothing younger
    // than the x loads is in flight and wait for everything.
    auto load_desc = [&](int32_t u) -> SfDesc {
        SfDesc d;
        const bool has = u < ns;
        const int32_t st = TRANS ? ns - 1 - u : u;
        const int32_t st_c = has ? st : 0;
        const int32_t pos = sp[st_c] + gi;
        d.act = has && pos < sp[st_c + 1];
        const int4 v = b.desc[d.act ? r0 + pos : 0];
        d.i = d.act ? v.x : r0;
        d.pb = d.act ? v.y : 0;
        d.pe = d.act ? v.z : 0;
        d.dpos = d.act ? v.w : 0;
        return d;
    };
    auto load_ent = [&](const SfDesc& d) -> SfEnt<T> {
        SfEnt<T> e;
        const int32_t p = d.pb + gl;
        const bool ok = d.act && p < d.pe;
        const int32_t pc = ok ? p : 0;
        const int32_t jj = idx[pc];
        int32_t vp = pc;
        if (TRANS) {
            const int32_t m = b.cmap[pc];
            vp = ok ? m : 0;
        }
        const T vv = vals[vp];
        const T dd = vals[d.act ? d.dpos : 0];
        e.j = ok ? jj : -1;
        e.v = ok ? vv : T(0);
        e.diag = d.act ? dd : T(1);
        return e;
    };
    // acc[tt] += v_p * x[j_p, q0 + tt] over this lane's entries p = p_start,
    // p_start + G, ... < pe, in ascending p.  The x values of U entries (and
    // all KT right-hand sides) are loaded together and only then checked, so
    // one memory latency covers them; a value still marked not ready is
    // waited for on its own.
    constexpr int U = 1;   // more entries per round lengthened the common one-entry path
    auto add_entries = [&](int32_t p_start, int32_t pe, int q0, T(&acc)[KT]) {
        for (int32_t p0 = p_start; p0 < pe; p0 += U * G) {
            int32_t jv[U];
            T vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t p = p0 + u * G;
                const bool ok = p < pe;
                const int32_t pc = ok ? p : p0;   // p0 < pe: always a valid entry
                const int32_t jj = idx[pc];
                const T v = value_at(pc);
                jv[u] = ok ? jj : -1;
                vv[u] = ok ? v : T(0);
            }
            T xv[U][KT];
            bool miss = false;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool local = TRANS ? (jv[u] < r1) : (jv[u] >= r0);
#pragma unroll
                for (int tt = 0; tt < KT; ++tt) {
                    xv[u][tt] = T(0);
                    if (jv[u] >= 0 && (KT == 1 || q0 + tt < k))
                        xv[u][tt] = local ? xs[(jv[u] - r0) * k + q0 + tt]
                                          : ld_relaxed(&X[jv[u] + (int64_t)(q0 + tt) * b.ldx]);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int tt = 0; tt < KT; ++tt) miss = miss || (jv[u] >= 0 && is_sentinel(xv[u][tt]));
            if (miss) {
                // rare: poll the values not yet published until all have
                // arrived (bounded by the watchdog; on expiry the error flag
                // is set and the missing values count as zero)
                const int64_t t0 = wall_clock64();
                for (;;) {
                    bool still = false;
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int tt = 0; tt < KT; ++tt)
                            if (jv[u] >= 0 && is_sentinel(xv[u][tt])) {
                                xv[u][tt] = ld_relaxed(&X[jv[u] + (int64_t)(q0 + tt) * b.ldx]);
                                still = still || is_sentinel(xv[u][tt]);
                            }
                    if (!still) break;
                    const bool expired = wall_clock64() - t0 > b.ticks;
                    if (expired)
                        __hip_atomic_store(err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                    if (expired || ld_relaxed(err) != 0) {
#pragma unroll
                        for (int u = 0; u < U; ++u)
#pragma unroll
                            for (int tt = 0; tt < KT; ++tt)
                                if (is_sentinel(xv[u][tt])) xv[u][tt] = T(0);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(0);
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int tt = 0; tt < KT; ++tt)
                    if (jv[u] >= 0 && (KT == 1 || q0 + tt < k)) acc[tt] += vv[u] * xv[u][tt];
        }
    };

    // A row solved without pipelining (rows beyond one per group, right-hand
    // sides beyond the first KT): all lanes of the wave call this together.
    auto solve_inline = [&](const SfDesc& d, const SfEnt<T>& e, int q_begin) {
        for (int q0 = q_begin; q0 < k; q0 += KT) {
            T acc[KT], bq[KT];
#pragma unroll
            for (int tt = 0; tt < KT; ++tt) {
                acc[tt] = T(0);
                bq[tt] = T(0);
                if (d.act && gl == 0 && (KT == 1 || q0 + tt < k)) bq[tt] = xs[(d.i - r0) * k + q0 + tt];
            }
            add_entries(d.pb + gl, d.pe, q0, acc);
#pragma unroll
            for (int tt = 0; tt < KT; ++tt) acc[tt] = group_sum(acc[tt], G);
            if (d.act && gl == 0) {
#pragma unroll
                for (int tt = 0; tt < KT; ++tt) {
                    const int q = q0 + tt;
                    if (KT == 1 || q < k) {
                        T xi = (bq[tt] - acc[tt]) / e.diag;
                        xs[(d.i - r0) * k + q] = xi;
                        if (d.i != b.hold_row) st_relaxed(&X[d.i + (int64_t)q * b.ldx], xi);
                    }
                }
            }
        }
    };

    // Pipelined level loop.  Per step, in this order: (1) load the x
    // values of the row's first entry (and b_i from LDS), (2) publish
    // the previous step's results, (3) load the data of the next steps,
    // (4) wait for (1) only.  Vector-memory counters retire in order, so
    // anything issued after (1) is not waited for by (4).
    SfDesc dc = load_desc(0);
    SfEnt<T> ec = load_ent(dc);
    SfDesc dn = load_desc(1);
    bool pend = false;
    int32_t pend_i = 0;
    T pend_x[KT];
#pragma unroll
    for (int tt = 0; tt < KT; ++tt) pend_x[tt] = T(0);
    for (int32_t u = 0; u < ns; ++u) {
        // (1)
        const bool have = dc.act && ec.j >= 0;
        const bool loc = have && (TRANS ? (ec.j < r1) : (ec.j >= r0));
        T xv[KT], bq[KT];
#pragma unroll
        for (int tt = 0; tt < KT; ++tt) {
            xv[tt] = T(0);
            bq[tt] = T(0);
            if (KT == 1 || tt < k) {
                if (have) xv[tt] = loc ? xs[(ec.j - r0) * k + tt]
                                       : ld_relaxed(&X[ec.j + (int64_t)tt * b.ldx]);
                if (dc.act && gl == 0) bq[tt] = xs[(dc.i - r0) * k + tt];
            }
        }
        // (2)
        if (pend) {
#pragma unroll
            for (int tt = 0; tt < KT; ++tt)
                if ((KT == 1 || tt < k) && pend_i != b.hold_row)
                    st_relaxed(&X[pend_i + (int64_t)tt * b.ldx], pend_x[tt]);
            pend = false;
        }
        // (3)
        const SfDesc dnn = load_desc(u + 2);
        const SfEnt<T> en = load_ent(dn);
        // (4)
        T acc[KT];
#pragma unroll
        for (int tt = 0; tt < KT; ++tt) {
            acc[tt] = T(0);
            if (KT == 1 || tt < k) {
                if (have && !loc && is_sentinel(xv[tt]))
                    xv[tt] = wait_value(&X[ec.j + (int64_t)tt * b.ldx], err, b.ticks);
                if (have) acc[tt] = ec.v * xv[tt];
            }
        }
        add_entries(dc.pb + gl + G, dc.pe, 0, acc);
#pragma unroll
        for (int tt = 0; tt < KT; ++tt) acc[tt] = group_sum(acc[tt], G);
        if (dc.act && gl == 0) {
#pragma unroll
            for (int tt = 0; tt < KT; ++tt) {
                if (KT == 1 || tt < k) {
                    T xi = (bq[tt] - acc[tt]) / ec.diag;
                    xs[(dc.i - r0) * k + tt] = xi;
                    pend_x[tt] = xi;
                }
            }
            pend = true;
            pend_i = dc.i;
        }
        // right-hand sides beyond the first KT of this row
        if (k > KT) solve_inline(dc, ec, KT);
        // rows of this step beyond one per group
        const int32_t st = TRANS ? ns - 1 - u : u;
        const int32_t beg = sp[st], end = sp[st + 1];
        for (int32_t base = beg + ngroups + wave_in_block * groups_per_wave; base < end;
             base += ngroups) {
            const int32_t pos = base + lane / G;
            SfDesc d;
            d.act = pos < end;
            d.i = d.pb = d.pe = d.dpos = 0;
            if (d.act) {
                const int4 v = b.desc[r0 + pos];
                d.i = v.x;
                d.pb = v.y;
                d.pe = v.z;
                d.dpos = v.w;
            }
            solve_inline(d, load_ent(d), 0);
        }
        lds_barrier();
        dc = dn;
        ec = en;
        dn = dnn;
    }
    if (pend) {
#pragma unroll
        for (int tt = 0; tt < KT; ++tt)
            if ((KT == 1 || tt < k) && pend_i != b.hold_row)
                st_relaxed(&X[pend_i + (int64_t)tt * b.ldx], pend_x[tt]);
    }
    __syncthreads();
}

}  // namespace rwt
