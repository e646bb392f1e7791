// Row-order wave walker: one wavefront solves a whole column of a
// triangular system in walk order, 64 rows (a chunk) at a time.
//
// Section 2.1 solves a row once all its dependencies are done; level-set
// and block schedules pay a synchronization per level (a barrier or a
// cross-workgroup hand-off, about 0.6-1.5 us on this part).  On deep,
// thin DAGs -- thousands of levels of a few rows each, dependencies spread
// over hundreds of rows -- a chunk of 64 consecutive rows spans only a few
// levels, so one wave can walk the rows in order and resolve the chunk's
// internal dependencies itself, in a few rounds of register ballots,
// instead of one global synchronization per level:
//   stage   the chunk's entry pointers are loaded two chunks ahead; its
//           contiguous CSR (or successor-list) entries one chunk ahead into
//           registers (coalesced, lane l holding entries l, l + 64, ...),
//           its right-hand sides likewise.  (Copies straight into LDS
//           would need no registers, but the compiler makes every later
//           LDS access wait for such a copy, which exposes a full memory
//           latency per chunk.);
//   flat    the wave turns the value of every staged entry whose dependency
//           lies before the chunk into the product v * x_dep (x from an LDS
//           ring of the last WK_W solved values, older ones from HBM), one
//           entry per lane and round, so a long row does not serialize a
//           lane;
//   sum     each lane adds its row's products in walk order;
//   rounds  a lane whose in-chunk dependencies (a 64-bit mask of lanes)
//           are all solved adds those terms and solves its row; a ballot
//           marks the newly solved rows; repeat until the chunk is done.
// A row's terms are always added in walk order of its dependencies
// (ascending column forward, descending successor row transposed), so
// the result does not depend on the chunking.  A chunk with more entries
// than the stage holds reads them from HBM instead.
//
// Positions: the walk visits position t = 0..n-1; forward t = row,
// transposed t = n-1-row (L^T is solved from the last row up through the
// successor lists).  Every dependency of the row at t has a smaller
// position.  Lane l of chunk c holds position 64c + l.
#pragma once

#include "common.hpp"

namespace rwt {

constexpr int WK_W = 2048;            // ring: the last WK_W solved values (power of 2)
constexpr int WK_ECAP = 960;          // entries staged per chunk (multiple of 64; a chunk
                                      // of rows of about 9 entries holds about 580)

constexpr int WK_U = WK_ECAP / WAVE;  // staged entries per lane

// Entries [0, count) of src (count <= WK_ECAP, the same in every lane) into
// registers: lane l takes entries l, l + 64, ...; slots past count repeat
// the last entry (never used).  Every slot is loaded, so the number of
// loads in flight is fixed and the compiler's waits for the loads issued
// before these stay exact (a variable count makes it wait for all of them);
// with count = 0 the loads read safe[0] instead, which must be readable
// (the value is never used).
template <typename V>
__device__ __forceinline__ void wk_fetch(const V* src, int32_t count, const void* safe,
                                         V (&dst)[WK_U]) {
    const int lane = lane_id();
    count = __builtin_amdgcn_readfirstlane(count);
    const V* s = count > 0 ? src : static_cast<const V*>(safe);
    const int32_t last = count > 0 ? count - 1 : 0;
#pragma unroll
    for (int u = 0; u < WK_U; ++u) dst[u] = s[min(u * WAVE + lane, last)];
}

// Wait for every vector memory access of this wave (vmcnt(0)), as an
// instruction the compiler knows of: its own later waits count from it.
__device__ __forceinline__ void wk_wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// Wave-wide reductions through DPP lane moves (ALU speed) instead of LDS
// shuffles; every lane must be active.  Lanes exchange partners inside
// quads (xor 1, xor 2), then across the two quads of each 8 (half mirror)
// and the two 8s of each 16 (mirror), so every lane of a 16-lane row holds
// the row's total; the four row totals are combined as (r0 + r1) +
// (r2 + r3).  A fixed order: the result is the same in every lane and on
// every run.
template <int CTRL>
__device__ __forceinline__ uint32_t wk_dpp(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ double wk_dpp(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = wk_dpp<CTRL>((uint32_t)b), hi = wk_dpp<CTRL>((uint32_t)(b >> 32));
    return __longlong_as_double((long long)((hi << 32) | lo));
}
template <int CTRL>
__device__ __forceinline__ float wk_dpp(float v) {
    return __uint_as_float(wk_dpp<CTRL>(__float_as_uint(v)));
}
template <int CTRL>
__device__ __forceinline__ uint64_t wk_dpp(uint64_t v) {
    const uint64_t lo = wk_dpp<CTRL>((uint32_t)v), hi = wk_dpp<CTRL>((uint32_t)(v >> 32));
    return (hi << 32) | lo;
}
template <int CTRL>
__device__ __forceinline__ int32_t wk_dpp(int32_t v) {
    return (int32_t)wk_dpp<CTRL>((uint32_t)v);
}
__device__ __forceinline__ uint32_t wk_lane_val(uint32_t v, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ int32_t wk_lane_val(int32_t v, int l) {
    return __builtin_amdgcn_readlane(v, l);
}
__device__ __forceinline__ double wk_lane_val(double v, int l) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint64_t lo = wk_lane_val((uint32_t)b, l), hi = wk_lane_val((uint32_t)(b >> 32), l);
    return __longlong_as_double((long long)((hi << 32) | lo));
}
__device__ __forceinline__ float wk_lane_val(float v, int l) {
    return __uint_as_float(wk_lane_val(__float_as_uint(v), l));
}
__device__ __forceinline__ uint64_t wk_lane_val(uint64_t v, int l) {
    return ((uint64_t)wk_lane_val((uint32_t)(v >> 32), l) << 32) | wk_lane_val((uint32_t)v, l);
}
constexpr int WK_DPP_XOR1 = 0xB1;          // quad_perm [1, 0, 3, 2]
constexpr int WK_DPP_XOR2 = 0x4E;          // quad_perm [2, 3, 0, 1]
constexpr int WK_DPP_HALF_MIRROR = 0x141;  // lane i <-> 7 - i within 8
constexpr int WK_DPP_MIRROR = 0x140;       // lane i <-> 15 - i within 16
template <typename V, typename Op>
__device__ __forceinline__ V wk_reduce(V v, Op op) {
    v = op(v, wk_dpp<WK_DPP_XOR1>(v));
    v = op(v, wk_dpp<WK_DPP_XOR2>(v));
    v = op(v, wk_dpp<WK_DPP_HALF_MIRROR>(v));
    v = op(v, wk_dpp<WK_DPP_MIRROR>(v));
    return op(op(wk_lane_val(v, 0), wk_lane_val(v, 16)), op(wk_lane_val(v, 32), wk_lane_val(v, 48)));
}
template <typename T>
__device__ __forceinline__ T wk_sum(T v) {
    return wk_reduce(v, [](T x, T y) { return x + y; });
}
__device__ __forceinline__ uint64_t wk_or(uint64_t v) {
    return wk_reduce(v, [](uint64_t x, uint64_t y) { return x | y; });
}
__device__ __forceinline__ int32_t wk_max(int32_t v) {
    return wk_reduce(v, [](int32_t x, int32_t y) { return x > y ? x : y; });
}

template <typename T>
struct WkLds {
    T xr[WK_W];                     // x at position t in xr[t & (WK_W - 1)]
    T ev[WK_ECAP];                  // the chunk's values; products for dependencies before it
    int32_t ej[WK_ECAP];            // the chunk's dependency rows
    uint64_t sm[WK_U];              // entry e's bit: forward, its dependency is in the chunk;
                                    // transposed, before it (where a row's second part starts)
    int32_t rp[WAVE + 1];           // entry starts of the chunk's rows, by local row index
};

template <typename T>
__host__ __device__ constexpr int wk_lds_bytes() {
    return (int)((sizeof(WkLds<T>) + 15) & ~size_t(15));
}

struct WkArgs {
    int32_t n;
    const int32_t* ptr;      // forward: rowptr; transposed: successor-list starts
    const int32_t* idx;      // forward: colidx; transposed: successor rows
    const void* vals;        // forward: CSR values; transposed: values in successor order
    const int32_t* rowptr;   // transposed: diagonal positions
    const void* dvals;       // transposed: CSR values (diagonals)
    const void* b;           // one column
    void* x;                 // one column
    int32_t* err;            // set when a chunk cannot finish (a dependency not below its row)
};

// chunk c holds rows [lo, lo + cnt)
struct WkChunk {
    int32_t lo, cnt;
};
template <bool TRANS>
__device__ __forceinline__ WkChunk wk_chunk(int32_t n, int32_t c) {
    const int32_t t0 = c * WAVE;
    const int32_t cnt = min(WAVE, n - t0);
    return WkChunk{TRANS ? n - t0 - cnt : t0, cnt};
}

// entry pointers of a chunk (loaded two chunks ahead)
struct WkPtr {
    int32_t rpv;     // ptr[lo + min(local index of this lane, cnt)]
    int32_t endv;    // ptr[lo + cnt]
    int32_t dpos;    // transposed: position of this lane's diagonal in the CSR
};

// Loads for a chunk past the last are clamped to the last chunk (their
// results are never used): every load is issued unconditionally, so the
// compiler's in-order wait counts stay exact.
template <bool TRANS>
__device__ __forceinline__ WkPtr wk_load_ptr(const WkArgs& a, int32_t c, int32_t nchunks) {
    const int lane = lane_id();
    const WkChunk ch = wk_chunk<TRANS>(a.n, min(c, nchunks - 1));
    WkPtr p;
    p.rpv = a.ptr[ch.lo + min(lane, ch.cnt)];
    p.endv = a.ptr[ch.lo + ch.cnt];
    p.dpos = 0;
    if (TRANS) p.dpos = a.rowptr[ch.lo + max(ch.cnt - 1 - lane, 0) + 1] - 1;
    return p;
}

template <typename T>
struct WkRhs {
    T b, diag;
};
template <typename T, bool TRANS>
__device__ __forceinline__ WkRhs<T> wk_load_rhs(const WkArgs& a, int32_t c, int32_t nchunks,
                                                const WkPtr& p) {
    const int lane = lane_id();
    const WkChunk ch = wk_chunk<TRANS>(a.n, min(c, nchunks - 1));
    const int32_t li = TRANS ? max(ch.cnt - 1 - lane, 0) : min(lane, ch.cnt - 1);
    WkRhs<T> r;
    r.b = static_cast<const T*>(a.b)[ch.lo + li];
    r.diag = TRANS ? static_cast<const T*>(a.dvals)[p.dpos] : T(1);
    return r;
}

// the chunk's entries (at most WK_ECAP) into registers
template <typename T>
struct WkStage {
    int32_t j[WK_U];
    T v[WK_U];
};
template <typename T>
__device__ __forceinline__ void wk_stage_entries(const WkArgs& a, const WkPtr& p, WkStage<T>& st) {
    const int32_t base = wk_lane_val(p.rpv, 0);
    const int32_t cnt = min(p.endv - base, WK_ECAP);
    // a.ptr holds n + 1 >= 2 words: 8 readable bytes for an empty chunk
    wk_fetch<int32_t>(a.idx + base, cnt, a.ptr, st.j);
    wk_fetch<T>(static_cast<const T*>(a.vals) + base, cnt, a.ptr, st.v);
}

constexpr int WK_LONG = 24;
constexpr int WK_KREG = 4;   // in-chunk dependencies a lane keeps in registers for the rounds
constexpr int WK_RWU = 4;    // list entries per lane a level walk requests at once for a rewritten row

// The in-chunk part of a chunk's rows (both walks of values): each row's
// sum of the terms before the chunk is acc, its in-chunk entries are
// forward [split, oe), transposed [eb, split]; dep holds the lanes of its
// in-chunk dependencies (need_dep: only from the first WK_KREG entries,
// the rest are added here).  Returns the row's x, also left in the ring.
template <typename T, bool TRANS, bool STAGED>
__device__ __forceinline__ T wk_rounds(const WkArgs& a, T* xr, const int32_t* ej, const T* ev,
                                       int32_t base, int32_t lo, int32_t cnt, int32_t t0,
                                       int32_t eb, int32_t oe, int32_t split, T acc, uint64_t dep,
                                       bool need_dep, T b_i, T diag) {
    const int lane = lane_id();
    const int32_t n = a.n;
    const int32_t hi = lo + cnt - 1;
    const T* vals = static_cast<const T*>(a.vals);
    auto pos_of = [&](int32_t r) { return TRANS ? n - 1 - r : r; };
    auto lane_of = [&](int32_t r) { return TRANS ? hi - r : r - lo; };
    auto J = [&](int32_t e) -> int32_t { return STAGED ? ej[e] : a.idx[base + e]; };
    auto V = [&](int32_t e) -> T { return STAGED ? ev[e] : vals[base + e]; };
    const bool act = lane < cnt;
    // x = (b - sum) times the diagonal's reciprocal, formed here, off the
    // rounds' dependent chain
    const T rdiag = T(1) / diag;
    // the in-chunk terms: the first WK_KREG of each row in registers, in
    // walk order (value and the lane holding the dependency's x), and the
    // mask of in-chunk dependencies (long rows have it already)
    const int32_t nk = act ? (TRANS ? split - eb + 1 : oe - split) : 0;
    T dv[WK_KREG];
    int32_t dl[WK_KREG];
#pragma unroll
    for (int k = 0; k < WK_KREG; ++k) {
        dv[k] = T(0);
        dl[k] = lane;
        if (k < nk) {
            const int32_t e = TRANS ? split - k : split + k;
            dv[k] = V(e);
            dl[k] = lane_of(J(e)) & (WAVE - 1);
            dep |= 1ull << dl[k];
        }
    }
    if (need_dep)
        for (int32_t k = WK_KREG; k < nk; ++k)
            dep |= 1ull << (lane_of(ej[TRANS ? split - k : split + k]) & (WAVE - 1));
    const bool kused[WK_KREG] = {__ballot(nk > 0) != 0, __ballot(nk > 1) != 0,
                                 __ballot(nk > 2) != 0, __ballot(nk > 3) != 0};
    // rounds: each solves at least the lowest unsolved position of a valid
    // (lower triangular) system, so at most WAVE of them.  The x of an
    // in-chunk dependency comes from its lane (solved in an earlier round);
    // terms past the first WK_KREG from the ring, which then takes each x
    // as it is solved (else once, after the rounds).
    const bool ring_rounds = __ballot(nk > WK_KREG) != 0;
    uint64_t done = __ballot(!act);
    T xi = T(0);
    for (int round = 0; done != ~0ull && round < WAVE; ++round) {
        const bool ready = act && !((done >> lane) & 1ull) && (dep & ~done) == 0;
        T xk[WK_KREG];
#pragma unroll
        for (int k = 0; k < WK_KREG; ++k) xk[k] = kused[k] ? __shfl(xi, dl[k]) : T(0);
        if (ready) {
            T s = acc;
#pragma unroll
            for (int k = 0; k < WK_KREG; ++k)
                if (k < nk) s += dv[k] * xk[k];
            if (nk > WK_KREG) {
                if (!TRANS) {
                    for (int32_t e = split + WK_KREG; e < oe; ++e)
                        s += V(e) * xr[pos_of(J(e)) & (WK_W - 1)];
                } else {
                    for (int32_t e = split - WK_KREG; e >= eb; --e)
                        s += V(e) * xr[pos_of(J(e)) & (WK_W - 1)];
                }
            }
            xi = (b_i - s) * rdiag;
            if (ring_rounds) xr[(t0 + lane) & (WK_W - 1)] = xi;
        }
        if (ring_rounds) asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        done |= __ballot(ready);
    }
    if (!ring_rounds && act) xr[(t0 + lane) & (WK_W - 1)] = xi;
    if (done != ~0ull && lane == 0)   // a dependency on or after its own row
        __hip_atomic_store(a.err, (int32_t)RWT_ERR_INVALID_ARG, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    return xi;
}

// One chunk's rows once the products of the dependencies before the chunk
// are known: each row's sum, then the rounds over the in-chunk
// dependencies.  STAGED: entries from LDS, products already formed; else
// from HBM (a chunk larger than the stage).  A row with more than WK_LONG
// dependencies, and every row of an unstaged chunk, is summed by the whole
// wave (64 entries a step, then a fixed-order reduction); the others by
// their own lane, in walk order.
template <typename T, bool TRANS, bool STAGED>
__device__ __forceinline__ T wk_rows(const WkArgs& a, T* xr, const int32_t* rp, const uint64_t* sm,
                                     const int32_t* ej, const T* ev, int32_t base, int32_t lo,
                                     int32_t cnt, int32_t t0, T b_i, T diag) {
    const int lane = lane_id();
    const int32_t n = a.n;
    const int32_t hi = lo + cnt - 1;
    const T* vals = static_cast<const T*>(a.vals);
    const T* X = static_cast<const T*>(a.x);
    auto pos_of = [&](int32_t r) { return TRANS ? n - 1 - r : r; };
    auto outside = [&](int32_t r) { return TRANS ? r > hi : r < lo; };
    auto lane_of = [&](int32_t r) { return TRANS ? hi - r : r - lo; };
    auto J = [&](int32_t e) -> int32_t { return STAGED ? ej[e] : a.idx[base + e]; };
    auto V = [&](int32_t e) -> T { return STAGED ? ev[e] : vals[base + e]; };
    // a product of a dependency before the chunk: formed already, or now
    auto term = [&](int32_t e, int32_t r) -> T {
        if (STAGED) return ev[e];
        const int32_t t = pos_of(r);
        const T x = t >= t0 + WAVE - WK_W ? xr[t & (WK_W - 1)] : ld_relaxed(&X[r]);
        return vals[base + e] * x;
    };
    const bool act = lane < cnt;
    const int32_t li = TRANS ? cnt - 1 - lane : lane;
    int32_t eb = 0, ee = 0;
    if (act) {
        eb = rp[li];
        ee = rp[li + 1];
    }
    // off-diagonal entries [eb, oe); forward rows end with their diagonal
    const int32_t oe = TRANS ? ee : ee - 1;
    if (act && !TRANS) diag = V(ee - 1);
    T acc = T(0);
    uint64_t dep = 0;
    // the in-chunk entries: forward a suffix [split, oe), transposed a
    // prefix [eb, split]
    int32_t split = TRANS ? eb - 1 : oe;
    const bool coop = act && (!STAGED || oe - eb > WK_LONG);
    for (uint64_t m = __ballot(coop); m != 0; m &= m - 1) {
        const int o = __builtin_ctzll(m);
        const int32_t cb = wk_lane_val(eb, o), ce = wk_lane_val(oe, o);
        T part = T(0);
        uint64_t dm = 0;
        int32_t nout = 0;   // entries outside the chunk (the same in every lane)
        for (int32_t e0 = cb; e0 < ce; e0 += WAVE) {
            const int32_t e = e0 + lane;
            bool out = false;
            if (e < ce) {
                const int32_t r = J(e);
                out = outside(r);
                if (out) part += term(e, r);
                else dm |= 1ull << lane_of(r);
            }
            nout += __builtin_popcountll(__ballot(out));
        }
        part = wk_sum(part);
        dm = wk_or(dm);
        if (lane == o) {
            acc = part;
            dep = dm;
            split = TRANS ? ce - 1 - nout : cb + nout;
        }
    }
    if (STAGED && act && !coop) {
        // where the row's second part starts, from the chunk's entry masks
        // (forward: outside entries [eb, split), in-chunk [split, oe);
        // transposed: in-chunk [eb, split], outside (split, oe))
        int32_t first = oe;
        for (int32_t w = eb >> 6; (w << 6) < oe; ++w) {
            uint64_t m = sm[w];
            if ((w << 6) < eb) m &= ~0ull << (eb & 63);
            if (m != 0) {
                first = min((w << 6) + (int32_t)__builtin_ctzll(m), oe);
                break;
            }
        }
        split = TRANS ? first - 1 : first;
        // the outside terms, four per step with their loads issued together,
        // added in walk order (forward ascending, transposed descending)
        constexpr int U4 = 4;
        if (!TRANS) {
            for (int32_t e0 = eb; e0 < split; e0 += U4) {
                T v[U4];
#pragma unroll
                for (int u = 0; u < U4; ++u) v[u] = ev[min(e0 + u, split - 1)];
#pragma unroll
                for (int u = 0; u < U4; ++u)
                    if (e0 + u < split) acc += v[u];
            }
        } else {
            for (int32_t e0 = oe - 1; e0 > split; e0 -= U4) {
                T v[U4];
#pragma unroll
                for (int u = 0; u < U4; ++u) v[u] = ev[max(e0 - u, split + 1)];
#pragma unroll
                for (int u = 0; u < U4; ++u)
                    if (e0 - u > split) acc += v[u];
            }
        }
    }
    return wk_rounds<T, TRANS, STAGED>(a, xr, ej, ev, base, lo, cnt, t0, eb, oe, split, acc, dep,
                                       STAGED && act && !coop, b_i, diag);
}

// Solve one column: rows in walk order, chunk by chunk.  Every lane of the
// wave calls it.
template <typename T, bool TRANS>
__device__ __forceinline__ void wk_solve(const WkArgs& a, WkLds<T>* L) {
    const int lane = lane_id();
    const int32_t n = a.n;
    if (n <= 0) return;
    const int32_t nchunks = (n + WAVE - 1) / WAVE;
    T* X = static_cast<T*>(a.x);
    WkPtr p_cur = wk_load_ptr<TRANS>(a, 0, nchunks);
    WkPtr p_nxt = wk_load_ptr<TRANS>(a, 1, nchunks);
    WkRhs<T> r_nxt = wk_load_rhs<T, TRANS>(a, 0, nchunks, p_cur);
    WkStage<T> st;
    wk_stage_entries<T>(a, p_cur, st);
    int32_t* ej = L->ej;
    T* ev = L->ev;
    // the previous chunk's solution: stored together with the next chunk's
    // loads, so that the wait for those loads (every load issued a chunk
    // earlier is waited for together) does not wait for a store just issued
    T x_prev = T(0);
    int32_t at_prev = -1;
    for (int32_t c = 0; c < nchunks; ++c) {
        const WkChunk ch = wk_chunk<TRANS>(n, c);
        const int32_t lo = ch.lo, cnt = ch.cnt, hi = lo + cnt - 1;
        const int32_t t0 = c * WAVE;                       // first position of the chunk
        const WkRhs<T> r_cur = r_nxt;
        const int32_t base = wk_lane_val(p_cur.rpv, 0);
        const int32_t E = p_cur.endv - base;
        L->rp[lane] = p_cur.rpv - base;
        if (lane == 0) L->rp[cnt] = E;
        const bool staged = E <= WK_ECAP;
        const int32_t ring_lo = t0 + WAVE - WK_W;
        if (!staged) {
            // the chunk reads its entries from HBM; the staged registers go
            // unused, but the wait below keeps the compiler's count of the
            // loads in flight the same on both paths
            wk_wait_vm();
        } else {
            // the staged entries into LDS, the value of every dependency
            // before the chunk multiplied by its x from the ring on the way;
            // dependencies older than the ring in a second pass (rare: it
            // waits for HBM)
            bool far = false;
            // every slot's ring value read and every slot written, the
            // padding past E included (no reader goes past E): no branches,
            // which would each save and restore the lane mask
            T xv[WK_U];
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                const int32_t e = lane + u * WAVE;
                const int32_t r = e < E ? st.j[u] : (TRANS ? hi : lo);   // padding: in the chunk
                const int32_t t = TRANS ? n - 1 - r : r;
                const T xo = L->xr[t & (WK_W - 1)];
                xv[u] = (t < t0 && t >= ring_lo) ? xo : T(1);
                far = far || t < ring_lo;
            }
            // slice masks: lane u keeps slice u's
            uint64_t smv = 0;
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                const int32_t e = lane + u * WAVE;
                const int32_t t = TRANS ? n - 1 - st.j[u] : st.j[u];
                const uint64_t m = __ballot(e < E && (TRANS ? t < t0 : t >= t0));
                smv = lane == u ? m : smv;
            }
            if (lane < WK_U) L->sm[lane] = smv;
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                const int32_t e = lane + u * WAVE;
                ej[e] = st.j[u];
                ev[e] = st.v[u] * xv[u];
            }
            if (__ballot(far) != 0) {
                for (int32_t e = lane; e < E; e += WAVE) {
                    const int32_t r = ej[e];
                    const int32_t t = TRANS ? n - 1 - r : r;
                    if (t < ring_lo) ev[e] = ev[e] * ld_relaxed(&X[r]);
                }
            }
        }
        // the next chunks' loads (the staging registers are free again) and
        // the previous chunk's store; the rows of a staged chunk wait for
        // none of them.  Pointers and right-hand sides first: the copies at
        // the end of the chunk wait for them (loads complete in order), not
        // for the staged entries.  Past the last chunk the loads repeat it.
        const WkPtr p_n2 = wk_load_ptr<TRANS>(a, c + 2, nchunks);
        r_nxt = wk_load_rhs<T, TRANS>(a, c + 1, nchunks, p_nxt);
        wk_stage_entries<T>(a, p_nxt, st);
        if (at_prev >= 0) X[at_prev] = x_prev;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        T xi;
        if (staged) {
            xi = wk_rows<T, TRANS, true>(a, L->xr, L->rp, L->sm, ej, ev, base, lo, cnt, t0, r_cur.b,
                                         r_cur.diag);
        } else {
            xi = wk_rows<T, TRANS, false>(a, L->xr, L->rp, L->sm, ej, ev, base, lo, cnt, t0, r_cur.b,
                                          r_cur.diag);
            wk_wait_vm();   // its own loads, so that both paths end with the same loads in flight
        }
        // rows contiguous: one coalesced store (issued with the next loads)
        x_prev = xi;
        at_prev = lane < cnt ? (TRANS ? hi - lane : lo + lane) : -1;
        p_cur = p_nxt;
        p_nxt = p_n2;
    }
    if (at_prev >= 0) X[at_prev] = x_prev;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// ---------------------------------------------------------------------------
// The walk of one column split over two waves of a workgroup, pipelined by
// chunk: while wave 1 (the solver) finishes chunk c -- the terms of its
// rows' dependencies in chunk c - 1, then the rounds -- wave 0 (the stager)
// prepares chunk c + 1: stages its entries in LDS, forms the products of
// every dependency older than chunk c and sums them per row.  One workgroup
// barrier per chunk.  A row's entries fall in three runs by the position of
// their dependency: older than the previous chunk, in the previous chunk
// ("late"), in the chunk; forward they come in that order along the row,
// transposed in the reverse one, and each run is added in walk order with
// every product rounded on its own, so the arithmetic is the one-wave
// walk's, bit for bit (a long row's terms outside the chunk are summed by
// the solver in the one-wave walk's single wave-wide pass).  A chunk with
// more entries than the stage is solved by the solver alone from HBM.
// ---------------------------------------------------------------------------
template <typename T>
struct WkLds2 {
    T xr[WK_W];                     // x at position t in xr[t & (WK_W - 1)]
    T ev[2][WK_ECAP];               // per chunk parity: values; products of older dependencies
    int32_t ej[2][WK_ECAP];
    uint64_t m1[2][WK_U];           // forward: dependency late or in the chunk; transposed: before the chunk
    uint64_t m2[2][WK_U];           // forward: in the chunk; transposed: older than the previous chunk
    int32_t rp[2][WAVE + 1];
    T acc[2][WAVE];                 // per lane: its row's sum of older terms (rows up to WK_LONG)
    int32_t b1[2][WAVE], b2[2][WAVE];   // per lane: first entries of the second and third runs
    int32_t base[2], E[2];
};

template <typename T>
__host__ __device__ constexpr int wk2_lds_bytes() {
    return (int)((sizeof(WkLds2<T>) + 15) & ~size_t(15));
}

// first set bit of the per-64-entry masks m at or after entry eb, before oe (else oe)
__device__ __forceinline__ int32_t wk_first_set(const uint64_t* m, int32_t eb, int32_t oe) {
    for (int32_t w = eb >> 6; (w << 6) < oe; ++w) {
        uint64_t v = m[w];
        if ((w << 6) < eb) v &= ~0ull << (eb & 63);
        if (v != 0) return min((w << 6) + (int32_t)__builtin_ctzll(v), oe);
    }
    return oe;
}

template <typename T, bool TRANS>
__device__ __forceinline__ void wk_solve2(const WkArgs& a, WkLds2<T>* L) {
    const int lane = lane_id();
    // wave 0 stages, wave 1 solves; further waves of the workgroup only
    // take part in the barriers
    const int wv = threadIdx.x / WAVE;
    const bool stager = wv == 0, solver = wv == 1;
    const int32_t n = a.n;
    if (n <= 0) return;
    const int32_t nchunks = (n + WAVE - 1) / WAVE;
    T* X = static_cast<T*>(a.x);
    auto pos_of = [&](int32_t r) { return TRANS ? n - 1 - r : r; };
    // stager state: pointers two chunks ahead, entries one ahead
    WkPtr p_cur, p_nxt;
    WkStage<T> st;
    // solver state: right-hand sides one chunk ahead (transposed: their
    // diagonals need the pointers, loaded two chunks ahead)
    WkRhs<T> r_nxt;
    WkPtr q_nxt;
    if (stager) {
        p_cur = wk_load_ptr<TRANS>(a, 0, nchunks);
        p_nxt = wk_load_ptr<TRANS>(a, 1, nchunks);
        wk_stage_entries<T>(a, p_cur, st);
    } else if (solver) {
        const WkPtr q0 = wk_load_ptr<TRANS>(a, 0, nchunks);
        q_nxt = wk_load_ptr<TRANS>(a, 1, nchunks);
        r_nxt = wk_load_rhs<T, TRANS>(a, 0, nchunks, q0);
    }
    // the stager prepares chunk c (older dependencies: before chunk c - 1)
    auto prepare = [&](int32_t c) {
        const int b = c & 1;
        const WkChunk ch = wk_chunk<TRANS>(n, c);
        const int32_t lo = ch.lo, cnt = ch.cnt, hi = lo + cnt - 1;
        const int32_t t0 = c * WAVE;
        const int32_t tl = t0 - WAVE;   // first position of the previous chunk
        const int32_t base = wk_lane_val(p_cur.rpv, 0);
        const int32_t E = p_cur.endv - base;
        L->rp[b][lane] = p_cur.rpv - base;
        if (lane == 0) {
            L->rp[b][cnt] = E;
            L->base[b] = base;
            L->E[b] = E;
        }
        const bool staged = E <= WK_ECAP;
        const int32_t ring_lo = t0 + WAVE - WK_W;
        if (!staged) {
            wk_wait_vm();
        } else {
            bool far = false;
            T xv[WK_U];
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                const int32_t e = lane + u * WAVE;
                const int32_t r = e < E ? st.j[u] : (TRANS ? hi : lo);
                const int32_t t = pos_of(r);
                xv[u] = (t < tl && t >= ring_lo) ? L->xr[t & (WK_W - 1)] : T(1);
                far = far || t < ring_lo;
            }
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                const int32_t e = lane + u * WAVE;
                if (e < E) {
                    L->ej[b][e] = st.j[u];
                    L->ev[b][e] = st.v[u] * xv[u];
                }
            }
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                if (u * WAVE >= E) break;
                const int32_t e = lane + u * WAVE;
                const int32_t t = pos_of(st.j[u]);
                const uint64_t m1 = __ballot(e < E && (TRANS ? t < t0 : t >= tl));
                const uint64_t m2 = __ballot(e < E && (TRANS ? t < tl : t >= t0));
                if (lane == 0) {
                    L->m1[b][u] = m1;
                    L->m2[b][u] = m2;
                }
            }
            if (__ballot(far) != 0) {
                for (int32_t e = lane; e < E; e += WAVE) {
                    const int32_t r = L->ej[b][e];
                    if (pos_of(r) < ring_lo) L->ev[b][e] = L->ev[b][e] * ld_relaxed(&X[r]);
                }
            }
        }
        // the next chunks' loads; nothing below waits for them (the
        // pointers rotate at the end, after the sums)
        const WkPtr p_n2 = wk_load_ptr<TRANS>(a, c + 2, nchunks);
        wk_stage_entries<T>(a, p_nxt, st);
        if (!staged) {
            p_cur = p_nxt;
            p_nxt = p_n2;
            return;
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        // per row: the runs, the sum of the older terms, long rows' masks
        const bool act = lane < cnt;
        const int32_t li = TRANS ? cnt - 1 - lane : lane;
        int32_t eb = 0, ee = 0;
        if (act) {
            eb = L->rp[b][li];
            ee = L->rp[b][li + 1];
        }
        const int32_t oe = TRANS ? ee : ee - 1;
        const int32_t* ej = L->ej[b];
        const T* ev = L->ev[b];
        int32_t b1 = act ? wk_first_set(L->m1[b], eb, oe) : 0;
        int32_t b2 = act ? wk_first_set(L->m2[b], eb, oe) : 0;
        // older run: forward [eb, b1), transposed [b2, oe)
        const int32_t ob = TRANS ? b2 : eb, oe2 = TRANS ? oe : b1;
        T acc = T(0);
        // long rows are summed by the solver in one pass (the one-wave
        // walk's order); the stager only marks their runs
        const bool coop = act && oe - eb > WK_LONG;
        if (act && !coop) {
            constexpr int U4 = 4;
            if (!TRANS) {
                for (int32_t e0 = ob; e0 < oe2; e0 += U4) {
                    T v[U4];
#pragma unroll
                    for (int u = 0; u < U4; ++u) v[u] = ev[min(e0 + u, oe2 - 1)];
#pragma unroll
                    for (int u = 0; u < U4; ++u)
                        if (e0 + u < oe2) acc += v[u];
                }
            } else {
                for (int32_t e0 = oe2 - 1; e0 >= ob; e0 -= U4) {
                    T v[U4];
#pragma unroll
                    for (int u = 0; u < U4; ++u) v[u] = ev[max(e0 - u, ob)];
#pragma unroll
                    for (int u = 0; u < U4; ++u)
                        if (e0 - u >= ob) acc += v[u];
                }
            }
        }
        L->acc[b][lane] = acc;
        L->b1[b][lane] = b1;
        L->b2[b][lane] = b2;
        p_cur = p_nxt;
        p_nxt = p_n2;
    };
    if (stager) prepare(0);
    __syncthreads();
    T x_prev = T(0);
    int32_t at_prev = -1;
    for (int32_t c = 0; c < nchunks; ++c) {
        if (stager) {
            if (c + 1 < nchunks) prepare(c + 1);
        } else if (solver) {
            // the solver finishes chunk c
            const int b = c & 1;
            const WkChunk ch = wk_chunk<TRANS>(n, c);
            const int32_t lo = ch.lo, cnt = ch.cnt, hi = lo + cnt - 1;
            const int32_t t0 = c * WAVE;
            const WkRhs<T> r_cur = r_nxt;
            const int32_t base = L->base[b], E = L->E[b];
            {   // right-hand sides of the next chunk
                const WkPtr q_n2 = wk_load_ptr<TRANS>(a, c + 2, nchunks);
                r_nxt = wk_load_rhs<T, TRANS>(a, c + 1, nchunks, q_nxt);
                q_nxt = q_n2;
            }
            if (at_prev >= 0) X[at_prev] = x_prev;
            T xi;
            if (E > WK_ECAP) {
                xi = wk_rows<T, TRANS, false>(a, L->xr, L->rp[b], nullptr, nullptr, nullptr, base, lo,
                                              cnt, t0, r_cur.b, r_cur.diag);
                wk_wait_vm();
            } else {
                const bool act = lane < cnt;
                const int32_t li = TRANS ? cnt - 1 - lane : lane;
                int32_t eb = 0, ee = 0;
                if (act) {
                    eb = L->rp[b][li];
                    ee = L->rp[b][li + 1];
                }
                const int32_t oe = TRANS ? ee : ee - 1;
                const int32_t* ej = L->ej[b];
                const T* ev = L->ev[b];
                T diag = r_cur.diag;
                if (act && !TRANS) diag = ev[ee - 1];
                T acc = L->acc[b][lane];
                const int32_t b1 = L->b1[b][lane], b2 = L->b2[b][lane];
                uint64_t dep = 0;
                // late run: forward [b1, b2), transposed [b1, b2) added from
                // its end; each product rounded on its own, as the one-wave
                // walk forms it in its flat pass.  Long rows: every term
                // outside the chunk in one wave-wide pass from the row's
                // start, as the one-wave walk sums them.
                const int32_t lb = b1, le = b2;
                const int32_t tl = t0 - WAVE;
                auto lane_of = [&](int32_t r) { return TRANS ? hi - r : r - lo; };
                const bool coop = act && oe - eb > WK_LONG;
                for (uint64_t m = __ballot(coop); m != 0; m &= m - 1) {
                    const int o = __builtin_ctzll(m);
                    const int32_t cb = wk_lane_val(eb, o), ce = wk_lane_val(oe, o);
                    T part = T(0);
                    uint64_t dm = 0;
                    for (int32_t e = cb + lane; e < ce; e += WAVE) {
                        const int32_t r = ej[e];
                        const int32_t t = pos_of(r);
                        if (t < t0) part += t >= tl ? mul_rn(ev[e], L->xr[t & (WK_W - 1)]) : ev[e];
                        else dm |= 1ull << (lane_of(r) & (WAVE - 1));
                    }
                    part = wk_sum(part);
                    dm = wk_or(dm);
                    if (lane == o) {
                        acc = part;
                        dep = dm;
                    }
                }
                if (act && !coop) {
                    if (!TRANS) {
                        for (int32_t e = lb; e < le; ++e)
                            acc += mul_rn(ev[e], L->xr[pos_of(ej[e]) & (WK_W - 1)]);
                    } else {
                        for (int32_t e = le - 1; e >= lb; --e)
                            acc += mul_rn(ev[e], L->xr[pos_of(ej[e]) & (WK_W - 1)]);
                    }
                }
                // in-chunk run: forward [b2, oe), transposed [eb, b1)
                const int32_t split = TRANS ? b1 - 1 : b2;
                xi = wk_rounds<T, TRANS, true>(a, L->xr, ej, ev, base, lo, cnt, t0, eb, oe, split,
                                               acc, dep, act && !coop, r_cur.b, diag);
            }
            x_prev = xi;
            at_prev = lane < cnt ? (TRANS ? hi - lane : lo + lane) : -1;
        }
        __syncthreads();
    }
    if (solver && at_prev >= 0) X[at_prev] = x_prev;
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// ---------------------------------------------------------------------------
// The same walk for the levels of a rewritten matrix L' (Section 2.1: the
// level of a row is 0 without dependencies, else 1 + the largest level of
// its dependencies), for one candidate rewrite set: rows keep L's
// dependencies unless rewritten, in which case their new list comes from
// the batched symbolic rewrite.  Levels are an order-free maximum, so a
// lane's in-chunk dependencies are read straight from its mask of lanes.
// ---------------------------------------------------------------------------
struct WkLvlLds {
    int32_t lr[WK_W];               // level at position t in lr[t & (WK_W - 1)]
    int32_t ej[WK_ECAP];            // the chunk's dependency rows
    int32_t el[WK_ECAP];            // their levels when before the chunk
    uint64_t sm[WK_U];              // entry e's bit: its dependency is in the chunk
    int32_t rp[WAVE + 1];
};

struct WkLvlArgs {
    int32_t n;
    const int32_t* rowptr;       // L
    const int32_t* colidx;
    int32_t* lev;                // per row: before the walk, rewritten rows hold
                                 // (tag << 24) | mark | list offset; after it,
                                 // (tag << 24) | level
    uint32_t tag, mark;
    const int32_t* pat_ptr;      // new dependency lists, by list position: start (diagonal last)
    const int32_t* pat_len;      // and length
    const int32_t* pat;
    int32_t qb;                  // the candidate's first list position (marks hold offsets from it)
    int32_t qmax;                // list positions < qmax (at least 1 entry in pat_ptr, pat_len)
    int32_t* err;
};

// slots of rows marked as rewritten this launch hold their list offset
__device__ __forceinline__ bool wk_marked(int32_t v, uint32_t tag, uint32_t mark) {
    return ((uint32_t)v >> 24) == tag && ((uint32_t)v & mark);
}

__device__ __forceinline__ void wk_levels(const WkLvlArgs& a, WkLvlLds* L) {
    const int lane = lane_id();
    const int32_t n = a.n;
    if (n <= 0) return;
    const int32_t nchunks = (n + WAVE - 1) / WAVE;
    const uint32_t tagbits = a.tag << 24;
    const int32_t lmask = (int32_t)(a.mark - 1u);
    // pointers and rewrite marks two chunks ahead, a rewritten row's list
    // bounds and the entries one chunk ahead; loads past the last chunk are
    // clamped to it (unused), so that every load is issued unconditionally
    struct P {
        int32_t rpv, endv, slot;
    };
    auto load_p = [&](int32_t c) -> P {
        const int32_t lo = min(c, nchunks - 1) * WAVE, cnt = min(WAVE, n - lo);
        P p;
        p.rpv = a.rowptr[lo + min(lane, cnt)];
        p.endv = a.rowptr[lo + cnt];
        p.slot = ld_relaxed(&a.lev[lo + min(lane, cnt - 1)]);
        return p;
    };
    struct Q {
        int32_t nb, ne;   // a rewritten row's new list (diagonal excluded); ne < nb: L's list
    };
    auto load_q = [&](const P& p) -> Q {
        const bool rw = wk_marked(p.slot, a.tag, a.mark);
        const int32_t q = max(min(a.qb + (rw ? (p.slot & lmask) : 0), a.qmax - 1), 0);
        const int32_t nb = a.pat_ptr[q], ne = nb + a.pat_len[q] - 1;
        return rw ? Q{nb, ne} : Q{0, -1};
    };
    int32_t sj[WK_U];   // the chunk's entries, staged in registers
    auto stage = [&](const P& p) {
        const int32_t base = wk_lane_val(p.rpv, 0);
        wk_fetch<int32_t>(a.colidx + base, min(p.endv - base, WK_ECAP), a.rowptr, sj);
    };
    P p_cur = load_p(0), p_nxt = load_p(1);
    Q q_nxt = load_q(p_cur);
    stage(p_cur);
    int32_t* ej = L->ej;
    for (int32_t c = 0; c < nchunks; ++c) {
        const int32_t lo = c * WAVE, cnt = min(WAVE, n - lo);
        const Q q_cur = q_nxt;
        const int32_t base = wk_lane_val(p_cur.rpv, 0);
        const int32_t E = p_cur.endv - base;
        const bool act = lane < cnt;
        const int32_t i = lo + lane;
        auto lvl_out = [&](int32_t r) -> int32_t {
            return r >= lo + WAVE - WK_W ? L->lr[r & (WK_W - 1)]
                                         : (ld_relaxed(&a.lev[r]) & lmask);
        };
        int32_t best = -1;       // largest level of the dependencies before the chunk
        uint64_t dep = 0;        // dependencies in the chunk, by lane
        // rewritten rows take their lists from HBM: the first WK_RWU * WAVE
        // entries of the chunk's first such row are requested now (a fixed
        // number of loads, a dummy address past the list), so that they
        // arrive while the chunk's entries are staged below
        const bool rw = act && q_cur.ne >= q_cur.nb;
        const uint64_t rwm = __ballot(rw);
        int32_t pre[WK_RWU];
        {
            int32_t f_nb = 0, f_ne = 0;
            if (rwm != 0) {
                const int o = __builtin_ctzll(rwm);
                f_nb = wk_lane_val(q_cur.nb, o);
                f_ne = wk_lane_val(q_cur.ne, o);
            }
#pragma unroll
            for (int u = 0; u < WK_RWU; ++u) {
                const int32_t pp = f_nb + u * WAVE + lane;
                pre[u] = *(pp < f_ne ? a.pat + pp : a.pat_ptr);
            }
        }
        L->rp[lane] = p_cur.rpv - base;
        if (lane == 0) L->rp[cnt] = E;
        if (E > WK_ECAP) {
            // the chunk reads its entries from HBM; the staged registers go
            // unused, but the wait keeps the compiler's count of the loads
            // in flight the same on both paths
            wk_wait_vm();
        } else {
            // the staged entries into LDS with the levels of the dependencies
            // before the chunk: ring, then (rare) older ones from HBM in a
            // second pass
            // Every slot is written and every ring slot read, the padding
            // past E included (no reader goes past E): no branches, which
            // would each save and restore the lane mask
            const int32_t ring_lo = lo + WAVE - WK_W;
            bool far = false;
            int32_t rv[WK_U];
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                const int32_t e = lane + u * WAVE;
                rv[u] = e < E ? sj[u] : lo;   // padding: an in-chunk row
                ej[e] = rv[u];
            }
            int32_t lv[WK_U];
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                lv[u] = L->lr[rv[u] & (WK_W - 1)];
                far = far || rv[u] < ring_lo;
            }
#pragma unroll
            for (int u = 0; u < WK_U; ++u)
                L->el[lane + u * WAVE] = (rv[u] < lo && rv[u] >= ring_lo) ? lv[u] : -1;
            // slice masks of in-chunk dependencies: lane u keeps slice u's
            uint64_t smv = 0;
#pragma unroll
            for (int u = 0; u < WK_U; ++u) {
                const uint64_t m = __ballot(lane + u * WAVE < E && rv[u] >= lo);
                smv = lane == u ? m : smv;
            }
            if (lane < WK_U) L->sm[lane] = smv;
            if (__ballot(far) != 0)
                for (int32_t e = lane; e < E; e += WAVE) {
                    const int32_t r = ej[e];
                    if (r < ring_lo) L->el[e] = ld_relaxed(&a.lev[r]) & lmask;
                }
        }
        // the rewritten rows, one at a time by the whole wave: the first
        // one's head from the registers above, the rest WK_RWU * WAVE entries
        // per request (before the next chunk's loads are issued, so that
        // waiting for these does not wait for those)
        for (uint64_t m = rwm; m != 0; m &= m - 1) {
            const int owner = __builtin_ctzll(m);
            const int32_t nb = wk_lane_val(q_cur.nb, owner), ne = wk_lane_val(q_cur.ne, owner);
            const int32_t io = lo + owner;
            int32_t mx = -1;
            uint64_t dm = 0;
            auto take = [&](int32_t pp, int32_t r) {
                if (pp >= ne) return;
                if (r < 0 || r >= io) {
                    __hip_atomic_store(a.err, (int32_t)RWT_ERR_INVALID_ARG, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                    return;
                }
                if (r < lo) mx = max(mx, lvl_out(r));
                else dm |= 1ull << (r - lo);
            };
            int32_t p0 = nb;
            if (m == rwm) {
#pragma unroll
                for (int u = 0; u < WK_RWU; ++u) take(nb + u * WAVE + lane, pre[u]);
                p0 += WK_RWU * WAVE;
            }
            for (; p0 < ne; p0 += WK_RWU * WAVE) {
                int32_t rr[WK_RWU];
#pragma unroll
                for (int u = 0; u < WK_RWU; ++u) {
                    const int32_t pp = p0 + u * WAVE + lane;
                    rr[u] = pp < ne ? a.pat[pp] : -1;
                }
#pragma unroll
                for (int u = 0; u < WK_RWU; ++u) take(p0 + u * WAVE + lane, rr[u]);
            }
            mx = wk_max(mx);
            dm = wk_or(dm);   // OR of the lanes' in-chunk masks
            if (lane == owner) {
                best = mx;
                dep = dm;
            }
        }
        // the next chunks' loads (the staging registers are free again):
        // pointers and list bounds first, since the copies at the end of the
        // chunk wait for them (loads complete in order), then the entries
        const P p_n2 = load_p(c + 2);
        q_nxt = load_q(p_nxt);
        stage(p_nxt);
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        // L's rows: long ones (and every row of an unstaged chunk) by the
        // whole wave, the others by their own lane
        const bool staged = E <= WK_ECAP;
        const int32_t eb = act ? L->rp[lane] : 0, ee = act ? L->rp[lane + 1] - 1 : 0;   // no diagonal
        const bool coop = act && !rw && (!staged || ee - eb > WK_LONG);
        for (uint64_t m = __ballot(coop); m != 0; m &= m - 1) {
            const int o = __builtin_ctzll(m);
            const int32_t cb = wk_lane_val(eb, o), ce = wk_lane_val(ee, o);
            int32_t mx = -1;
            uint64_t dm = 0;
            // (two loops, so that no pointer selects between LDS and HBM)
            if (staged) {
                for (int32_t e = cb + lane; e < ce; e += WAVE) {
                    const int32_t r = ej[e];
                    if (r < lo) mx = max(mx, L->el[e]);
                    else dm |= 1ull << (r - lo);
                }
            } else {
                for (int32_t e = cb + lane; e < ce; e += WAVE) {
                    const int32_t r = a.colidx[base + e];
                    if (r < lo) mx = max(mx, lvl_out(r));
                    else dm |= 1ull << (r - lo);
                }
            }
            mx = wk_max(mx);
            dm = wk_or(dm);
            if (lane == o) {
                best = mx;
                dep = dm;
            }
        }
        if (!staged) wk_wait_vm();   // as in the row walk: the same loads in flight on both paths
        if (act && !rw && !coop) {
            // dependencies before the chunk [eb, split), in it [split, ee)
            int32_t split = ee;
            for (int32_t w = eb >> 6; (w << 6) < ee; ++w) {
                uint64_t m = L->sm[w];
                if ((w << 6) < eb) m &= ~0ull << (eb & 63);
                if (m != 0) {
                    split = min((w << 6) + (int32_t)__builtin_ctzll(m), ee);
                    break;
                }
            }
            constexpr int U4 = 4;
            for (int32_t e0 = eb; e0 < split; e0 += U4) {
                int32_t v[U4];
#pragma unroll
                for (int u = 0; u < U4; ++u) v[u] = L->el[min(e0 + u, split - 1)];
#pragma unroll
                for (int u = 0; u < U4; ++u) best = max(best, v[u]);
            }
            for (int32_t e = split; e < ee; ++e) dep |= 1ull << ((ej[e] - lo) & (WAVE - 1));
        }
        // rounds as in the row walk: the levels of the first WK_KREG in-chunk
        // dependencies from their lanes, any others from the ring
        int32_t dl[WK_KREG];
        uint64_t drest = dep;
#pragma unroll
        for (int k = 0; k < WK_KREG; ++k) {
            dl[k] = drest != 0 ? __builtin_ctzll(drest) : lane;
            drest &= drest - 1;
        }
        const bool kused[WK_KREG] = {__ballot(dep != 0) != 0,
                                     __ballot(__builtin_popcountll(dep) > 1) != 0,
                                     __ballot(__builtin_popcountll(dep) > 2) != 0,
                                     __ballot(__builtin_popcountll(dep) > 3) != 0};
        uint64_t done = __ballot(!act);
        int32_t li = -1;   // level of this lane's row once solved
        for (int round = 0; done != ~0ull && round < WAVE; ++round) {
            const bool ready = act && !((done >> lane) & 1ull) && (dep & ~done) == 0;
            int32_t lk[WK_KREG];
#pragma unroll
            for (int k = 0; k < WK_KREG; ++k) lk[k] = kused[k] ? __shfl(li, dl[k]) : -1;
            if (ready) {
                int32_t mx = best;
#pragma unroll
                // unused slots read -1: their own unsolved lane, or none
                for (int k = 0; k < WK_KREG; ++k) mx = max(mx, lk[k]);
                for (uint64_t d = drest; d != 0; d &= d - 1)
                    mx = max(mx, L->lr[(lo + __builtin_ctzll(d)) & (WK_W - 1)]);
                li = mx + 1;
                L->lr[i & (WK_W - 1)] = li;
            }
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
            done |= __ballot(ready);
        }
        if (done != ~0ull && lane == 0)   // a dependency on or after its own row
            __hip_atomic_store(a.err, (int32_t)RWT_ERR_INVALID_ARG, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
        if (act) st_relaxed(&a.lev[i], (int32_t)(tagbits | (uint32_t)max(li, 0)));
        p_cur = p_nxt;
        p_nxt = p_n2;
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

}  // namespace rwt
