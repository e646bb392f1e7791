// Rewrite-list generator: the environment of Section 4.1 (level table
// updated per move without touching the DAG, relaxed thin-level threshold)
// driven by a fixed policy, with the node choice of Section 4.3 and the
// target selection of Algorithm 1, for many environments (parameter sets)
// over one matrix in one launch.
//
// One wave runs one environment.  The moves of an environment are
// sequential, so the wave keeps the source and target levels' sums in
// registers and uses its 64 lanes only for the searches; three facts keep
// those short:
//   - a level never turns thin again once it is not (only sources lose
//     rows, and a source is thin already), and never becomes a valid source
//     again once it is not; so the next source is the first valid level of
//     one fixed (row count, level) order of all levels, found by a cursor
//     that only moves forward;
//   - while a source is being emptied no level above it loses rows, so the
//     nearest non-empty level p above it is fixed, and the levels between
//     p and the current target stay non-thin: a target that turns thick is
//     replaced by a search that starts just above it;
//   - the lowest level that may still be thin only rises (a cursor), which
//     decides between rejection (a thin level exists beyond max_dist) and
//     the fallback to p (no thin level above at all).
// The result equals taking the fewest-rows source and the nearest thin
// target afresh at every step.
#include "common.hpp"
#include "levtab.hpp"
#include "prim.hpp"
#include "u128.hpp"

#pragma clang fp contract(off)

namespace rwt {
namespace {

constexpr uint8_t GEN_TGT = 1;   // the level received a row
constexpr uint8_t GEN_REJ = 2;   // a step from this level was rejected

struct GenWs {
    int2* ent;          // (row, dependencies) in (level, dependencies, row) order [n]
    int32_t* rows0;     // rows per level [D]
    int64_t* deps0;     // dependencies per level [D]
    uint32_t* keys;
    uint32_t* tkeys;
    int32_t* vals;      // after the last sort: levels 1..D-1 in (rows, level) order
    int32_t* tvals;
    void* rws;
    rwt_gen_params* prm;   // [num_env]
    int64_t* st_cost;      // [num_env * D]
    int64_t* st_deps;
    int32_t* st_rows;
    uint8_t* st_flags;
};

size_t carve_gen(void* base, int32_t n, int32_t D, int32_t ne, GenWs* g) {
    Carver cv(base);
    const size_t nn = n > 0 ? (size_t)n : 1, dd = D > 0 ? (size_t)D : 1;
    const size_t ee = ne > 0 ? (size_t)ne : 1;
    g->ent = cv.take<int2>(nn);
    g->rows0 = cv.take<int32_t>(dd);
    g->deps0 = cv.take<int64_t>(dd);
    g->keys = cv.take<uint32_t>(nn);
    g->tkeys = cv.take<uint32_t>(nn);
    g->vals = cv.take<int32_t>(nn);
    g->tvals = cv.take<int32_t>(nn);
    g->rws = cv.take<char>(radix_ws((int64_t)nn));
    g->prm = cv.take<rwt_gen_params>(ee);
    g->st_cost = cv.take<int64_t>(ee * dd);
    g->st_deps = cv.take<int64_t>(ee * dd);
    g->st_rows = cv.take<int32_t>(ee * dd);
    g->st_flags = cv.take<uint8_t>(ee * dd);
    return cv.used();
}

// per-level rows and dependencies (cost = 2 deps + rows), and the sort keys
// of levels 1..D-1 by row count
__global__ void k_gen_levels(const int32_t* lptr, const int64_t* cost, int32_t D, int32_t* rows0,
                             int64_t* deps0, uint32_t* keys, int32_t* vals) {
    for (int32_t l = blockIdx.x * blockDim.x + threadIdx.x; l < D; l += gridDim.x * blockDim.x) {
        const int32_t r = lptr[l + 1] - lptr[l];
        rows0[l] = r;
        deps0[l] = (cost[l] - r) / 2;
        if (l >= 1) {
            keys[l - 1] = (uint32_t)r;
            vals[l - 1] = l;
        }
    }
}

struct GenArgs {
    const int2* ent;
    const int32_t* lorder;
    const int32_t* lptr;
    const int32_t* rows0;
    const int64_t* cost0;
    const int64_t* deps0;
    const rwt_level_stats* stats;
    const rwt_gen_params* prm;
    int64_t* st_cost;
    int64_t* st_deps;
    int32_t* st_rows;
    uint8_t* st_flags;
    int32_t n, D, cap;
    int32_t* mv_row;
    int32_t* mv_src;
    int32_t* mv_tgt;
    rwt_gen_result* res;
    int64_t* out_cost;
    int32_t* out_rows;
    int64_t* out_deps;
};

// The stop test thin / T0 < thin_stop (double division) is monotone in the
// thin count, which only falls: it holds exactly when thin <= the largest
// k in [0, T0] that passes it (-1 when none does).
__device__ __forceinline__ int32_t thin_stop_count(int32_t T0, double ts) {
    if (T0 <= 0) return -1;
    auto pass = [&](int32_t k) { return (double)k / (double)T0 < ts; };
    if (!pass(0)) return -1;
    int32_t lo = 0, hi = T0;            // pass(lo) holds
    if (pass(hi)) return hi;
    while (hi - lo > 1) {                // pass(hi) fails
        const int32_t mid = lo + (hi - lo) / 2;
        if (pass(mid)) lo = mid;
        else hi = mid;
    }
    return lo;
}

// a value that lane 0 stored earlier, read by lane 0 and given to every lane
template <typename T>
__device__ __forceinline__ T lane0_load(const T* p) {
    T v = T(0);
    if (lane_id() == 0) v = *p;
    if constexpr (sizeof(T) < 4)
        return (T)__shfl((int)v, 0);
    else
        return __shfl(v, 0);
}

__global__ void __launch_bounds__(WAVE) k_gen_env(GenArgs a) {
    const int32_t e = blockIdx.x;
    const int lane = lane_id();
    const int32_t D = a.D;
    const rwt_gen_params prm = a.prm[e];
    int64_t* cost = a.st_cost + (size_t)e * D;
    int64_t* deps = a.st_deps + (size_t)e * D;
    int32_t* rows = a.st_rows + (size_t)e * D;
    uint8_t* flags = a.st_flags + (size_t)e * D;

    // relaxed thin-level threshold of Section 4.1, from the input's ALC and
    // CV, rounded step by step
    double relax = 1.0 - a.stats->cv;
    if (relax < 0.0) relax = 0.0;
    const double scaled = prm.alpha * relax;
    const double factor = 1.0 + scaled;
    const double thr = a.stats->alc * factor;
    const int64_t cb = cost_bound(thr);

    int32_t T0 = 0;
    for (int32_t l = lane; l < D; l += WAVE) {
        const int32_t r = a.rows0[l];
        const int64_t c = a.cost0[l];
        rows[l] = r;
        cost[l] = c;
        deps[l] = a.deps0[l];
        flags[l] = 0;
        T0 += thin_of(r, c, cb) ? 1 : 0;
    }
    T0 = wave_sum(T0);
    const int32_t kstop = thin_stop_count(T0, prm.thin_stop);
    const int32_t maxm = prm.max_moves > 0 && prm.max_moves < a.cap ? prm.max_moves : a.cap;
    int64_t ms = prm.max_steps > 0 ? prm.max_steps : 2 * (int64_t)D;
    if (prm.max_steps <= 0 && ms < 6144) ms = 6144;
    const int32_t maxs = ms > INT32_MAX ? INT32_MAX : (int32_t)ms;

    int32_t moves = 0, steps = 0, rej = 0, thin = T0, stop = RWT_GEN_NO_SOURCE;
    int32_t src = -1, p = 0, cursor = 0, mt = 0, s_end = 0;
    int32_t s_rows = 0;
    int64_t s_cost = 0, s_deps = 0;
    int32_t tc = -1;                  // target: level >= 0, -1 unknown, -2 fallback p
    int32_t t_rows = 0, t_flags = 0;
    int64_t t_cost = 0, t_deps = 0;
    int32_t pf_q = -1;                // table position of the prefetched entry
    int2 pf_en = make_int2(0, 0);
    __syncthreads();
    for (;;) {
        if (thin <= kstop) {
            stop = RWT_GEN_THIN;
            break;
        }
        if (moves >= maxm) {
            stop = RWT_GEN_MOVES;
            break;
        }
        if (steps >= maxs) {
            stop = RWT_GEN_STEPS;
            break;
        }
        if (src < 0) {
            __syncthreads();
            // the next valid source in (row count, level) order
            int32_t found = -1;
            while (cursor < D - 1) {
                const int32_t q = cursor + lane;
                int32_t l = 0;
                bool ok = false;
                if (q < D - 1) {
                    l = a.lorder[q];
                    ok = flags[l] == 0 && thin_of(rows[l], cost[l], cb);
                }
                const uint64_t m = __ballot(ok);
                if (m) {
                    const int f = __builtin_ctzll(m);
                    found = __shfl(l, f);
                    cursor += f;
                    break;
                }
                cursor += WAVE;
            }
            if (found < 0) {
                stop = RWT_GEN_NO_SOURCE;
                break;
            }
            src = found;
            s_rows = lane0_load(&rows[src]);
            s_cost = lane0_load(&cost[src]);
            s_deps = lane0_load(&deps[src]);
            s_end = a.lptr[src + 1];
            // nearest non-empty level above (level 0 never loses rows)
            p = -1;
            for (int32_t base = src - 1; base >= 0 && p < 0; base -= WAVE) {
                const int32_t l = base - lane;
                const uint64_t m = __ballot(l >= 0 && rows[l] > 0);
                if (m) p = base - __builtin_ctzll(m);
            }
            tc = -1;
            if (p == 0) {
                tc = 0;
                t_rows = lane0_load(&rows[0]);
                t_cost = lane0_load(&cost[0]);
                t_deps = lane0_load(&deps[0]);
                t_flags = lane0_load(&flags[0]);
            }
        }
        // next row of the source in (deps, row) order; an index outside the
        // table means the level arrays were not the analysis of L
        const int32_t qn = s_end - s_rows;
        if (qn < 0 || qn >= a.n || p < 0) {
            stop = RWT_GEN_NO_SOURCE;
            break;
        }
        ++steps;
        // the entry was loaded one step ahead while the source stays the
        // same; the load of the next one is in flight during this step
        const int2 en = qn == pf_q ? pf_en : a.ent[qn];
        pf_q = qn + 1 < a.n ? qn + 1 : qn;
        pf_en = a.ent[pf_q];

        // Algorithm 1
        int32_t t = -1;
        if (p == 0) {
            if (thin_of(t_rows, t_cost, cb)) t = 0;
        } else {
            if (tc == -1 || (tc >= 0 && !thin_of(t_rows, t_cost, cb))) {
                const int32_t start = tc == -1 ? p : tc - 1;
                const int32_t lo = src - prm.max_dist > 0 ? src - prm.max_dist : 0;
                __syncthreads();
                int32_t f = -1;
                for (int32_t base = start; base >= lo && f < 0; base -= WAVE) {
                    const int32_t l = base - lane;
                    const uint64_t m = __ballot(l >= lo && thin_of(rows[l], cost[l], cb));
                    if (m) f = base - __builtin_ctzll(m);
                }
                if (f >= 0) {
                    tc = f;
                } else {
                    // none within reach: any thin level further up?
                    bool beyond = false;
                    while (mt < lo) {
                        const int32_t l = mt + lane;
                        const uint64_t m = __ballot(l < lo && thin_of(rows[l], cost[l], cb));
                        if (m) {
                            mt += __builtin_ctzll(m);
                            beyond = true;
                            break;
                        }
                        mt = mt + WAVE < lo ? mt + WAVE : lo;
                    }
                    tc = beyond ? -3 : -2;
                }
                if (tc >= 0 || tc == -2) {
                    const int32_t tl = tc >= 0 ? tc : p;
                    t_rows = lane0_load(&rows[tl]);
                    t_cost = lane0_load(&cost[tl]);
                    t_deps = lane0_load(&deps[tl]);
                    t_flags = lane0_load(&flags[tl]);
                }
            }
            t = tc >= 0 ? tc : (tc == -2 ? p : -1);
        }
        if (t >= 0 && src - t > prm.max_dist) t = -1;
        if (t < 0) {
            if (lane == 0) flags[src] = GEN_REJ;   // a valid source had no flag
            ++rej;
            src = -1;
            continue;
        }

        // the move: state of Section 4.1, the row keeping its original cost
        const int64_t d = en.y, c = 2 * d + 1;
        const int32_t before = (thin_of(s_rows, s_cost, cb) ? 1 : 0) + (thin_of(t_rows, t_cost, cb) ? 1 : 0);
        s_rows -= 1;
        s_cost -= c;
        s_deps -= d;
        t_rows += 1;
        t_cost += c;
        t_deps += d;
        thin += (thin_of(s_rows, s_cost, cb) ? 1 : 0) + (thin_of(t_rows, t_cost, cb) ? 1 : 0) - before;
        if (lane == 0) {
            rows[src] = s_rows;
            cost[src] = s_cost;
            deps[src] = s_deps;
            rows[t] = t_rows;
            cost[t] = t_cost;
            deps[t] = t_deps;
            if (!(t_flags & GEN_TGT)) flags[t] = (uint8_t)(t_flags | GEN_TGT);
            const size_t o = (size_t)e * a.cap + moves;
            a.mv_row[o] = en.x;
            a.mv_src[o] = src;
            a.mv_tgt[o] = t;
        }
        t_flags |= GEN_TGT;
        ++moves;
        if (s_rows == 0) src = -1;
    }

    __syncthreads();
    int32_t ne = 0, th = 0;
    uint64_t s1 = 0;
    U128 s2{0, 0};
    for (int32_t l = lane; l < D; l += WAVE) {
        const int32_t r = rows[l];
        const int64_t c = cost[l];
        if (r > 0) {
            ++ne;
            s1 += (uint64_t)c;
            s2 = u128_add(s2, u128_sq((uint64_t)c));
        }
        th += thin_of(r, c, cb) ? 1 : 0;
        if (a.out_cost) a.out_cost[(size_t)e * D + l] = c;
        if (a.out_rows) a.out_rows[(size_t)e * D + l] = r;
        if (a.out_deps) a.out_deps[(size_t)e * D + l] = deps[l];
    }
    ne = wave_sum(ne);
    th = wave_sum(th);
    s1 = wave_sum(s1);
    s2 = wave_sum128(s2);
    if (lane == 0) {
        rwt_gen_result r;
        r.moves = moves;
        r.steps = steps;
        r.stop = stop;
        r.levels = ne;
        r.thin = th;
        r.thin0 = T0;
        r.rejected = rej;
        r.pad_ = 0;
        r.threshold = thr;
        r.S1 = s1;
        r.S2_lo = s2.lo;
        r.S2_hi = s2.hi;
        r.cv = cv_exact((uint64_t)ne, s1, s2);
        a.res[e] = r;
    }
}

__global__ void k_gen_empty(const rwt_gen_params* prm, int32_t ne, rwt_gen_result* res) {
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    (void)prm;
    rwt_gen_result r{};
    r.stop = RWT_GEN_NO_SOURCE;
    res[e] = r;
}

// --- candidate row sets from the move lists ---------------------------------

struct RsWs {
    int32_t* counts;   // [num_env]
    uint32_t* keys;
    uint32_t* tkeys;
    int32_t* vals;
    int32_t* tvals;
    int32_t* arow;
    int32_t* atgt;
    int32_t* aenv;
    void* sws;
    void* rws;
};

size_t carve_rs(void* base, int32_t ne, int64_t total, RsWs* w) {
    Carver cv(base);
    const size_t ee = ne > 0 ? (size_t)ne : 1, tt = total > 0 ? (size_t)total : 1;
    w->counts = cv.take<int32_t>(ee + 1);
    w->keys = cv.take<uint32_t>(tt);
    w->tkeys = cv.take<uint32_t>(tt);
    w->vals = cv.take<int32_t>(tt);
    w->tvals = cv.take<int32_t>(tt);
    w->arow = cv.take<int32_t>(tt);
    w->atgt = cv.take<int32_t>(tt);
    w->aenv = cv.take<int32_t>(tt);
    w->sws = cv.take<char>(scan_ws((int64_t)ee + 1));
    w->rws = cv.take<char>(radix_ws((int64_t)tt));
    return cv.used();
}

__global__ void k_rs_counts(const rwt_gen_result* res, int32_t ne, int32_t cap, int32_t* counts) {
    const int32_t e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ne) {
        const int32_t m = res[e].moves;
        counts[e] = m < 0 ? 0 : (m > cap ? cap : m);
    }
}

// every slot of the capacity gets a key: moves keep (row, env), unused
// slots sort last (row n, env ne)
__global__ void k_rs_gather(const rwt_gen_result* res, const int32_t* mv_row, const int32_t* mv_tgt,
                            int32_t ne, int32_t cap, int32_t n, uint32_t* keys, int32_t* vals,
                            int32_t* arow, int32_t* atgt, int32_t* aenv) {
    const int64_t total = (int64_t)ne * cap;
    for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < total;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int32_t e = (int32_t)(s / cap), q = (int32_t)(s - (int64_t)e * cap);
        const bool used = q < res[e].moves;
        const int32_t row = used ? mv_row[s] : n;
        keys[s] = (uint32_t)row;
        vals[s] = (int32_t)s;
        arow[s] = row;
        atgt[s] = used ? mv_tgt[s] : 0;
        aenv[s] = used ? e : ne;
    }
}

__global__ void k_rs_envkeys(const int32_t* vals, const int32_t* aenv, int64_t total, uint32_t* keys) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x)
        keys[q] = (uint32_t)aenv[vals[q]];
}

__global__ void k_rs_scatter(const int32_t* vals, const int32_t* arow, const int32_t* atgt,
                             const int32_t* ptr, int32_t ne, int32_t* rows, int32_t* tgts) {
    const int32_t total = ptr[ne];
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int32_t v = vals[q];
        rows[q] = arow[v];
        if (tgts) tgts[q] = atgt[v];
    }
}

rwt_status check_params(const rwt_gen_params* h, int32_t ne) {
    for (int32_t e = 0; e < ne; ++e) {
        const rwt_gen_params& p = h[e];
        RWT_REQUIRE(p.alpha >= 0.0 && p.alpha <= 1e300 && p.thin_stop >= 0.0 &&
                        p.thin_stop <= 1e300 && p.max_dist >= 0 && p.max_moves >= 0 &&
                        p.max_steps >= 0,
                    RWT_ERR_INVALID_ARG, "generator parameters of environment %d are invalid", e);
    }
    return RWT_OK;
}

}  // namespace
}  // namespace rwt

using namespace rwt;

extern "C" rwt_status rwt_generate_ws(int32_t n, int32_t num_levels, int32_t num_env,
                                      size_t* h_bytes) {
    RWT_REQUIRE(h_bytes && n >= 0 && num_levels >= 0 && num_levels <= (n > 0 ? n : 0) &&
                    num_env >= 0,
                RWT_ERR_INVALID_ARG, "bad generator sizes");
    GenWs g;
    *h_bytes = carve_gen(nullptr, n, num_levels, num_env, &g);
    return RWT_OK;
}

extern "C" rwt_status rwt_generate(const rwt_csr* L, const int32_t* d_level,
                                   const int32_t* d_level_ptr, const int64_t* d_cost,
                                   const rwt_level_stats* d_stats, int32_t num_levels,
                                   int32_t num_env, const rwt_gen_params* h_params, int32_t cap,
                                   int32_t* d_mv_row, int32_t* d_mv_src, int32_t* d_mv_tgt,
                                   rwt_gen_result* d_res, int64_t* d_lev_cost,
                                   int32_t* d_lev_rows, int64_t* d_lev_deps, void* d_ws,
                                   size_t ws_bytes, rwt_stream_t stream) {
    RWT_REQUIRE(L != nullptr, RWT_ERR_INVALID_ARG, "NULL matrix");
    const int32_t n = L->n, D = num_levels;
    RWT_REQUIRE(n >= 0 && num_env >= 0 && cap >= 0, RWT_ERR_INVALID_ARG, "negative size");
    RWT_REQUIRE(n == 0 ? D == 0 : (D >= 1 && D <= n), RWT_ERR_INVALID_ARG,
                "num_levels must be the analysis' level count");
    if (num_env == 0) return RWT_OK;
    RWT_REQUIRE(h_params && d_res, RWT_ERR_INVALID_ARG, "NULL parameters or results");
    RWT_REQUIRE(cap == 0 || (d_mv_row && d_mv_src && d_mv_tgt), RWT_ERR_INVALID_ARG,
                "NULL move arrays");
    RWT_REQUIRE(n == 0 || (L->rowptr && d_level && d_level_ptr && d_cost && d_stats),
                RWT_ERR_INVALID_ARG, "NULL analysis arrays");
    RWT_TRY(check_params(h_params, num_env));
    GenWs g;
    const size_t need = carve_gen(nullptr, n, D, num_env, &g);
    RWT_REQUIRE(d_ws && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "generator workspace must hold %zu bytes", need);
    carve_gen(d_ws, n, D, num_env, &g);
    hipStream_t s = hs(stream);
    RWT_HIP(hipMemcpyAsync(g.prm, h_params, sizeof(rwt_gen_params) * (size_t)num_env,
                           hipMemcpyHostToDevice, s));
    if (n == 0) {
        hipLaunchKernelGGL(k_gen_empty, dim3(blocks_for(num_env, 256)), dim3(256), 0, s, g.prm,
                           num_env, d_res);
        RWT_LAUNCHED();
        return RWT_OK;
    }
    RWT_TRY(rows_by_level_and_deps(L->rowptr, d_level, n, D, g.keys, g.vals, g.tkeys, g.tvals,
                                   g.rws, g.ent, s));
    hipLaunchKernelGGL(k_gen_levels, dim3(blocks_for(D, 256, 4096)), dim3(256), 0, s, d_level_ptr,
                       d_cost, D, g.rows0, g.deps0, g.keys, g.vals);
    RWT_LAUNCHED();
    if (D > 1)
        RWT_TRY(radix_sort(g.keys, g.vals, g.tkeys, g.tvals, D - 1, bits_for((uint64_t)n), g.rws, s));
    GenArgs a;
    a.ent = g.ent;
    a.lorder = g.vals;
    a.lptr = d_level_ptr;
    a.rows0 = g.rows0;
    a.cost0 = d_cost;
    a.deps0 = g.deps0;
    a.stats = d_stats;
    a.prm = g.prm;
    a.st_cost = g.st_cost;
    a.st_deps = g.st_deps;
    a.st_rows = g.st_rows;
    a.st_flags = g.st_flags;
    a.n = n;
    a.D = D;
    a.cap = cap;
    a.mv_row = d_mv_row;
    a.mv_src = d_mv_src;
    a.mv_tgt = d_mv_tgt;
    a.res = d_res;
    a.out_cost = d_lev_cost;
    a.out_rows = d_lev_rows;
    a.out_deps = d_lev_deps;
    hipLaunchKernelGGL(k_gen_env, dim3(num_env), dim3(WAVE), 0, s, a);
    RWT_LAUNCHED();
    return RWT_OK;
}

extern "C" rwt_status rwt_gen_rowsets_ws(int32_t num_env, int32_t cap, size_t* h_bytes) {
    RWT_REQUIRE(h_bytes && num_env >= 0 && cap >= 0, RWT_ERR_INVALID_ARG, "bad sizes");
    RWT_REQUIRE((int64_t)num_env * cap < (int64_t(1) << 31), RWT_ERR_TOO_LARGE,
                "num_env * cap must stay below 2^31");
    RsWs w;
    *h_bytes = carve_rs(nullptr, num_env, (int64_t)num_env * cap, &w);
    return RWT_OK;
}

extern "C" rwt_status rwt_gen_rowsets(int32_t n, int32_t num_env, int32_t cap,
                                      const rwt_gen_result* d_res, const int32_t* d_mv_row,
                                      const int32_t* d_mv_tgt, int32_t* d_cand_ptr,
                                      int32_t* d_cand_rows, int32_t* d_cand_targets, void* d_ws,
                                      size_t ws_bytes, rwt_stream_t stream) {
    RWT_REQUIRE(n >= 0 && num_env >= 0 && cap >= 0, RWT_ERR_INVALID_ARG, "negative size");
    RWT_REQUIRE((int64_t)num_env * cap < (int64_t(1) << 31), RWT_ERR_TOO_LARGE,
                "num_env * cap must stay below 2^31");
    RWT_REQUIRE(n < INT32_MAX, RWT_ERR_TOO_LARGE, "n too large");
    if (num_env == 0) return RWT_OK;
    RWT_REQUIRE(d_res && d_cand_ptr, RWT_ERR_INVALID_ARG, "NULL results or offsets");
    RWT_REQUIRE(cap == 0 || (d_mv_row && d_cand_rows && (d_mv_tgt || !d_cand_targets)),
                RWT_ERR_INVALID_ARG, "NULL move or row arrays");
    const int64_t total = (int64_t)num_env * cap;
    RsWs w;
    const size_t need = carve_rs(nullptr, num_env, total, &w);
    RWT_REQUIRE(d_ws && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "row-set workspace must hold %zu bytes", need);
    carve_rs(d_ws, num_env, total, &w);
    hipStream_t s = hs(stream);
    hipLaunchKernelGGL(k_rs_counts, dim3(blocks_for(num_env, 256)), dim3(256), 0, s, d_res, num_env,
                       cap, w.counts);
    RWT_LAUNCHED();
    RWT_TRY(scan_exclusive(w.counts, d_cand_ptr, num_env, w.sws, s));
    if (total == 0) return RWT_OK;
    const unsigned gb = blocks_for(total, 256, 4096);
    hipLaunchKernelGGL(k_rs_gather, dim3(gb), dim3(256), 0, s, d_res, d_mv_row,
                       d_mv_tgt ? d_mv_tgt : d_mv_row, num_env, cap, n, w.keys, w.vals, w.arow,
                       w.atgt, w.aenv);
    RWT_LAUNCHED();
    RWT_TRY(radix_sort(w.keys, w.vals, w.tkeys, w.tvals, total, bits_for((uint64_t)n), w.rws, s));
    hipLaunchKernelGGL(k_rs_envkeys, dim3(gb), dim3(256), 0, s, w.vals, w.aenv, total, w.keys);
    RWT_LAUNCHED();
    RWT_TRY(radix_sort(w.keys, w.vals, w.tkeys, w.tvals, total, bits_for((uint64_t)num_env),
                       w.rws, s));
    hipLaunchKernelGGL(k_rs_scatter, dim3(gb), dim3(256), 0, s, w.vals, w.arow, w.atgt, d_cand_ptr,
                       num_env, d_cand_rows, d_cand_targets);
    RWT_LAUNCHED();
    return RWT_OK;
}
