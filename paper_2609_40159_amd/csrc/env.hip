// Environment step of Sections 4.1-4.5 for many environments over one
// matrix: the caller's policy picks a source level per environment, one
// launch applies every action (node choice of Section 4.3, target of
// Algorithm 1 with the target affinities and the search window), updates
// the level table incrementally and returns the reward of Algorithm 2; a
// second launch writes the observation of Table 1 and the action mask.
//
// One wave serves one environment in the step: the move itself is a
// handful of scalar updates; the 64 lanes are used for the searches (the
// nearest non-empty level above the source, the window of thin levels, a
// scan of the rows that moved into the source).  Everything the reward
// needs is kept incrementally: the exact integer sums of squared level
// costs and row counts (CV after the move without a pass over the levels),
// the thin, non-empty and single-row level counts.  The observation is a
// streaming kernel over levels, one workgroup per environment.
//
// Readings the paper leaves open (constants of the reward, the
// abandonment penalty, affinities, the invalid-action reward) follow the
// documentation of rwt_env_step in rwtrsv.h.
#include "common.hpp"
#include "levtab.hpp"
#include "prim.hpp"
#include "u128.hpp"

#pragma clang fp contract(off)

namespace rwt {
namespace {

constexpr int32_t ENV_MAGIC = 0x52574531;   // set by init; kernels refuse other workspaces

struct EnvMeta {
    int32_t magic, n, D, E, cap, T0, max_steps, ones0;
    double thr, alc, arl, cv0, cvr0;
    int64_t cb;            // thin: cost < cb (cb = ceil(thr), exact for integer costs)
    uint64_t S1;           // sum of level costs (constant)
    uint64_t S2_lo, S2_hi; // initial sum of squared level costs
    uint64_t S2r;          // initial sum of squared row counts
    int32_t done0, pad_;
    rwt_env_params prm;
};

struct EnvHdr {
    int32_t steps, moves, last_src, last_collapse;
    int32_t levels, thin, ones, done;
    uint64_t S2_lo, S2_hi, S2r;
    double cv, cv_rows;
};

struct EnvWs {
    EnvMeta* meta;
    rwt_env_params* prm;   // staging of the host parameters (init)
    int2* ent;          // (row, dependencies) in (level, dependencies, row) order [n]
    int32_t* lptr;      // [D+1]
    int32_t* rows0;     // [D]
    int64_t* cost0;     // [D]
    int64_t* deps0;     // [D]
    uint32_t* keys;     // sort scratch (init only)
    uint32_t* tkeys;
    int32_t* vals;
    int32_t* tvals;
    void* rws;
    EnvHdr* hdr;        // [E]
    int64_t* cost;      // per environment and level [E*D]
    int64_t* deps;
    int32_t* rows;
    int32_t* cursor;    // next unmoved original row of the level (position in ent)
    int32_t* movedin;   // rows on the level that moved in
    int32_t* init;      // initial size (abandonment)
    int32_t* first;     // first-touch step, 0 = none
    int32_t* sstamp;    // step of the last choice as source, 0 = never
    int32_t* tstamp;    // step of the last received row, 0 = never
    uint8_t* tgt;       // the level ever received a row
    int32_t* prow;      // per environment and move [E*cap]: the moved row,
    int32_t* plev;      //   the level it is on now (-1 once it moved again),
    int32_t* pdeps;     //   its dependency count
};

size_t carve_env(void* base, int32_t n, int32_t D, int32_t E, int32_t cap, EnvWs* w) {
    Carver cv(base);
    const size_t nn = n > 0 ? (size_t)n : 1, dd = D > 0 ? (size_t)D : 1;
    const size_t ee = E > 0 ? (size_t)E : 1, cc = cap > 0 ? (size_t)cap : 1;
    w->meta = cv.take<EnvMeta>(1);
    w->prm = cv.take<rwt_env_params>(1);
    w->ent = cv.take<int2>(nn);
    w->lptr = cv.take<int32_t>(dd + 1);
    w->rows0 = cv.take<int32_t>(dd);
    w->cost0 = cv.take<int64_t>(dd);
    w->deps0 = cv.take<int64_t>(dd);
    w->keys = cv.take<uint32_t>(nn);
    w->tkeys = cv.take<uint32_t>(nn);
    w->vals = cv.take<int32_t>(nn);
    w->tvals = cv.take<int32_t>(nn);
    w->rws = cv.take<char>(radix_ws((int64_t)nn));
    w->hdr = cv.take<EnvHdr>(ee);
    w->cost = cv.take<int64_t>(ee * dd);
    w->deps = cv.take<int64_t>(ee * dd);
    w->rows = cv.take<int32_t>(ee * dd);
    w->cursor = cv.take<int32_t>(ee * dd);
    w->movedin = cv.take<int32_t>(ee * dd);
    w->init = cv.take<int32_t>(ee * dd);
    w->first = cv.take<int32_t>(ee * dd);
    w->sstamp = cv.take<int32_t>(ee * dd);
    w->tstamp = cv.take<int32_t>(ee * dd);
    w->tgt = cv.take<uint8_t>(ee * dd);
    w->prow = cv.take<int32_t>(ee * cc);
    w->plev = cv.take<int32_t>(ee * cc);
    w->pdeps = cv.take<int32_t>(ee * cc);
    return cv.used();
}

__device__ __forceinline__ bool meta_ok(const EnvMeta& m, int32_t n, int32_t D, int32_t E,
                                        int32_t cap) {
    return m.magic == ENV_MAGIC && m.n == n && m.D == D && m.E == E && m.cap == cap;
}

// episode end, checked after reset and after every step, in this order
__device__ __forceinline__ int32_t stop_of(const EnvMeta& m, int32_t thin, int32_t moves,
                                           int32_t steps, int32_t levels) {
    if (m.T0 > 0 && (double)thin / (double)m.T0 < m.prm.thin_stop) return RWT_GEN_THIN;
    if (moves >= m.cap) return RWT_GEN_MOVES;
    if (steps >= m.max_steps) return RWT_GEN_STEPS;
    if (levels <= 1) return RWT_GEN_NO_SOURCE;   // level 0 never empties
    return -1;
}

// ---------------------------------------------------------------- init ----

__global__ void k_env_levels(const int32_t* lptr_in, const int64_t* cost, int32_t D,
                             int32_t* lptr, int32_t* rows0, int64_t* cost0, int64_t* deps0) {
    for (int32_t l = blockIdx.x * blockDim.x + threadIdx.x; l <= D; l += gridDim.x * blockDim.x) {
        lptr[l] = lptr_in[l];
        if (l < D) {
            const int32_t r = lptr_in[l + 1] - lptr_in[l];
            rows0[l] = r;
            cost0[l] = cost[l];
            deps0[l] = (cost[l] - r) / 2;
        }
    }
}

// One workgroup of 256: the constants of every environment's initial state.
__global__ void __launch_bounds__(256) k_env_meta(EnvMeta* meta, const rwt_level_stats* st,
                                                  const rwt_env_params* prm, const int32_t* rows0,
                                                  const int64_t* cost0, int32_t n, int32_t D,
                                                  int32_t E, int32_t cap) {
    __shared__ uint64_t s_s1[4], s_s2r[4], s_s2lo[4], s_s2hi[4];
    __shared__ int32_t s_t0[4], s_ones[4];
    const rwt_env_params p = *prm;
    double relax = 1.0 - st->cv;
    if (relax < 0.0) relax = 0.0;
    const double scaled = p.alpha * relax;
    const double factor = 1.0 + scaled;
    const double thr = st->alc * factor;
    const int64_t cb = cost_bound(thr);
    uint64_t s1 = 0, s2r = 0;
    U128 s2{0, 0};
    int32_t t0 = 0, ones = 0;
    for (int32_t l = threadIdx.x; l < D; l += blockDim.x) {
        const int32_t r = rows0[l];
        const int64_t c = cost0[l];
        s1 += (uint64_t)c;
        s2 = u128_add(s2, u128_sq((uint64_t)c));
        s2r += (uint64_t)r * (uint64_t)r;
        t0 += thin_of(r, c, cb) ? 1 : 0;
        ones += (l >= 1 && r == 1) ? 1 : 0;
    }
    s1 = wave_sum(s1);
    s2r = wave_sum(s2r);
    s2 = wave_sum128(s2);
    t0 = wave_sum(t0);
    ones = wave_sum(ones);
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
        s_s1[w] = s1;
        s_s2r[w] = s2r;
        s_s2lo[w] = s2.lo;
        s_s2hi[w] = s2.hi;
        s_t0[w] = t0;
        s_ones[w] = ones;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    EnvMeta m;
    m.magic = ENV_MAGIC;
    m.n = n;
    m.D = D;
    m.E = E;
    m.cap = cap;
    m.T0 = 0;
    m.ones0 = 0;
    m.S1 = 0;
    m.S2r = 0;
    U128 a{0, 0};
    for (int i = 0; i < 4; ++i) {
        m.S1 += s_s1[i];
        m.S2r += s_s2r[i];
        a = u128_add(a, U128{s_s2lo[i], s_s2hi[i]});
        m.T0 += s_t0[i];
        m.ones0 += s_ones[i];
    }
    m.S2_lo = a.lo;
    m.S2_hi = a.hi;
    int64_t ms = 2 * (int64_t)D < 6144 ? 6144 : 2 * (int64_t)D;
    if (ms > INT32_MAX) ms = INT32_MAX;
    m.max_steps = p.max_steps > 0 ? p.max_steps : (int32_t)ms;
    m.thr = thr;
    m.cb = cb;
    m.alc = st->alc;
    m.arl = (double)n / (double)D;
    m.cv0 = cv_exact((uint64_t)D, m.S1, a);
    m.cvr0 = cv_exact((uint64_t)D, (uint64_t)n, U128{m.S2r, 0});
    m.prm = p;
    m.pad_ = 0;
    m.done0 = stop_of(m, m.T0, 0, 0, D);
    *meta = m;
}

// Initial state of the selected environments (all when which is null).
__global__ void __launch_bounds__(256) k_env_reset(EnvWs w, const uint8_t* which, int32_t n,
                                                   int32_t D, int32_t E, int32_t cap) {
    const int32_t e = blockIdx.x;
    if (e >= E || (which && !which[e])) return;
    const EnvMeta& m = *w.meta;
    if (!meta_ok(m, n, D, E, cap)) return;
    const size_t o = (size_t)e * D;
    for (int32_t l = threadIdx.x; l < D; l += blockDim.x) {
        const int32_t r = w.rows0[l];
        w.cost[o + l] = w.cost0[l];
        w.deps[o + l] = w.deps0[l];
        w.rows[o + l] = r;
        w.cursor[o + l] = w.lptr[l];
        w.movedin[o + l] = 0;
        w.init[o + l] = r;
        w.first[o + l] = 0;
        w.sstamp[o + l] = 0;
        w.tstamp[o + l] = 0;
        w.tgt[o + l] = 0;
    }
    if (threadIdx.x == 0) {
        EnvHdr h;
        h.steps = 0;
        h.moves = 0;
        h.last_src = -1;
        h.last_collapse = 0;
        h.levels = D;
        h.thin = m.T0;
        h.ones = m.ones0;
        h.done = m.done0;
        h.S2_lo = m.S2_lo;
        h.S2_hi = m.S2_hi;
        h.S2r = m.S2r;
        h.cv = m.cv0;
        h.cv_rows = m.cvr0;
        w.hdr[e] = h;
    }
}

// ---------------------------------------------------------------- step ----

__device__ __forceinline__ void fill_result(rwt_env_result& r, const EnvHdr& h, const EnvMeta& m) {
    r.done = h.done;
    r.steps = h.steps;
    r.moves = h.moves;
    r.levels = h.levels;
    r.thin = h.thin;
    r.thin0 = m.T0;
    r.cv = h.cv;
    r.cv_rows = h.cv_rows;
}

// One environment's step, run by one wave (no workgroup barrier inside).
__device__ void env_step_body(const EnvWs& w, const int32_t* action, int32_t n, int32_t D,
                              int32_t E, int32_t cap, rwt_env_result* res, int32_t* mv_row,
                              int32_t* mv_src, int32_t* mv_tgt, int32_t e) {
    const int lane = lane_id();
    const EnvMeta m = *w.meta;
    rwt_env_result r{};
    r.node = r.src = r.tgt = -1;
    if (!meta_ok(m, n, D, E, cap)) {
        if (lane == 0) {
            r.outcome = RWT_ENV_ERROR;
            r.done = RWT_GEN_NO_SOURCE;
            res[e] = r;
        }
        return;
    }
    const rwt_env_params& p = m.prm;
    const size_t o = (size_t)e * D, po = (size_t)e * cap;
    int64_t* cost = w.cost + o;
    int64_t* deps = w.deps + o;
    int32_t* rows = w.rows + o;
    EnvHdr h = w.hdr[e];
    if (h.done >= 0) {
        if (lane == 0) {
            r.outcome = RWT_ENV_IGNORED;
            fill_result(r, h, m);
            res[e] = r;
        }
        return;
    }
    const int32_t a = action[e];
    const int32_t step = h.steps + 1;
    const double ra = p.reward_alpha;
    const int64_t cb = m.cb;

    int32_t outcome = RWT_ENV_MOVED, node = -1, nd = 0, from = -1, t = -1;
    if (a < 1 || a >= D || rows[a] <= 0) {
        outcome = RWT_ENV_INVALID;
    } else {
        // node: fewest dependencies, ties to the lower row; the unmoved
        // original rows of the level are a suffix of its table entries, the
        // rows that moved in are found in this environment's move pool
        const int32_t cur = w.cursor[o + a], end = w.lptr[a + 1];
        uint64_t best = ~0ull;
        if (cur >= w.lptr[a] && cur < end) {
            const int2 en = w.ent[cur];
            best = ((uint64_t)(uint32_t)en.y << 32) | (uint32_t)en.x;
        }
        if (w.movedin[o + a] > 0) {
            uint64_t mine = ~0ull;
            int32_t mq = -1;
            const int32_t mv = h.moves < cap ? h.moves : cap;
            for (int32_t q = lane; q < mv; q += WAVE) {
                if (w.plev[po + q] == a) {
                    const uint64_t k = ((uint64_t)(uint32_t)w.pdeps[po + q] << 32) |
                                       (uint32_t)w.prow[po + q];
                    if (k < mine) {
                        mine = k;
                        mq = q;
                    }
                }
            }
            const uint64_t wmin = wave_min(mine);
            const uint64_t hit = __ballot(mine == wmin && mq >= 0);
            if (hit && wmin < best) {
                best = wmin;
                from = __shfl(mq, __builtin_ctzll(hit));
            }
        }
        if (best == ~0ull) {
            outcome = RWT_ENV_ERROR;   // the level's rows were not found: corrupt state
        } else {
            node = (int32_t)(uint32_t)best;
            nd = (int32_t)(best >> 32);
            // Algorithm 1: p = nearest non-empty level above the source
            int32_t pl = -1;
            for (int32_t base = a - 1; base >= 0 && pl < 0; base -= WAVE) {
                const int32_t l = base - lane;
                const uint64_t mk = __ballot(l >= 0 && rows[l] > 0);
                if (mk) pl = base - __builtin_ctzll(mk);
            }
            if (pl < 0) {
                outcome = RWT_ENV_ERROR;
            } else if (pl == 0) {
                t = thin_of(rows[0], cost[0], cb) ? 0 : -1;
            } else {
                // the search_window nearest thin levels at or above p: the
                // one that most recently received a row, ties to the nearest
                int32_t found = 0, bt = -1, bs = -1;
                const int32_t W = p.search_window;
                for (int32_t base = pl; base >= 0 && found < W; base -= WAVE) {
                    const int32_t l = base - lane;
                    const bool th = l >= 0 && thin_of(rows[l], cost[l], cb);
                    const uint64_t mk = __ballot(th);
                    if (!mk) continue;
                    const bool take = th && lanes_below(mk) < W - found;
                    const int64_t key = take ? (((int64_t)w.tstamp[o + l] << 8) | (int64_t)(63 - lane))
                                             : (int64_t)-1;
                    const int64_t km = wave_max(key);
                    const int32_t cs = (int32_t)(km >> 8);
                    const int32_t cl = base - (63 - (int32_t)(km & 0xff));
                    if (bt < 0 || cs > bs) {
                        bt = cl;
                        bs = cs;
                    }
                    const int32_t pc = __popcll(mk);
                    found += pc < W - found ? pc : W - found;
                }
                if (bt >= 0) t = bt;
                else t = thin_of(rows[a], cost[a], cb) ? pl : -1;
            }
            if (t >= 0 && a - t > p.max_dist) t = -1;
            if (outcome == RWT_ENV_MOVED && t < 0) outcome = RWT_ENV_REJECTED;
        }
    }

    if (outcome != RWT_ENV_MOVED) {
        h.steps = step;
        if (outcome != RWT_ENV_ERROR) h.done = stop_of(m, h.thin, h.moves, h.steps, h.levels);
        else h.done = RWT_GEN_NO_SOURCE;
        if (lane == 0) {
            r.outcome = outcome;
            if (outcome == RWT_ENV_REJECTED) {
                r.node = node;
                r.src = a;
            }
            r.reward = -ra;
            fill_result(r, h, m);
            res[e] = r;
            w.hdr[e] = h;
        }
        return;
    }

    // the move, on values every lane holds
    const int32_t rs = rows[a], rt = rows[t];
    const int64_t cs = cost[a], ct = cost[t], ds = deps[a], dt = deps[t];
    const bool src_thin = thin_of(rs, cs, cb);
    const double cv_before = h.cv;

    // abandonment of the previous source, on the state before the move
    double r_ab = 0.0;
    const int32_t A = h.last_src;
    bool reset_A = false;
    if (A >= 1 && A != a) {
        const int32_t rA = rows[A];
        if (w.tgt[o + A]) {
            reset_A = true;
        } else if (rA > 0) {
            if (!(h.ones > 0 && thin_of(rA, cost[A], cb))) {
                const double q = (double)rA / ((double)w.init[o + A] + 1.0);
                const double c = 1.0 - q;
                const double pen = (1.0 - c) * log1p((double)(step - w.first[o + A]));
                r_ab = -pen;
            }
        }
    }

    const int64_t wgt = 2 * (int64_t)nd + 1;
    const int32_t rs1 = rs - 1, rt1 = rt + 1;
    const int64_t cs1 = cs - wgt, ct1 = ct + wgt;
    h.thin += (thin_of(rs1, cs1, cb) ? 1 : 0) + (thin_of(rt1, ct1, cb) ? 1 : 0) -
              (src_thin ? 1 : 0) - (thin_of(rt, ct, cb) ? 1 : 0);
    h.ones += (rs1 == 1 ? 1 : 0) - (rs == 1 ? 1 : 0);
    if (t >= 1) h.ones += (rt1 == 1 ? 1 : 0) - (rt == 1 ? 1 : 0);
    U128 s2{h.S2_lo, h.S2_hi};
    s2 = u128_add(s2, u128_sq((uint64_t)cs1));
    s2 = u128_add(s2, u128_sq((uint64_t)ct1));
    s2 = u128_sub(s2, u128_sq((uint64_t)cs));
    s2 = u128_sub(s2, u128_sq((uint64_t)ct));
    h.S2_lo = s2.lo;
    h.S2_hi = s2.hi;
    h.S2r = h.S2r + (uint64_t)rs1 * (uint64_t)rs1 + (uint64_t)rt1 * (uint64_t)rt1 -
            (uint64_t)rs * (uint64_t)rs - (uint64_t)rt * (uint64_t)rt;
    const bool collapsed = rs1 == 0;
    if (collapsed) {
        h.levels -= 1;
        h.last_collapse = step;
    }
    h.cv = cv_exact((uint64_t)h.levels, m.S1, s2);
    h.cv_rows = cv_exact((uint64_t)h.levels, (uint64_t)n, U128{h.S2r, 0});
    const int32_t q = h.moves;
    h.moves += 1;
    h.steps = step;
    h.last_src = a;
    h.done = stop_of(m, h.thin, h.moves, h.steps, h.levels);

    // reward (Algorithm 2)
    const double D0 = (double)D;
    const double dcv = cv_before - h.cv;
    double r_cv = 0.0;
    if (dcv < -p.eps) r_cv = -ra;
    else if (dcv > p.eps) r_cv = D0 * dcv;
    const double s = log(1.0 + (double)rs + 1.0);
    double r_cp;
    if (collapsed) r_cp = ra * (D0 / (double)h.levels) * (1.0 + 1.0 / s);
    else if (src_thin) r_cp = ra / s;
    else r_cp = -1.0 * ra * (1.0 + s);
    const int32_t dist = a - t, thd = p.dist_threshold;
    double r_rw;
    if (dist < thd) r_rw = log1p((double)(thd - dist)) / D0;
    else r_rw = -log1p((double)(dist - thd)) / D0;
    const double w1 = 0.80 * r_cv, w2 = 0.80 * r_cp, w3 = 0.05 * r_rw, w4 = 0.50 * r_ab;
    double sum = w1 + w2;
    sum = sum + w3;

    if (lane == 0) {
        if (reset_A) {
            w.init[o + A] = rows[A];
            w.first[o + A] = 0;
        }
        rows[a] = rs1;
        cost[a] = cs1;
        deps[a] = ds - nd;
        rows[t] = rt1;
        cost[t] = ct1;
        deps[t] = dt + nd;
        w.tgt[o + t] = 1;
        w.tstamp[o + t] = step;
        w.sstamp[o + a] = step;
        if (w.first[o + a] == 0) w.first[o + a] = step;
        if (from >= 0) {
            w.plev[po + from] = -1;
            w.movedin[o + a] -= 1;
        } else {
            w.cursor[o + a] += 1;
        }
        w.movedin[o + t] += 1;
        // q < cap: a full pool ends the episode (MOVES) before another move
        w.prow[po + q] = node;
        w.plev[po + q] = t;
        w.pdeps[po + q] = nd;
        mv_row[po + q] = node;
        mv_src[po + q] = a;
        mv_tgt[po + q] = t;
        r.outcome = RWT_ENV_MOVED;
        r.node = node;
        r.src = a;
        r.tgt = t;
        r.collapsed = collapsed ? 1 : 0;
        r.reward = sum + w4;
        r.r_cv = r_cv;
        r.r_cp = r_cp;
        r.r_rwdist = r_rw;
        r.r_abandon = r_ab;
        fill_result(r, h, m);
        res[e] = r;
        w.hdr[e] = h;
    }
}

// ------------------------------------------------------------- observe ----

template <typename T>
__device__ __forceinline__ T block_max256(T v, T* sm) {
    v = wave_max(v);
    __syncthreads();
    if (lane_id() == 0) sm[threadIdx.x / WAVE] = v;
    __syncthreads();
    T r = sm[0];
    for (int i = 1; i < 4; ++i) r = sm[i] > r ? sm[i] : r;
    return r;
}

// One environment's observation and mask, run by a whole workgroup of 256
// (its early returns depend only on values uniform over the workgroup).
__device__ void env_observe_body(const EnvWs& w, int32_t n, int32_t D, int32_t E, int32_t cap,
                                 float* obs_level, float* obs_global, uint8_t* mask, int32_t e,
                                 int64_t* s_red) {
    const EnvMeta m = *w.meta;
    if (!meta_ok(m, n, D, E, cap)) return;
    const rwt_env_params& p = m.prm;
    const EnvHdr h = w.hdr[e];
    const size_t o = (size_t)e * D;
    const int64_t cb = m.cb;
    if (obs_level) {
        float* f = obs_level + (size_t)e * 6 * D;
        for (int32_t l = threadIdx.x; l < D; l += blockDim.x) {
            const int32_t r = w.rows[o + l];
            const int64_t c = w.cost[o + l];
            const bool empty = r == 0, th = thin_of(r, c, cb);
            const int32_t ss = w.sstamp[o + l], ts = w.tstamp[o + l];
            double sa, ta;
            if (empty || w.tgt[o + l]) sa = -1.0;
            else if (ss == 0) sa = 0.0;
            else sa = pow(p.decay, (double)(h.steps - ss));
            if (!th) ta = -1.0;
            else if (ts == 0) ta = 0.0;
            else ta = pow(p.decay, (double)(h.steps - ts));
            const double qq = (double)r / ((double)w.init[o + l] + 1.0);
            f[0 * (size_t)D + l] = (float)((double)c / m.alc);
            f[1 * (size_t)D + l] = (float)((double)r / m.arl);
            f[2 * (size_t)D + l] = (float)sa;
            f[3 * (size_t)D + l] = (float)ta;
            f[4 * (size_t)D + l] = (float)(1.0 - qq);
            f[5 * (size_t)D + l] = th ? 1.0f : 0.0f;
        }
    }
    if (obs_global && threadIdx.x == 0) {
        float* g = obs_global + (size_t)e * 9;
        g[0] = (float)h.cv;
        g[1] = 1.0f;
        g[2] = (float)h.cv_rows;
        g[3] = 1.0f;
        g[4] = (float)((double)h.levels / (double)n);
        g[5] = (float)((double)h.moves / (double)n);
        g[6] = (float)(m.T0 > 0 ? (double)h.thin / (double)m.T0 : 0.0);
        g[7] = (float)((double)h.levels / (double)D);
        g[8] = (float)(h.levels > 0 ? (double)h.thin / (double)h.levels : 0.0);
    }
    if (!mask) return;
    uint8_t* mk = mask + o;
    const bool running = h.done < 0;
    const bool forced = running && h.last_src >= 1 && h.last_src < D && w.rows[o + h.last_src] == 1;
    const bool stalled = running && !forced && p.stall_steps > 0 &&
                         h.steps - h.last_collapse >= p.stall_steps;
    for (int32_t l = threadIdx.x; l < D; l += blockDim.x) {
        bool v = running && l >= 1 && w.rows[o + l] > 0;
        if (forced) v = l == h.last_src;
        if (stalled) v = false;
        mk[l] = v ? 1 : 0;
    }
    if (!stalled) return;
    // keep_top valid levels by source affinity: key = -1 for levels that
    // received rows, else the source stamp; ties to the lower level.  Keys
    // are made distinct by the level, so round j takes the largest key
    // below round j-1's.
    int64_t last = INT64_MAX;
    for (int32_t j = 0; j < p.keep_top; ++j) {
        int64_t bestk = -1;
        for (int32_t l = threadIdx.x; l < D; l += blockDim.x) {
            if (l < 1 || w.rows[o + l] <= 0) continue;
            const int64_t key = w.tgt[o + l] ? 0 : (int64_t)w.sstamp[o + l] + 1;
            const int64_t k = (key << 32) | (int64_t)(uint32_t)(D - 1 - l);
            if (k < last && k > bestk) bestk = k;
        }
        bestk = block_max256(bestk, s_red);
        if (bestk < 0) break;
        if (threadIdx.x == 0) mk[D - 1 - (int32_t)(bestk & 0xffffffff)] = 1;
        last = bestk;
    }
}

__global__ void __launch_bounds__(WAVE) k_env_step(EnvWs w, const int32_t* action, int32_t n,
                                                   int32_t D, int32_t E, int32_t cap,
                                                   rwt_env_result* res, int32_t* mv_row,
                                                   int32_t* mv_src, int32_t* mv_tgt) {
    env_step_body(w, action, n, D, E, cap, res, mv_row, mv_src, mv_tgt, blockIdx.x);
}

__global__ void __launch_bounds__(256) k_env_observe(EnvWs w, int32_t n, int32_t D, int32_t E,
                                                     int32_t cap, float* obs_level,
                                                     float* obs_global, uint8_t* mask) {
    __shared__ int64_t s_red[4];
    env_observe_body(w, n, D, E, cap, obs_level, obs_global, mask, blockIdx.x, s_red);
}

// The step by the first wave, then the observation of the new state by the
// whole workgroup: the barrier makes the step's writes visible to it.
__global__ void __launch_bounds__(256) k_env_step_observe(EnvWs w, const int32_t* action,
                                                          int32_t n, int32_t D, int32_t E,
                                                          int32_t cap, rwt_env_result* res,
                                                          int32_t* mv_row, int32_t* mv_src,
                                                          int32_t* mv_tgt, float* obs_level,
                                                          float* obs_global, uint8_t* mask) {
    __shared__ int64_t s_red[4];
    if (threadIdx.x < WAVE)
        env_step_body(w, action, n, D, E, cap, res, mv_row, mv_src, mv_tgt, blockIdx.x);
    __syncthreads();
    env_observe_body(w, n, D, E, cap, obs_level, obs_global, mask, blockIdx.x, s_red);
}

__global__ void k_env_read(EnvWs w, int32_t n, int32_t D, int32_t E, int32_t cap, int64_t* cost,
                           int32_t* rows, int64_t* deps) {
    const size_t total = (size_t)E * D;
    if (!meta_ok(*w.meta, n, D, E, cap)) return;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < total;
         q += (size_t)gridDim.x * blockDim.x) {
        if (cost) cost[q] = w.cost[q];
        if (rows) rows[q] = w.rows[q];
        if (deps) deps[q] = w.deps[q];
    }
}

rwt_status check_sizes(int32_t n, int32_t D, int32_t E, int32_t cap) {
    RWT_REQUIRE(n >= 1 && D >= 1 && D <= n && E >= 1 && cap >= 1, RWT_ERR_INVALID_ARG,
                "environment sizes: need n >= 1, 1 <= num_levels <= n, num_env >= 1, cap >= 1");
    RWT_REQUIRE((int64_t)E * D < (int64_t(1) << 40) && (int64_t)E * cap < (int64_t(1) << 40),
                RWT_ERR_TOO_LARGE, "num_env * num_levels and num_env * cap must stay below 2^40");
    return RWT_OK;
}

rwt_status check_ws(int32_t n, int32_t D, int32_t E, int32_t cap, const void* d_ws, size_t bytes,
                    EnvWs* w) {
    RWT_TRY(check_sizes(n, D, E, cap));
    const size_t need = carve_env(nullptr, n, D, E, cap, w);
    RWT_REQUIRE(d_ws && bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "environment workspace must hold %zu bytes", need);
    carve_env(const_cast<void*>(d_ws), n, D, E, cap, w);
    return RWT_OK;
}

}  // namespace
}  // namespace rwt

using namespace rwt;

extern "C" rwt_status rwt_env_ws(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                                 size_t* h_bytes) {
    RWT_REQUIRE(h_bytes != nullptr, RWT_ERR_INVALID_ARG, "NULL size pointer");
    RWT_TRY(check_sizes(n, num_levels, num_env, cap));
    EnvWs w;
    *h_bytes = carve_env(nullptr, n, num_levels, num_env, cap, &w);
    return RWT_OK;
}

extern "C" rwt_status rwt_env_init(const rwt_csr* L, const int32_t* d_level,
                                   const int32_t* d_level_ptr, const int64_t* d_cost,
                                   const rwt_level_stats* d_stats, int32_t num_levels,
                                   int32_t num_env, int32_t cap, const rwt_env_params* h_params,
                                   void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    RWT_REQUIRE(L != nullptr && h_params != nullptr, RWT_ERR_INVALID_ARG,
                "NULL matrix or parameters");
    const int32_t n = L->n, D = num_levels, E = num_env;
    EnvWs w;
    RWT_TRY(check_ws(n, D, E, cap, d_ws, ws_bytes, &w));
    RWT_REQUIRE(L->rowptr && d_level && d_level_ptr && d_cost && d_stats, RWT_ERR_INVALID_ARG,
                "NULL analysis arrays");
    const rwt_env_params& p = *h_params;
    RWT_REQUIRE(p.alpha >= 0.0 && p.alpha <= 1e300 && p.thin_stop >= 0.0 && p.thin_stop <= 1e300 &&
                    p.reward_alpha >= 0.0 && p.reward_alpha <= 1e300 && p.eps >= 0.0 &&
                    p.eps <= 1e300 && p.decay > 0.0 && p.decay < 1.0 && p.max_dist >= 0 &&
                    p.search_window >= 1 && p.dist_threshold >= 0 && p.max_steps >= 0 &&
                    p.stall_steps >= 0 && p.keep_top >= 1,
                RWT_ERR_INVALID_ARG, "environment parameters are invalid");
    hipStream_t s = hs(stream);
    RWT_HIP(hipMemcpyAsync(w.prm, h_params, sizeof(rwt_env_params), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_env_levels, dim3(blocks_for((size_t)D + 1, 256, 4096)), dim3(256), 0, s,
                       d_level_ptr, d_cost, D, w.lptr, w.rows0, w.cost0, w.deps0);
    RWT_LAUNCHED();
    hipLaunchKernelGGL(k_env_meta, dim3(1), dim3(256), 0, s, w.meta, d_stats, w.prm, w.rows0,
                       w.cost0, n, D, E, cap);
    RWT_LAUNCHED();
    RWT_TRY(rows_by_level_and_deps(L->rowptr, d_level, n, D, w.keys, w.vals, w.tkeys, w.tvals,
                                   w.rws, w.ent, s));
    hipLaunchKernelGGL(k_env_reset, dim3(E), dim3(256), 0, s, w, (const uint8_t*)nullptr, n, D, E,
                       cap);
    RWT_LAUNCHED();
    // the host parameters are read by the copy above before this returns
    RWT_HIP(hipStreamSynchronize(s));
    return RWT_OK;
}

extern "C" rwt_status rwt_env_reset(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                                    const uint8_t* d_which, void* d_ws, size_t ws_bytes,
                                    rwt_stream_t stream) {
    EnvWs w;
    RWT_TRY(check_ws(n, num_levels, num_env, cap, d_ws, ws_bytes, &w));
    hipLaunchKernelGGL(k_env_reset, dim3(num_env), dim3(256), 0, hs(stream), w, d_which, n,
                       num_levels, num_env, cap);
    RWT_LAUNCHED();
    return RWT_OK;
}

extern "C" rwt_status rwt_env_step(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                                   const int32_t* d_action, rwt_env_result* d_res,
                                   int32_t* d_mv_row, int32_t* d_mv_src, int32_t* d_mv_tgt,
                                   void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    EnvWs w;
    RWT_TRY(check_ws(n, num_levels, num_env, cap, d_ws, ws_bytes, &w));
    RWT_REQUIRE(d_action && d_res && d_mv_row && d_mv_src && d_mv_tgt, RWT_ERR_INVALID_ARG,
                "NULL action, result or move arrays");
    hipLaunchKernelGGL(k_env_step, dim3(num_env), dim3(WAVE), 0, hs(stream), w, d_action, n,
                       num_levels, num_env, cap, d_res, d_mv_row, d_mv_src, d_mv_tgt);
    RWT_LAUNCHED();
    return RWT_OK;
}

extern "C" rwt_status rwt_env_step_observe(int32_t n, int32_t num_levels, int32_t num_env,
                                           int32_t cap, const int32_t* d_action,
                                           rwt_env_result* d_res, int32_t* d_mv_row,
                                           int32_t* d_mv_src, int32_t* d_mv_tgt,
                                           float* d_obs_level, float* d_obs_global,
                                           uint8_t* d_mask, void* d_ws, size_t ws_bytes,
                                           rwt_stream_t stream) {
    EnvWs w;
    RWT_TRY(check_ws(n, num_levels, num_env, cap, d_ws, ws_bytes, &w));
    RWT_REQUIRE(d_action && d_res && d_mv_row && d_mv_src && d_mv_tgt, RWT_ERR_INVALID_ARG,
                "NULL action, result or move arrays");
    hipLaunchKernelGGL(k_env_step_observe, dim3(num_env), dim3(256), 0, hs(stream), w, d_action, n,
                       num_levels, num_env, cap, d_res, d_mv_row, d_mv_src, d_mv_tgt, d_obs_level,
                       d_obs_global, d_mask);
    RWT_LAUNCHED();
    return RWT_OK;
}

extern "C" rwt_status rwt_env_observe(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                                      float* d_obs_level, float* d_obs_global, uint8_t* d_mask,
                                      const void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    EnvWs w;
    RWT_TRY(check_ws(n, num_levels, num_env, cap, d_ws, ws_bytes, &w));
    if (!d_obs_level && !d_obs_global && !d_mask) return RWT_OK;
    hipLaunchKernelGGL(k_env_observe, dim3(num_env), dim3(256), 0, hs(stream), w, n, num_levels,
                       num_env, cap, d_obs_level, d_obs_global, d_mask);
    RWT_LAUNCHED();
    return RWT_OK;
}

extern "C" rwt_status rwt_env_levels(int32_t n, int32_t num_levels, int32_t num_env, int32_t cap,
                                     int64_t* d_cost, int32_t* d_rows, int64_t* d_deps,
                                     const void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    EnvWs w;
    RWT_TRY(check_ws(n, num_levels, num_env, cap, d_ws, ws_bytes, &w));
    if (!d_cost && !d_rows && !d_deps) return RWT_OK;
    const size_t total = (size_t)num_env * num_levels;
    hipLaunchKernelGGL(k_env_read, dim3(blocks_for(total, 256, 4096)), dim3(256), 0, hs(stream), w,
                       n, num_levels, num_env, cap, d_cost, d_rows, d_deps);
    RWT_LAUNCHED();
    return RWT_OK;
}
