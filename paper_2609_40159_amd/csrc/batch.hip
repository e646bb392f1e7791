// Batched launch: solves of many matrices and level statistics of many
// candidate rewrite sets in one persistent kernel (plus setup kernels),
// optionally replayed from a captured hipGraph.
//
// Work is a table of row-block tasks.  A chain is the sequence of blocks of
// one matrix's solve, or of one candidate's level computation; inside a
// chain the tasks follow row order, so a task only ever waits for rows of
// tasks with earlier tickets (deadlock-free for any number of resident
// workgroups).  Chains are interleaved by their relative position, so that
// every chain advances while others wait on dependencies.
//
//   solve task      one row block of matrix m: the sync-free block body
//                   shared with the single-matrix solve (x values in LDS,
//                   sentinel-checked reads of rows outside the block).
//   level task      one row block of candidate c: the levels of the
//                   rewritten matrix L' (Section 2.1 level of a row: 1 +
//                   the largest level of its dependencies), taking rewritten
//                   rows' new dependency lists from the batched symbolic
//                   rewrite.  Rows are visited in the original (level, row)
//                   order, which is topological for L' as well: a rewritten
//                   row's new dependencies all sit on earlier original
//                   levels.  Levels are published tagged with the launch
//                   epoch (readiness without clearing the arrays).
//   finalize        the workgroup finishing a candidate's last block builds
//                   the level-cost histogram (cost 2*nnz'_row - 1) in LDS and
//                   the exact S1 / S2 / CV.
#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "batch.hpp"
#include "plan.hpp"
#include "prim.hpp"
#include "sf_block.hpp"
#include "u128.hpp"
#include "walk.hpp"

namespace rwt {

namespace {

constexpr int BT_THREADS = 256;
// row-order walks: solve tasks run two columns (waves 0 and 1), level
// tasks four candidates (one per wave)
constexpr int WK_SOLVE_WAVES = 2;
constexpr int WK_LEVEL_WAVES = 4;
// share of the early task claims that go to walk tasks: one in this many
constexpr size_t WALK_CLAIM_EVERY = 5;
constexpr int BT_LDS = SF_LDS_BUDGET;
// candidate rows whose rewritten pattern outgrows both LDS tiers are redone
// in workspace slabs (one wave each, n + 1 entries per buffer), this many at
// a time
constexpr int NSLAB_B = 64;
// setup control words: [0] first overflow count, [3] too large, [4]
// capacity error, [5] rejected row lists, [6] bad list offsets, [7] second
// overflow count, [9] the one-pass patterns did not fit (the two passes
// follow), [16, 16 + PATTERN_BUMPS) entries of each part of the pattern
// overflow region in use
constexpr int RWCTRL_WORDS = 16 + PATTERN_BUMPS;
// one-pass patterns: a fixed slot of this many entries per candidate row
// (power-law rows rewritten one level down average about 18 entries, a few
// percent exceed 32), used when the pattern capacity holds at least
// PATTERN_ONE_PASS_MIN entries per row; else the lengths pass, a scan and
// the pattern pass
constexpr int PATTERN_SLOT = 32;
constexpr int PATTERN_ONE_PASS_MIN = 48;

struct BatchMatDev {
    int32_t n, R, lanes, nblocks, k, kc;   // kc: right-hand sides per solve chain
    int32_t D, sweep;                      // levels; candidates take the level sweep
    int32_t walk, pad_w;                   // solves and candidates take the row-order walk
    int64_t ldb, ldx;
    const int32_t* perm;                   // rows in (level, row) order
    const int32_t* lptr;                   // level offsets in perm
    const int32_t* rowptr;
    const int32_t* colidx;
    const int32_t* level;
    const double* vals;
    const int4* desc;
    const int32_t* step_pos;
    const int32_t* blk_step;
    const double* B;
    double* X;
};

struct BatchCandDev {
    int32_t m;
    int32_t pad;
    uint32_t* bitmap;   // rewritten rows
    int32_t* lev;       // levels of L', tagged with the launch epoch
};

// the tables' pointers, marked global (in_global)
__device__ __forceinline__ BatchMatDev mat_g(const BatchMatDev& m) {
    BatchMatDev o = m;
    o.perm = in_global(m.perm);
    o.lptr = in_global(m.lptr);
    o.rowptr = in_global(m.rowptr);
    o.colidx = in_global(m.colidx);
    o.level = in_global(m.level);
    o.vals = in_global(m.vals);
    o.desc = in_global(m.desc);
    o.step_pos = in_global(m.step_pos);
    o.blk_step = in_global(m.blk_step);
    o.B = in_global(m.B);
    o.X = in_global(m.X);
    return o;
}
__device__ __forceinline__ BatchCandDev cand_g(const BatchCandDev& c) {
    BatchCandDev o = c;
    o.bitmap = in_global(c.bitmap);
    o.lev = in_global(c.lev);
    return o;
}

struct BatchKArgs {
    const BatchMatDev* mats;
    const BatchCandDev* cands;
    const int4* tasks;
    int32_t ntasks;
    int32_t C;
    const int32_t* cand_ptr;
    const int32_t* rows;
    const int32_t* counts_q;
    const int32_t* pat_ptr;
    const int32_t* pat;
    const unsigned char* cand_bad;
    int32_t* cand_done;
    rwt_cand_stats* stats;
    Ctrl* ctrl;
    const uint32_t* epoch;
    int64_t ticks;
    int32_t hist_cap;   // level-cost histogram entries that fit the launch's LDS
    int32_t qcap;       // capacity of the candidate row lists (pat_ptr holds qcap + 1)
};

__device__ __forceinline__ uint32_t epoch_tag(uint32_t e) { return (e % 255u) + 1u; }

__device__ __forceinline__ void lds_sync() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// level of row j of candidate c, written by another workgroup
__device__ __forceinline__ int32_t wait_level(const int32_t* p, uint32_t tag, int32_t* err,
                                              int64_t ticks) {
    int32_t v = ld_relaxed(p);
    if (((uint32_t)v >> 24) == tag) return v & 0xffffff;
    int64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(0);
        v = ld_relaxed(p);
        if (((uint32_t)v >> 24) == tag) return v & 0xffffff;
        if (ld_relaxed(err) != 0) return 0;
        if (wall_clock64() - t0 > ticks) {
            __hip_atomic_store(err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
    }
}

template <typename T>
__device__ T group_max_i(T v, int G) {
    for (int o = G / 2; o > 0; o >>= 1) {
        T u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    return v;
}

__device__ int32_t lower_bound_g(const int32_t* a, int32_t lo, int32_t hi, int32_t x) {
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// All levels of a group of gs <= SG candidates of one matrix by one
// workgroup: the original levels in order, each one's rows all at once (one
// lane per row).  A row's dependencies -- its own, or a rewritten row's new
// list -- lie on earlier original levels, published by this workgroup before
// the barrier that ended their level.  The group's levels are interleaved,
// lev[i*gs + s] for candidate c0+s, so one dependency read serves every
// candidate that keeps the row's original list.  A load that still shows
// another launch's tag (a stale cache line) is repeated with a device-scope
// load.
constexpr int SG = 8;
// Before the sweep, each rewritten row's slot holds its position in the
// candidate's row list: this launch's tag, bit 23 set, the offset below it
// (levels stay below 2^23 on this path, so bit 23 tells the two apart).
constexpr uint32_t MARK = 0x800000u;

// a level published in this launch (tag, bit 23 clear), waiting for it
__device__ int32_t wait_level_sw(const int32_t* p, uint32_t tag, int32_t* err, int64_t ticks) {
    int32_t v = ld_relaxed(p);
    if (((uint32_t)v >> 24) == tag && !((uint32_t)v & MARK)) return v & 0x7fffff;
    int64_t t0 = wall_clock64();
    for (;;) {
        __builtin_amdgcn_s_sleep(0);
        v = ld_relaxed(p);
        if (((uint32_t)v >> 24) == tag && !((uint32_t)v & MARK)) return v & 0x7fffff;
        if (ld_relaxed(err) != 0) return 0;
        if (wall_clock64() - t0 > ticks) {
            __hip_atomic_store(err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
    }
}

__device__ __forceinline__ int32_t level_of(int32_t* lev, int32_t idx, int32_t v, uint32_t tag,
                                            int32_t* err, int64_t ticks) {
    return (((uint32_t)v >> 24) == tag && !((uint32_t)v & MARK)) ? (v & 0x7fffff)
                                                                 : wait_level_sw(&lev[idx], tag, err, ticks);
}

__device__ __forceinline__ void sweep_group(const BatchKArgs& a, const BatchMatDev& M, int32_t c0,
                                            int32_t gs, int32_t* lev, uint32_t tag) {
    int32_t* err = &a.ctrl->err;
    const bool marks = M.D < (int32_t)MARK;
    if (marks) {
        for (int32_t s = 0; s < gs; ++s) {
            const int32_t c = c0 + s;
            if (a.cand_bad[c]) continue;
            const BatchCandDev Cd = cand_g(a.cands[c]);
            const int32_t qb = a.cand_ptr[c], qe = a.cand_ptr[c + 1];
            for (int32_t q = qb + threadIdx.x; q < qe; q += blockDim.x) {
                const int32_t r = a.rows[q];
                if (q - qb < (int32_t)MARK && ((Cd.bitmap[r >> 5] >> (r & 31)) & 1u))
                    st_relaxed(&lev[r * gs + s], (int32_t)((tag << 24) | MARK | (uint32_t)(q - qb)));
            }
        }
        __syncthreads();
    }
    for (int32_t l = 0; l < M.D; ++l) {
        const int32_t beg = M.lptr[l], end = M.lptr[l + 1];
        for (int32_t pos = beg + threadIdx.x; pos < end; pos += blockDim.x) {
            const int32_t i = M.perm[pos];
            const int32_t db = M.rowptr[i], de = M.rowptr[i + 1] - 1;   // without the diagonal
            uint32_t rw = 0;   // candidates of the group that rewrite row i
#pragma unroll
            for (int s = 0; s < SG; ++s) {
                if (s >= gs) break;
                const BatchCandDev Cd = cand_g(a.cands[c0 + s]);
                if (!a.cand_bad[c0 + s] && ((Cd.bitmap[i >> 5] >> (i & 31)) & 1u)) rw |= 1u << s;
            }
            int32_t mx[SG];
#pragma unroll
            for (int s = 0; s < SG; ++s) mx[s] = -1;
            const uint32_t all = (1u << gs) - 1u;
            if (rw != all) {
                // U dependencies at a time: their columns, then all their
                // slots' levels, are loaded together
                constexpr int U = 4;
                for (int32_t p0 = db; p0 < de; p0 += U) {
                    int32_t jv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        const int32_t p = p0 + u;
                        const int32_t jj = M.colidx[p < de ? p : p0];
                        const bool ok = p < de && jj >= 0 && jj < i;
                        if (p < de && !ok)
                            __hip_atomic_store(err, (int32_t)RWT_ERR_INVALID_ARG, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        jv[u] = ok ? jj : -1;
                    }
                    int32_t v[U][SG];
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int s = 0; s < SG; ++s)
                            v[u][s] = (s < gs && jv[u] >= 0) ? lev[jv[u] * gs + s] : 0;
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        if (jv[u] < 0) continue;
#pragma unroll
                        for (int s = 0; s < SG; ++s) {
                            if (s >= gs || ((rw >> s) & 1u)) continue;
                            const int32_t lj = level_of(lev, jv[u] * gs + s, v[u][s], tag, err, a.ticks);
                            mx[s] = lj > mx[s] ? lj : mx[s];
                        }
                    }
                }
            }
            for (uint32_t m = rw; m != 0; m &= m - 1) {
                const int s = __builtin_ctz(m);
                const int32_t c = c0 + s;
                const int32_t qb = a.cand_ptr[c];
                const uint32_t mv = marks ? (uint32_t)ld_relaxed(&lev[i * gs + s]) : 0u;
                const int32_t q = ((mv >> 24) == tag && (mv & MARK))
                                      ? qb + (int32_t)(mv & (MARK - 1))
                                      : lower_bound_g(a.rows, qb, a.cand_ptr[c + 1], i);
                const int32_t nb = a.pat_ptr[q], ne = nb + a.counts_q[q] - 1;   // new diagonal last
                int32_t best = -1;
                for (int32_t p = nb; p < ne; ++p) {
                    const int32_t j = a.pat[p];
                    if (j < 0 || j >= i) {
                        __hip_atomic_store(err, (int32_t)RWT_ERR_INVALID_ARG, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        continue;
                    }
                    const int32_t lj = level_of(lev, j * gs + s, lev[j * gs + s], tag, err, a.ticks);
                    best = lj > best ? lj : best;
                }
#pragma unroll
                for (int t = 0; t < SG; ++t)
                    if (t == s) mx[t] = best;
            }
#pragma unroll
            for (int s = 0; s < SG; ++s)
                if (s < gs) st_relaxed(&lev[i * gs + s], (int32_t)((tag << 24) | (uint32_t)(mx[s] + 1)));
        }
        __syncthreads();
        if (ld_relaxed(err) != 0) return;
    }
}

// One row block of the level chains of a group of gs <= SG candidates of one
// matrix: the block's rows in the original (level, row) order, step by
// step, G lanes per row.  Levels of the block's rows live in LDS (lv[(i -
// r0) * gs + s]); rows before the block are read from the group's
// interleaved level arrays, published by earlier blocks (tag-checked, waited
// for).  Before the steps, each rewritten row's LDS slot holds its position
// in its candidate's row list (top bit set), so its new dependency list is
// found without a search.
constexpr uint32_t LDS_MARK = 0x80000000u;

__device__ __forceinline__ int32_t level_blk(const int32_t* lev, int32_t idx, uint32_t tag,
                                             int32_t* err, int64_t ticks) {
    const int32_t v = ld_relaxed(&lev[idx]);
    return ((uint32_t)v >> 24) == tag ? (v & 0xffffff) : wait_level(&lev[idx], tag, err, ticks);
}

__device__ __forceinline__ void level_block_group(const BatchKArgs& a, const BatchMatDev& M,
                                                  int32_t c0, int32_t gs, int32_t* lev, int32_t blk,
                                                  uint32_t tag, unsigned char* s_raw) {
    const int32_t R = M.R;
    const int32_t r0 = blk * R, r1 = min(M.n, r0 + R);
    const int32_t sb = M.blk_step[blk], ns = M.blk_step[blk + 1] - sb;
    int32_t* lv = reinterpret_cast<int32_t*>(s_raw);
    int32_t* sp = reinterpret_cast<int32_t*>(s_raw + ((R * gs * 4 + 15) & ~15));
    int32_t* qr = sp + ((ns + 1 + 3) & ~3);   // [2 * SG]: the block's range of each list
    int32_t* err = &a.ctrl->err;
    for (int32_t u = threadIdx.x; u <= ns; u += blockDim.x) sp[u] = M.step_pos[sb + u] - r0;
    if (threadIdx.x < (unsigned)gs) {
        const int32_t c = c0 + (int32_t)threadIdx.x;
        int32_t lo = 0, hi = 0;
        if (!a.cand_bad[c]) {
            const int32_t qb = a.cand_ptr[c], qe = a.cand_ptr[c + 1];
            lo = lower_bound_g(a.rows, qb, qe, r0);
            hi = lower_bound_g(a.rows, lo, qe, r1);
        }
        qr[2 * threadIdx.x] = lo;
        qr[2 * threadIdx.x + 1] = hi;
    }
    __syncthreads();
    for (int32_t s = 0; s < gs; ++s) {
        const BatchCandDev Cd = cand_g(a.cands[c0 + s]);
        const int32_t qb = a.cand_ptr[c0 + s];
        for (int32_t q = qr[2 * s] + threadIdx.x; q < qr[2 * s + 1]; q += blockDim.x) {
            const int32_t r = a.rows[q];
            if ((Cd.bitmap[r >> 5] >> (r & 31)) & 1u)
                lv[(r - r0) * gs + s] = (int32_t)(LDS_MARK | (uint32_t)(q - qb));
        }
    }
    __syncthreads();
    const int G = M.lanes;
    const int gl = threadIdx.x & (G - 1);
    const int lane = lane_id();
    const int gpw = WAVE / G;
    const int wib = threadIdx.x / WAVE;
    const int32_t stride = (blockDim.x / WAVE) * gpw;
    const uint32_t all = (1u << gs) - 1u;
    for (int32_t u = 0; u < ns; ++u) {
        const int32_t beg = sp[u], end = sp[u + 1];
        for (int32_t base = beg + wib * gpw; base < end; base += stride) {
            const int32_t pos = base + lane / G;
            const bool act = pos < end;
            int32_t i = r0, db = 0, de = 0;
            uint32_t rw = 0;
            if (act) {
                const int4 d = M.desc[r0 + pos];
                i = d.x;
                db = d.y;
                de = d.z;   // forward pattern without the diagonal
#pragma unroll
                for (int s = 0; s < SG; ++s) {
                    if (s >= gs) break;
                    const BatchCandDev Cd = cand_g(a.cands[c0 + s]);
                    if (!a.cand_bad[c0 + s] && ((Cd.bitmap[i >> 5] >> (i & 31)) & 1u))
                        rw |= 1u << s;
                }
            }
            int32_t mx[SG];
#pragma unroll
            for (int s = 0; s < SG; ++s) mx[s] = -1;
            if (act && rw != all) {
                constexpr int U = 4;
                for (int32_t p0 = db + gl; p0 < de; p0 += U * G) {
                    int32_t jv[U];
#pragma unroll
                    for (int u2 = 0; u2 < U; ++u2) {
                        const int32_t p = p0 + u2 * G;
                        const int32_t jj = M.colidx[p < de ? p : p0];
                        const bool ok = p < de && jj >= 0 && jj < i;
                        if (p < de && !ok)
                            __hip_atomic_store(err, (int32_t)RWT_ERR_INVALID_ARG, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        jv[u2] = ok ? jj : -1;
                    }
#pragma unroll
                    for (int u2 = 0; u2 < U; ++u2) {
                        const int32_t j = jv[u2];
                        if (j < 0) continue;
#pragma unroll
                        for (int s = 0; s < SG; ++s) {
                            if (s >= gs || ((rw >> s) & 1u)) continue;
                            const int32_t lj = j >= r0 ? lv[(j - r0) * gs + s]
                                                       : level_blk(lev, j * gs + s, tag, err, a.ticks);
                            mx[s] = lj > mx[s] ? lj : mx[s];
                        }
                    }
                }
            }
            for (uint32_t m = act ? rw : 0u; m != 0; m &= m - 1) {
                const int s = __builtin_ctz(m);
                const int32_t q = a.cand_ptr[c0 + s] + (int32_t)((uint32_t)lv[(i - r0) * gs + s] & ~LDS_MARK);
                const int32_t nb = a.pat_ptr[q], ne = nb + a.counts_q[q] - 1;   // new diagonal last
                int32_t best = -1;
                for (int32_t p = nb + gl; p < ne; p += G) {
                    const int32_t j = a.pat[p];
                    if (j < 0 || j >= i) {
                        __hip_atomic_store(err, (int32_t)RWT_ERR_INVALID_ARG, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                        continue;
                    }
                    const int32_t lj = j >= r0 ? lv[(j - r0) * gs + s]
                                               : level_blk(lev, j * gs + s, tag, err, a.ticks);
                    best = lj > best ? lj : best;
                }
#pragma unroll
                for (int t = 0; t < SG; ++t)
                    if (t == s) mx[t] = best;
            }
#pragma unroll
            for (int s = 0; s < SG; ++s) {
                if (s >= gs) break;
                mx[s] = group_max_i(mx[s], G);
            }
            if (act && gl == 0) {
#pragma unroll
                for (int s = 0; s < SG; ++s) {
                    if (s >= gs) break;
                    const int32_t L = mx[s] + 1;
                    lv[(i - r0) * gs + s] = L;
                    st_relaxed(&lev[i * gs + s], (int32_t)((tag << 24) | (uint32_t)L));
                }
            }
        }
        lds_sync();
    }
}

__device__ U128 block_sum_u128_bt(U128 v, unsigned char* scratch) {
    uint64_t* s = reinterpret_cast<uint64_t*>(scratch);
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        U128 u;
        u.lo = __shfl_xor(v.lo, o);
        u.hi = __shfl_xor(v.hi, o);
        v = u128_add(v, u);
    }
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane_id() == 0) {
        s[2 * w] = v.lo;
        s[2 * w + 1] = v.hi;
    }
    __syncthreads();
    U128 r{0, 0};
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) r = u128_add(r, U128{s[2 * i], s[2 * i + 1]});
    __syncthreads();
    return r;
}

__device__ int32_t block_max_bt(int32_t v, int32_t* scratch) {
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        int32_t u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    const int w = threadIdx.x / WAVE;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    int32_t r = scratch[0];
    for (int i = 1; i < (int)(blockDim.x / WAVE); ++i) r = scratch[i] > r ? scratch[i] : r;
    __syncthreads();
    return r;
}

// statistics of the gs candidates of a sweep group (levels interleaved):
// each candidate's level count, then its level-cost histogram in LDS level
// range by level range, and the exact S1 / S2 / CV
__device__ __forceinline__ void finalize_group(const BatchKArgs& a, const BatchMatDev& M,
                                               int32_t c0, int32_t gs, int32_t* lev, uint32_t tag,
                                               bool marks, unsigned char* s_raw) {
    // sweeps mark slots with bit 23 (levels below 2^23); chains use 24 bits
    const int32_t lmask = marks ? 0x7fffff : 0xffffff;
    int32_t* err = &a.ctrl->err;
    const int32_t n = M.n;
    int32_t D[SG];
    int32_t dmax = 0;
    {
        int32_t mx[SG];
#pragma unroll
        for (int s = 0; s < SG; ++s) mx[s] = -1;
        // every level is published (the sweep ended with a barrier): the
        // loads of a row's slots are issued together and only a value not
        // yet visible here is waited for
        for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
            int32_t v[SG];
#pragma unroll
            for (int s = 0; s < SG; ++s) v[s] = s < gs ? ld_relaxed(&lev[i * gs + s]) : 0;
#pragma unroll
            for (int s = 0; s < SG; ++s) {
                if (s >= gs) break;
                const int32_t L =
                    marks ? level_of(lev, i * gs + s, v[s], tag, err, a.ticks)
                          : (((uint32_t)v[s] >> 24) == tag ? (v[s] & 0xffffff)
                                                           : wait_level(&lev[i * gs + s], tag, err, a.ticks));
                mx[s] = L > mx[s] ? L : mx[s];
            }
        }
#pragma unroll
        for (int s = 0; s < SG; ++s) {
            D[s] = s < gs ? block_max_bt(mx[s], reinterpret_cast<int32_t*>(s_raw)) + 1 : 0;
            dmax = D[s] > dmax ? D[s] : dmax;
        }
    }
    uint32_t* hist = reinterpret_cast<uint32_t*>(s_raw + 256);
    const int32_t W = a.hist_cap / gs;   // levels per range, per candidate
    uint64_t s1[SG];
    U128 s2[SG];
#pragma unroll
    for (int s = 0; s < SG; ++s) {
        s1[s] = 0;
        s2[s] = U128{0, 0};
    }
    for (int32_t lb = 0; lb < dmax; lb += W) {
        const int32_t le = min(dmax, lb + W);
        for (int32_t e = threadIdx.x; e < gs * W; e += blockDim.x) hist[e] = 0u;
        __syncthreads();
        for (int32_t i = threadIdx.x; i < n; i += blockDim.x) {
            const uint32_t cost = (uint32_t)(2 * (M.rowptr[i + 1] - M.rowptr[i]) - 1);
            int32_t v[SG];
#pragma unroll
            for (int s = 0; s < SG; ++s) v[s] = s < gs ? ld_relaxed(&lev[i * gs + s]) : 0;
#pragma unroll
            for (int s = 0; s < SG; ++s) {
                if (s >= gs) break;
                const int32_t L = v[s] & lmask;
                if (L >= lb && L < le) atomicAdd(&hist[s * W + (L - lb)], cost);
            }
        }
        // rewritten rows: cost of the new row instead of the old one (a
        // rejected candidate's list is never read: its bounds may be invalid)
        for (int32_t s = 0; s < gs; ++s) {
            const int32_t c = c0 + s;
            const BatchCandDev Cd = cand_g(a.cands[c]);
            const int32_t qb = a.cand_ptr[c], qe = a.cand_bad[c] ? qb : a.cand_ptr[c + 1];
            for (int32_t q = qb + threadIdx.x; q < qe; q += blockDim.x) {
                const int32_t r = a.rows[q];
                if (!((Cd.bitmap[r >> 5] >> (r & 31)) & 1u)) continue;
                const int32_t L = ld_relaxed(&lev[r * gs + s]) & lmask;
                if (L >= lb && L < le)
                    atomicAdd(&hist[s * W + (L - lb)],
                              (uint32_t)(2 * (a.counts_q[q] - (M.rowptr[r + 1] - M.rowptr[r]))));
            }
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < SG; ++s) {
            if (s >= gs) break;
            for (int32_t l = threadIdx.x; l < le - lb; l += blockDim.x) {
                const uint64_t v = hist[s * W + l];
                s1[s] += v;
                s2[s] = u128_add(s2[s], U128{v * v, __umul64hi(v, v)});
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int s = 0; s < SG; ++s) {
        if (s >= gs) break;
        const U128 s1w = block_sum_u128_bt(U128{s1[s], 0}, s_raw);
        const U128 s2w = block_sum_u128_bt(s2[s], s_raw);
        if (threadIdx.x == 0) {
            rwt_cand_stats o;
            o.num_levels = D[s];
            o.valid = a.cand_bad[c0 + s] ? 0 : 1;
            o.S1 = s1w.lo;
            o.S2_lo = s2w.lo;
            o.S2_hi = s2w.hi;
            o.cv = cv_exact((uint64_t)D[s], s1w.lo, s2w);
            a.stats[c0 + s] = o;
        }
    }
}

__global__ void __launch_bounds__(BT_THREADS) k_batch_main(BatchKArgs a) {
    extern __shared__ __align__(16) unsigned char s_raw[];
    __shared__ int32_t s_task;
    __shared__ int32_t s_last;
    const uint32_t tag = epoch_tag(*a.epoch);
    for (;;) {
        if (threadIdx.x == 0) s_task = (int32_t)fetch_add(&a.ctrl->ticket, 1u);
        __syncthreads();
        const int32_t t = s_task;
        __syncthreads();
        if (t >= a.ntasks) break;
        const int4 tk = a.tasks[t];
        if (tk.x == 0) {
            const BatchMatDev M = mat_g(a.mats[tk.y]);
            const int32_t q0 = tk.w * M.kc;   // this chain's first column
            SfBlockArgs b;
            b.r0 = tk.z * M.R;
            b.r1 = min(M.n, b.r0 + M.R);
            b.sb = M.blk_step[tk.z];
            b.ns = M.blk_step[tk.z + 1] - b.sb;
            b.k = min(M.kc, M.k - q0);
            b.lanes = M.lanes;
            b.stage_x = 0;   // read by the staged body only
            b.ldb = M.ldb;
            b.ldx = M.ldx;
            b.colidx = M.colidx;
            b.crow = nullptr;
            b.cmap = nullptr;
            b.vals = M.vals;
            b.desc = M.desc;
            b.step_pos = M.step_pos;
            b.B = M.B + (int64_t)q0 * M.ldb;
            b.X = M.X + (int64_t)q0 * M.ldx;
            b.err = &a.ctrl->err;
            b.ticks = a.ticks;
            b.lds_rows = M.R;
            b.hold_row = -1;
            if (M.kc == 1) sf_block<double, false, 1>(b, s_raw);
            else sf_block<double, false, 4>(b, s_raw);
        } else if (tk.x == 3) {
            // row-order walks of columns tk.z .. tk.z + tk.w - 1 of matrix tk.y,
            // one wave each
            const BatchMatDev M = mat_g(a.mats[tk.y]);
            const int w = threadIdx.x / WAVE;
            if (w < tk.w) {
                const int32_t q = tk.z + w;
                WkArgs wa;
                wa.n = M.n;
                wa.ptr = M.rowptr;
                wa.idx = M.colidx;
                wa.vals = M.vals;
                wa.rowptr = M.rowptr;
                wa.dvals = M.vals;
                wa.b = M.B + (int64_t)q * M.ldb;
                wa.x = M.X + (int64_t)q * M.ldx;
                wa.err = &a.ctrl->err;
                wk_solve<double, false>(
                    wa, reinterpret_cast<WkLds<double>*>(s_raw + (size_t)w * wk_lds_bytes<double>()));
            }
        } else if (tk.x == 4) {
            // row-order walks of the levels of candidates tk.y .. tk.y + tk.z - 1
            // (one matrix), one wave each, then their statistics
            const int32_t c0 = tk.y, gs = tk.z;
            const BatchMatDev M = mat_g(a.mats[a.cands[c0].m]);
            const int w = threadIdx.x / WAVE;
            if (w < gs) {
                const int32_t c = c0 + w;
                const BatchCandDev Cd = cand_g(a.cands[c]);
                // each rewritten row's slot holds its offset in the row list
                const int32_t qb = a.cand_ptr[c], qe = a.cand_bad[c] ? qb : a.cand_ptr[c + 1];
                for (int32_t q = qb + lane_id(); q < qe; q += WAVE) {
                    const int32_t r = a.rows[q];
                    if (q - qb < (int32_t)MARK && ((Cd.bitmap[r >> 5] >> (r & 31)) & 1u))
                        st_relaxed(&Cd.lev[r], (int32_t)((tag << 24) | MARK | (uint32_t)(q - qb)));
                }
                asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
                WkLvlArgs la;
                la.n = M.n;
                la.rowptr = M.rowptr;
                la.colidx = M.colidx;
                la.lev = Cd.lev;
                la.tag = tag;
                la.mark = MARK;
                la.pat_ptr = a.pat_ptr;
                la.pat_len = a.counts_q;
                la.pat = a.pat;
                la.qb = qb;
                la.qmax = a.qcap;
                la.err = &a.ctrl->err;
                wk_levels(la, reinterpret_cast<WkLvlLds*>(s_raw + (size_t)w * sizeof(WkLvlLds)));
            }
            __syncthreads();
            for (int32_t s = 0; s < gs; ++s)
                finalize_group(a, M, c0 + s, 1, in_global(a.cands[c0 + s].lev), tag, true, s_raw);
        } else if (tk.x == 2) {
            // a sweep group: candidates tk.y .. tk.y + tk.z - 1 of one matrix,
            // levels interleaved in the first one's (and its neighbours')
            // level arrays
            const BatchCandDev Cd = cand_g(a.cands[tk.y]);
            const BatchMatDev M = mat_g(a.mats[Cd.m]);
            sweep_group(a, M, tk.y, tk.z, Cd.lev, tag);
            __syncthreads();
            finalize_group(a, M, tk.y, tk.z, Cd.lev, tag, true, s_raw);
        } else {
            // one row block of the level chains of candidates tk.y .. tk.y + tk.w - 1
            const int32_t c0 = tk.y;
            const BatchCandDev Cd = cand_g(a.cands[c0]);
            const BatchMatDev M = mat_g(a.mats[Cd.m]);
            level_block_group(a, M, c0, tk.w, Cd.lev, tk.z, tag, s_raw);
            __syncthreads();
            if (threadIdx.x == 0)
                s_last = (fetch_add(&a.cand_done[c0], 1) == M.nblocks - 1) ? 1 : 0;
            __syncthreads();
            if (s_last) finalize_group(a, M, c0, tk.w, Cd.lev, tag, false, s_raw);
        }
        __syncthreads();
        if (ld_relaxed(&a.ctrl->err) != 0) break;
    }
}

// Lowest level among the rows of each row block (tasks are ordered by when
// their first rows can start).
__global__ void k_block_minlev(const int32_t* level, int32_t n, int32_t R, int32_t* out) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n; i += nth) atomicMin(&out[i / R], level[i]);
}

__global__ void k_fill_i32max(int32_t* p, int64_t n) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < n; i += nth) p[i] = 0x7fffffff;
}

__global__ void k_batch_epoch(uint32_t* epoch) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *epoch = *epoch + 1u;
}

// Reset per-launch state: counters, bitmaps, overflow marks, X sentinels,
// and every level array once per 255 launches (before its tags repeat).
__global__ void k_batch_begin(const BatchMatDev* mats, int32_t count, uint32_t* bitmaps,
                              int64_t bitmap_words, int32_t* levs, int64_t lev_words,
                              const uint32_t* epoch, int32_t* cand_done, unsigned char* cand_bad,
                              int32_t C, int32_t* counts_q, unsigned char* ovf_mark, int32_t qcap,
                              Ctrl* ctrl, int32_t* rwctrl) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    if (tid == 0) {
        ctrl->bar_count = 0;
        ctrl->bar_gen = 0;
        ctrl->ticket = 0;
        ctrl->err = 0;
        ctrl->heartbeat = 0;
        for (int i = 0; i < RWCTRL_WORDS; ++i) rwctrl[i] = 0;
    }
    for (int64_t i = tid; i < C; i += nth) {
        cand_done[i] = 0;
        cand_bad[i] = 0;
    }
    for (int64_t i = tid; i < bitmap_words; i += nth) bitmaps[i] = 0u;
    for (int64_t i = tid; i <= qcap; i += nth) counts_q[i] = 0;
    for (int64_t i = tid; i < qcap; i += nth) ovf_mark[i] = 0;
    if ((*epoch % 255u) == 0u)
        for (int64_t i = tid; i < lev_words; i += nth) levs[i] = 0;
    const double s = sentinel_value<double>();
    for (int32_t m = 0; m < count; ++m) {
        const BatchMatDev M = mat_g(mats[m]);
        const int64_t total = (int64_t)M.n * M.k;
        for (int64_t e = tid; e < total; e += nth) {
            const int64_t q = e / M.n, i = e - q * M.n;
            M.X[i + q * M.ldx] = s;
        }
    }
}

// Before the two-pass patterns that follow one-pass patterns that did not
// fit: the overflow lists and marks start again.  Only when *gate != 0.
__global__ void k_batch_redo_reset(const int32_t* gate, int32_t* rwctrl, int32_t* counts_q,
                                   unsigned char* ovf_mark, int32_t qcap) {
    if (ld_relaxed(gate) == 0) return;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    if (tid == 0) {
        rwctrl[0] = 0;
        rwctrl[7] = 0;
    }
    for (int64_t i = tid; i <= qcap; i += nth) counts_q[i] = 0;
    for (int64_t i = tid; i < qcap; i += nth) ovf_mark[i] = 0;
}

// dst[0 .. count) = src[...], only when *gate != 0
__global__ void k_copy_gated(const int32_t* gate, const int32_t* src, int32_t* dst, int64_t count) {
    if (ld_relaxed(gate) == 0) return;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = tid; i < count; i += nth) dst[i] = src[i];
}

// The candidate list as a whole: offsets start at 0, never decrease and end
// within the row capacity.  Otherwise every candidate is rejected.
__global__ void k_batch_ptrcheck(const int32_t* cand_ptr, int32_t C, int32_t qcap,
                                 int32_t* rwctrl) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    bool bad = false;
    if (tid == 0) bad = cand_ptr[0] != 0 || cand_ptr[C] > qcap;
    for (int64_t c = tid; c < C; c += nth) bad = bad || cand_ptr[c] > cand_ptr[c + 1];
    if (bad) atomicExch(&rwctrl[6], 1);
}

// One wave per candidate: check its row list, then mark the rows that the
// rewrite changes (level >= 1 and target below the level).
__global__ void k_batch_bitmap(const BatchMatDev* mats, const BatchCandDev* cands, int32_t C,
                               const int32_t* cand_ptr, const int32_t* rows, const int32_t* targets,
                               int32_t qcap, unsigned char* cand_bad, int32_t* rwctrl) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int lane = lane_id();
    const bool list_ok = ld_relaxed(&rwctrl[6]) == 0;
    for (int64_t c = wave; c < C; c += nw) {
        const BatchCandDev Cd = cand_g(cands[c]);
        const BatchMatDev M = mat_g(mats[Cd.m]);
        const int32_t qb = cand_ptr[c], qe = cand_ptr[c + 1];
        bool bad = !list_ok || qe < qb || qb < 0 || qe > qcap;
        if (!bad) {
            for (int32_t q = qb + lane; q < qe; q += WAVE) {
                const int32_t r = rows[q];
                if (r < 0 || r >= M.n || (q > qb && rows[q - 1] >= r) || (targets && targets[q] < 0))
                    bad = true;
            }
        }
        bad = __ballot(bad) != 0;
        if (bad) {
            if (lane == 0) {
                cand_bad[c] = 1;
                atomicExch(&rwctrl[5], 1);
            }
            continue;
        }
        for (int32_t q = qb + lane; q < qe; q += WAVE) {
            const int32_t r = rows[q];
            const int32_t lvl = M.level[r];
            const int32_t t = targets ? targets[q] : lvl - 1;
            if (lvl > 0 && t < lvl) atomicOr(&Cd.bitmap[r >> 5], 1u << (r & 31));
        }
    }
}

}  // namespace
}  // namespace rwt

using namespace rwt;

struct rwt_batch {
    rwt_batch_desc desc;
    std::vector<rwt_batch_matrix> mats;
    std::vector<int32_t> cand_mat;
    std::vector<rwt_plan*> plans;
    // device state
    BatchMatDev* d_mats = nullptr;
    BatchCandDev* d_cands = nullptr;
    BatchRwMat* d_rwmats = nullptr;
    int32_t* d_cand_mat = nullptr;
    int4* d_tasks = nullptr;
    int32_t ntasks = 0, solve_tasks = 0, sweep_cands = 0;
    int32_t lds_bytes = BT_LDS;   // dynamic LDS of the persistent launch
    uint32_t* bitmaps = nullptr;
    int64_t bitmap_words = 0;
    int32_t* levs = nullptr;
    int64_t lev_words = 0;
    int32_t* cand_done = nullptr;
    unsigned char* cand_bad = nullptr;
    rwt_cand_stats* stats = nullptr;
    int32_t* counts_q = nullptr;
    int32_t* pat_ptr = nullptr;
    int32_t* pat_ptr2 = nullptr;
    int32_t* pat = nullptr;
    int32_t* ovf = nullptr;
    int32_t* ovf2 = nullptr;
    unsigned char* ovf_mark = nullptr;
    int32_t* rwctrl = nullptr;
    unsigned char* slab = nullptr;
    int64_t slab_stride = 0;
    int32_t slab_cap = 0;
    void* scan_ws = nullptr;
    Ctrl* ctrl = nullptr;
    uint32_t* epoch = nullptr;
    int32_t qcap = 0, pat_cap = 0;
    int32_t slot_len = 0;          // one-pass patterns: fixed slot per row (0: two passes)
    int grid = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    double create_ms = 0;
};

namespace {

rwt_plan_opts batch_plan_opts(const rwt_batch_desc* d, const rwt_batch_matrix& m) {
    rwt_plan_opts o;
    memset(&o, 0, sizeof o);
    o.algo = RWT_ALGO_SYNCFREE;   // block size (or one whole-matrix block) is tuned
    // The largest block that fits, unless given: solve chains and candidate
    // level chains share the block tables, and in a batch -- where many
    // chains compete for workgroups -- fewer, larger blocks mean fewer level
    // steps in all (measured on the 256-matrix batch: 1.5x faster launches
    // than per-matrix tuned sizes, and no tuning solves at creation).
    o.block_rows = m.block_rows > 0 ? m.block_rows : (1 << 16);
    o.kmax = m.k > 0 ? m.k : 1;
    o.rhs_chunk = 1;   // one column per solve chain: parallel chains to spare
    o.tune_cols = 1;
    o.stage_outside = 1;   // no timing solves at creation
    o.narrow_rows = -1;
    o.watchdog_ms = d->watchdog_ms;
    return o;
}

struct BatchLayout {
    std::vector<size_t> plan_off, plan_bytes;
    size_t mats, cands, candmat, rwmats, tasks, bitmaps, levs, done, bad, stats, counts, patptr, patptr2, pat, ovf, ovf2,
        ovfmark, rwctrl, slab, scan, ctrl, epoch, blkmin, total;
    int64_t bitmap_words, lev_words, slab_stride;
    int32_t qcap, pat_cap, slab_cap, ntasks_max;
};

rwt_status layout_batch(const rwt_batch_desc* d, BatchLayout* L) {
    RWT_REQUIRE(d != nullptr && d->count >= 0 && d->num_cand >= 0, RWT_ERR_INVALID_ARG,
                "bad batch descriptor");
    RWT_REQUIRE(d->count == 0 || d->mats != nullptr, RWT_ERR_INVALID_ARG, "null matrix list");
    RWT_REQUIRE(d->cand_mode >= 0 && d->cand_mode <= 3, RWT_ERR_INVALID_ARG,
                "cand_mode must be 0, 1, 2 or 3");
    RWT_REQUIRE(d->num_cand == 0 ||
                    (d->h_cand_mat && d->d_cand_ptr && d->d_cand_rows && d->cand_rows_cap >= 0),
                RWT_ERR_INVALID_ARG, "null candidate arrays");
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~size_t(255);
        size_t o = off;
        off += bytes;
        return o;
    };
    int32_t nmax = 1;
    int64_t blocks_max = 0;
    for (int32_t m = 0; m < d->count; ++m) {
        const rwt_batch_matrix& M = d->mats[m];
        RWT_REQUIRE(M.L.dt == RWT_F64, RWT_ERR_INVALID_ARG, "batched matrices must be FP64");
        RWT_REQUIRE(M.k >= 0 && M.k <= 16, RWT_ERR_INVALID_ARG,
                    "matrix %d: 0..16 right-hand sides per matrix in a batch", m);
        RWT_REQUIRE(M.k == 0 || (M.B && M.X && M.ldb >= M.L.n && M.ldx >= M.L.n),
                    RWT_ERR_INVALID_ARG, "matrix %d: bad right-hand sides", m);
        RWT_REQUIRE(M.block_rows >= 0 && M.block_rows <= (1 << 20), RWT_ERR_INVALID_ARG,
                    "matrix %d: block size outside 0..2^20", m);
        rwt_plan_opts o = batch_plan_opts(d, M);
        size_t pb = 0;
        RWT_TRY(rwt_plan_ws(&M.L, &o, &pb));
        L->plan_bytes.push_back(pb);
        L->plan_off.push_back(take(pb));
        nmax = std::max(nmax, M.L.n);
        blocks_max += (M.L.n + 31) / 32;
    }
    for (int32_t c = 0; c < d->num_cand; ++c) {
        int32_t m = d->h_cand_mat[c];
        RWT_REQUIRE(m >= 0 && m < d->count, RWT_ERR_INVALID_ARG, "candidate %d: bad matrix", c);
        RWT_REQUIRE(d->mats[m].L.n < (1 << 24), RWT_ERR_TOO_LARGE,
                    "candidate analysis supports matrices below 2^24 rows");
        RWT_REQUIRE(d->mats[m].L.n > 0, RWT_ERR_INVALID_ARG, "candidate %d: empty matrix", c);
    }
    L->bitmap_words = 0;
    L->lev_words = 0;
    for (int32_t c = 0; c < d->num_cand; ++c) {
        const int32_t n = d->mats[d->h_cand_mat[c]].L.n;
        L->bitmap_words += (n + 31) / 32 + 1;
        L->lev_words += n;
    }
    L->qcap = d->cand_rows_cap;
    int64_t pc = d->pattern_cap > 0 ? d->pattern_cap : (int64_t)64 * (L->qcap > 0 ? L->qcap : 1);
    RWT_REQUIRE(pc < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "pattern capacity too large");
    L->pat_cap = (int32_t)pc;
    L->slab_cap = nmax + 1;
    L->slab_stride = (int64_t)batch_rw_slab_stride(nmax);
    int64_t ntask = 0;
    for (int32_t m = 0; m < d->count; ++m)   // at most one chain per column
        if (d->mats[m].k > 0) ntask += (int64_t)d->mats[m].k * ((d->mats[m].L.n + 31) / 32);
    for (int32_t c = 0; c < d->num_cand; ++c) ntask += (d->mats[d->h_cand_mat[c]].L.n + 31) / 32;
    RWT_REQUIRE(ntask < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "too many tasks");
    L->ntasks_max = (int32_t)ntask;
    L->mats = take(sizeof(BatchMatDev) * std::max(1, d->count));
    L->cands = take(sizeof(BatchCandDev) * std::max(1, d->num_cand));
    L->candmat = take(sizeof(int32_t) * std::max(1, d->num_cand));
    L->rwmats = take(sizeof(BatchRwMat) * std::max(1, d->count));
    L->tasks = take(sizeof(int4) * std::max<int64_t>(1, ntask));
    L->bitmaps = take(sizeof(uint32_t) * std::max<int64_t>(1, L->bitmap_words));
    L->levs = take(sizeof(int32_t) * std::max<int64_t>(1, L->lev_words));
    L->done = take(sizeof(int32_t) * std::max(1, d->num_cand));
    L->bad = take(std::max(1, d->num_cand));
    L->stats = take(sizeof(rwt_cand_stats) * std::max(1, d->num_cand));
    L->counts = take(sizeof(int32_t) * ((size_t)L->qcap + 1));
    L->patptr = take(sizeof(int32_t) * ((size_t)L->qcap + 2));
    L->patptr2 = take(sizeof(int32_t) * ((size_t)L->qcap + 2));   // two-pass starts after one pass
    L->pat = take(sizeof(int32_t) * (size_t)L->pat_cap);
    L->ovf = take(sizeof(int32_t) * std::max(1, L->qcap));
    L->ovf2 = take(sizeof(int32_t) * std::max(1, L->qcap));
    L->ovfmark = take(std::max(1, L->qcap));
    L->rwctrl = take(sizeof(int32_t) * RWCTRL_WORDS);
    L->slab = take((size_t)NSLAB_B * (size_t)L->slab_stride);
    L->scan = take(scan_ws((int64_t)L->qcap + 1));
    L->ctrl = take(sizeof(Ctrl));
    L->epoch = take(sizeof(uint32_t));
    L->blkmin = take(sizeof(int32_t) * std::max<int64_t>(1, blocks_max));
    L->total = (off + 255) & ~size_t(255);
    return RWT_OK;
}

template <typename P>
P* at(void* base, size_t off) {
    return reinterpret_cast<P*>(static_cast<char*>(base) + off);
}

rwt_status enqueue_setup(rwt_batch* b, hipStream_t s);
rwt_status enqueue_main(rwt_batch* b, hipStream_t s);

rwt_status enqueue_run(rwt_batch* b, hipStream_t s, bool setup = true, bool main = true);

rwt_status enqueue_run(rwt_batch* b, hipStream_t s, bool setup, bool main) {
    if (setup) RWT_TRY(enqueue_setup(b, s));
    if (main) RWT_TRY(enqueue_main(b, s));
    return RWT_OK;
}

rwt_status enqueue_setup(rwt_batch* b, hipStream_t s) {
    const rwt_batch_desc& d = b->desc;
    const int32_t C = d.num_cand;
    hipLaunchKernelGGL(k_batch_epoch, dim3(1), dim3(64), 0, s, b->epoch);
    RWT_LAUNCHED();
    const int64_t work = std::max<int64_t>(std::max<int64_t>(b->bitmap_words, b->lev_words / 4),
                                           (int64_t)b->qcap + 1);
    const unsigned gb = std::max<unsigned>(blocks_for(work, 256, 4096), (unsigned)std::min(d.count, 4096));
    hipLaunchKernelGGL(k_batch_begin, dim3(gb), dim3(256), 0, s, b->d_mats, d.count, b->bitmaps,
                       b->bitmap_words, b->levs, b->lev_words, b->epoch, b->cand_done, b->cand_bad, C,
                       b->counts_q, b->ovf_mark, b->qcap, b->ctrl, b->rwctrl);
    RWT_LAUNCHED();
    if (C > 0) {
        hipLaunchKernelGGL(k_batch_ptrcheck, dim3(blocks_for((size_t)C, 256, 1024)), dim3(256), 0, s,
                           d.d_cand_ptr, C, b->qcap, b->rwctrl);
        RWT_LAUNCHED();
        hipLaunchKernelGGL(k_batch_bitmap, dim3(blocks_for((size_t)C * WAVE, 256, 4096)), dim3(256),
                           0, s, b->d_mats, b->d_cands, C, d.d_cand_ptr, d.d_cand_rows,
                           d.d_cand_targets, b->qcap, b->cand_bad, b->rwctrl);
        RWT_LAUNCHED();
        BatchRwArgs ra;
        ra.mats = b->d_rwmats;
        ra.cand_ptr = d.d_cand_ptr;
        ra.cand_mat = nullptr;
        ra.C = C;
        ra.qcap = b->qcap;
        ra.rows = d.d_cand_rows;
        ra.targets = d.d_cand_targets;
        ra.counts_q = b->counts_q;
        ra.pat_ptr = b->pat_ptr;
        ra.pat = b->pat;
        ra.pat_cap = b->pat_cap;
        ra.slot_len = b->slot_len;
        ra.bump = b->rwctrl + 16;
        ra.redo = b->rwctrl + 9;
        ra.gate = nullptr;
        ra.ovf = b->ovf;
        ra.ovf2 = b->ovf2;
        ra.ovf_mark = b->ovf_mark;
        ra.ctrl = b->rwctrl;
        ra.cand_bad = b->cand_bad;
        ra.slab = b->slab;
        ra.slab_stride = b->slab_stride;
        ra.slab_cap = b->slab_cap;
        ra.nslab = NSLAB_B;
        ra.cand_mat = b->d_cand_mat;
        if (b->slot_len > 0) {
            RWT_TRY(batch_rewrite_pass(ra, 3, s));
            // the two passes, which run only if the one pass did not fit
            const unsigned gq = blocks_for((size_t)b->qcap + 1, 256, 4096);
            ra.gate = b->rwctrl + 9;
            hipLaunchKernelGGL(k_batch_redo_reset, dim3(gq), dim3(256), 0, s, ra.gate, b->rwctrl,
                               b->counts_q, b->ovf_mark, b->qcap);
            RWT_LAUNCHED();
            RWT_TRY(batch_rewrite_pass(ra, 1, s));
            RWT_TRY(scan_exclusive(b->counts_q, b->pat_ptr2, b->qcap, b->scan_ws, s));
            ra.pat_ptr = b->pat_ptr2;
            RWT_TRY(batch_rewrite_pass(ra, 2, s));
            hipLaunchKernelGGL(k_copy_gated, dim3(gq), dim3(256), 0, s, ra.gate, b->pat_ptr2,
                               b->pat_ptr, (int64_t)b->qcap + 1);
            RWT_LAUNCHED();
        } else {
            RWT_TRY(batch_rewrite_pass(ra, 1, s));
            RWT_TRY(scan_exclusive(b->counts_q, b->pat_ptr, b->qcap, b->scan_ws, s));
            RWT_TRY(batch_rewrite_pass(ra, 2, s));
        }
    }
    return RWT_OK;
}

rwt_status enqueue_main(rwt_batch* b, hipStream_t s) {
    const rwt_batch_desc& d = b->desc;
    const int32_t C = d.num_cand;
    BatchKArgs ka;
    ka.mats = b->d_mats;
    ka.cands = b->d_cands;
    ka.tasks = b->d_tasks;
    ka.ntasks = b->ntasks;
    ka.C = C;
    ka.cand_ptr = d.d_cand_ptr;
    ka.rows = d.d_cand_rows;
    ka.counts_q = b->counts_q;
    ka.pat_ptr = b->pat_ptr;
    ka.pat = b->pat;
    ka.cand_bad = b->cand_bad;
    ka.cand_done = b->cand_done;
    ka.stats = b->stats;
    ka.ctrl = b->ctrl;
    ka.epoch = b->epoch;
    ka.ticks = watchdog_ticks(d.watchdog_ms);
    ka.hist_cap = (b->lds_bytes - 256) / 4;
    ka.qcap = b->qcap;
    if (b->ntasks > 0) {
        hipLaunchKernelGGL(k_batch_main, dim3(b->grid), dim3(BT_THREADS), b->lds_bytes, s, ka);
        RWT_LAUNCHED();
    }
    return RWT_OK;
}

}  // namespace

// LDS of a row-block level task of gs candidates (levels, step starts, list
// ranges) and the group size of a matrix's chains: as many candidates as fit
// in half the LDS budget, so that the launch keeps four workgroups per CU
size_t chain_lds(size_t R, int32_t gs) {
    return ((R * (size_t)gs * 4 + 15) & ~size_t(15)) + (((R + 1 + 3) & ~size_t(3)) * 4) +
           2 * SG * 4 + 16;
}
int32_t chain_group(int32_t R) {
    int32_t gs = SG;
    while (gs > 1 && chain_lds((size_t)R, gs) > (size_t)BT_LDS / 2) --gs;
    return gs;
}

extern "C" rwt_status rwt_batch_ws(const rwt_batch_desc* desc, size_t* h_bytes) {
    RWT_REQUIRE(h_bytes != nullptr, RWT_ERR_INVALID_ARG, "h_bytes is NULL");
    BatchLayout L;
    RWT_TRY(layout_batch(desc, &L));
    *h_bytes = L.total;
    return RWT_OK;
}

extern "C" rwt_status rwt_batch_create(const rwt_batch_desc* desc, void* d_ws, size_t ws_bytes,
                                       rwt_batch** out, rwt_stream_t stream) {
    RWT_REQUIRE(out != nullptr, RWT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    const auto t0 = std::chrono::steady_clock::now();
    BatchLayout L;
    RWT_TRY(layout_batch(desc, &L));
    RWT_REQUIRE(d_ws != nullptr && ws_bytes >= L.total, RWT_ERR_BUFFER_TOO_SMALL,
                "batch workspace must hold %zu bytes", L.total);
    hipStream_t s = hs(stream);
    rwt_batch* b = new (std::nothrow) rwt_batch();
    RWT_REQUIRE(b != nullptr, RWT_ERR_INVALID_ARG, "out of host memory");
    auto fail = [&](rwt_status e) {
        for (rwt_plan* p : b->plans) rwt_plan_destroy(p);
        delete b;
        return e;
    };
    b->desc = *desc;
    b->mats.assign(desc->mats, desc->mats + desc->count);
    b->cand_mat.assign(desc->h_cand_mat, desc->h_cand_mat + desc->num_cand);
    b->desc.mats = b->mats.data();
    b->desc.h_cand_mat = b->cand_mat.data();
    // per-matrix plans: analysis, schedule, autotuned block size
    std::vector<BatchMatDev> hm(desc->count);
    std::vector<BatchRwMat> hr(desc->count);
    for (int32_t m = 0; m < desc->count; ++m) {
        const rwt_batch_matrix& M = b->mats[m];
        rwt_plan_opts o = batch_plan_opts(desc, M);
        rwt_plan* p = nullptr;
        rwt_status st = rwt_plan_create(&M.L, &o, at<char>(d_ws, L.plan_off[m]), L.plan_bytes[m],
                                        &p, stream);
        if (st != RWT_OK) return fail(st);
        b->plans.push_back(p);
        // the row-order walk where the plan's model finds that consecutive
        // rows span few levels (deep, thin DAGs); the plan then solves with
        // it too, so per-matrix solves match the batch bit for bit
        const bool walk = p->walk_ok;
        if (walk) p->fwd = p->bwd = Algo::Walk;
        BatchMatDev& d = hm[m];
        memset(&d, 0, sizeof d);
        d.n = M.L.n;
        d.R = p->R;
        d.lanes = p->lanes;
        d.nblocks = p->nblocks;
        d.k = M.k;
        d.kc = p->kc;
        d.ldb = M.ldb;
        d.ldx = M.ldx;
        d.rowptr = M.L.rowptr;
        d.colidx = M.L.colidx;
        d.level = p->level;
        d.vals = static_cast<const double*>(M.L.vals);
        d.desc = p->desc_f;
        d.step_pos = p->step_pos;
        d.blk_step = p->blk_step;
        d.D = p->D;
        d.perm = p->perm;
        d.lptr = p->level_ptr;
        d.B = static_cast<const double*>(M.B);
        d.X = static_cast<double*>(M.X);
        d.walk = walk ? 1 : 0;
        d.pad_w = 0;
        hr[m].n = M.L.n;
        hr[m].pad = 0;
        hr[m].rowptr = M.L.rowptr;
        hr[m].colidx = M.L.colidx;
        hr[m].level = p->level;
    }
    b->d_mats = at<BatchMatDev>(d_ws, L.mats);
    b->d_cands = at<BatchCandDev>(d_ws, L.cands);
    b->d_rwmats = at<BatchRwMat>(d_ws, L.rwmats);
    b->d_cand_mat = at<int32_t>(d_ws, L.candmat);
    b->d_tasks = at<int4>(d_ws, L.tasks);
    b->bitmaps = at<uint32_t>(d_ws, L.bitmaps);
    b->bitmap_words = L.bitmap_words;
    b->levs = at<int32_t>(d_ws, L.levs);
    b->lev_words = L.lev_words;
    b->cand_done = at<int32_t>(d_ws, L.done);
    b->cand_bad = at<unsigned char>(d_ws, L.bad);
    b->stats = at<rwt_cand_stats>(d_ws, L.stats);
    b->counts_q = at<int32_t>(d_ws, L.counts);
    b->pat_ptr = at<int32_t>(d_ws, L.patptr);
    b->pat_ptr2 = at<int32_t>(d_ws, L.patptr2);
    b->pat = at<int32_t>(d_ws, L.pat);
    b->ovf = at<int32_t>(d_ws, L.ovf);
    b->ovf2 = at<int32_t>(d_ws, L.ovf2);
    b->ovf_mark = at<unsigned char>(d_ws, L.ovfmark);
    b->rwctrl = at<int32_t>(d_ws, L.rwctrl);
    b->slab = at<unsigned char>(d_ws, L.slab);
    b->slab_stride = L.slab_stride;
    b->slab_cap = L.slab_cap;
    b->scan_ws = at<char>(d_ws, L.scan);
    b->ctrl = at<Ctrl>(d_ws, L.ctrl);
    b->epoch = at<uint32_t>(d_ws, L.epoch);
    b->qcap = L.qcap;
    b->pat_cap = L.pat_cap;
    b->slot_len = (int64_t)L.pat_cap >= (int64_t)PATTERN_ONE_PASS_MIN * L.qcap ? PATTERN_SLOT : 0;
    // candidates: matrix, bitmap and level array slices
    std::vector<BatchCandDev> hc(desc->num_cand);
    {
        int64_t bw = 0, lw = 0;
        for (int32_t c = 0; c < desc->num_cand; ++c) {
            const int32_t n = b->mats[b->cand_mat[c]].L.n;
            hc[c].m = b->cand_mat[c];
            hc[c].pad = 0;
            hc[c].bitmap = b->bitmaps + bw;
            hc[c].lev = b->levs + lw;
            bw += (n + 31) / 32 + 1;
            lw += n;
        }
    }
    // task table.  A chain (one matrix's solve, or one candidate's levels)
    // is its row blocks in row order.  A task is keyed by the level at which
    // it can first do work: the lowest level of its rows, raised to the
    // running maximum along the chain so that keys never decrease inside a
    // chain.  Sorting all tasks by key (stably) keeps each chain in row
    // order -- a task waits only for tasks with earlier tickets, so the
    // schedule is deadlock-free for any number of resident workgroups --
    // and claims a task roughly when its dependencies are done, instead of
    // letting tasks of deep chains hold workgroups while they wait.
    std::vector<int64_t> blk_off(desc->count + 1, 0);
    for (int32_t m = 0; m < desc->count; ++m) blk_off[m + 1] = blk_off[m] + hm[m].nblocks;
    std::vector<int32_t> minlev(std::max<int64_t>(1, blk_off[desc->count]), 0);
    {
        int32_t* d_min = at<int32_t>(d_ws, L.blkmin);
        const int64_t tot = blk_off[desc->count];
        if (tot > 0) {
            hipLaunchKernelGGL(k_fill_i32max, dim3(blocks_for(tot, 256, 1024)), dim3(256), 0, s, d_min,
                               tot);
            for (int32_t m = 0; m < desc->count; ++m)
                if (hm[m].n > 0)
                    hipLaunchKernelGGL(k_block_minlev, dim3(blocks_for(hm[m].n, 256, 1024)), dim3(256), 0,
                                       s, hm[m].level, hm[m].n, hm[m].R, d_min + blk_off[m]);
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(minlev.data(), d_min, sizeof(int32_t) * tot, hipMemcpyDeviceToHost, s) !=
                    hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                set_hip_error(hipGetLastError(), "batch task keys");
                return fail(RWT_ERR_HIP);
            }
        }
    }
    std::vector<int32_t> cand_count(desc->count, 0);
    // candidate mode per matrix: the level sweep when the block chain has
    // many more level steps than the matrix has levels
    {
        std::vector<int32_t> steps(desc->count, 0);
        for (int32_t m = 0; m < desc->count; ++m)
            if (hm[m].nblocks > 0 &&
                hipMemcpyAsync(&steps[m], hm[m].blk_step + hm[m].nblocks, sizeof(int32_t),
                               hipMemcpyDeviceToHost, s) != hipSuccess) {
                set_hip_error(hipGetLastError(), "batch step counts");
                return fail(RWT_ERR_HIP);
            }
        if (hipStreamSynchronize(s) != hipSuccess) {
            set_hip_error(hipGetLastError(), "batch step counts");
            return fail(RWT_ERR_HIP);
        }
        for (int32_t c = 0; c < desc->num_cand; ++c) cand_count[hc[c].m] += 1;
        for (int32_t m = 0; m < desc->count; ++m) {
            // candidates: the walk (levels below 2^23, the walk's matrices, or
            // every matrix with cand_mode 3), else the sweep or the chains
            hm[m].walk = hm[m].D < (1 << 23) &&
                         (desc->cand_mode == 3 || (desc->cand_mode == 0 && hm[m].walk));
            hm[m].sweep = !hm[m].walk && hm[m].D < (1 << 23) &&
                          (desc->cand_mode == 2 ||
                           (desc->cand_mode == 0 && (int64_t)steps[m] >= 4 * (int64_t)hm[m].D));
        }
    }
    {
        DeviceInfo di;
        rwt_status st0 = device_info(&di);
        if (st0 != RWT_OK) return fail(st0);
        // LDS of the launch: what its task bodies use (solve blocks: x values
        // and step starts; level blocks: levels and step starts), at least
        // 16 KB for the histogram of the statistics -- not the whole budget,
        // so that more workgroups fit on a compute unit
        {
            size_t need = 16384;
            for (int32_t m = 0; m < desc->count; ++m) {
                const size_t R = (size_t)hm[m].R;
                if (b->plans[m]->fwd == Algo::Walk && b->mats[m].k > 0)
                    need = std::max(need, (size_t)WK_SOLVE_WAVES * wk_lds_bytes<double>());
                if (hm[m].walk && cand_count[m] > 0)
                    need = std::max(need, (size_t)WK_LEVEL_WAVES * sizeof(WkLvlLds));
                if (b->mats[m].k > 0 && b->plans[m]->fwd != Algo::Walk)
                    need = std::max(need, (size_t)sf_x_bytes((int)R, hm[m].kc, 8) + (R + 1) * 4 + 16);
                if (!hm[m].sweep && !hm[m].walk && cand_count[m] > 0)
                    need = std::max(need, chain_lds(R, chain_group(R)));
            }
            need = (need + 255) & ~size_t(255);
            b->lds_bytes = (int32_t)std::min<size_t>(need, BT_LDS);
        }
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_batch_main, BT_THREADS,
                                                          b->lds_bytes) != hipSuccess ||
            per_cu < 1)
            per_cu = 1;
        b->grid = di.cus * std::min(per_cu, 8);
    }
    struct T {
        int32_t key;
        int4 t;
    };
    std::vector<T> tv;
    auto add_chain = [&](int32_t m, int kind, int32_t id, int32_t chunk) {
        int32_t run = 0;
        for (int32_t k = 0; k < hm[m].nblocks; ++k) {
            run = std::max(run, minlev[blk_off[m] + k]);
            tv.push_back({run, make_int4(kind, id, k, chunk)});
        }
    };
    // one solve chain per chunk of kc right-hand-side columns; row-order
    // walks, which wait on nothing, longest first (interleaved below)
    for (int32_t m = 0; m < desc->count; ++m) {
        if (b->plans[m]->fwd == Algo::Walk) {
            for (int32_t q = 0; q < b->mats[m].k; q += WK_SOLVE_WAVES)
                tv.push_back({-hm[m].n, make_int4(3, m, q, std::min(WK_SOLVE_WAVES, b->mats[m].k - q))});
            continue;
        }
        for (int32_t c = 0; c * hm[m].kc < b->mats[m].k; ++c) add_chain(m, 0, m, c);
    }
    b->solve_tasks = (int32_t)tv.size();
    // sweep candidates go in groups: up to gmax consecutive candidates of one
    // matrix (their level arrays are adjacent), one task each, ready at once.
    // Larger groups read less (one read of a dependency serves the group)
    // but leave fewer tasks; gmax keeps about two thirds of the grid busy.
    int32_t nsweep = 0;
    for (int32_t c = 0; c < desc->num_cand; ++c) nsweep += hm[hc[c].m].sweep ? 1 : 0;
    const int32_t gmax = std::max<int32_t>(
        1, std::min<int32_t>(SG, (nsweep + (2 * b->grid / 3) - 1) / std::max(1, 2 * b->grid / 3)));
    b->sweep_cands = 0;
    for (int32_t c = 0; c < desc->num_cand;) {
        const int32_t m = hc[c].m;
        if (hm[m].walk) {
            int32_t gs = 1;
            while (gs < WK_LEVEL_WAVES && c + gs < desc->num_cand && hc[c + gs].m == m) ++gs;
            tv.push_back({-hm[m].n, make_int4(4, c, gs, 0)});
            c += gs;
            continue;
        }
        if (!hm[m].sweep) {
            // level chains in groups too: up to chain_group(R) consecutive
            // candidates of the matrix share each row-block task
            const int32_t gb = chain_group(hm[m].R);
            int32_t gs = 1;
            while (gs < gb && c + gs < desc->num_cand && hc[c + gs].m == m) ++gs;
            add_chain(m, 1, c, gs);
            c += gs;
            continue;
        }
        int32_t gs = 1;
        while (gs < gmax && c + gs < desc->num_cand && hc[c + gs].m == m) ++gs;
        tv.push_back({0, make_int4(2, c, gs, 0)});
        b->sweep_cands += gs;
        c += gs;
    }
    std::stable_sort(tv.begin(), tv.end(), [](const T& x, const T& y) { return x.key < y.key; });
    // Walks (kinds 3 and 4, longest first) wait on nothing but hold their
    // workgroup for the whole walk while using little of the compute unit;
    // claimed all at once they would fill the grid and hold back the level
    // chains and sweeps. They are interleaved instead, one claim in
    // WALK_CLAIM_EVERY, for as long as both lists last; the other tasks keep
    // their order, which is topological along every chain.
    std::vector<int4> tasks(tv.size());
    {
        std::vector<int4> walks, rest;
        for (const T& x : tv) (x.t.x == 3 || x.t.x == 4 ? walks : rest).push_back(x.t);
        size_t iw = 0, ir = 0;
        for (size_t p = 0; p < tv.size(); ++p) {
            const bool walk = iw < walks.size() &&
                              (ir >= rest.size() || iw * WALK_CLAIM_EVERY < p + 1);
            tasks[p] = walk ? walks[iw++] : rest[ir++];
        }
    }
    b->ntasks = (int32_t)tasks.size();
    if (hipMemcpyAsync(b->d_mats, hm.data(), sizeof(BatchMatDev) * hm.size(), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        hipMemcpyAsync(b->d_rwmats, hr.data(), sizeof(BatchRwMat) * hr.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->d_cands, hc.data(), sizeof(BatchCandDev) * hc.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(b->d_tasks, tasks.data(), sizeof(int4) * tasks.size(), hipMemcpyHostToDevice,
                       s) != hipSuccess ||
        (desc->num_cand > 0 &&
         hipMemcpyAsync(b->d_cand_mat, b->cand_mat.data(), sizeof(int32_t) * b->cand_mat.size(),
                        hipMemcpyHostToDevice, s) != hipSuccess)) {
        set_hip_error(hipGetLastError(), "batch table upload");
        return fail(RWT_ERR_HIP);
    }
    rwt_status st;
    if ((st = fill_u8(b->levs, (int64_t)sizeof(int32_t) * std::max<int64_t>(1, b->lev_words), s)) !=
            RWT_OK ||
        (st = fill_u8(b->epoch, sizeof(uint32_t), s)) != RWT_OK)
        return fail(st);
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_hip_error(hipGetLastError(), "batch creation");
        return fail(RWT_ERR_HIP);
    }
    b->create_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    *out = b;
    return RWT_OK;
}

extern "C" rwt_status rwt_batch_run(rwt_batch* b, rwt_stream_t stream) {
    RWT_REQUIRE(b != nullptr, RWT_ERR_INVALID_ARG, "null batch");
    return enqueue_run(b, hs(stream));
}

extern "C" rwt_status rwt_batch_run_setup(rwt_batch* b, rwt_stream_t stream) {
    RWT_REQUIRE(b != nullptr, RWT_ERR_INVALID_ARG, "null batch");
    return enqueue_setup(b, hs(stream));
}

extern "C" rwt_status rwt_batch_run_main(rwt_batch* b, rwt_stream_t stream) {
    RWT_REQUIRE(b != nullptr, RWT_ERR_INVALID_ARG, "null batch");
    return enqueue_main(b, hs(stream));
}

extern "C" rwt_status rwt_batch_capture(rwt_batch* b, rwt_stream_t stream) {
    RWT_REQUIRE(b != nullptr, RWT_ERR_INVALID_ARG, "null batch");
    RWT_REQUIRE(stream != nullptr, RWT_ERR_INVALID_ARG, "capture needs a non-default stream");
    hipStream_t s = hs(stream);
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    RWT_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    rwt_status st = enqueue_run(b, s);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != RWT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    RWT_HIP(e);
    b->graph = g;
    RWT_HIP(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return RWT_OK;
}

extern "C" rwt_status rwt_batch_launch(rwt_batch* b, rwt_stream_t stream) {
    RWT_REQUIRE(b != nullptr && b->exec != nullptr, RWT_ERR_INVALID_ARG,
                "no captured graph: call rwt_batch_capture first");
    RWT_HIP(hipGraphLaunch(b->exec, hs(stream)));
    return RWT_OK;
}

extern "C" rwt_status rwt_batch_stats(const rwt_batch* b, rwt_cand_stats* h_out,
                                      rwt_stream_t stream) {
    RWT_REQUIRE(b != nullptr, RWT_ERR_INVALID_ARG, "null batch");
    hipStream_t s = hs(stream);
    Ctrl hc;
    int32_t rc[8];
    RWT_HIP(hipMemcpyAsync(&hc, b->ctrl, sizeof hc, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipMemcpyAsync(rc, b->rwctrl, sizeof rc, hipMemcpyDeviceToHost, s));
    if (h_out && b->desc.num_cand > 0)
        RWT_HIP(hipMemcpyAsync(h_out, b->stats, sizeof(rwt_cand_stats) * b->desc.num_cand,
                               hipMemcpyDeviceToHost, s));
    RWT_HIP(hipStreamSynchronize(s));
    if (hc.err != 0) {
        set_error("a device wait expired in the batch (watchdog)");
        return RWT_ERR_DEADLOCK;
    }
    if (rc[3] != 0 || rc[4] != 0) {
        set_error("rewritten-row patterns exceeded the batch capacity");
        return RWT_ERR_TOO_LARGE;
    }
    if (rc[5] != 0) {
        set_error("some candidate row lists were rejected (unsorted, out of range or over capacity)");
        return RWT_ERR_BAD_ROWSET;
    }
    return RWT_OK;
}

extern "C" rwt_status rwt_batch_get_info(const rwt_batch* b, rwt_batch_info* h) {
    RWT_REQUIRE(b != nullptr && h != nullptr, RWT_ERR_INVALID_ARG, "null argument");
    h->tasks = b->ntasks;
    h->solve_tasks = b->solve_tasks;
    h->grid = b->grid;
    h->captured = b->exec != nullptr;
    h->create_ms = b->create_ms;
    h->sweep_cands = b->sweep_cands;
    h->pattern_slot = b->slot_len;
    return RWT_OK;
}

extern "C" rwt_status rwt_batch_plan(const rwt_batch* b, int32_t m, const rwt_plan** out) {
    RWT_REQUIRE(b != nullptr && out != nullptr && m >= 0 && m < (int32_t)b->plans.size(),
                RWT_ERR_INVALID_ARG, "bad matrix index");
    *out = b->plans[m];
    return RWT_OK;
}

extern "C" rwt_status rwt_batch_destroy(rwt_batch* b) {
    if (!b) return RWT_OK;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    for (rwt_plan* p : b->plans) rwt_plan_destroy(p);
    delete b;
    return RWT_OK;
}
