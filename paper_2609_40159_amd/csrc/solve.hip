// Forward substitution L X = B and its transpose L^T Y = G (paper Section
// 2.1: x_i = (b_i - sum_j L_ij x_j) / L_ii once every dependency j is done;
// the transposed system runs the same recurrence over successors, levels in
// reverse order).
//
// Readiness travels with the data: before a solve X is filled with a
// signalling-NaN sentinel, a row's result is published with one
// device-scope store, and a reader of another workgroup's row spins
// (bounded) until the sentinel is gone.  No device-scope fences are used.
//
// Two schedules:
//   level-scheduled  (k_solve_level): one level after another, each spread
//       over the whole grid, every wave taking the same share of each level
//       in turn (Section 2.1; the level-set method of Section 7).  No grid
//       barrier between levels: a row reads its dependencies with the
//       sentinel wait, so a wave starts its share of the next level as soon
//       as its own share of this one is done, and waits only for the values
//       it needs.  Its first group of rows of each level is loaded ahead
//       (bounds, descriptors, first entries: three, two and one levels
//       ahead), so that a level's critical path is the dependencies' values
//       alone.  Deadlock-free: every workgroup is resident (one per compute
//       unit) and waits only on earlier levels.
//   sync-free        (k_solve_sf): blocks of consecutive rows are claimed
//       in row order from a ticket counter (deadlock-free: a block waits
//       only on rows of earlier tickets).  Inside a block the rows go level
//       by level with workgroup barriers and the block's x values live in
//       LDS; dependencies outside the block are read from HBM with the
//       sentinel wait (Section 7, synchronization-free methods).
// A row is processed by a group of G lanes (rows-per-wavefront = 64/G):
// strided partial dot products, then a butterfly reduction in the group.
#include "solve.hpp"

#include "sf_block.hpp"
#include "sf_staged.hpp"
#include "walk.hpp"

#include "prim.hpp"

namespace rwt {

namespace {

constexpr int SV_THREADS = 256;

template <typename T, bool TRANS, int KT, bool LOCAL>
__device__ __forceinline__ void solve_row(const SolveArgs& a, bool active, int32_t i, int gl, int G,
                                          T* xs, int32_t r0, int32_t r1) {
    const T* vals = static_cast<const T*>(a.vals);
    const T* B = static_cast<const T*>(a.B);
    T* X = static_cast<T*>(a.X);
    int32_t pb = 0, pe = 0;
    T diag = T(1);
    if (active) {
        if (!TRANS) {
            pb = a.rowptr[i];
            pe = a.rowptr[i + 1] - 1;
            diag = vals[pe];
        } else {
            pb = a.cptr[i];
            pe = a.cptr[i + 1];
            diag = vals[a.rowptr[i + 1] - 1];
        }
    }
    int32_t* err = &a.ctrl->err;
    for (int q0 = 0; q0 < a.k; q0 += KT) {
        T acc[KT];
#pragma unroll
        for (int t = 0; t < KT; ++t) acc[t] = T(0);
        for (int32_t p = pb + gl; p < pe; p += G) {
            int32_t j;
            T v;
            if (!TRANS) {
                j = a.colidx[p];
                v = vals[p];
            } else {
                j = a.crow[p];
                v = vals[a.cmap[p]];
            }
            const bool local = LOCAL && (TRANS ? (j < r1) : (j >= r0));
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const int q = q0 + t;
                if (KT == 1 || q < a.k) {
                    T xj = local ? xs[(int64_t)(j - r0) * a.k + q]
                                 : wait_value(&X[j + (int64_t)q * a.ldx], err, a.ticks);
                    acc[t] += v * xj;
                }
            }
        }
#pragma unroll
        for (int t = 0; t < KT; ++t) acc[t] = group_sum(acc[t], G);
        if (active && gl == 0) {
#pragma unroll
            for (int t = 0; t < KT; ++t) {
                const int q = q0 + t;
                if (KT == 1 || q < a.k) {
                    T xi = (B[i + (int64_t)q * a.ldb] - acc[t]) / diag;
                    if (LOCAL) xs[(int64_t)(i - r0) * a.k + q] = xi;
                    if (i != a.hold_row) st_relaxed(&X[i + (int64_t)q * a.ldx], xi);
                }
            }
        }
    }
}

// Sentinel prefill of the n x k solution block (column stride ldx) and reset
// of the solve's control words, in one launch.
static_assert(sizeof(Ctrl) % 4 == 0 && sizeof(Ctrl) / 4 <= 256, "control words");
template <typename T>
__global__ void __launch_bounds__(256) k_prefill(T* X, int64_t ldx, int32_t n, int32_t k,
                                                 uint32_t* ctrl) {
    if (blockIdx.x == 0 && threadIdx.x < sizeof(Ctrl) / 4) ctrl[threadIdx.x] = 0u;
    const T s = sentinel_value<T>();
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 1 || ldx == n) {   // one contiguous run of n * k values
        const int64_t total = (int64_t)n * k;
        for (int64_t t = t0; t < total; t += st) X[t] = s;
    } else {
        for (int32_t q = 0; q < k; ++q)
            for (int64_t i = t0; i < n; i += st) X[i + (int64_t)q * ldx] = s;
    }
}

// A wave's first group of rows of one level, loaded ahead of the level in
// three stages: the level's bounds (three levels ahead), the rows'
// descriptors (two ahead), each lane's first entry and the diagonal (one
// ahead).  Forward descriptors {row, first entry, last off-diagonal entry,
// diagonal}; transposed {row, successor-list start, end, diagonal}.
template <typename T>
struct LvlAhead {
    int32_t beg, end;   // level bounds in level order
    int4 d;             // this lane's row (d.x < 0: no row)
    int32_t j, m;       // first entry: dependency row; transposed: value position
    T v, diag;
};

template <typename T, bool TRANS, int KT>
__global__ void __launch_bounds__(SV_THREADS) k_solve_level(SolveArgs a) {
    const int G = a.lanes;
    const int gl = threadIdx.x & (G - 1);
    const int lane = lane_id();
    const int groups_per_wave = WAVE / G;
    const int wave_in_block = threadIdx.x / WAVE;
    const int waves_per_block = blockDim.x / WAVE;
    const int32_t gwave = blockIdx.x * waves_per_block + wave_in_block;
    const int32_t stride = gridDim.x * waves_per_block * groups_per_wave;
    const int32_t first = gwave * groups_per_wave + lane / G;   // offset of this lane's row in a level
    const int32_t D = a.nlev;
    const T* vals = static_cast<const T*>(a.vals);
    const T* B = static_cast<const T*>(a.B);
    T* X = static_cast<T*>(a.X);
    int32_t* err = &a.ctrl->err;
    // level of the li-th step (levels past the last repeat it; never used)
    auto lvl = [&](int32_t li) { li = min(li, D - 1); return TRANS ? D - 1 - li : li; };
    auto stage_bounds = [&](LvlAhead<T>& s, int32_t li) {
        const int32_t l = lvl(li);
        s.beg = a.level_ptr[l];
        s.end = a.level_ptr[l + 1];
    };
    auto stage_desc = [&](LvlAhead<T>& s) {
        const int32_t q = s.beg + first;
        s.d = q < s.end ? a.ldesc[q] : make_int4(-1, 0, 0, 0);
    };
    auto stage_entry = [&](LvlAhead<T>& s) {
        const bool act = s.d.x >= 0;
        const int32_t p0 = s.d.y + gl;
        const bool has = act && p0 < s.d.z;
        s.j = 0;
        s.m = 0;
        s.v = T(0);
        if (has) {
            s.j = TRANS ? a.crow[p0] : a.colidx[p0];
            if (TRANS) s.m = a.cmap[p0];
            else s.v = vals[p0];
        }
        s.diag = act ? vals[s.d.w] : T(1);
    };
    // one group of rows: the lane's first entry from the stage, the others
    // loaded here; the same order of terms as solve_row
    auto run_group = [&](const LvlAhead<T>& s) {
        const bool act = s.d.x >= 0;
        const int32_t i = s.d.x, pb = s.d.y, pe = s.d.z;
        const bool has = act && pb + gl < pe;
        const T v0 = TRANS ? (has ? vals[s.m] : T(0)) : s.v;
        for (int q0 = 0; q0 < a.k; q0 += KT) {
            T acc[KT];
#pragma unroll
            for (int t = 0; t < KT; ++t) acc[t] = T(0);
            if (has) {
#pragma unroll
                for (int t = 0; t < KT; ++t) {
                    const int q = q0 + t;
                    if (KT == 1 || q < a.k)
                        acc[t] += v0 * wait_value(&X[s.j + (int64_t)q * a.ldx], err, a.ticks);
                }
            }
            for (int32_t p = pb + gl + G; act && p < pe; p += G) {
                const int32_t j = TRANS ? a.crow[p] : a.colidx[p];
                const T v = TRANS ? vals[a.cmap[p]] : vals[p];
#pragma unroll
                for (int t = 0; t < KT; ++t) {
                    const int q = q0 + t;
                    if (KT == 1 || q < a.k) acc[t] += v * wait_value(&X[j + (int64_t)q * a.ldx], err, a.ticks);
                }
            }
#pragma unroll
            for (int t = 0; t < KT; ++t) acc[t] = group_sum(acc[t], G);
            if (act && gl == 0) {
#pragma unroll
                for (int t = 0; t < KT; ++t) {
                    const int q = q0 + t;
                    if (KT == 1 || q < a.k) {
                        const T xi = (B[i + (int64_t)q * a.ldb] - acc[t]) / s.diag;
                        if (i != a.hold_row) st_relaxed(&X[i + (int64_t)q * a.ldx], xi);
                    }
                }
            }
        }
    };
    if (D <= 0) return;
    // the pipeline: s0 = this level, s1 = next (descriptor and entry
    // loaded), s2 = the one after (descriptor), s3 = bounds only
    LvlAhead<T> s0, s1, s2, s3;
    stage_bounds(s0, 0);
    stage_bounds(s1, 1);
    stage_bounds(s2, 2);
    stage_desc(s0);
    stage_desc(s1);
    stage_entry(s0);
    for (int32_t li = 0; li < D; ++li) {
        // the next levels' loads first: nothing below waits for them
        stage_bounds(s3, li + 3);
        stage_desc(s2);
        stage_entry(s1);
        run_group(s0);
        // rows of this level past the wave's first group (levels wider
        // than the grid's groups): loaded as they come
        for (int32_t base = s0.beg + gwave * groups_per_wave + stride; base < s0.end;
             base += stride) {
            const int32_t q = base + lane / G;
            const bool act = q < s0.end;
            solve_row<T, TRANS, KT, false>(a, act, act ? a.perm[q] : 0, gl, G, nullptr, 0, 0);
        }
        s0 = s1;
        s1 = s2;
        s2 = s3;
    }
}

template <typename T, bool TRANS, int KT>
__global__ void __launch_bounds__(SV_THREADS) k_solve_sf(SolveArgs a) {
    extern __shared__ __align__(16) unsigned char s_raw[];
    __shared__ int32_t s_blk;
    SfBlockArgs b;
    b.k = a.k;
    b.lanes = a.lanes;
    b.stage_x = a.stage_x;
    b.ldb = a.ldb;
    b.ldx = a.ldx;
    b.colidx = a.colidx;
    b.crow = a.crow;
    b.cmap = a.cmap;
    b.vals = a.vals;
    b.desc = a.desc;
    b.step_pos = a.step_pos;
    b.B = a.B;
    b.X = a.X;
    b.err = &a.ctrl->err;
    b.ticks = a.ticks;
    b.lds_rows = a.block_rows;
    b.hold_row = a.hold_row;
    // tasks: (row block, column chunk) with the chunks of one block on
    // consecutive tickets; each chunk's blocks follow row order (reverse for
    // the transposed solve), so a task waits only on earlier tickets
    const int32_t nch = (a.k + a.kc - 1) / a.kc;
    const int64_t ntask = (int64_t)a.nblocks * nch;
    for (;;) {
        if (threadIdx.x == 0) s_blk = (int32_t)fetch_add(&a.ctrl->ticket, 1u);
        __syncthreads();
        const int64_t t = (uint32_t)s_blk;
        __syncthreads();
        if (t >= ntask) break;
        const int32_t tb = (int32_t)(t / nch), c = (int32_t)(t - (int64_t)tb * nch);
        const int32_t blk = TRANS ? a.nblocks - 1 - tb : tb;
        const int32_t q0 = c * a.kc;
        b.k = min(a.kc, a.k - q0);
        b.B = static_cast<const T*>(a.B) + (int64_t)q0 * a.ldb;
        b.X = static_cast<T*>(a.X) + (int64_t)q0 * a.ldx;
        b.r0 = blk * a.block_rows;
        b.r1 = min(a.n, b.r0 + a.block_rows);
        b.sb = a.blk_step[blk];
        b.ns = a.blk_step[blk + 1] - b.sb;
        sf_block_staged<T, TRANS, KT>(b, s_raw);
        if (ld_relaxed(&a.ctrl->err) != 0) break;
    }
}

// One column per workgroup of two waves (walk.hpp, the two-wave walk: one
// wave stages and sums each chunk's older terms while the other finishes
// the chunk before).
template <typename T, bool TRANS>
__global__ void __launch_bounds__(2 * WAVE) k_solve_walk(SolveArgs a) {
    extern __shared__ __align__(16) unsigned char s_raw[];
    const int32_t q = blockIdx.x;
    if (q >= a.k) return;
    WkLds2<T>* L = reinterpret_cast<WkLds2<T>*>(s_raw);
    WkArgs wa;
    wa.n = a.n;
    wa.ptr = TRANS ? a.cptr : a.rowptr;
    wa.idx = TRANS ? a.crow : a.colidx;
    wa.vals = TRANS ? a.vt : a.vals;
    wa.rowptr = a.rowptr;
    wa.dvals = a.vals;
    wa.b = static_cast<const T*>(a.B) + (int64_t)q * a.ldb;
    wa.x = static_cast<T*>(a.X) + (int64_t)q * a.ldx;
    wa.err = &a.ctrl->err;
    wk_solve2<T, TRANS>(wa, L);
}

template <typename T>
__global__ void k_gather_vals(const int32_t* map, int64_t m, const T* vals, T* out) {
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += st)
        out[p] = vals[map[p]];
}

// The rounds the walk would take on each 64-row chunk (the longest chain
// of dependencies inside the chunk, plus one), summed over the chunks: the
// walk's rounds without its values, one wave per chunk.
__global__ void k_chunk_rounds(const int32_t* rowptr, const int32_t* colidx, int32_t n,
                               unsigned long long* out) {
    const int lane = lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int64_t nch = ((int64_t)n + WAVE - 1) / WAVE;
    unsigned long long acc = 0;
    for (int64_t c = wave; c < nch; c += nw) {
        const int32_t lo = (int32_t)(c * WAVE);
        const int32_t i = lo + lane;
        uint64_t dep = 0;
        if (i < n)
            for (int32_t p = rowptr[i + 1] - 2; p >= rowptr[i]; --p) {   // last entry: diagonal
                const int32_t j = colidx[p];
                if (j < lo) break;                                     // columns ascend
                if (j < i) dep |= 1ull << (j - lo);
            }
        uint64_t done = __ballot(i >= n);
        int rounds = 0;
        while (done != ~0ull && rounds < WAVE) {
            done |= __ballot(!((done >> lane) & 1ull) && (dep & ~done) == 0);
            ++rounds;
        }
        acc += (unsigned long long)rounds;
    }
    if (lane == 0 && acc != 0) atomicAdd(out, acc);
}

template <typename T, bool TRANS>
rwt_status launch_typed(const SolveArgs& a, Algo algo, unsigned grid, hipStream_t s) {
    const bool multi = (algo == Algo::Level ? a.k : a.kc) > 1;
    if (algo == Algo::Level) {
        if (multi)
            hipLaunchKernelGGL((k_solve_level<T, TRANS, 4>), dim3(grid), dim3(SV_THREADS), 0, s, a);
        else
            hipLaunchKernelGGL((k_solve_level<T, TRANS, 1>), dim3(grid), dim3(SV_THREADS), 0, s, a);
    } else {
        const size_t lds = (size_t)a.lds_bytes;
        if (multi)
            hipLaunchKernelGGL((k_solve_sf<T, TRANS, 4>), dim3(grid), dim3(SV_THREADS), lds, s, a);
        else
            hipLaunchKernelGGL((k_solve_sf<T, TRANS, 1>), dim3(grid), dim3(SV_THREADS), lds, s, a);
    }
    RWT_LAUNCHED();
    return RWT_OK;
}

}  // namespace

unsigned solve_grid(Algo algo, rwt_dtype dt, bool transposed, int k, size_t lds, int cus) {
    const void* f = nullptr;
    const bool multi = k > 1;
#define RWT_PICK(T, TR)                                                                     \
    if (algo == Algo::Level)                                                                \
        f = multi ? (const void*)k_solve_level<T, TR, 4> : (const void*)k_solve_level<T, TR, 1>; \
    else                                                                                    \
        f = multi ? (const void*)k_solve_sf<T, TR, 4> : (const void*)k_solve_sf<T, TR, 1>;
    if (dt == RWT_F64) {
        if (transposed) { RWT_PICK(double, true) } else { RWT_PICK(double, false) }
    } else {
        if (transposed) { RWT_PICK(float, true) } else { RWT_PICK(float, false) }
    }
#undef RWT_PICK
    if (algo == Algo::Level) return (unsigned)cus;   // one workgroup per compute unit
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, SV_THREADS, lds) != hipSuccess ||
        per_cu < 1)
        per_cu = 1;
    if (per_cu > 8) per_cu = 8;
    return (unsigned)(cus * per_cu);
}

int syncfree_lds_bytes(int block_rows, int k, rwt_dtype dt, int lanes) {
    const int s = (int)dtype_size(dt);
    return sf_stage_offset(block_rows, k, s) + sf_stage_bytes(lanes, k == 1 ? 1 : 4, s);
}

rwt_status solve_prepare(const SolveArgs& a, rwt_dtype dt, hipStream_t s) {
    const int64_t total = (int64_t)a.n * a.k;
    if (total == 0) return fill_u8(a.ctrl, sizeof(Ctrl), s);
    // about four values per thread
    const unsigned g = blocks_for(total, 1024, 4096);
    uint32_t* cw = reinterpret_cast<uint32_t*>(a.ctrl);
    if (dt == RWT_F64)
        hipLaunchKernelGGL(k_prefill<double>, dim3(g), dim3(256), 0, s, static_cast<double*>(a.X),
                           a.ldx, a.n, a.k, cw);
    else
        hipLaunchKernelGGL(k_prefill<float>, dim3(g), dim3(256), 0, s, static_cast<float*>(a.X),
                           a.ldx, a.n, a.k, cw);
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status walk_launch(const SolveArgs& a, rwt_dtype dt, bool transposed, hipStream_t s) {
    if (a.n == 0 || a.k == 0) return RWT_OK;
    const dim3 grid((unsigned)a.k), blk(2 * WAVE);
    if (dt == RWT_F64) {
        const size_t lds = (size_t)wk2_lds_bytes<double>();
        if (transposed) hipLaunchKernelGGL((k_solve_walk<double, true>), grid, blk, lds, s, a);
        else hipLaunchKernelGGL((k_solve_walk<double, false>), grid, blk, lds, s, a);
    } else {
        const size_t lds = (size_t)wk2_lds_bytes<float>();
        if (transposed) hipLaunchKernelGGL((k_solve_walk<float, true>), grid, blk, lds, s, a);
        else hipLaunchKernelGGL((k_solve_walk<float, false>), grid, blk, lds, s, a);
    }
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status walk_gather_vals(const int32_t* map, int64_t m, const void* vals, void* out,
                            rwt_dtype dt, hipStream_t s) {
    if (m <= 0) return RWT_OK;
    const unsigned g = blocks_for((size_t)m, 256, 8192);
    if (dt == RWT_F64)
        hipLaunchKernelGGL(k_gather_vals<double>, dim3(g), dim3(256), 0, s, map, m,
                           static_cast<const double*>(vals), static_cast<double*>(out));
    else
        hipLaunchKernelGGL(k_gather_vals<float>, dim3(g), dim3(256), 0, s, map, m,
                           static_cast<const float*>(vals), static_cast<float*>(out));
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status chunk_rounds(const int32_t* rowptr, const int32_t* colidx, int32_t n,
                        unsigned long long* d_out, hipStream_t s) {
    RWT_TRY(fill_u8(d_out, sizeof(unsigned long long), s));
    if (n <= 0) return RWT_OK;
    const unsigned g = blocks_for(((size_t)n + WAVE - 1) / WAVE * WAVE, 256, 2048);
    hipLaunchKernelGGL(k_chunk_rounds, dim3(g), dim3(256), 0, s, rowptr, colidx, n, d_out);
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status solve_launch(const SolveArgs& a, rwt_dtype dt, Algo algo, bool transposed, unsigned grid,
                        hipStream_t s) {
    if (a.n == 0 || a.k == 0) return RWT_OK;
    if (dt == RWT_F64)
        return transposed ? launch_typed<double, true>(a, algo, grid, s)
                          : launch_typed<double, false>(a, algo, grid, s);
    return transposed ? launch_typed<float, true>(a, algo, grid, s)
                      : launch_typed<float, false>(a, algo, grid, s);
}

}  // namespace rwt
