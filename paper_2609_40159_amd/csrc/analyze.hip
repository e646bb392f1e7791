// Validation and level-set analysis (paper Section 2.1 level-set method;
// Section 4.1 / Table 1 level features; Section 3 ALC / ARL / AIR).
//
//   validate      one thread per row, first error of the lowest row wins
//   build_csc     successor lists = stable radix sort of the off-diagonal
//                 entries by column (rows stay ascending inside a column)
//   levelize      Kahn frontier BFS in one persistent launch: in-degree =
//                 off-diagonal count; the rows of the current frontier get
//                 the current level and decrement their successors'
//                 in-degrees; rows reaching zero are appended to the next
//                 frontier with wave-ballot compaction (one atomic per wave).
//                 Narrow frontiers are handled by workgroup 0 alone with
//                 workgroup barriers; wide ones by the whole grid with a
//                 device-wide barrier per level.
//   perm          stable radix sort of the rows by level
//   level stats   per-level rows and cost (2*nnz_row - 1), exact S1 / S2,
//                 CV, ALC, ARL, AIR, thin threshold and thin count
#include <cstdarg>
#include <cstdio>
#include <mutex>

#include "analyze.hpp"
#include "prim.hpp"
#include "u128.hpp"

namespace rwt {

// ---------------------------------------------------------------------------
// error strings
// ---------------------------------------------------------------------------
static thread_local char g_err[512] = "";
static thread_local int g_hip_err = 0;

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void set_hip_error(hipError_t e, const char* where) {
    g_hip_err = static_cast<int>(e);
    snprintf(g_err, sizeof g_err, "HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), where);
}

rwt_status device_info(DeviceInfo* out) {
    RWT_HIP(hipGetDevice(&out->device));
    RWT_HIP(hipDeviceGetAttribute(&out->cus, hipDeviceAttributeMultiprocessorCount, out->device));
    return RWT_OK;
}

double cv_from_sums(int32_t D, uint64_t S1, uint64_t S2_lo, uint64_t S2_hi) {
    return cv_exact((uint64_t)D, S1, U128{S2_lo, S2_hi});
}

// ---------------------------------------------------------------------------
// validate
// ---------------------------------------------------------------------------
// error key: (row << 8) | code rank; rowptr errors set a separate flag
template <typename T>
__global__ void k_validate(const int32_t* rowptr, const int32_t* colidx, const T* vals, int32_t n,
                           int64_t nnz, unsigned long long* key, int32_t* bad_ptr) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        if (rowptr[0] != 0 || (int64_t)rowptr[n] != nnz) atomicExch(bad_ptr, 1);
    }
    if (i >= n) return;
    int32_t b = rowptr[i], e = rowptr[i + 1];
    if (e < b || b < 0 || (int64_t)e > nnz) {
        atomicExch(bad_ptr, 1);
        return;
    }
    int code = 0;
    for (int32_t p = b; p < e; ++p) {
        int32_t c = colidx[p];
        if (c < 0 || c > i) { code = -RWT_ERR_NOT_LOWER; break; }
        if (p > b && c <= colidx[p - 1]) { code = -RWT_ERR_UNSORTED_OR_DUP; break; }
    }
    if (!code) {
        if (e == b || colidx[e - 1] != i) code = -RWT_ERR_MISSING_DIAG;
        else if (vals && vals[e - 1] == T(0)) code = -RWT_ERR_ZERO_DIAG;
    }
    if (code) atomicMin(key, ((unsigned long long)i << 8) | (unsigned long long)code);
}

// Validate on the device; 16 bytes of workspace; synchronizes the stream.
rwt_status validate_device(const rwt_csr& L, bool check_vals, void* ws16, int32_t* bad_row,
                           hipStream_t s) {
    if (bad_row) *bad_row = -1;
    unsigned long long* key = static_cast<unsigned long long*>(ws16);
    int32_t* bad_ptr = reinterpret_cast<int32_t*>(static_cast<char*>(ws16) + 8);
    unsigned long long init[2] = {~0ull, 0ull};
    RWT_HIP(hipMemcpyAsync(ws16, init, 16, hipMemcpyHostToDevice, s));
    if (L.n > 0) {
        const unsigned g = blocks_for(L.n, 256);
        const void* v = check_vals ? L.vals : nullptr;
        if (L.dt == RWT_F64)
            hipLaunchKernelGGL(k_validate<double>, dim3(g), dim3(256), 0, s, L.rowptr, L.colidx,
                               static_cast<const double*>(v), L.n, L.nnz, key, bad_ptr);
        else
            hipLaunchKernelGGL(k_validate<float>, dim3(g), dim3(256), 0, s, L.rowptr, L.colidx,
                               static_cast<const float*>(v), L.n, L.nnz, key, bad_ptr);
        RWT_LAUNCHED();
    }
    unsigned long long res[2];
    RWT_HIP(hipMemcpyAsync(res, ws16, 16, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipStreamSynchronize(s));
    if ((int32_t)(res[1] & 0xffffffffu) != 0 || (L.n == 0 && L.nnz != 0)) {
        set_error("row pointers are not a valid nondecreasing array from 0 to nnz");
        return RWT_ERR_INVALID_ARG;
    }
    if (res[0] != ~0ull) {
        int32_t row = (int32_t)(res[0] >> 8);
        if (bad_row) *bad_row = row;
        int code = -(int)(res[0] & 0xff);
        set_error("row %d: %s", row,
                  code == RWT_ERR_NOT_LOWER ? "entry above the diagonal or negative column"
                  : code == RWT_ERR_UNSORTED_OR_DUP ? "columns not strictly ascending"
                  : code == RWT_ERR_MISSING_DIAG ? "last entry is not the diagonal"
                                                 : "zero diagonal");
        return (rwt_status)code;
    }
    return RWT_OK;
}

// ---------------------------------------------------------------------------
// successor lists
// ---------------------------------------------------------------------------
__global__ void k_csc_keys(const int32_t* rowptr, const int32_t* colidx, const int32_t* rowidx,
                           int64_t nnz, int32_t n, uint32_t* keys, int32_t* vals) {
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; p < nnz; p += st) {
        int32_t c = colidx[p];
        keys[p] = (c == rowidx[p]) ? (uint32_t)n : (uint32_t)c;   // diagonal sorts last
        vals[p] = (int32_t)p;
    }
}

// the row of each successor (its CSR position came out of the sort)
__global__ void k_csc_rows(const int32_t* pos, const int32_t* rowidx, int64_t noff, int32_t* crow) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; q < noff; q += st) crow[q] = rowidx[pos[q]];
}

size_t csc_ws(int32_t n, int64_t nnz) {
    Carver cv(nullptr);
    cv.take<int32_t>(nnz);     // rowidx
    cv.take<uint32_t>(nnz);    // keys
    cv.take<uint32_t>(nnz);    // tmp keys
    cv.take<int32_t>(nnz);     // values (positions)
    cv.take<int32_t>(nnz);     // tmp values
    cv.take<char>(radix_ws(nnz));
    return cv.used();
}

rwt_status build_csc(const rwt_csr& L, const Csc& out, void* ws, hipStream_t s) {
    const int32_t n = L.n;
    const int64_t nnz = L.nnz;
    Carver cv(ws);
    int32_t* rowidx = cv.take<int32_t>(nnz);
    uint32_t* keys = cv.take<uint32_t>(nnz);
    uint32_t* tkeys = cv.take<uint32_t>(nnz);
    int32_t* pos = cv.take<int32_t>(nnz);
    int32_t* tpos = cv.take<int32_t>(nnz);
    void* rws = cv.take<char>(radix_ws(nnz));
    RWT_TRY(expand_rows(L.rowptr, n, rowidx, s));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_csc_keys, dim3(blocks_for(nnz, 256, 8192)), dim3(256), 0, s, L.rowptr,
                           L.colidx, rowidx, nnz, n, keys, pos);
        RWT_LAUNCHED();
        RWT_TRY(radix_sort(keys, pos, tkeys, tpos, nnz, bits_for((uint64_t)n), rws, s));
    }
    const int64_t noff = nnz - n;
    RWT_TRY(segment_starts(keys, noff, n, out.ptr, nullptr, s));
    if (noff > 0) {
        hipLaunchKernelGGL(k_csc_rows, dim3(blocks_for(noff, 256, 8192)), dim3(256), 0, s, pos,
                           rowidx, noff, out.row);
        RWT_LAUNCHED();
    }
    if (noff > 0 && out.map)
        RWT_HIP(hipMemcpyAsync(out.map, pos, (size_t)noff * 4, hipMemcpyDeviceToDevice, s));
    return RWT_OK;
}

// ---------------------------------------------------------------------------
// frontier levelization
// ---------------------------------------------------------------------------
constexpr int LV_THREADS = 256;

// in-degree, empty queue, level-0 flags
__global__ void k_lv_init(const int32_t* rowptr, int32_t n, int32_t* indeg, int32_t* queue,
                          int32_t* flag) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        int32_t d = rowptr[i + 1] - rowptr[i] - 1;
        indeg[i] = d;
        queue[i] = -1;
        flag[i] = d == 0 ? 1 : 0;
    }
}

// level-0 rows, in row order, at the head of the queue
__global__ void k_lv_seed(const int32_t* flag, const int32_t* pos, int32_t n, int32_t* queue,
                          Ctrl* ctrl) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st)
        if (flag[i]) queue[pos[i]] = (int32_t)i;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctrl->i0 = pos[n];   // end of the level-0 frontier
        ctrl->i1 = pos[n];   // append cursor
    }
}

// Wait-free drain of this wave's outstanding memory operations.
__device__ __forceinline__ void drain() { __builtin_amdgcn_s_waitcnt(0); }

// Pacing barrier over the whole grid.  It does not order data: every value
// one workgroup hands to another goes through device-scope atomics and is
// checked for readiness by the reader.  Each wave drains its own memory
// operations first, so any counter it advanced is already performed.
// The last workgroup to arrive copies the append cursor into the snapshot
// slot of the new generation: that copy, not the live cursor (which fast
// workgroups may already be advancing for the next level), is the frontier
// end every workgroup reads after the barrier.
__device__ bool pace_barrier(Ctrl* c, uint32_t& gen, int64_t ticks, int32_t* snap) {
    drain();
    __syncthreads();
    __shared__ int s_ok;
    if (threadIdx.x == 0) {
        const uint32_t nb = gridDim.x;
        uint32_t prev = fetch_add(&c->bar_count, 1u);
        int ok = 1;
        if (prev == nb * (gen + 1) - 1) {
            int32_t cur = fetch_add(&c->i1, 0);
            __hip_atomic_exchange(&snap[(gen + 1) & 1], cur, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            drain();
            __hip_atomic_exchange(&c->bar_gen, gen + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = wait_generation(c, gen, ticks) ? 1 : 0;
        }
        s_ok = ok;
    }
    __syncthreads();
    gen += 1;
    return s_ok != 0;
}

// queue entries are -1 until written: read with a bounded wait
__device__ __forceinline__ int32_t queue_get(const int32_t* q, int32_t* err, int64_t ticks) {
    int32_t v = ld_relaxed(q);
    if (v >= 0) return v;
    int64_t t0 = wall_clock64();
    while ((v = ld_relaxed(q)) < 0) {
        if (wall_clock64() - t0 > ticks) {
            __hip_atomic_store(err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            return 0;
        }
    }
    return v;
}

// Expand one frontier row u: record its level, decrement its successors'
// in-degrees and append the rows that become free.  The append is
// aggregated per wave: one ballot, one counter update by the lowest lane,
// each lane's slot from the count of set ballot bits below it.
template <bool WIDE>
__device__ void lv_expand(int32_t u, bool active, int32_t cur, const int32_t* cptr,
                          const int32_t* crow, int32_t* indeg, int32_t* queue, int32_t* level,
                          int32_t* g_cursor, int32_t* s_cursor, int32_t n, int32_t* err) {
    int32_t b = 0, e = 0;
    if (active) {
        level[u] = cur;
        b = cptr[u];
        e = cptr[u + 1];
    }
    // all lanes of the wave iterate together until every lane is done
    for (int32_t p = b;; ++p) {
        const bool mine = p < e;
        if (__ballot(mine) == 0) break;
        bool ready = false;
        int32_t s = 0;
        if (mine) {
            s = crow[p];
            int32_t old = __hip_atomic_fetch_add(&indeg[s], -1, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            ready = old == 1;
        }
        const uint64_t m = __ballot(ready);
        if (m) {
            const int leader = __builtin_ctzll(m);
            int32_t base = 0;
            if (lane_id() == leader) {
                if (WIDE) base = fetch_add(g_cursor, (int32_t)__popcll(m));
                else base = atomicAdd(s_cursor, (int32_t)__popcll(m));
            }
            base = __shfl(base, leader);
            const int32_t slot = base + lanes_below(m);
            if (ready) {
                if (slot < n) st_relaxed(&queue[slot], s);
                else __hip_atomic_store(err, (int32_t)RWT_ERR_NOT_LOWER, __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ void __launch_bounds__(LV_THREADS) k_levelize(int32_t n, const int32_t* cptr,
                                                        const int32_t* crow, int32_t* indeg,
                                                        int32_t* queue, int32_t* level, Ctrl* ctrl,
                                                        int32_t* snap, int32_t narrow, int64_t ticks) {
    __shared__ int32_t s_cursor;
    __shared__ int32_t s_fb, s_fe, s_cur;
    uint32_t gen = 0;
    int32_t fb = 0;
    int32_t fe = ctrl->i0;
    int32_t cur = 0;
    const int64_t gtid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t gthreads = (int64_t)gridDim.x * blockDim.x;
    while (fb < fe) {
        if (fe - fb <= narrow) {
            if (blockIdx.x == 0) {
                // workgroup 0 alone: levels follow each other with workgroup barriers
                if (threadIdx.x == 0) { s_fb = fb; s_fe = fe; s_cur = cur; s_cursor = fe; }
                __syncthreads();
                for (;;) {
                    int32_t b = s_fb, e = s_fe, c = s_cur;
                    // every wave runs whole rounds so its ballots see all lanes
                    for (int32_t q0 = b; q0 < e; q0 += blockDim.x) {
                        const int32_t q = q0 + threadIdx.x;
                        const bool act = q < e;
                        int32_t u = act ? queue_get(&queue[q], &ctrl->err, ticks) : 0;
                        lv_expand<false>(u, act, c, cptr, crow, indeg, queue, level, nullptr,
                                         &s_cursor, n, &ctrl->err);
                    }
                    drain();
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        s_fb = e;
                        s_fe = s_cursor;
                        s_cur = c + 1;
                        __hip_atomic_fetch_add(&ctrl->heartbeat, 1u, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                    }
                    __syncthreads();
                    int32_t sz = s_fe - s_fb;
                    if (sz == 0 || sz > narrow || ld_relaxed(&ctrl->err) != 0) break;
                }
                if (threadIdx.x == 0) {
                    // publish with read-modify-writes so the values are performed
                    __hip_atomic_exchange(&ctrl->i1, s_fe, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_exchange(&ctrl->i2, s_cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    __hip_atomic_exchange(&ctrl->l0, (int64_t)s_fb, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (!pace_barrier(ctrl, gen, ticks, snap)) return;
            fb = (int32_t)fetch_add(&ctrl->l0, (int64_t)0);
            fe = fetch_add(&snap[gen & 1], 0);
            cur = fetch_add(&ctrl->i2, 0);
        } else {
            for (int64_t q0 = fb + gtid - threadIdx.x % WAVE; q0 < fe; q0 += gthreads) {
                const int64_t q = q0 + threadIdx.x % WAVE;
                const bool act = q < fe;
                int32_t u = act ? queue_get(&queue[q], &ctrl->err, ticks) : 0;
                lv_expand<true>(u, act, cur, cptr, crow, indeg, queue, level, &ctrl->i1, nullptr, n,
                                &ctrl->err);
            }
            if (!pace_barrier(ctrl, gen, ticks, snap)) return;
            fb = fe;
            fe = fetch_add(&snap[gen & 1], 0);
            cur += 1;
        }
        if (ld_relaxed(&ctrl->err) != 0) return;
    }
    if (gtid == 0) {
        ctrl->i2 = cur;            // D
        ctrl->l1 = fe;             // rows reached (n for a valid matrix)
    }
}

// ---------------------------------------------------------------------------
// permutation, level pointers, statistics
// ---------------------------------------------------------------------------
__global__ void k_perm_keys(const int32_t* level, int32_t n, uint32_t* keys, int32_t* vals) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        keys[i] = (uint32_t)level[i];
        vals[i] = (int32_t)i;
    }
}

// one wave per level: rows and cost = sum of (2*nnz_row - 1)
__global__ void k_level_cost(const int32_t* rowptr, const int32_t* perm, const int32_t* level_ptr,
                             const Ctrl* ctrl, int32_t* rows, int64_t* cost) {
    const int32_t D = ctrl->i2;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const int lane = lane_id();
    for (int64_t l = wave; l < D; l += nwaves) {
        int32_t b = level_ptr[l], e = level_ptr[l + 1];
        int64_t acc = 0;
        for (int32_t q = b + lane; q < e; q += WAVE) {
            int32_t i = perm[q];
            acc += 2 * (int64_t)(rowptr[i + 1] - rowptr[i]) - 1;
        }
        acc = wave_sum(acc);
        if (lane == 0) {
            rows[l] = e - b;
            cost[l] = acc;
        }
    }
}

constexpr int ST_THREADS = 1024;

__device__ U128 block_sum_u128(U128 v) {
    __shared__ uint64_t s_lo[ST_THREADS / WAVE], s_hi[ST_THREADS / WAVE];
    // wave reduce with carries: shuffle the two halves
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        U128 u;
        u.lo = __shfl_xor(v.lo, o);
        u.hi = __shfl_xor(v.hi, o);
        v = u128_add(v, u);
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) { s_lo[w] = v.lo; s_hi[w] = v.hi; }
    __syncthreads();
    U128 r{0, 0};
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) r = u128_add(r, U128{s_lo[i], s_hi[i]});
    __syncthreads();
    return r;
}

__device__ int64_t block_sum_i64(int64_t v) {
    __shared__ int64_t s[ST_THREADS / WAVE];
    v = wave_sum(v);
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) s[w] = v;
    __syncthreads();
    int64_t r = 0;
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) r += s[i];
    __syncthreads();
    return r;
}

__device__ int64_t block_max_i64(int64_t v) {
    __shared__ int64_t s[ST_THREADS / WAVE];
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        int64_t u = __shfl_xor(v, o);
        v = u > v ? u : v;
    }
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) s[w] = v;
    __syncthreads();
    int64_t r = 0;
    for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) r = s[i] > r ? s[i] : r;
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(ST_THREADS) k_level_stats(const int32_t* rows, const int64_t* cost,
                                                          const Ctrl* ctrl, int32_t n, int64_t nnz,
                                                          rwt_level_stats* st) {
    const int32_t D = ctrl->i2;
    U128 s2{0, 0}, r2{0, 0};
    int64_t s1 = 0, rmax = 0;
    for (int64_t l = threadIdx.x; l < D; l += blockDim.x) {
        uint64_t c = (uint64_t)cost[l];
        uint64_t r = (uint64_t)rows[l];
        s1 += (int64_t)c;
        s2 = u128_add(s2, u128_sq(c));
        r2 = u128_add(r2, u128_sq(r));
        rmax = (int64_t)r > rmax ? (int64_t)r : rmax;
    }
    s1 = block_sum_i64(s1);
    s2 = block_sum_u128(s2);
    r2 = block_sum_u128(r2);
    rmax = block_max_i64(rmax);
    __shared__ double s_thr;
    __shared__ double s_cv, s_cvr, s_alc;
    if (threadIdx.x == 0) {
        s_cv = cv_exact((uint64_t)D, (uint64_t)s1, s2);
        s_cvr = cv_exact((uint64_t)D, (uint64_t)n, r2);
        s_alc = D > 0 ? (double)s1 / (double)D : 0.0;
        double relax = 1.0 - s_cv;
        if (relax < 0.0) relax = 0.0;
        s_thr = s_alc * (1.0 + 1.0 * relax);
    }
    __syncthreads();
    const double thr = s_thr;
    int64_t thin = 0;
    for (int64_t l = threadIdx.x; l < D; l += blockDim.x)
        if ((double)cost[l] < thr) ++thin;
    thin = block_sum_i64(thin);
    if (threadIdx.x == 0) {
        rwt_level_stats o;
        o.num_levels = D;
        o.thin_count = (int32_t)thin;
        o.S1 = (uint64_t)s1;
        o.S2_lo = s2.lo;
        o.S2_hi = s2.hi;
        o.cv = s_cv;
        o.cv_rows = s_cvr;
        o.alc = s_alc;
        o.arl = D > 0 ? (double)n / (double)D : 0.0;
        o.air = n > 0 ? (double)(nnz - n) / (double)n : 0.0;
        o.thin_threshold = thr;
        o.max_level_rows = (int32_t)rmax;
        o.pad_ = 0;
        *st = o;
    }
}

size_t levels_ws(int32_t n, int64_t nnz) {
    (void)nnz;
    Carver cv(nullptr);
    cv.take<int32_t>(n);       // indeg
    cv.take<int32_t>(n);       // queue
    cv.take<int32_t>(n);       // flags
    cv.take<int32_t>(n + 1);   // flag positions
    cv.take<uint32_t>(n);      // keys
    cv.take<uint32_t>(n);      // tmp keys
    cv.take<int32_t>(n);       // tmp vals
    cv.take<int32_t>(2);       // frontier-end snapshots
    cv.take<char>(scan_ws(n));
    cv.take<char>(radix_ws(n));
    return cv.used();
}

// Levels in row order, without level barriers (Section 2.1: the level of a
// row is 0 without dependencies, else 1 + the largest level among them).
// Waves claim chunks of WAVE/G consecutive rows in row order; a row reads
// its dependencies' levels from level[] (-1: not known yet) and publishes
// its own as soon as all are known.  A lane never spins on a row of its own
// wave: the wave publishes the rows it could finish, then retries the rest
// (a chain inside a chunk resolves one row per pass).  Every wait is for a
// lower row, which a running wave has already claimed, so the kernel cannot
// deadlock for any number of resident workgroups.  D (max level + 1) and
// the number of rows reached go to ctrl->i2 and ctrl->l1.
__global__ void __launch_bounds__(LV_THREADS) k_levels_sf(const int32_t* rowptr,
                                                          const int32_t* colidx, int32_t n, int G,
                                                          int32_t* level, Ctrl* ctrl, int64_t ticks) {
    __shared__ int32_t s_max[LV_THREADS / WAVE];
    __shared__ int64_t s_cnt[LV_THREADS / WAVE];
    const int lane = lane_id();
    const int w = threadIdx.x / WAVE;
    const int gl = lane & (G - 1);
    const int CH = WAVE / G;
    int32_t* err = &ctrl->err;
    int32_t wmax = -1;
    int64_t wcnt = 0;
    bool abort = false;
    while (!abort) {
        int32_t c = 0;
        if (lane == 0) c = (int32_t)fetch_add(&ctrl->ticket, 1u);
        c = __shfl(c, 0);
        if ((int64_t)c * CH >= n) break;
        const int64_t i64 = (int64_t)c * CH + lane / G;
        const bool act = i64 < n;
        const int32_t i = act ? (int32_t)i64 : 0;
        const int32_t rb = act ? rowptr[i] : 0;
        const int32_t re = act ? rowptr[i + 1] - 1 : 0;   // off-diagonal entries [rb, re)
        bool done = !act;
        int32_t res = 0;
        const int64_t t0 = wall_clock64();
        for (;;) {
            int32_t mx = -1;
            int miss = 0;
            if (!done)
                for (int32_t p = rb + gl; p < re; p += G) {
                    const int32_t lj = ld_relaxed(&level[colidx[p]]);
                    miss |= lj < 0 ? 1 : 0;
                    mx = lj > mx ? lj : mx;
                }
            for (int o = G / 2; o > 0; o >>= 1) {
                const int32_t m2 = __shfl_xor(mx, o);
                mx = m2 > mx ? m2 : mx;
                miss |= __shfl_xor(miss, o);
            }
            if (!done && !miss) {
                res = mx + 1;
                if (gl == 0) st_relaxed(&level[i], res);
                done = true;
            }
            if (__ballot(!done) == 0) break;
            // the wave's own stores complete before it reads again
            __builtin_amdgcn_s_waitcnt(0);
            __builtin_amdgcn_s_sleep(1);
            if (ld_relaxed(err) != 0) {
                abort = true;
                break;
            }
            if (wall_clock64() - t0 > ticks) {
                __hip_atomic_store(err, (int32_t)RWT_ERR_DEADLOCK, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
                abort = true;
                break;
            }
        }
        if (act && gl == 0 && done) {
            wmax = res > wmax ? res : wmax;
            ++wcnt;
        }
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const int32_t m2 = __shfl_xor(wmax, o);
        wmax = m2 > wmax ? m2 : wmax;
        wcnt += __shfl_xor(wcnt, o);
    }
    if (lane == 0) {
        s_max[w] = wmax;
        s_cnt[w] = wcnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t m = -1;
        int64_t cnt = 0;
        for (int k = 0; k < LV_THREADS / WAVE; ++k) {
            m = s_max[k] > m ? s_max[k] : m;
            cnt += s_cnt[k];
        }
        if (m >= 0) atomicMax(&ctrl->i2, m + 1);
        __hip_atomic_fetch_add(&ctrl->l1, cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Sum of dependency distances i - j over the off-diagonal entries (chooses
// the levelization method).
__global__ void k_dist_sum(const int32_t* rowptr, const int32_t* colidx, int32_t n,
                           unsigned long long* sum) {
    uint64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t p = rowptr[i]; p < rowptr[i + 1] - 1; ++p) acc += (uint64_t)(i - colidx[p]);
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (lane_id() == 0) atomicAdd(sum, (unsigned long long)acc);
}

rwt_status compute_levels(const rwt_csr& L, const Csc& csc, const LevelOut& out, Ctrl* ctrl,
                          void* ws, hipStream_t s, int watchdog_ms) {
    const int32_t n = L.n;
    Carver cv(ws);
    int32_t* indeg = cv.take<int32_t>(n);
    int32_t* queue = cv.take<int32_t>(n);
    int32_t* flag = cv.take<int32_t>(n);
    int32_t* fpos = cv.take<int32_t>(n + 1);
    uint32_t* keys = cv.take<uint32_t>(n);
    uint32_t* tkeys = cv.take<uint32_t>(n);
    int32_t* tvals = cv.take<int32_t>(n);
    int32_t* snap = cv.take<int32_t>(2);
    void* sws = cv.take<char>(scan_ws(n));
    void* rws = cv.take<char>(radix_ws(n));

    RWT_TRY(fill_u8(ctrl, sizeof(Ctrl), s));
    const unsigned gb = blocks_for(n, 256, 8192);
    DeviceInfo di;
    RWT_TRY(device_info(&di));
    // Method: the row-order kernel keeps a window of consecutive rows in
    // flight and needs no level barrier, which wins on deep DAGs whose
    // dependencies are short-range; the frontier search works a whole level
    // at a time, which wins when a level spans much of the row range.  The
    // mean dependency distance against n separates the two.
    unsigned long long* dsum = reinterpret_cast<unsigned long long*>(snap);   // 8 bytes
    RWT_TRY(fill_u8(dsum, sizeof(unsigned long long), s));
    hipLaunchKernelGGL(k_dist_sum, dim3(blocks_for(n, 256, 2048)), dim3(256), 0, s, L.rowptr,
                       L.colidx, n, dsum);
    RWT_LAUNCHED();
    unsigned long long hsum = 0;
    RWT_HIP(hipMemcpyAsync(&hsum, dsum, sizeof hsum, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipStreamSynchronize(s));
    const int64_t noff = L.nnz - n;
    const double mean_dist = noff > 0 ? (double)hsum / (double)noff : 0.0;
    const bool row_order = noff > 0 && mean_dist * 400.0 < (double)n;
    if (row_order) {
        RWT_TRY(fill_i32(out.level, n, -1, s));
        // lanes per row: a power of two near the mean dependency count
        const double mean = (double)noff / n;
        int G = 1;
        while (G < 16 && G < mean) G *= 2;
        hipLaunchKernelGGL(k_levels_sf, dim3(di.cus * 8), dim3(LV_THREADS), 0, s, L.rowptr, L.colidx,
                           n, G, out.level, ctrl, watchdog_ticks(watchdog_ms));
        RWT_LAUNCHED();
    } else {
        RWT_TRY(fill_u8(snap, 2 * sizeof(int32_t), s));
        hipLaunchKernelGGL(k_lv_init, dim3(gb), dim3(256), 0, s, L.rowptr, n, indeg, queue, flag);
        RWT_LAUNCHED();
        RWT_TRY(scan_exclusive(flag, fpos, n, sws, s));
        hipLaunchKernelGGL(k_lv_seed, dim3(gb), dim3(256), 0, s, flag, fpos, n, queue, ctrl);
        RWT_LAUNCHED();
        // one resident workgroup per compute unit
        const int32_t narrow = 2 * LV_THREADS;
        hipLaunchKernelGGL(k_levelize, dim3(di.cus), dim3(LV_THREADS), 0, s, n, csc.ptr, csc.row,
                           indeg, queue, out.level, ctrl, snap, narrow, watchdog_ticks(watchdog_ms));
        RWT_LAUNCHED();
    }

    hipLaunchKernelGGL(k_perm_keys, dim3(gb), dim3(256), 0, s, out.level, n, keys, out.perm);
    RWT_LAUNCHED();
    RWT_TRY(radix_sort(keys, out.perm, tkeys, tvals, n, bits_for((uint64_t)(n > 0 ? n - 1 : 0)),
                       rws, s));
    RWT_TRY(segment_starts(keys, n, n, out.level_ptr, &ctrl->i2, s));
    hipLaunchKernelGGL(k_level_cost, dim3(blocks_for((size_t)n * WAVE, 256, 4096)), dim3(256), 0, s,
                       L.rowptr, out.perm, out.level_ptr, ctrl, out.rows, out.cost);
    RWT_LAUNCHED();
    hipLaunchKernelGGL(k_level_stats, dim3(1), dim3(ST_THREADS), 0, s, out.rows, out.cost, ctrl, n,
                       L.nnz, out.stats);
    RWT_LAUNCHED();
    return RWT_OK;
}

}  // namespace rwt

// ===========================================================================
// C entry points
// ===========================================================================
using namespace rwt;

extern "C" const char* rwt_last_error_string(void) { return g_err; }
extern "C" int rwt_last_hip_error(void) { return g_hip_err; }
#ifndef RWT_SOURCE_HASH
#define RWT_SOURCE_HASH "unknown"
#endif
extern "C" const char* rwt_version(void) { return "rwtrsv 0.3 gfx950"; }
extern "C" const char* rwt_source_hash(void) { return RWT_SOURCE_HASH; }

static rwt_status check_csr(const rwt_csr* L, bool need_vals) {
    RWT_REQUIRE(L != nullptr, RWT_ERR_INVALID_ARG, "L is NULL");
    RWT_REQUIRE(L->n >= 0 && L->nnz >= 0, RWT_ERR_INVALID_ARG, "negative size");
    RWT_REQUIRE(L->nnz < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "nnz must be < 2^31");
    RWT_REQUIRE(L->nnz >= L->n, RWT_ERR_MISSING_DIAG, "nnz < n: some diagonal is missing");
    RWT_REQUIRE(L->rowptr != nullptr && (L->colidx != nullptr || L->nnz == 0),
                RWT_ERR_INVALID_ARG, "null pattern pointer");
    RWT_REQUIRE(!need_vals || L->vals != nullptr, RWT_ERR_INVALID_ARG, "values required");
    RWT_REQUIRE(L->dt == RWT_F64 || L->dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    return RWT_OK;
}

extern "C" size_t rwt_validate_ws(void) { return 256; }

extern "C" rwt_status rwt_validate(const rwt_csr* L, void* d_ws, size_t ws_bytes, int32_t* h_bad_row,
                                   rwt_stream_t stream) {
    RWT_REQUIRE(L != nullptr && h_bad_row != nullptr, RWT_ERR_INVALID_ARG, "null argument");
    *h_bad_row = -1;
    RWT_REQUIRE(L->n >= 0 && L->nnz >= 0 && L->rowptr != nullptr, RWT_ERR_INVALID_ARG,
                "bad sizes or null rowptr");
    RWT_REQUIRE(L->nnz < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "nnz must be < 2^31");
    RWT_REQUIRE(L->nnz == 0 || L->colidx != nullptr, RWT_ERR_INVALID_ARG, "null colidx");
    RWT_REQUIRE(L->dt == RWT_F64 || L->dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    RWT_REQUIRE(d_ws != nullptr && ws_bytes >= rwt_validate_ws(), RWT_ERR_BUFFER_TOO_SMALL,
                "validate workspace must hold %zu bytes", rwt_validate_ws());
    return validate_device(*L, L->vals != nullptr, d_ws, h_bad_row, hs(stream));
}

static size_t analyze_ws_bytes(int32_t n, int64_t nnz) {
    Carver cv(nullptr);
    cv.take<Ctrl>(1);
    cv.take<int32_t>(n + 1);                      // csc ptr
    cv.take<int32_t>(nnz > n ? nnz - n : 1);      // csc rows
    cv.take<char>(csc_ws(n, nnz));
    cv.take<char>(levels_ws(n, nnz));
    return cv.used();
}

extern "C" rwt_status rwt_analyze_ws(const rwt_csr* L, size_t* h_bytes) {
    RWT_TRY(check_csr(L, false));
    RWT_REQUIRE(h_bytes != nullptr, RWT_ERR_INVALID_ARG, "h_bytes is NULL");
    *h_bytes = analyze_ws_bytes(L->n, L->nnz);
    return RWT_OK;
}

extern "C" rwt_status rwt_analyze(const rwt_csr* L, void* d_ws, size_t ws_bytes, int32_t* d_level,
                                  int32_t* d_perm, int32_t* d_level_ptr, int32_t* d_rows,
                                  int64_t* d_cost, rwt_level_stats* d_stats,
                                  rwt_level_stats* h_stats, rwt_stream_t stream) {
    RWT_TRY(check_csr(L, false));
    RWT_REQUIRE(d_level && d_perm && d_level_ptr && d_rows && d_cost && d_stats,
                RWT_ERR_INVALID_ARG, "null output pointer");
    const size_t need = analyze_ws_bytes(L->n, L->nnz);
    RWT_REQUIRE(d_ws != nullptr && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "analyze workspace must hold %zu bytes", need);
    hipStream_t s = hs(stream);
    if (L->n == 0) {
        rwt_level_stats z;
        memset(&z, 0, sizeof z);
        RWT_HIP(hipMemcpyAsync(d_stats, &z, sizeof z, hipMemcpyHostToDevice, s));
        int32_t zero = 0;
        RWT_HIP(hipMemcpyAsync(d_level_ptr, &zero, 4, hipMemcpyHostToDevice, s));
        if (h_stats) {
            RWT_HIP(hipStreamSynchronize(s));
            *h_stats = z;
        }
        return RWT_OK;
    }
    Carver cv(d_ws);
    Ctrl* ctrl = cv.take<Ctrl>(1);
    RWT_TRY(validate_device(*L, false, ctrl, nullptr, s));   // pattern only; before any indexing
    Csc csc;
    csc.ptr = cv.take<int32_t>(L->n + 1);
    csc.row = cv.take<int32_t>(L->nnz > L->n ? L->nnz - L->n : 1);
    csc.map = nullptr;
    void* cws = cv.take<char>(csc_ws(L->n, L->nnz));
    void* lws = cv.take<char>(levels_ws(L->n, L->nnz));
    RWT_TRY(build_csc(*L, csc, cws, s));
    LevelOut out{d_level, d_perm, d_level_ptr, d_rows, d_cost, d_stats};
    RWT_TRY(compute_levels(*L, csc, out, ctrl, lws, s, 0));
    Ctrl hc;
    RWT_HIP(hipMemcpyAsync(&hc, ctrl, sizeof hc, hipMemcpyDeviceToHost, s));
    if (h_stats) RWT_HIP(hipMemcpyAsync(h_stats, d_stats, sizeof *h_stats, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipStreamSynchronize(s));
    if (hc.err != 0) {
        set_error("levelization watchdog expired");
        return RWT_ERR_DEADLOCK;
    }
    if (hc.l1 != L->n) {
        set_error("only %lld of %d rows were reached: the pattern is not lower triangular",
                  (long long)hc.l1, L->n);
        return RWT_ERR_NOT_LOWER;
    }
    return RWT_OK;
}
