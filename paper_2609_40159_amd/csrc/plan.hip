// Solve plans: analysis + transposed pattern + schedules + autotuning, and
// the solve entry points.
#include <algorithm>
#include <new>
#include <vector>

#include "plan.hpp"
#include "prim.hpp"

namespace rwt {

namespace {

// keys for grouping the level-ordered rows by row block (stable)
__global__ void k_block_keys(const int32_t* perm, int32_t n, int32_t R, uint32_t* keys,
                             int32_t* vals) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; q < n; q += st) {
        int32_t i = perm[q];
        keys[q] = (uint32_t)(i / R);
        vals[q] = i;
    }
}

// a step starts at each block start and wherever the level changes
__global__ void k_step_flags(const int32_t* bperm, const int32_t* level, int32_t n, int32_t R,
                             int32_t* flag) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; q < n; q += st)
        flag[q] = (q % R == 0 || level[bperm[q]] != level[bperm[q - 1]]) ? 1 : 0;
}

__global__ void k_step_pos(const int32_t* flag, const int32_t* pos, int32_t n, int32_t R,
                           int32_t nblocks, int32_t* step_pos, int32_t* blk_step) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; q < n; q += st) {
        if (flag[q]) step_pos[pos[q]] = (int32_t)q;
        if (q % R == 0) blk_step[q / R] = pos[q];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        step_pos[pos[n]] = n;
        blk_step[nblocks] = pos[n];
    }
}

// {row, first entry, end, diagonal position} of every row, in block order
__global__ void k_row_desc(const int32_t* bperm, const int32_t* rowptr, const int32_t* cptr,
                           int32_t n, int4* df, int4* dt) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; q < n; q += st) {
        const int32_t i = bperm[q];
        const int32_t d = rowptr[i + 1] - 1;
        df[q] = make_int4(i, rowptr[i], d, d);
        dt[q] = make_int4(i, cptr[i], cptr[i + 1], d);
    }
}

template <typename T>
__global__ void k_fill_val(T* p, int64_t n, T v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

template <typename T>
__global__ void k_copy_block(const T* src, int64_t lds, T* dst, int64_t ldd, int32_t n, int32_t k) {
    int64_t total = (int64_t)n * k;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; t < total; t += st) {
        int64_t q = t / n, i = t - q * n;
        dst[i + q * ldd] = src[i + q * lds];
    }
}

int pow2_floor(int v) {
    int p = 1;
    while (p * 2 <= v) p *= 2;
    return p;
}

}  // namespace

rwt_status copy_block(const void* src, int64_t lds, void* dst, int64_t ldd, int32_t n, int32_t k,
                      rwt_dtype dt, hipStream_t s) {
    int64_t total = (int64_t)n * k;
    if (total == 0) return RWT_OK;
    const unsigned g = blocks_for(total, 256, 8192);
    if (dt == RWT_F64)
        hipLaunchKernelGGL(k_copy_block<double>, dim3(g), dim3(256), 0, s,
                           static_cast<const double*>(src), lds, static_cast<double*>(dst), ldd, n, k);
    else
        hipLaunchKernelGGL(k_copy_block<float>, dim3(g), dim3(256), 0, s,
                           static_cast<const float*>(src), lds, static_cast<float*>(dst), ldd, n, k);
    RWT_LAUNCHED();
    return RWT_OK;
}

}  // namespace rwt

using namespace rwt;



namespace {

struct PlanLayout {
    size_t bytes;
};

constexpr int R_MIN = 32;       // smallest row block (sizes the block tables)
constexpr int TUNE_COLS = 64;   // right-hand sides the autotuner solves with (at most)
constexpr int32_t TUNE_ROWS = 1 << 21;   // rows the sync-free candidates are timed on (at most)
constexpr double WALK_ROUNDS_MAX = 12.0;   // largest mean rounds per chunk the walk is tried at

// A row block size is usable when the block's x values and step starts fit
// the LDS budget at the largest right-hand-side count.
bool block_rows_ok(int R, int kmax, rwt_dtype dt, int lanes) {
    return R >= R_MIN && syncfree_lds_bytes(R, kmax, dt, lanes) <= SF_LDS_BUDGET;
}

// Block sizes to try for chains of kc right-hand-side columns.
std::vector<int> block_candidates(const rwt_plan_opts& o, rwt_dtype dt, int32_t n, int kc,
                                  int lanes) {
    const int kmax = kc;
    std::vector<int> out;
    // the whole matrix in one workgroup, level after level with workgroup
    // barriers, when its x values fit in LDS
    const bool whole =
        n > 0 && n <= (1 << 20) && syncfree_lds_bytes(n, kmax, dt, lanes) <= SF_LDS_BUDGET;
    if (o.block_rows > 0) {
        int R = o.block_rows;
        while (R > R_MIN && !block_rows_ok(R, kmax, dt, lanes)) R /= 2;
        out.push_back(R < R_MIN ? R_MIN : R);
        return out;
    }
    if (whole) out.push_back(n);
    for (int R : {4096, 2048, 1024, 512, 256, 128, 64, 32})
        if (R < n && block_rows_ok(R, kmax, dt, lanes)) out.push_back(R);
    if (out.empty()) out.push_back(R_MIN);
    return out;
}

int default_lanes(int64_t nnz, int32_t n) {
    double mean = n > 0 ? (double)(nnz - n) / n : 0.0;
    int G = 1;
    while (G < 64 && G < mean) G *= 2;
    if (G < 2) G = 2;
    return G;
}

// Carve the plan's device state; with base == nullptr only sizes are computed.
struct PlanPtrs {
    Ctrl* ctrl;
    Ctrl* actrl;
    int32_t *level, *perm, *level_ptr, *rows;
    int64_t* cost;
    rwt_level_stats* dstats;
    Csc csc;
    int32_t* seg;
    int32_t *bperm, *step_pos, *blk_step;
    int4 *desc_f, *desc_t;
    int4 *ldesc_f, *ldesc_t;
    void* xtmp;
    void* xtmp2;
    void* vt;
    unsigned long long* span;
    void* scratch;
    size_t scratch_bytes;
};

size_t carve_plan(void* base, const rwt_csr& L, int kmax, PlanPtrs* p) {
    const int32_t n = L.n;
    const int64_t noff = L.nnz - n > 0 ? L.nnz - n : 1;
    const int32_t nblocks = (n + R_MIN - 1) / R_MIN;
    const size_t s = dtype_size(L.dt);
    Carver cv(base);
    p->ctrl = cv.take<Ctrl>(1);
    p->actrl = cv.take<Ctrl>(1);
    p->level = cv.take<int32_t>(n);
    p->perm = cv.take<int32_t>(n);
    p->level_ptr = cv.take<int32_t>(n + 1);
    p->rows = cv.take<int32_t>(n);
    p->cost = cv.take<int64_t>(n);
    p->dstats = cv.take<rwt_level_stats>(1);
    p->csc.ptr = cv.take<int32_t>(n + 1);
    p->csc.row = cv.take<int32_t>(noff);
    p->csc.map = cv.take<int32_t>(noff);
    p->seg = cv.take<int32_t>(3 * (size_t)n + 3);
    p->bperm = cv.take<int32_t>(n);
    p->step_pos = cv.take<int32_t>(n + 1);
    p->blk_step = cv.take<int32_t>(nblocks + 1);
    p->desc_f = cv.take<int4>(n);
    p->desc_t = cv.take<int4>(n);
    p->ldesc_f = cv.take<int4>(n);
    p->ldesc_t = cv.take<int4>(n);
    p->xtmp = cv.take<char>((size_t)n * kmax * s);
    p->xtmp2 = cv.take<char>((size_t)n * std::min(kmax, TUNE_COLS) * s);
    p->vt = cv.take<char>((size_t)noff * s);
    p->span = cv.take<unsigned long long>(1);
    // scratch shared by the construction steps
    size_t sched = 0;
    {
        Carver sc(nullptr);
        sc.take<uint32_t>(n);
        sc.take<uint32_t>(n);
        sc.take<int32_t>(n);
        sc.take<int32_t>(n + 1);
        sc.take<char>(radix_ws(n));
        sc.take<char>(scan_ws(n));
        sched = sc.used();
    }
    size_t scr = std::max(std::max(csc_ws(n, L.nnz), levels_ws(n, L.nnz)), sched);
    p->scratch = cv.take<char>(scr);
    p->scratch_bytes = scr;
    return cv.used();
}

rwt_status check_opts(const rwt_csr* L, const rwt_plan_opts* o) {
    RWT_REQUIRE(L != nullptr && o != nullptr, RWT_ERR_INVALID_ARG, "null argument");
    RWT_REQUIRE(L->n >= 0 && L->nnz >= L->n, RWT_ERR_INVALID_ARG, "bad sizes");
    RWT_REQUIRE(L->nnz < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "nnz must be < 2^31");
    RWT_REQUIRE(L->rowptr && (L->nnz == 0 || (L->colidx && L->vals)), RWT_ERR_INVALID_ARG,
                "a plan needs pattern and values");
    RWT_REQUIRE(L->dt == RWT_F64 || L->dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    RWT_REQUIRE(o->algo >= RWT_ALGO_AUTO && o->algo <= RWT_ALGO_WALK, RWT_ERR_INVALID_ARG,
                "bad algorithm");
    RWT_REQUIRE(o->kmax >= 0 && o->kmax <= 4096, RWT_ERR_INVALID_ARG, "kmax out of range");
    RWT_REQUIRE(o->lanes_per_row == 0 ||
                    (o->lanes_per_row >= 1 && o->lanes_per_row <= 64 &&
                     (o->lanes_per_row & (o->lanes_per_row - 1)) == 0),
                RWT_ERR_INVALID_ARG, "lanes_per_row must be 0 or a power of two <= 64");
    RWT_REQUIRE(o->block_rows >= 0 && o->block_rows <= (1 << 20), RWT_ERR_INVALID_ARG,
                "block_rows outside 0..2^20");
    RWT_REQUIRE(o->rhs_chunk >= 0 && o->rhs_chunk <= 4, RWT_ERR_INVALID_ARG,
                "rhs_chunk must be 0..4");
    RWT_REQUIRE(o->tune_cols >= 0, RWT_ERR_INVALID_ARG, "negative tune_cols");
    RWT_REQUIRE(o->stage_outside >= 0 && o->stage_outside <= 2, RWT_ERR_INVALID_ARG,
                "stage_outside must be 0..2");
    return RWT_OK;
}

SolveArgs make_args(const rwt_plan* p) {
    SolveArgs a;
    memset(&a, 0, sizeof a);
    a.n = p->L.n;
    a.rowptr = p->L.rowptr;
    a.colidx = p->L.colidx;
    a.vals = p->L.vals;
    a.cptr = p->csc.ptr;
    a.crow = p->csc.row;
    a.cmap = p->csc.map;
    a.perm = p->perm;
    a.level_ptr = p->level_ptr;
    a.nlev = p->D;
    a.ldesc = p->ldesc_f;
    a.seg = p->seg;
    a.nseg = p->nseg;
    a.block_rows = p->R;
    a.nblocks = p->nblocks;
    a.bperm = p->bperm;
    a.step_pos = p->step_pos;
    a.blk_step = p->blk_step;
    a.lanes = p->lanes;
    a.kc = p->kc;
    a.stage_x = p->stage_x == 1;
    a.ctrl = p->ctrl;
    a.ticks = watchdog_ticks(p->opts.watchdog_ms);
    a.hold_row = -1;
    return a;
}

// rows > 0: solve only the leading rows x rows block (a forward sync-free
// solve of whole row blocks; used by the autotuner)
rwt_status run_solve(const rwt_plan* p, bool transposed, Algo algo, const void* B, int32_t k,
                     int64_t ldb, void* X, int64_t ldx, hipStream_t s, int32_t rows = 0,
                     int32_t hold_row = -1) {
    SolveArgs a = make_args(p);
    a.hold_row = hold_row;
    a.vt = p->vt;
    if (rows > 0 && rows < a.n) {
        a.n = rows;
        a.nblocks = (rows + p->R - 1) / p->R;
    }
    a.k = k;
    a.X = X;
    a.ldx = ldx;
    if (B == X) {
        RWT_TRY(copy_block(B, ldb, p->xtmp, p->L.n, p->L.n, k, p->L.dt, s));
        a.B = p->xtmp;
        a.ldb = p->L.n;
    } else {
        a.B = B;
        a.ldb = ldb;
    }
    if (algo == Algo::Walk) {
        // no cross-wave readiness: only the control words are reset; the
        // transposed walk reads the values in successor-list order
        RWT_TRY(fill_u8(a.ctrl, sizeof(Ctrl), s));
        if (transposed)
            RWT_TRY(walk_gather_vals(p->csc.map, (int64_t)p->L.nnz - p->L.n, p->L.vals, p->vt,
                                     p->L.dt, s));
        return walk_launch(a, p->L.dt, transposed, s);
    }
    RWT_TRY(solve_prepare(a, p->L.dt, s));
    a.ldesc = transposed ? p->ldesc_t : p->ldesc_f;
    size_t lds = 0;
    int kg = k;
    if (algo == Algo::SyncFree) {
        a.kc = std::min(p->kc, k);
        kg = a.kc;
        a.desc = transposed ? p->desc_t : p->desc_f;
        a.lds_bytes = syncfree_lds_bytes(p->R, a.kc, p->L.dt, p->lanes);
        lds = (size_t)a.lds_bytes;
    }
    unsigned grid = solve_grid(algo, p->L.dt, transposed, kg, lds, p->cus);
    return solve_launch(a, p->L.dt, algo, transposed, grid, s);
}

// The sync-free candidates are timed on the leading rows only: whole row
// blocks covering up to TUNE_ROWS rows (the leading block of a lower
// triangular matrix is one on its own, and per-level costs carry over).
int32_t tune_rows(const rwt_plan* p) {
    if (p->R >= p->L.n) return p->L.n;
    const int32_t r = (TUNE_ROWS / p->R) * p->R;
    return r > 0 && r < p->L.n ? r : p->L.n;
}

double time_solve(rwt_plan* p, Algo algo, int kt, hipStream_t s, int reps);

// the sync-free schedule timed on every row
double time_solve_full(rwt_plan* p, int kt, hipStream_t s);

// Median-free timing: best of reps - 1 runs after one warm-up, on kt
// columns of ones. A warm-up run longer than cutoff ms ends the timing and
// its own time is returned.
double time_solve_rows(rwt_plan* p, Algo algo, int kt, hipStream_t s, int reps, int32_t rows,
                       double cutoff = 1e30) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 1e30;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return 1e30;
    }
    double best = 1e30;
    for (int r = 0; r < reps; ++r) {
        (void)hipEventRecord(e0, s);
        rwt_status st = run_solve(p, false, algo, p->xtmp, kt, p->L.n, p->xtmp2, p->L.n, s, rows);
        (void)hipEventRecord(e1, s);
        if (st != RWT_OK || hipEventSynchronize(e1) != hipSuccess) { best = 1e30; break; }
        float ms = 0;
        (void)hipEventElapsedTime(&ms, e0, e1);
        Ctrl hc;
        if (hipMemcpy(&hc, p->ctrl, sizeof hc, hipMemcpyDeviceToHost) != hipSuccess || hc.err != 0) {
            best = 1e30;
            break;
        }
        if (r > 0 && ms < best) best = ms;   // the first run warms up
        if (reps == 1 || (r == 0 && ms > cutoff)) {
            best = ms;
            break;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

double time_solve(rwt_plan* p, Algo algo, int kt, hipStream_t s, int reps) {
    return time_solve_rows(p, algo, kt, s, reps, algo == Algo::SyncFree ? tune_rows(p) : 0);
}

double time_solve_full(rwt_plan* p, int kt, hipStream_t s) {
    return time_solve_rows(p, Algo::SyncFree, kt, s, 2, 0);
}

}  // namespace

namespace rwt {
rwt_status plan_solve(const rwt_plan* p, bool transposed, const void* B, int32_t k, int64_t ldb,
                      void* X, int64_t ldx, hipStream_t s) {
    return run_solve(p, transposed, transposed ? p->bwd : p->fwd, B, k, ldb, X, ldx, s);
}
}  // namespace rwt

extern "C" rwt_status rwt_plan_ws(const rwt_csr* L, const rwt_plan_opts* opts, size_t* h_bytes) {
    RWT_TRY(check_opts(L, opts));
    RWT_REQUIRE(h_bytes != nullptr, RWT_ERR_INVALID_ARG, "h_bytes is NULL");
    PlanPtrs pp;
    int kmax = opts->kmax > 0 ? opts->kmax : 1;
    *h_bytes = carve_plan(nullptr, *L, kmax, &pp);
    return RWT_OK;
}

extern "C" rwt_status rwt_plan_create(const rwt_csr* L, const rwt_plan_opts* opts, void* d_ws,
                                      size_t ws_bytes, rwt_plan** out, rwt_stream_t stream) {
    RWT_TRY(check_opts(L, opts));
    RWT_REQUIRE(out != nullptr, RWT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    const int kmax = opts->kmax > 0 ? opts->kmax : 1;
    // right-hand-side chunk candidates (columns per sync-free chain)
    std::vector<int> kcs;
    if (opts->rhs_chunk > 0) kcs.push_back(std::min(opts->rhs_chunk, kmax));
    else if (kmax == 1) kcs.push_back(1);
    else kcs = {std::min(kmax, 4), 1};
    const int lanes = opts->lanes_per_row > 0 ? opts->lanes_per_row : default_lanes(L->nnz, L->n);
    int R = block_candidates(*opts, L->dt, L->n, kcs.front(), lanes).front();
    PlanPtrs pp;
    const size_t need = carve_plan(nullptr, *L, kmax, &pp);
    RWT_REQUIRE(d_ws != nullptr && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "plan workspace must hold %zu bytes", need);
    carve_plan(d_ws, *L, kmax, &pp);
    hipStream_t s = hs(stream);
    rwt_plan* p = new (std::nothrow) rwt_plan();
    RWT_REQUIRE(p != nullptr, RWT_ERR_INVALID_ARG, "out of host memory");
    p->L = *L;
    p->opts = *opts;
    p->opts.kmax = kmax;
    p->R = R;
    p->nblocks = (L->n + R - 1) / R;
    p->ctrl = pp.ctrl;
    p->level = pp.level;
    p->perm = pp.perm;
    p->level_ptr = pp.level_ptr;
    p->csc = pp.csc;
    p->seg = pp.seg;
    p->bperm = pp.bperm;
    p->step_pos = pp.step_pos;
    p->blk_step = pp.blk_step;
    p->desc_f = pp.desc_f;
    p->desc_t = pp.desc_t;
    p->ldesc_f = pp.ldesc_f;
    p->ldesc_t = pp.ldesc_t;
    p->xtmp = pp.xtmp;
    p->xtmp2 = pp.xtmp2;
    p->vt = pp.vt;
    p->span = pp.span;
    p->lanes = lanes;
    p->kc = kcs.front();
    DeviceInfo di;
    rwt_status st = device_info(&di);
    if (st != RWT_OK) { delete p; return st; }
    p->cus = di.cus;
    memset(&p->stats, 0, sizeof p->stats);
    const int32_t n = L->n;
    auto fail = [&](rwt_status e) {
        delete p;
        return e;
    };
    if (n == 0) {
        *out = p;
        return RWT_OK;
    }
    // the pattern and diagonal are checked before any kernel indexes with them
    if ((st = validate_device(*L, true, pp.actrl, nullptr, s)) != RWT_OK) return fail(st);
    // analysis
    if ((st = build_csc(*L, p->csc, pp.scratch, s)) != RWT_OK) return fail(st);
    LevelOut lo{pp.level, pp.perm, pp.level_ptr, pp.rows, pp.cost, pp.dstats};
    if ((st = compute_levels(*L, p->csc, lo, pp.actrl, pp.scratch, s, opts->watchdog_ms)) != RWT_OK)
        return fail(st);
    if ((st = chunk_rounds(L->rowptr, L->colidx, n, pp.span, s)) != RWT_OK) return fail(st);
    hipLaunchKernelGGL(k_row_desc, dim3(blocks_for((size_t)n, 256, 4096)), dim3(256), 0, s, pp.perm,
                       L->rowptr, p->csc.ptr, n, pp.ldesc_f, pp.ldesc_t);
    if (hipError_t e = hipGetLastError(); e != hipSuccess) {
        set_hip_error(e, "level-order row descriptors");
        return fail(RWT_ERR_HIP);
    }
    Ctrl hc;
    unsigned long long span_sum = 0;
    if (hipMemcpyAsync(&span_sum, pp.span, sizeof span_sum, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&hc, pp.actrl, sizeof hc, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(&p->stats, pp.dstats, sizeof p->stats, hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
        set_hip_error(hipGetLastError(), "plan analysis readback");
        return fail(RWT_ERR_HIP);
    }
    if (hc.err != 0) {
        set_error("levelization watchdog expired");
        return fail(RWT_ERR_DEADLOCK);
    }
    if (hc.l1 != n) {
        set_error("only %lld of %d rows reached: pattern not lower triangular", (long long)hc.l1, n);
        return fail(RWT_ERR_NOT_LOWER);
    }
    p->D = p->stats.num_levels;
    // the row-order walk resolves a chunk's internal dependencies in rounds,
    // one per link of the chunk's longest internal chain: it suits matrices
    // whose chunks of consecutive rows need few rounds (deep, thin DAGs with
    // spread-out dependencies), not grids in natural order (each row depends
    // on the one before: 64 rounds)
    p->chunk_rounds = (double)span_sum / (double)((n + 63) / 64);
    p->walk_ok = p->chunk_rounds <= WALK_ROUNDS_MAX;
    // level segments: runs of narrow levels go to one workgroup
    std::vector<int32_t> rows(p->D);
    if (hipMemcpy(rows.data(), pp.rows, sizeof(int32_t) * p->D, hipMemcpyDeviceToHost) != hipSuccess) {
        set_hip_error(hipGetLastError(), "level sizes readback");
        return fail(RWT_ERR_HIP);
    }
    // default: a level that one workgroup finishes in up to 4 rounds
    const int narrow = opts->narrow_rows >= 0 ? opts->narrow_rows : 4 * (256 / p->lanes);
    p->opts.narrow_rows = narrow;
    std::vector<int32_t> seg;
    for (int32_t l = 0; l < p->D;) {
        if (rows[l] <= narrow) {
            int32_t e = l;
            while (e < p->D && rows[e] <= narrow) ++e;
            seg.insert(seg.end(), {l, e, 1});
            l = e;
        } else {
            seg.insert(seg.end(), {l, l + 1, 0});
            ++l;
        }
    }
    p->nseg = (int32_t)(seg.size() / 3);
    if (hipMemcpyAsync(p->seg, seg.data(), sizeof(int32_t) * seg.size(), hipMemcpyHostToDevice, s) !=
        hipSuccess) {
        set_hip_error(hipGetLastError(), "segment upload");
        return fail(RWT_ERR_HIP);
    }
    // sync-free blocks: rows grouped by block, each block in (level, row) order
    auto build_blocks = [&](int Rb) -> rwt_status {
        p->R = Rb;
        p->nblocks = (n + Rb - 1) / Rb;
        Carver sc(pp.scratch);
        uint32_t* keys = sc.take<uint32_t>(n);
        uint32_t* tkeys = sc.take<uint32_t>(n);
        int32_t* tvals = sc.take<int32_t>(n);
        int32_t* pos = sc.take<int32_t>(n + 1);
        void* rws = sc.take<char>(radix_ws(n));
        void* sws = sc.take<char>(scan_ws(n));
        const unsigned g = blocks_for(n, 256, 8192);
        hipLaunchKernelGGL(k_block_keys, dim3(g), dim3(256), 0, s, p->perm, n, Rb, keys, p->bperm);
        RWT_LAUNCHED();
        RWT_TRY(radix_sort(keys, p->bperm, tkeys, tvals, n, bits_for((uint64_t)(p->nblocks - 1)),
                           rws, s));
        int32_t* flag = reinterpret_cast<int32_t*>(keys);   // keys no longer needed
        hipLaunchKernelGGL(k_step_flags, dim3(g), dim3(256), 0, s, p->bperm, p->level, n, Rb, flag);
        RWT_LAUNCHED();
        RWT_TRY(scan_exclusive(flag, pos, n, sws, s));
        hipLaunchKernelGGL(k_step_pos, dim3(g), dim3(256), 0, s, flag, pos, n, Rb, p->nblocks,
                           p->step_pos, p->blk_step);
        RWT_LAUNCHED();
        hipLaunchKernelGGL(k_row_desc, dim3(g), dim3(256), 0, s, p->bperm, L->rowptr, p->csc.ptr, n,
                           p->desc_f, p->desc_t);
        RWT_LAUNCHED();
        return RWT_OK;
    };
    // algorithm, RHS chunk and block size: measured on the plan's own matrix
    // (with kt = min(kmax, TUNE_COLS) columns) unless forced
    p->fwd = p->bwd = opts->algo == RWT_ALGO_LEVEL ? Algo::Level
                      : opts->algo == RWT_ALGO_WALK  ? Algo::Walk
                                                     : Algo::SyncFree;
    const int kt = std::min(kmax, opts->tune_cols > 0 ? opts->tune_cols : TUNE_COLS);
    const bool tune_algo = opts->algo == RWT_ALGO_AUTO;
    const bool blocks_used = opts->algo == RWT_ALGO_AUTO || opts->algo == RWT_ALGO_SYNCFREE;
    const bool tune_sf = blocks_used &&
                         (kcs.size() > 1 ||
                          block_candidates(*opts, L->dt, n, kcs.front(), lanes).size() > 1);
    const bool tune_stage = blocks_used && opts->stage_outside == 0 && n > 0;
    p->stage_x = opts->stage_outside == 2 ? 2 : 1;
    if (tune_algo || tune_sf || tune_stage) {
        const int64_t nf = (int64_t)n * kt;
        const unsigned g = blocks_for(nf, 256, 8192);
        if (L->dt == RWT_F64)
            hipLaunchKernelGGL(k_fill_val<double>, dim3(g), dim3(256), 0, s,
                               static_cast<double*>(p->xtmp), nf, 1.0);
        else
            hipLaunchKernelGGL(k_fill_val<float>, dim3(g), dim3(256), 0, s,
                               static_cast<float*>(p->xtmp), nf, 1.0f);
    }
    // staging of outside x values in the helper waves (on or off), decided
    // first, on the largest block candidate, so that the block size is tuned
    // with it: both timed alternately after two warm-up solves, best of
    // three each
    if (tune_stage) {
        if ((st = build_blocks(R)) != RWT_OK) return fail(st);
        if (p->nblocks > 1) {
            double t[2] = {1e30, 1e30};
            for (int w = 0; w < 2; ++w) (void)time_solve(p, Algo::SyncFree, kt, s, 1);
            for (int r = 0; r < 3; ++r)
                for (int m = 0; m < 2; ++m) {
                    p->stage_x = m + 1;
                    t[m] = std::min(t[m], time_solve(p, Algo::SyncFree, kt, s, 1));
                }
            p->stage_x = t[1] < t[0] ? 2 : 1;
        }
    }
    if (tune_algo || tune_sf) {
        // per chunk, candidates run from large blocks to small, each the best
        // of three timed solves after a warm-up; stop after two in a row that
        // are more than 10% slower than the best so far
        double best_sf = 1e30;
        int best_R = R, best_kc = kcs.front();
        for (int kc : kcs) {
            p->kc = kc;
            double best_here = 1e30;
            int worse = 0;
            for (int Rc : block_candidates(*opts, L->dt, n, kc, lanes)) {
                if ((st = build_blocks(Rc)) != RWT_OK) return fail(st);
                double ms = time_solve(p, Algo::SyncFree, kt, s, 4);   // best of 3
                if (ms < best_sf) { best_sf = ms; best_R = Rc; best_kc = kc; }
                if (ms < best_here) best_here = ms;
                worse = ms > 1.1 * best_here ? worse + 1 : 0;
                if (worse >= 2) break;
            }
        }
        p->tuned_sf = best_sf;
        R = best_R;
        p->kc = best_kc;
        if (tune_algo) {
            // the level-scheduled solve is timed on the whole matrix: time the
            // chosen sync-free schedule on the whole matrix as well
            if ((st = build_blocks(R)) != RWT_OK) return fail(st);
            if (tune_rows(p) < n) {
                best_sf = time_solve_full(p, kt, s);
                p->tuned_sf = best_sf;
            }
            // the row-order walk, on the whole matrix, where the model says
            // it may win
            const double walk_ms =
                p->walk_ok ? time_solve_rows(p, Algo::Walk, kt, s, 3, 0) : 1e30;
            if (p->walk_ok) p->tuned_walk = walk_ms;
            // the level-scheduled solve: a warm-up run over four times the
            // best time so far cannot win and is not repeated (on deep
            // power-law matrices it takes seconds)
            p->tuned_level = time_solve_rows(p, Algo::Level, kt, s, 3, 0,
                                             4.0 * std::min(best_sf, walk_ms));
            if (p->tuned_level >= 1e30 && best_sf >= 1e30 && walk_ms >= 1e30) {
                set_error("autotuning solves failed");
                return fail(RWT_ERR_DEADLOCK);
            }
            Algo pick = Algo::SyncFree;
            double pick_ms = best_sf;
            if (p->tuned_level < pick_ms) { pick = Algo::Level; pick_ms = p->tuned_level; }
            if (walk_ms < pick_ms) pick = Algo::Walk;
            p->fwd = p->bwd = pick;
        }
    }
    if ((st = build_blocks(R)) != RWT_OK) return fail(st);
    if (hipStreamSynchronize(s) != hipSuccess) {
        set_hip_error(hipGetLastError(), "plan creation");
        return fail(RWT_ERR_HIP);
    }
    *out = p;
    return RWT_OK;
}

extern "C" rwt_status rwt_plan_get_info(const rwt_plan* p, rwt_plan_info* h) {
    RWT_REQUIRE(p != nullptr && h != nullptr, RWT_ERR_INVALID_ARG, "null argument");
    memset(h, 0, sizeof *h);
    h->stats = p->stats;
    auto code = [](Algo a) {
        return a == Algo::Level ? RWT_ALGO_LEVEL : a == Algo::Walk ? RWT_ALGO_WALK : RWT_ALGO_SYNCFREE;
    };
    h->algo_fwd = code(p->fwd);
    h->algo_bwd = code(p->bwd);
    h->block_rows = p->R;
    h->lanes_per_row = p->lanes;
    h->narrow_rows = p->opts.narrow_rows;
    h->num_blocks = p->nblocks;
    h->rhs_chunk = p->kc;
    h->stage_outside = p->stage_x;
    h->grid = (int32_t)solve_grid(p->fwd, p->L.dt, false, p->fwd == Algo::SyncFree ? p->kc : 1,
                                  p->fwd == Algo::SyncFree
                                      ? syncfree_lds_bytes(p->R, p->kc, p->L.dt, p->lanes)
                                      : 0,
                                  p->cus);
    if (p->fwd == Algo::Walk) h->grid = p->opts.kmax;   // one workgroup (two waves) per column
    h->tuned_ms_level = p->tuned_level;
    h->tuned_ms_syncfree = p->tuned_sf;
    h->tuned_ms_walk = p->tuned_walk;
    h->chunk_rounds = p->chunk_rounds;
    return RWT_OK;
}

extern "C" rwt_status rwt_plan_levels(const rwt_plan* p, const int32_t** d_level,
                                      const int32_t** d_perm, const int32_t** d_level_ptr) {
    RWT_REQUIRE(p != nullptr, RWT_ERR_INVALID_ARG, "null plan");
    if (d_level) *d_level = p->level;
    if (d_perm) *d_perm = p->perm;
    if (d_level_ptr) *d_level_ptr = p->level_ptr;
    return RWT_OK;
}

extern "C" rwt_status rwt_plan_destroy(rwt_plan* p) {
    delete p;
    return RWT_OK;
}

static rwt_status solve_common(const rwt_plan* p, bool transposed, const void* B, int32_t k,
                               int64_t ldb, void* X, int64_t ldx, rwt_stream_t stream,
                               int32_t hold_row = -1) {
    RWT_REQUIRE(p != nullptr, RWT_ERR_INVALID_ARG, "null plan");
    RWT_REQUIRE(k >= 0 && k <= p->opts.kmax, RWT_ERR_INVALID_ARG, "k=%d outside [0, kmax=%d]", k,
                p->opts.kmax);
    RWT_REQUIRE(k == 0 || p->L.n == 0 || (B != nullptr && X != nullptr), RWT_ERR_INVALID_ARG,
                "null right-hand side");
    RWT_REQUIRE(ldb >= p->L.n && ldx >= p->L.n, RWT_ERR_INVALID_ARG, "leading dimension < n");
    if (k == 0 || p->L.n == 0) return RWT_OK;
    Algo algo = transposed ? p->bwd : p->fwd;
    return run_solve(p, transposed, algo, B, k, ldb, X, ldx, hs(stream), 0, hold_row);
}

extern "C" rwt_status rwt_solve(const rwt_plan* p, const void* d_B, int32_t k, int64_t ldb,
                                void* d_X, int64_t ldx, rwt_stream_t stream) {
    return solve_common(p, false, d_B, k, ldb, d_X, ldx, stream);
}

extern "C" rwt_status rwt_solve_transpose(const rwt_plan* p, const void* d_G, int32_t k,
                                          int64_t ldg, void* d_Y, int64_t ldy,
                                          rwt_stream_t stream) {
    return solve_common(p, true, d_G, k, ldg, d_Y, ldy, stream);
}

extern "C" rwt_status rwt_solve_withhold(const rwt_plan* p, int32_t row, const void* d_B,
                                         int32_t k, int64_t ldb, void* d_X, int64_t ldx,
                                         rwt_stream_t stream) {
    RWT_REQUIRE(p != nullptr, RWT_ERR_INVALID_ARG, "null plan");
    RWT_REQUIRE(row >= 0 && row < p->L.n, RWT_ERR_INVALID_ARG, "row %d outside [0, %d)", row,
                p->L.n);
    return solve_common(p, false, d_B, k, ldb, d_X, ldx, stream, row);
}

extern "C" rwt_status rwt_plan_check(const rwt_plan* p, rwt_stream_t stream) {
    RWT_REQUIRE(p != nullptr, RWT_ERR_INVALID_ARG, "null plan");
    if (p->L.n == 0) return RWT_OK;
    Ctrl hc;
    RWT_HIP(hipMemcpyAsync(&hc, p->ctrl, sizeof hc, hipMemcpyDeviceToHost, hs(stream)));
    RWT_HIP(hipStreamSynchronize(hs(stream)));
    if (hc.err != 0) {
        set_error("a device wait expired in the last solve (watchdog)");
        return RWT_ERR_DEADLOCK;
    }
    return RWT_OK;
}
