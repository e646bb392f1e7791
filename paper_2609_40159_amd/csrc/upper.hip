// Upper-triangular solves and the L-then-U pair (the preconditioner
// application of an incomplete LU factorization, which is what repeated
// solves with one rewritten factor amortize over).
//
// U (CSR, diagonal first in each row) is solved through the lower
// triangular matrix L_U = J U J, J the reversal permutation (row and column
// i <-> n-1-i): row i' of L_U is row n-1-i' of U with its columns mapped to
// n-1-j and their order reversed, so its columns ascend and the diagonal
// comes last.  U x = b is L_U (J x) = J b, so every solve schedule, the
// autotuner and the level analysis of the lower path apply unchanged.  The
// pattern of L_U and the position map from its entries to U's are built
// once; the values are gathered at creation and by rwt_upper_refresh.  A
// solve reverses B into a workspace block, solves into X and reverses X in
// place: 4 n k value moves on top of the solve.
#include "common.hpp"
#include "plan.hpp"
#include "prim.hpp"

struct rwt_upper {
    rwt_csr U;          // the caller's matrix (pattern and values)
    rwt_csr LU;         // J U J, in the workspace
    int32_t* map;       // entry q of L_U is entry map[q] of U
    void* tmp;          // n * kmax values
    int32_t* flag;      // device word for the row-pointer check
    void* vws;          // validation workspace
    rwt_plan* plan;     // the plan of L_U
    int32_t kmax;
};

namespace rwt {
namespace {

struct UpWs {
    int32_t* rowptr;
    int32_t* colidx;
    void* vals;
    int32_t* map;
    void* tmp;
    int32_t* flag;
    void* vws;
    void* sws;
    void* plan_ws;
};

size_t carve_up(void* base, const rwt_csr& U, int32_t kmax, size_t plan_bytes, UpWs* w) {
    Carver cv(base);
    const size_t s = dtype_size(U.dt);
    const size_t nnz = U.nnz > 0 ? (size_t)U.nnz : 1;
    w->rowptr = cv.take<int32_t>((size_t)U.n + 1);
    w->colidx = cv.take<int32_t>(nnz);
    w->vals = cv.take<char>(nnz * s);
    w->map = cv.take<int32_t>(nnz);
    w->tmp = cv.take<char>((size_t)(U.n > 0 ? U.n : 1) * (size_t)kmax * s);
    w->flag = cv.take<int32_t>(1);
    w->vws = cv.take<char>(rwt_validate_ws());
    w->sws = cv.take<char>(scan_ws((int64_t)U.n + 1));
    w->plan_ws = cv.take<char>(plan_bytes);
    return cv.used();
}

// row pointers start at 0, never decrease and end at nnz
__global__ void k_up_rowptr(const int32_t* rowptr, int32_t n, int64_t nnz, int32_t* flag) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t a = rowptr[i], b = rowptr[i + 1];
        if (b < a || (i == 0 && a != 0) || (i == n - 1 && (int64_t)b != nnz)) *flag = 1;
    }
}

__global__ void k_up_lens(const int32_t* rowptr, int32_t n, int32_t* lens) {
    for (int32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x) {
        const int32_t i = n - 1 - r;
        lens[r] = rowptr[i + 1] - rowptr[i];
    }
}

__global__ void k_up_scatter(const int32_t* rowptr, const int32_t* colidx, int32_t n,
                             const int32_t* rp2, int32_t* ci2, int32_t* map) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int32_t b = rowptr[i], len = rowptr[i + 1] - b;
        const int32_t q0 = rp2[n - 1 - i];
        for (int32_t t = 0; t < len; ++t) {
            const int32_t q = q0 + len - 1 - t;
            ci2[q] = n - 1 - colidx[b + t];
            map[q] = b + t;
        }
    }
}

template <typename T>
__global__ void k_up_gather(const T* uv, const int32_t* map, int64_t nnz, T* v2) {
    for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < nnz;
         q += (int64_t)gridDim.x * blockDim.x)
        v2[q] = uv[map[q]];
}

// D[i + q ldd] = S[n-1-i + q lds]
template <typename T>
__global__ void k_rev_copy(const T* S, int64_t lds, T* D, int64_t ldd, int32_t n, int32_t k) {
    const int64_t total = (int64_t)n * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = (int32_t)(e / n), i = (int32_t)(e - (int64_t)q * n);
        D[i + q * ldd] = S[(n - 1 - i) + q * lds];
    }
}

template <typename T>
__global__ void k_rev_inplace(T* X, int64_t ldx, int32_t n, int32_t k) {
    const int32_t h = n / 2;
    const int64_t total = (int64_t)h * k;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = (int32_t)(e / h), i = (int32_t)(e - (int64_t)q * h);
        T* c = X + q * ldx;
        const T a = c[i], b = c[n - 1 - i];
        c[i] = b;
        c[n - 1 - i] = a;
    }
}

rwt_status rev_copy(const void* S, int64_t lds, void* D, int64_t ldd, int32_t n, int32_t k,
                    rwt_dtype dt, hipStream_t s) {
    if (n == 0 || k == 0) return RWT_OK;
    const unsigned g = blocks_for((size_t)n * k, 256, 8192);
    if (dt == RWT_F64)
        hipLaunchKernelGGL(k_rev_copy<double>, dim3(g), dim3(256), 0, s,
                           static_cast<const double*>(S), lds, static_cast<double*>(D), ldd, n, k);
    else
        hipLaunchKernelGGL(k_rev_copy<float>, dim3(g), dim3(256), 0, s,
                           static_cast<const float*>(S), lds, static_cast<float*>(D), ldd, n, k);
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status rev_inplace(void* X, int64_t ldx, int32_t n, int32_t k, rwt_dtype dt, hipStream_t s) {
    if (n < 2 || k == 0) return RWT_OK;
    const unsigned g = blocks_for((size_t)(n / 2) * k, 256, 8192);
    if (dt == RWT_F64)
        hipLaunchKernelGGL(k_rev_inplace<double>, dim3(g), dim3(256), 0, s, static_cast<double*>(X),
                           ldx, n, k);
    else
        hipLaunchKernelGGL(k_rev_inplace<float>, dim3(g), dim3(256), 0, s, static_cast<float*>(X),
                           ldx, n, k);
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status gather_vals(const rwt_upper* up, hipStream_t s) {
    if (up->U.nnz == 0) return RWT_OK;
    const unsigned g = blocks_for((size_t)up->U.nnz, 256, 8192);
    if (up->U.dt == RWT_F64)
        hipLaunchKernelGGL(k_up_gather<double>, dim3(g), dim3(256), 0, s,
                           static_cast<const double*>(up->U.vals), up->map, up->U.nnz,
                           static_cast<double*>(const_cast<void*>(up->LU.vals)));
    else
        hipLaunchKernelGGL(k_up_gather<float>, dim3(g), dim3(256), 0, s,
                           static_cast<const float*>(up->U.vals), up->map, up->U.nnz,
                           static_cast<float*>(const_cast<void*>(up->LU.vals)));
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status up_args(const rwt_csr* U, const rwt_plan_opts* opts, rwt_csr* LU, size_t* plan_bytes) {
    RWT_REQUIRE(U != nullptr && opts != nullptr, RWT_ERR_INVALID_ARG, "null argument");
    RWT_REQUIRE(U->n >= 0 && U->nnz >= U->n, RWT_ERR_INVALID_ARG, "bad sizes");
    RWT_REQUIRE(U->nnz < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "nnz must be < 2^31");
    RWT_REQUIRE(U->rowptr && (U->nnz == 0 || (U->colidx && U->vals)), RWT_ERR_INVALID_ARG,
                "an upper plan needs pattern and values");
    *LU = *U;   // sizes and type; pointers are replaced by the workspace's
    return rwt_plan_ws(LU, opts, plan_bytes);
}

}  // namespace
}  // namespace rwt

using namespace rwt;

extern "C" rwt_status rwt_upper_ws(const rwt_csr* U, const rwt_plan_opts* opts, size_t* h_bytes) {
    RWT_REQUIRE(h_bytes != nullptr, RWT_ERR_INVALID_ARG, "h_bytes is NULL");
    rwt_csr LU;
    size_t pb = 0;
    RWT_TRY(up_args(U, opts, &LU, &pb));
    UpWs w;
    *h_bytes = carve_up(nullptr, *U, opts->kmax > 0 ? opts->kmax : 1, pb, &w);
    return RWT_OK;
}

extern "C" rwt_status rwt_upper_create(const rwt_csr* U, const rwt_plan_opts* opts, void* d_ws,
                                       size_t ws_bytes, rwt_upper** out, rwt_stream_t stream) {
    RWT_REQUIRE(out != nullptr, RWT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    rwt_csr LU;
    size_t pb = 0;
    RWT_TRY(up_args(U, opts, &LU, &pb));
    const int32_t kmax = opts->kmax > 0 ? opts->kmax : 1;
    UpWs w;
    const size_t need = carve_up(nullptr, *U, kmax, pb, &w);
    RWT_REQUIRE(d_ws && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "upper plan workspace must hold %zu bytes", need);
    carve_up(d_ws, *U, kmax, pb, &w);
    hipStream_t s = hs(stream);
    const int32_t n = U->n;
    // row pointers first: the reversal scatters by them
    RWT_TRY(fill_i32(w.flag, 1, 0, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_up_rowptr, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, U->rowptr, n,
                           U->nnz, w.flag);
        RWT_LAUNCHED();
    }
    int32_t hflag = 0;
    RWT_HIP(hipMemcpyAsync(&hflag, w.flag, sizeof hflag, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipStreamSynchronize(s));
    RWT_REQUIRE(hflag == 0, RWT_ERR_INVALID_ARG, "U row pointers are not a valid CSR index");
    if (n > 0) {
        hipLaunchKernelGGL(k_up_lens, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, U->rowptr, n,
                           w.rowptr);
        RWT_LAUNCHED();
    }
    RWT_TRY(scan_exclusive(w.rowptr, w.rowptr, n, w.sws, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_up_scatter, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, U->rowptr,
                           U->colidx, n, w.rowptr, w.colidx, w.map);
        RWT_LAUNCHED();
    }
    rwt_upper* up = new rwt_upper;
    up->U = *U;
    up->LU = *U;
    up->LU.rowptr = w.rowptr;
    up->LU.colidx = w.colidx;
    up->LU.vals = w.vals;
    up->map = w.map;
    up->tmp = w.tmp;
    up->flag = w.flag;
    up->vws = w.vws;
    up->plan = nullptr;
    up->kmax = kmax;
    rwt_status st = gather_vals(up, s);
    // U is valid exactly when L_U is (the reversal maps "above the
    // diagonal", "unsorted", "diagonal not first" and "zero diagonal" of a
    // row of U onto the lower checks of its reversed row)
    int32_t bad = -1;
    if (st == RWT_OK) {
        st = rwt_validate(&up->LU, w.vws, rwt_validate_ws(), &bad, stream);
        if (st != RWT_OK) {
            const int32_t urow = bad >= 0 ? n - 1 - bad : -1;
            set_error("U row %d: %s", urow,
                      st == RWT_ERR_NOT_LOWER ? "entry below the diagonal or column out of range"
                      : st == RWT_ERR_UNSORTED_OR_DUP ? "columns not strictly ascending"
                      : st == RWT_ERR_MISSING_DIAG ? "first entry is not the diagonal"
                      : st == RWT_ERR_ZERO_DIAG ? "zero diagonal"
                                                : "invalid");
        }
    }
    if (st == RWT_OK) st = rwt_plan_create(&up->LU, opts, w.plan_ws, pb, &up->plan, stream);
    if (st != RWT_OK) {
        delete up;
        return st;
    }
    *out = up;
    return RWT_OK;
}

extern "C" rwt_status rwt_upper_refresh(rwt_upper* up, rwt_stream_t stream) {
    RWT_REQUIRE(up != nullptr, RWT_ERR_INVALID_ARG, "NULL upper plan");
    return gather_vals(up, hs(stream));
}

extern "C" rwt_status rwt_upper_get_info(const rwt_upper* up, rwt_plan_info* h_info) {
    RWT_REQUIRE(up != nullptr, RWT_ERR_INVALID_ARG, "NULL upper plan");
    return rwt_plan_get_info(up->plan, h_info);
}

static rwt_status upper_run(const rwt_upper* up, bool transposed, const void* d_B, int32_t k,
                            int64_t ldb, void* d_X, int64_t ldx, rwt_stream_t stream) {
    RWT_REQUIRE(up != nullptr, RWT_ERR_INVALID_ARG, "NULL upper plan");
    const int32_t n = up->U.n;
    RWT_REQUIRE(k >= 0 && k <= up->kmax, RWT_ERR_INVALID_ARG, "k must be 0..kmax");
    RWT_REQUIRE(k == 0 || n == 0 || (d_B && d_X && ldb >= n && ldx >= n), RWT_ERR_INVALID_ARG,
                "bad dense blocks");
    if (n == 0 || k == 0) return RWT_OK;
    hipStream_t s = hs(stream);
    RWT_TRY(rev_copy(d_B, ldb, up->tmp, n, n, k, up->U.dt, s));
    if (transposed)
        RWT_TRY(rwt_solve_transpose(up->plan, up->tmp, k, n, d_X, ldx, stream));
    else
        RWT_TRY(rwt_solve(up->plan, up->tmp, k, n, d_X, ldx, stream));
    return rev_inplace(d_X, ldx, n, k, up->U.dt, s);
}

extern "C" rwt_status rwt_upper_levels(const rwt_upper* up, const int32_t** d_level,
                                       const int32_t** d_perm, const int32_t** d_level_ptr) {
    RWT_REQUIRE(up != nullptr, RWT_ERR_INVALID_ARG, "null upper plan");
    return rwt_plan_levels(up->plan, d_level, d_perm, d_level_ptr);
}

extern "C" rwt_status rwt_upper_solve(const rwt_upper* up, const void* d_B, int32_t k, int64_t ldb,
                                      void* d_X, int64_t ldx, rwt_stream_t stream) {
    return upper_run(up, false, d_B, k, ldb, d_X, ldx, stream);
}

extern "C" rwt_status rwt_upper_solve_transpose(const rwt_upper* up, const void* d_G, int32_t k,
                                                int64_t ldg, void* d_Y, int64_t ldy,
                                                rwt_stream_t stream) {
    return upper_run(up, true, d_G, k, ldg, d_Y, ldy, stream);
}

extern "C" rwt_status rwt_solve_pair(const rwt_plan* L, const rwt_upper* U, const void* d_B,
                                     int32_t k, int64_t ldb, void* d_X, int64_t ldx,
                                     rwt_stream_t stream) {
    RWT_REQUIRE(L != nullptr && U != nullptr, RWT_ERR_INVALID_ARG, "NULL plan");
    RWT_REQUIRE(L->L.n == U->U.n && L->L.dt == U->U.dt, RWT_ERR_INVALID_ARG,
                "L and U must have the same size and value type");
    RWT_REQUIRE(k >= 0 && k <= U->kmax, RWT_ERR_INVALID_ARG, "k must be 0..kmax of U");
    RWT_TRY(rwt_solve(L, d_B, k, ldb, d_X, ldx, stream));
    return upper_run(U, false, d_X, k, ldx, d_X, ldx, stream);
}

extern "C" rwt_status rwt_upper_check(const rwt_upper* up, rwt_stream_t stream) {
    RWT_REQUIRE(up != nullptr, RWT_ERR_INVALID_ARG, "NULL upper plan");
    return rwt_plan_check(up->plan, stream);
}

extern "C" rwt_status rwt_upper_destroy(rwt_upper* up) {
    if (up == nullptr) return RWT_OK;
    rwt_status st = rwt_plan_destroy(up->plan);
    delete up;
    return st;
}
