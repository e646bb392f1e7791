// Adjoint helpers for differentiating X = L^{-1} B through a rewritten
// system L' = M L, B' = M B (M = I - C, paper Section 2.2 rewriting):
//   grad_B = M^T L'^{-T} G = Y - C^T Y   (Y from the transposed solve)
//   grad_L = -grad_B X^T on the stored pattern of L.
// C^T is built with the stable radix sort so every sum runs in a fixed
// order: the results do not depend on the schedule.
#include <mutex>
#include <vector>

#include "prim.hpp"
#include "rowmap.hpp"

namespace rwt {

namespace {


__global__ void k_ct_keys(const int32_t* ccol, int64_t nc, uint32_t* keys, int32_t* vals) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; e < nc; e += st) {
        keys[e] = (uint32_t)ccol[e];
        vals[e] = (int32_t)e;
    }
}

// out[j,q] = Y[j,q] - sum over substitutions e of column j (ascending e)
//            of cval[e] * Y[crow[e], q]
template <typename T>
__global__ void k_apply_mt(const int32_t* ptr, const int32_t* ent, const int32_t* crow,
                           const T* cval, const T* Y, int64_t ldy, T* out, int64_t ldo, int32_t n,
                           int32_t k) {
    int64_t total = (int64_t)n * k;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; t < total; t += st) {
        int64_t q = t / n, j = t - q * n;
        T v = Y[j + q * ldy];
        for (int32_t p = ptr[j]; p < ptr[j + 1]; ++p) {
            int32_t e = ent[p];
            v = sub_rn(v, mul_rn(cval[e], Y[crow[e] + q * ldy]));
        }
        out[j + q * ldo] = v;
    }
}

// out[r,q] = B[r,q] - sum over the substitutions e of row r, in their order,
// of cval[e] * B[ccol[e], q]  (B' = M B; rows without substitutions copied)
template <typename T>
__global__ void k_apply_m(const int32_t* ptr, const int32_t* ccol, const T* cval, const T* B,
                          int64_t ldb, T* out, int64_t ldo, int32_t n, int32_t k) {
    const int64_t total = (int64_t)n * k;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = t / n, r = t - q * n;
        T v = B[r + q * ldb];
        for (int32_t e = ptr[r]; e < ptr[r + 1]; ++e) {
            const int32_t j = ccol[e];
            if ((uint32_t)j < (uint32_t)n) v = sub_rn(v, mul_rn(cval[e], B[j + q * ldb]));
        }
        out[r + q * ldo] = v;
    }
}

// grad_vals[p] = 0 - sum_q gB[row_p, q] * X[col_p, q]: a workgroup takes 256
// rows and their contiguous entries; each thread finds its row in an LDS
// map of entry -> row (binary search when the rows' entries exceed it).
template <typename T>
__global__ void __launch_bounds__(256) k_grad_vals(const int32_t* rowptr, const int32_t* colidx,
                                                   int32_t n, const T* gB, int64_t ldg, const T* X,
                                                   int64_t ldx, int32_t k, T* gv) {
    __shared__ int32_t s_ptr[257];
    __shared__ unsigned char s_row[ROW_MAP];
    const int32_t r0 = blockIdx.x * 256;
    const int32_t r1 = min(n, r0 + 256);
    for (int32_t i = threadIdx.x; i <= r1 - r0; i += blockDim.x) s_ptr[i] = rowptr[r0 + i];
    __syncthreads();
    const int32_t nr = r1 - r0;
    const int32_t pb = s_ptr[0], pe = s_ptr[nr];
    const bool mapped = map_rows(s_ptr, nr, s_row);
    for (int32_t p = pb + threadIdx.x; p < pe; p += blockDim.x) {
        const int32_t i = r0 + row_of(s_ptr, nr, s_row, mapped, p);
        const int32_t j = colidx[p];
        T s = T(0);
        for (int32_t q = 0; q < k; ++q) s = add_rn(s, mul_rn(gB[i + (int64_t)q * ldg], X[j + (int64_t)q * ldx]));
        gv[p] = sub_rn(T(0), s);
    }
}

struct MtWs {
    uint32_t* keys;
    uint32_t* tkeys;
    int32_t* vals;
    int32_t* tvals;
    int32_t* ptr;
    void* rws;
};

size_t carve_mt(void* base, int32_t n, int64_t nc, MtWs* w) {
    Carver cv(base);
    int64_t c = nc > 0 ? nc : 1;
    w->keys = cv.take<uint32_t>(c);
    w->tkeys = cv.take<uint32_t>(c);
    w->vals = cv.take<int32_t>(c);
    w->tvals = cv.take<int32_t>(c);
    w->ptr = cv.take<int32_t>((size_t)n + 1);
    w->rws = cv.take<char>(radix_ws(c));
    return cv.used();
}

}  // namespace
}  // namespace rwt

using namespace rwt;

extern "C" rwt_status rwt_apply_MT_ws(int32_t n, int64_t nC, size_t* h_bytes) {
    RWT_REQUIRE(h_bytes != nullptr && n >= 0 && nC >= 0, RWT_ERR_INVALID_ARG, "bad argument");
    RWT_REQUIRE(nC < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "too many multipliers");
    MtWs w;
    *h_bytes = carve_mt(nullptr, n, nC, &w);
    return RWT_OK;
}

static rwt_status mt_checks(int32_t n, int64_t nC, size_t ws_bytes, const void* d_ws) {
    RWT_REQUIRE(n >= 0 && nC >= 0, RWT_ERR_INVALID_ARG, "negative size");
    RWT_REQUIRE(nC < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "too many multipliers");
    MtWs w;
    size_t need = carve_mt(nullptr, n, nC, &w);
    RWT_REQUIRE(d_ws != nullptr && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "apply_MT workspace must hold %zu bytes", need);
    return RWT_OK;
}

extern "C" rwt_status rwt_apply_MT_prepare(int32_t n, int64_t nC, const int32_t* d_ccol,
                                           void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    RWT_TRY(mt_checks(n, nC, ws_bytes, d_ws));
    RWT_REQUIRE(nC == 0 || d_ccol, RWT_ERR_INVALID_ARG, "null multiplier columns");
    MtWs w;
    carve_mt(d_ws, n, nC, &w);
    hipStream_t s = hs(stream);
    if (nC > 0) {
        hipLaunchKernelGGL(k_ct_keys, dim3(blocks_for(nC, 256, 4096)), dim3(256), 0, s, d_ccol, nC,
                           w.keys, w.vals);
        RWT_LAUNCHED();
        RWT_TRY(radix_sort(w.keys, w.vals, w.tkeys, w.tvals, nC, bits_for((uint64_t)n), w.rws, s));
    }
    if (n > 0) RWT_TRY(segment_starts(w.keys, nC, n, w.ptr, nullptr, s));
    return RWT_OK;
}

extern "C" rwt_status rwt_apply_MT_apply(int32_t n, int64_t nC, const int32_t* d_crow,
                                         const void* d_cval, rwt_dtype dt, const void* d_Y,
                                         int32_t k, int64_t ldy, void* d_out, int64_t ldo,
                                         const void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    RWT_TRY(mt_checks(n, nC, ws_bytes, d_ws));
    RWT_REQUIRE(k >= 0, RWT_ERR_INVALID_ARG, "negative k");
    RWT_REQUIRE(dt == RWT_F64 || dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    RWT_REQUIRE(nC == 0 || (d_crow && d_cval), RWT_ERR_INVALID_ARG, "null multipliers");
    RWT_REQUIRE(k == 0 || n == 0 || (d_Y && d_out && ldy >= n && ldo >= n), RWT_ERR_INVALID_ARG,
                "bad dense blocks");
    RWT_REQUIRE(k == 0 || n == 0 || d_Y != d_out, RWT_ERR_INVALID_ARG, "output may not alias Y");
    if (n == 0 || k == 0) return RWT_OK;
    MtWs w;
    carve_mt(const_cast<void*>(d_ws), n, nC, &w);
    hipStream_t s = hs(stream);
    const unsigned g = blocks_for((size_t)n * k, 256, 8192);
    if (dt == RWT_F64)
        hipLaunchKernelGGL(k_apply_mt<double>, dim3(g), dim3(256), 0, s, w.ptr, w.vals, d_crow,
                           static_cast<const double*>(d_cval), static_cast<const double*>(d_Y), ldy,
                           static_cast<double*>(d_out), ldo, n, k);
    else
        hipLaunchKernelGGL(k_apply_mt<float>, dim3(g), dim3(256), 0, s, w.ptr, w.vals, d_crow,
                           static_cast<const float*>(d_cval), static_cast<const float*>(d_Y), ldy,
                           static_cast<float*>(d_out), ldo, n, k);
    RWT_LAUNCHED();
    return RWT_OK;
}

extern "C" rwt_status rwt_apply_MT(int32_t n, int64_t nC, const int32_t* d_crow,
                                   const int32_t* d_ccol, const void* d_cval, rwt_dtype dt,
                                   const void* d_Y, int32_t k, int64_t ldy, void* d_out,
                                   int64_t ldo, void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    RWT_TRY(mt_checks(n, nC, ws_bytes, d_ws));
    RWT_REQUIRE(k >= 0, RWT_ERR_INVALID_ARG, "negative k");
    RWT_REQUIRE(dt == RWT_F64 || dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    RWT_REQUIRE(nC == 0 || (d_crow && d_ccol && d_cval), RWT_ERR_INVALID_ARG, "null multipliers");
    RWT_REQUIRE(k == 0 || n == 0 || (d_Y && d_out && ldy >= n && ldo >= n), RWT_ERR_INVALID_ARG,
                "bad dense blocks");
    RWT_REQUIRE(k == 0 || n == 0 || d_Y != d_out, RWT_ERR_INVALID_ARG, "output may not alias Y");
    if (n == 0 || k == 0) return RWT_OK;
    RWT_TRY(rwt_apply_MT_prepare(n, nC, d_ccol, d_ws, ws_bytes, stream));
    return rwt_apply_MT_apply(n, nC, d_crow, d_cval, dt, d_Y, k, ldy, d_out, ldo, d_ws, ws_bytes,
                              stream);
}

extern "C" rwt_status rwt_apply_M_ws(int32_t n, size_t* h_bytes) {
    RWT_REQUIRE(h_bytes != nullptr && n >= 0, RWT_ERR_INVALID_ARG, "bad argument");
    *h_bytes = (((size_t)n + 1) * sizeof(int32_t) + 255) & ~size_t(255);
    return RWT_OK;
}

static rwt_status apply_m_checks(int32_t n, int64_t nC, const int32_t* d_crow,
                                 const int32_t* d_ccol, const void* d_cval, rwt_dtype dt,
                                 const void* d_B, int32_t k, int64_t ldb, void* d_out,
                                 int64_t ldo) {
    RWT_REQUIRE(n >= 0 && nC >= 0 && k >= 0, RWT_ERR_INVALID_ARG, "negative size");
    RWT_REQUIRE(nC < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "too many multipliers");
    RWT_REQUIRE(dt == RWT_F64 || dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    RWT_REQUIRE(nC == 0 || (d_crow && d_ccol && d_cval), RWT_ERR_INVALID_ARG, "null multipliers");
    RWT_REQUIRE(k == 0 || n == 0 || (d_B && d_out && ldb >= n && ldo >= n), RWT_ERR_INVALID_ARG,
                "bad dense blocks");
    RWT_REQUIRE(k == 0 || n == 0 || d_B != d_out, RWT_ERR_INVALID_ARG, "output may not alias B");
    return RWT_OK;
}

// M B with the row offsets of the multipliers built in ptr[n+1] (device)
static rwt_status apply_m_run(int32_t n, int64_t nC, const int32_t* d_crow, const int32_t* d_ccol,
                              const void* d_cval, rwt_dtype dt, const void* d_B, int32_t k,
                              int64_t ldb, void* d_out, int64_t ldo, int32_t* ptr, hipStream_t s) {
    // the multipliers come grouped by row, rows ascending (rwt_rewrite_numeric)
    RWT_TRY(segment_starts(reinterpret_cast<const uint32_t*>(d_crow), nC, n, ptr, nullptr, s));
    const unsigned g = blocks_for((size_t)n * k, 256, 8192);
    if (dt == RWT_F64)
        hipLaunchKernelGGL(k_apply_m<double>, dim3(g), dim3(256), 0, s, ptr, d_ccol,
                           static_cast<const double*>(d_cval), static_cast<const double*>(d_B), ldb,
                           static_cast<double*>(d_out), ldo, n, k);
    else
        hipLaunchKernelGGL(k_apply_m<float>, dim3(g), dim3(256), 0, s, ptr, d_ccol,
                           static_cast<const float*>(d_cval), static_cast<const float*>(d_B), ldb,
                           static_cast<float*>(d_out), ldo, n, k);
    RWT_LAUNCHED();
    return RWT_OK;
}

extern "C" rwt_status rwt_apply_M(int32_t n, int64_t nC, const int32_t* d_crow,
                                  const int32_t* d_ccol, const void* d_cval, rwt_dtype dt,
                                  const void* d_B, int32_t k, int64_t ldb, void* d_out,
                                  int64_t ldo, void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    RWT_TRY(apply_m_checks(n, nC, d_crow, d_ccol, d_cval, dt, d_B, k, ldb, d_out, ldo));
    size_t need = 0;
    RWT_TRY(rwt_apply_M_ws(n, &need));
    RWT_REQUIRE(d_ws && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "apply_M workspace must hold %zu bytes", need);
    if (n == 0 || k == 0) return RWT_OK;
    return apply_m_run(n, nC, d_crow, d_ccol, d_cval, dt, d_B, k, ldb, d_out, ldo,
                       static_cast<int32_t*>(d_ws), hs(stream));
}

// ---------------------------------------------------------------------------
// rwt_apply_M without a workspace: the row offsets live in a file-scope
// device array.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); the device address of each
// GPU's copy is looked up once per device and kept.
// ---------------------------------------------------------------------------
__device__ __align__(256) int32_t scratch[RWT_APPLY_M_NOALLOC_MAX_N + 1];

namespace {
std::mutex g_scratch_mu;
std::vector<int32_t*> g_scratch_ptr;   // per device ordinal; nullptr until looked up

rwt_status scratch_for_current_device(int32_t** out) {
    int dev = -1;
    RWT_HIP(hipGetDevice(&dev));
    RWT_REQUIRE(dev >= 0, RWT_ERR_INVALID_ARG, "no current device");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr.size() <= (size_t)dev) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        RWT_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        RWT_REQUIRE(p != nullptr, RWT_ERR_HIP, "no device address for the apply_M scratch array");
        g_scratch_ptr[dev] = static_cast<int32_t*>(p);
    }
    *out = g_scratch_ptr[dev];
    return RWT_OK;
}
}  // namespace

extern "C" rwt_status rwt_apply_M_noalloc(int32_t n, int64_t nC, const int32_t* d_crow,
                                          const int32_t* d_ccol, const void* d_cval, rwt_dtype dt,
                                          const void* d_B, int32_t k, int64_t ldb, void* d_out,
                                          int64_t ldo, rwt_stream_t stream) {
    RWT_TRY(apply_m_checks(n, nC, d_crow, d_ccol, d_cval, dt, d_B, k, ldb, d_out, ldo));
    RWT_REQUIRE(n <= RWT_APPLY_M_NOALLOC_MAX_N, RWT_ERR_TOO_LARGE,
                "apply_M_noalloc handles at most %d rows (n = %d); use rwt_apply_M",
                (int)RWT_APPLY_M_NOALLOC_MAX_N, (int)n);
    int32_t* ptr = nullptr;
    RWT_TRY(scratch_for_current_device(&ptr));
    if (n == 0 || k == 0) return RWT_OK;
    // every entry ptr[0..n] is rewritten by the segment-start kernel before
    // the product reads it, so nothing left by an earlier call is read
    return apply_m_run(n, nC, d_crow, d_ccol, d_cval, dt, d_B, k, ldb, d_out, ldo, ptr,
                       hs(stream));
}

extern "C" rwt_status rwt_grad_vals(const rwt_csr* L, const void* d_gB, int64_t ldg,
                                    const void* d_X, int64_t ldx, int32_t k, void* d_gvals,
                                    rwt_stream_t stream) {
    RWT_REQUIRE(L != nullptr && L->n >= 0 && L->nnz >= 0 && k >= 0, RWT_ERR_INVALID_ARG,
                "bad arguments");
    RWT_REQUIRE(L->nnz < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "nnz must be < 2^31");
    RWT_REQUIRE(L->dt == RWT_F64 || L->dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    RWT_REQUIRE(L->n == 0 || (L->rowptr && L->colidx && d_gvals), RWT_ERR_INVALID_ARG,
                "null pointer");
    RWT_REQUIRE(k == 0 || L->n == 0 || (d_gB && d_X && ldg >= L->n && ldx >= L->n), RWT_ERR_INVALID_ARG,
                "bad dense blocks");
    if (L->n == 0) return RWT_OK;
    hipStream_t s = hs(stream);
    const unsigned g = (unsigned)((L->n + 255) / 256);
    if (L->dt == RWT_F64)
        hipLaunchKernelGGL(k_grad_vals<double>, dim3(g), dim3(256), 0, s, L->rowptr, L->colidx, L->n,
                           static_cast<const double*>(d_gB), ldg, static_cast<const double*>(d_X),
                           ldx, k, static_cast<double*>(d_gvals));
    else
        hipLaunchKernelGGL(k_grad_vals<float>, dim3(g), dim3(256), 0, s, L->rowptr, L->colidx, L->n,
                           static_cast<const float*>(d_gB), ldg, static_cast<const float*>(d_X), ldx,
                           k, static_cast<float*>(d_gvals));
    RWT_LAUNCHED();
    return RWT_OK;
}
