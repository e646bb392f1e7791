// Prefix sums and a stable radix sort built from wave64 ballot / mbcnt
// primitives.  Used by the analysis (level-ordered permutation, transposed
// pattern), the rewrite (new row pointers) and the adjoint (C^T).
#include "prim.hpp"

namespace rwt {

namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// inclusive scan of one value per thread across the block; returns the
// exclusive prefix and writes the block total to *total
template <typename T>
__device__ T block_exclusive(T v, T* total) {
    __shared__ T s_wave[SCAN_THREADS / WAVE];
    const int lane = lane_id();
    const int w = threadIdx.x / WAVE;
    T inc = v;
    for (int o = 1; o < WAVE; o <<= 1) {
        T u = __shfl_up(inc, o);
        if (lane >= o) inc += u;
    }
    if (lane == WAVE - 1) s_wave[w] = inc;
    __syncthreads();
    T wave_off = 0, tot = 0;
    for (int i = 0; i < SCAN_THREADS / WAVE; ++i) {
        if (i < w) wave_off += s_wave[i];
        tot += s_wave[i];
    }
    __syncthreads();
    *total = tot;
    return wave_off + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_tile_sums(const T* in, int64_t n, T* sums) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t e = base + (int64_t)i * SCAN_THREADS + threadIdx.x;
        if (e < n) acc += in[e];
    }
    T tot;
    (void)block_exclusive(acc, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums(T* sums, int64_t nt, T* total_out) {
    T carry = 0;
    for (int64_t b = 0; b < nt; b += SCAN_THREADS) {
        int64_t e = b + threadIdx.x;
        T v = e < nt ? sums[e] : T(0);
        T tot;
        T ex = block_exclusive(v, &tot);
        if (e < nt) sums[e] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

template <typename T>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_apply(const T* in, T* out, int64_t n,
                                                           const T* sums) {
    int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    T v[SCAN_ITEMS];
    T acc = 0;
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t e = base + i;
        v[i] = e < n ? in[e] : T(0);
        acc += v[i];
    }
    T tot;
    T ex = block_exclusive(acc, &tot) + sums[blockIdx.x];
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        int64_t e = base + i;
        if (e < n) out[e] = ex;
        ex += v[i];
    }
}

template <typename T>
rwt_status scan_impl(const T* in, T* out, int64_t n, void* ws, hipStream_t s) {
    int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nt < 1) nt = 1;
    T* sums = static_cast<T*>(ws);
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s, in, n, sums);
    RWT_LAUNCHED();
    hipLaunchKernelGGL(k_scan_sums<T>, dim3(1), dim3(SCAN_THREADS), 0, s, sums, nt, out + n);
    RWT_LAUNCHED();
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s, in, out, n,
                       (const T*)sums);
    RWT_LAUNCHED();
    return RWT_OK;
}

// ---------------------------------------------------------------------------
// radix sort, 8-bit digits
// ---------------------------------------------------------------------------
constexpr int RX_THREADS = 256;
constexpr int RX_ITEMS = 16;
constexpr int RX_TILE = RX_THREADS * RX_ITEMS;
constexpr int RX_WAVES = RX_THREADS / WAVE;

__global__ void __launch_bounds__(RX_THREADS) k_rx_hist(const uint32_t* keys, int64_t n, int shift,
                                                      uint32_t* hist, int64_t nb) {
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * RX_TILE;
    for (int i = 0; i < RX_ITEMS; ++i) {
        int64_t e = base + (int64_t)i * RX_THREADS + threadIdx.x;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(RX_THREADS) k_rx_scatter(const uint32_t* kin, const int32_t* vin,
                                                         uint32_t* kout, int32_t* vout, int64_t n,
                                                         int shift, const int32_t* offs,
                                                         int64_t nb) {
    __shared__ int32_t s_base[256];
    __shared__ int32_t s_wave[RX_WAVES][256];
    const int t = threadIdx.x;
    const int w = t / WAVE;
    s_base[t] = offs[(int64_t)t * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * RX_TILE;
    const uint64_t lt = (1ull << lane_id()) - 1ull;
    for (int c = 0; c < RX_ITEMS; ++c) {
        for (int q = 0; q < RX_WAVES; ++q) s_wave[q][t] = 0;
        __syncthreads();
        const int64_t e = base + (int64_t)c * RX_THREADS + t;
        const bool valid = e < n;
        uint32_t key = valid ? kin[e] : 0u;
        int32_t val = valid ? vin[e] : 0;
        uint32_t d = (key >> shift) & 255u;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        int rank = __popcll(m & lt);
        if (valid && rank == 0) s_wave[w][d] = __popcll(m);
        __syncthreads();
        {
            int32_t acc = s_base[t];
            for (int q = 0; q < RX_WAVES; ++q) {
                int32_t v = s_wave[q][t];
                s_wave[q][t] = acc;
                acc += v;
            }
            s_base[t] = acc;
        }
        __syncthreads();
        if (valid) {
            int32_t pos = s_wave[w][d] + rank;
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
    }
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) p[i] = v;
}

__global__ void k_zero_bytes(unsigned char* p, int64_t bytes) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < bytes; i += st) p[i] = 0;
}

// one wave per 64 rows: each lane writes its row's indices (short rows),
// long rows are written by the whole wave
__global__ void k_expand_rows(const int32_t* rowptr, int32_t n, int32_t* rowidx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        int32_t b = rowptr[i], e = rowptr[i + 1];
        for (int32_t p = b; p < e; ++p) rowidx[p] = (int32_t)i;
    }
}

__global__ void k_segment_starts(const uint32_t* keys, int64_t nkeys, int64_t nseg, int32_t* ptr,
                                 const int32_t* nseg_dev) {
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    const int64_t last = nseg_dev ? (int64_t)*nseg_dev : nseg;
    for (; c <= last; c += st) {
        int64_t lo = 0, hi = nkeys;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)keys[mid] < c) lo = mid + 1;
            else hi = mid;
        }
        ptr[c] = (int32_t)lo;
    }
}

}  // namespace

rwt_status segment_starts(const uint32_t* keys, int64_t nkeys, int64_t nseg, int32_t* ptr,
                          const int32_t* nseg_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_segment_starts, dim3(blocks_for(nseg + 1, 256, 8192)), dim3(256), 0, s,
                       keys, nkeys, nseg, ptr, nseg_dev);
    RWT_LAUNCHED();
    return RWT_OK;
}

size_t scan_ws(int64_t n) {
    int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
    if (nt < 1) nt = 1;
    return (size_t)nt * 8 + 256;
}

rwt_status scan_exclusive(const int32_t* in, int32_t* out, int64_t n, void* ws, hipStream_t s) {
    return scan_impl<int32_t>(in, out, n, ws, s);
}
rwt_status scan_exclusive(const int64_t* in, int64_t* out, int64_t n, void* ws, hipStream_t s) {
    return scan_impl<int64_t>(in, out, n, ws, s);
}

size_t radix_ws(int64_t n) {
    int64_t nb = (n + RX_TILE - 1) / RX_TILE;
    if (nb < 1) nb = 1;
    size_t hist = (size_t)(256 * nb + 1) * 4;
    hist = (hist + 255) & ~size_t(255);
    return hist + scan_ws(256 * nb);
}

rwt_status radix_sort(uint32_t* keys, int32_t* vals, uint32_t* tkeys, int32_t* tvals, int64_t n,
                      int key_bits, void* ws, hipStream_t s) {
    if (n <= 1) return RWT_OK;
    int64_t nb = (n + RX_TILE - 1) / RX_TILE;
    size_t hist_bytes = ((size_t)(256 * nb + 1) * 4 + 255) & ~size_t(255);
    uint32_t* hist = static_cast<uint32_t*>(ws);
    void* sws = static_cast<char*>(ws) + hist_bytes;
    uint32_t* ka = keys;
    int32_t* va = vals;
    uint32_t* kb = tkeys;
    int32_t* vb = tvals;
    int passes = (key_bits + 7) / 8;
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_rx_hist, dim3((unsigned)nb), dim3(RX_THREADS), 0, s, ka, n, shift,
                           hist, nb);
        RWT_LAUNCHED();
        RWT_TRY(scan_exclusive(reinterpret_cast<int32_t*>(hist), reinterpret_cast<int32_t*>(hist),
                               256 * nb, sws, s));
        hipLaunchKernelGGL(k_rx_scatter, dim3((unsigned)nb), dim3(RX_THREADS), 0, s, ka, va, kb, vb,
                           n, shift, reinterpret_cast<const int32_t*>(hist), nb);
        RWT_LAUNCHED();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        RWT_HIP(hipMemcpyAsync(keys, ka, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
        RWT_HIP(hipMemcpyAsync(vals, va, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
    }
    return RWT_OK;
}

rwt_status fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return RWT_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(blocks_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status fill_u8(void* p, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return RWT_OK;
    hipLaunchKernelGGL(k_zero_bytes, dim3(blocks_for(bytes, 256, 4096)), dim3(256), 0, s,
                       static_cast<unsigned char*>(p), bytes);
    RWT_LAUNCHED();
    return RWT_OK;
}

rwt_status expand_rows(const int32_t* rowptr, int32_t n, int32_t* rowidx, hipStream_t s) {
    if (n <= 0) return RWT_OK;
    hipLaunchKernelGGL(k_expand_rows, dim3(blocks_for(n, 256, 8192)), dim3(256), 0, s, rowptr, n,
                       rowidx);
    RWT_LAUNCHED();
    return RWT_OK;
}

}  // namespace rwt
