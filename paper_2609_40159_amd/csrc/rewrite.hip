// Equation rewriting (paper Section 2.2; the <node, source, target> rewriting
// list of Algorithm 1).
//
// One wave per rewritten row r with target level t.  The row lives in an
// LDS accumulator kept sorted by column.  Repeatedly: take the largest
// column j != r whose level is >= t, set c = acc[j] / L_jj, drop j and merge
// the off-diagonal entries of the input row j scaled by -c into the
// accumulator (B'[r,:] -= c * B[j,:] likewise), until no such column is
// left.  Because j decreases at every step and row j only holds columns
// below j, a dropped column never comes back.
//
// The merge is wave-parallel: duplicates of row j's columns in the
// accumulator are found by binary search, a wave prefix sum over the
// non-duplicates gives each entry its output slot, and each accumulator
// entry finds its partner in row j by binary search.  Every value update
// is one rounded multiply and one rounded subtract in elimination order,
// exactly as written in the recurrence (no fused multiply-add), so L' and
// B' do not depend on the parallel schedule.
//
// Symbolic pass: output lengths and substitution counts (row pointers of L'
// and of the multiplier list).  Numeric pass: values, B' and multipliers.
// Rows whose accumulator outgrows the LDS capacity are redone by a
// fallback kernel whose buffers are in the workspace.
#include "analyze.hpp"
#include "batch.hpp"
#include "prim.hpp"
#include "rowmap.hpp"

namespace rwt {

namespace {

// Rows are rewritten by one wave each with the accumulator in LDS, in two
// capacity tiers: most rows fit the small tier, whose low LDS use keeps
// many waves resident; rows that overflow it retry in the large tier, and
// rows that overflow that one use workspace slabs in global memory.
constexpr int RW_CAP1 = 128;               // small tier: entries per accumulator / staged row
constexpr int RW_WAVES1 = 4;               // small tier: waves per workgroup
constexpr int RW_CAP2 = 640;               // large tier
constexpr int RW_WAVES2 = 2;
constexpr int NSLAB = 2;                   // concurrent fallback rows

// LDS bytes of one wave's buffers at capacity CAP (value size S)
constexpr int rw_wave_bytes(int CAP, int S) {
    return 2 * CAP * (4 + S + 1) + CAP * (4 + S) + (CAP + 1) * 4 + CAP + 64;
}

struct Bufs {
    int32_t* acol[2];
    double* aval[2];          // used as float storage for FP32 via reinterpret (see below)
    unsigned char* aelig[2];
    int32_t* bcol;
    double* bval;
    int32_t* nd;              // exclusive prefix of non-duplicate flags of row j, cap + 1
    unsigned char* bdup;
    int32_t cap;
    int32_t capb;
};

struct RwArgs {
    int32_t n;
    const int32_t* rowptr;
    const int32_t* colidx;
    const void* vals;
    const int32_t* level;
    const int32_t* set_rows;
    const int32_t* targets;
    int32_t m;
    // symbolic outputs
    int32_t* counts;          // n (+1 for the scan total)
    int32_t* csub;            // m (+1)
    unsigned char* rewritten; // n
    int32_t* ovf;             // rows that overflowed the small LDS tier (set indices)
    int32_t* ovf2;            // rows that overflowed the large LDS tier
    unsigned char* ovf_mark;  // m: 0 small tier, 1 large tier, 2 slab
    int32_t* ctrl;            // [0] overflow count, [1] skipped, [2] error, [3] too-large,
                              // [4] capacity mismatch, [5] second overflow count
    // numeric inputs / outputs
    const int32_t* rowptr_out;
    int32_t* colidx_out;
    void* vals_out;
    const int32_t* cptr;
    int32_t* crow;
    int32_t* ccol;
    void* cval;
    const void* B;
    int64_t ldb;
    void* Bp;
    int64_t ldbp;
    int32_t k;
    // fallback slabs
    unsigned char* slab;
    int64_t slab_stride;
    int32_t slab_cap;
    // outputs indexed by set position (batched candidate analysis)
    int32_t* counts_q;
    const int32_t* pat_ptr;
    int32_t* pat_out;
    int32_t pat_cap;
    unsigned char* cand_bad_out;   // batched: candidate rejected when its pattern does not fit
    int32_t cand_index;
    int32_t* pat_start_out;        // batched, one pass: start of each position's pattern
    int32_t slot_len;              // batched, one pass: fixed slot per position
    int32_t* bump;                 // batched, one pass: overflow region in use
    int32_t* redo;                 // batched, one pass: set when the overflow region is full
    int32_t qcap;
};

// One-pass batched patterns: where position q's pattern of len entries
// goes (its fixed slot, or the overflow region after qcap slots); -1 when
// the capacity is exceeded, which asks for the two-pass form (lengths, a
// scan, exact places) after this pass.  Wave-uniform.
__device__ __forceinline__ int64_t pattern_place(const RwArgs& a, int32_t q, int32_t len) {
    int64_t ob;
    if (len <= a.slot_len) {
        ob = (int64_t)q * a.slot_len;
    } else {
        // the overflow region is split in PATTERN_BUMPS parts with a
        // counter each (position q takes part q mod PATTERN_BUMPS), so that
        // the atomics spread over as many addresses
        const int64_t base = (int64_t)a.qcap * a.slot_len;
        const int64_t part = ((int64_t)a.pat_cap - base) / PATTERN_BUMPS;
        const int32_t k = q & (PATTERN_BUMPS - 1);
        int32_t o = 0;
        if (lane_id() == 0) o = atomicAdd(a.bump + k, len);
        o = __shfl(o, 0);
        // (a counter past 2^31 - 1 reads negative: full as well)
        ob = (o < 0 || o + (int64_t)len > part) ? (int64_t)a.pat_cap : base + k * part + o;
    }
    if (ob + len > a.pat_cap) {
        if (lane_id() == 0) atomicExch(a.redo, 1);
        return -1;
    }
    return ob;
}

// Order this wave's earlier buffer writes before its later reads (the
// buffers may be LDS or global memory).
__device__ __forceinline__ void phase_sync() {
    __builtin_amdgcn_s_waitcnt(0);
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int lower_bound_lds(const int32_t* a, int len, int32_t x) {
    int lo = 0, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}


// Rewrite one row with one wave.  Returns false on capacity overflow.
// QMODE 0: symbolic or numeric rewrite of one matrix; QMODE 1: only the new
// row length, stored at counts_q[q]; QMODE 2: only the new pattern, stored
// at pat_out[pat_ptr[q]...]; QMODE 3: both, the pattern placed by
// pattern_place.
template <typename T, bool NUMERIC, int QMODE = 0>
__device__ __forceinline__ bool rewrite_row(const RwArgs& a, int32_t q, const Bufs& bf) {
    const int lane = lane_id();
    const int32_t r = a.set_rows[q];
    const int32_t t = a.targets ? a.targets[q] : a.level[r] - 1;
    const T* vals = static_cast<const T*>(a.vals);
    int cur = 0;
    int32_t* acol = bf.acol[0];
    T* aval = reinterpret_cast<T*>(bf.aval[0]);
    unsigned char* aelig = bf.aelig[0];
    // load row r
    const int32_t rb = a.rowptr[r], re = a.rowptr[r + 1];
    int32_t alen = re - rb;
    if (alen > bf.cap) return false;
    for (int32_t p = lane; p < alen; p += WAVE) {
        int32_t c = a.colidx[rb + p];
        acol[p] = c;
        if (NUMERIC) aval[p] = vals[rb + p];
        aelig[p] = (c != r && a.level[c] >= t) ? 1 : 0;
    }
    if (NUMERIC) {
        T* Bp = static_cast<T*>(a.Bp);
        const T* B = static_cast<const T*>(a.B);
        for (int32_t c = lane; c < a.k; c += WAVE) Bp[r + c * a.ldbp] = B[r + c * a.ldb];
    }
    phase_sync();
    int32_t nsub = 0;
    int32_t csub_base = NUMERIC ? a.cptr[q] : 0;
    for (;;) {
        // largest eligible column: scan from the top in chunks of 64
        int32_t jpos = -1;
        for (int32_t top = alen - 1; top >= 0 && jpos < 0; top -= WAVE) {
            int32_t p = top - lane;
            bool e = p >= 0 && aelig[p];
            uint64_t bal = __ballot(e);
            if (bal) jpos = top - (int32_t)__builtin_ctzll(bal);
        }
        if (jpos < 0) break;
        const int32_t j = acol[jpos];
        const int32_t jb = a.rowptr[j], je = a.rowptr[j + 1] - 1;   // off-diagonal part
        const int32_t blen = je - jb;
        if (blen > bf.capb) return false;
        T cm = T(0);
        if (NUMERIC) {
            // the symbolic pass sized the substitution slots of this row
            if (csub_base + nsub >= a.cptr[q + 1]) {
                if (lane == 0) atomicExch(&a.ctrl[4], 1);
                return true;
            }
            cm = aval[jpos] / vals[je];
            if (lane == 0 && a.crow) {
                a.crow[csub_base + nsub] = r;
                a.ccol[csub_base + nsub] = j;
                static_cast<T*>(a.cval)[csub_base + nsub] = cm;
            }
            T* Bp = static_cast<T*>(a.Bp);
            const T* B = static_cast<const T*>(a.B);
            for (int32_t c = lane; c < a.k; c += WAVE)
                Bp[r + c * a.ldbp] = sub_rn(Bp[r + c * a.ldbp], mul_rn(cm, B[j + c * a.ldb]));
        }
        ++nsub;
        // stage row j
        T* bval = reinterpret_cast<T*>(bf.bval);
        for (int32_t p = lane; p < blen; p += WAVE) {
            bf.bcol[p] = a.colidx[jb + p];
            if (NUMERIC) bval[p] = vals[jb + p];
        }
        phase_sync();
        // duplicates and the exclusive prefix of non-duplicates
        int32_t run = 0;
        for (int32_t b0 = 0; b0 < blen; b0 += WAVE) {
            int32_t b = b0 + lane;
            bool valid = b < blen;
            bool dup = false;
            if (valid) {
                int32_t x = bf.bcol[b];
                int lb = lower_bound_lds(acol, alen, x);
                dup = lb < alen && acol[lb] == x;
                bf.bdup[b] = dup ? 1 : 0;
            }
            uint64_t nd = __ballot(valid && !dup);
            if (valid) bf.nd[b] = run + lanes_below(nd);
            run += (int32_t)__popcll(nd);
        }
        if (lane == 0) bf.nd[blen] = run;
        phase_sync();
        const int32_t nlen = alen - 1 + run;
        if (nlen > bf.cap) return false;
        const int nxt = cur ^ 1;
        // select, not index: a dynamically indexed pointer array would live in scratch
        int32_t* ocol = nxt ? bf.acol[1] : bf.acol[0];
        T* oval = reinterpret_cast<T*>(nxt ? bf.aval[1] : bf.aval[0]);
        unsigned char* oelig = nxt ? bf.aelig[1] : bf.aelig[0];
        // accumulator entries (except j)
        for (int32_t p = lane; p < alen; p += WAVE) {
            if (p == jpos) continue;
            int32_t x = acol[p];
            int lb = lower_bound_lds(bf.bcol, blen, x);
            int32_t o = (p > jpos ? p - 1 : p) + bf.nd[lb];
            ocol[o] = x;
            oelig[o] = aelig[p];
            if (NUMERIC) {
                T v = aval[p];
                if (lb < blen && bf.bcol[lb] == x) v = sub_rn(v, mul_rn(cm, bval[lb]));
                oval[o] = v;
            }
        }
        // new entries from row j
        for (int32_t b = lane; b < blen; b += WAVE) {
            if (bf.bdup[b]) continue;
            int32_t x = bf.bcol[b];
            int32_t o = bf.nd[b] + lower_bound_lds(acol, alen, x);
            ocol[o] = x;
            oelig[o] = a.level[x] >= t ? 1 : 0;
            if (NUMERIC) oval[o] = sub_rn(T(0), mul_rn(cm, bval[b]));
        }
        phase_sync();
        cur = nxt;
        acol = ocol;
        aval = oval;
        aelig = oelig;
        alen = nlen;
    }
    if (NUMERIC) {
        int32_t ob = a.rowptr_out[r];
        if (a.rowptr_out[r + 1] - ob != alen) {
            if (lane == 0) atomicExch(&a.ctrl[4], 1);
            return true;
        }
        T* vo = static_cast<T*>(a.vals_out);
        for (int32_t p = lane; p < alen; p += WAVE) {
            a.colidx_out[ob + p] = acol[p];
            vo[ob + p] = aval[p];
        }
    } else if (QMODE == 1) {
        if (lane == 0) a.counts_q[q] = alen;
    } else if (QMODE == 2) {
        const int32_t ob = a.pat_ptr[q];
        if (a.pat_ptr[q + 1] - ob != alen || (int64_t)ob + alen > a.pat_cap) {
            if (lane == 0) {
                atomicExch(&a.ctrl[4], 1);
                if (a.cand_bad_out) a.cand_bad_out[a.cand_index] = 1;
            }
            return true;
        }
        for (int32_t p = lane; p < alen; p += WAVE) a.pat_out[ob + p] = acol[p];
    } else if (QMODE == 3) {
        const int64_t ob = pattern_place(a, q, alen);
        if (ob < 0) return true;
        for (int32_t p = lane; p < alen; p += WAVE) a.pat_out[ob + p] = acol[p];
        if (lane == 0) {
            a.counts_q[q] = alen;
            a.pat_start_out[q] = (int32_t)ob;
        }
    } else if (lane == 0) {
        a.counts[r] = alen;
        a.csub[q] = nsub;
        a.rewritten[r] = 1;
    }
    return true;
}

__device__ __forceinline__ bool row_is_noop(const RwArgs& a, int32_t q) {
    const int32_t r = a.set_rows[q];
    const int32_t lv = a.level[r];
    const int32_t t = a.targets ? a.targets[q] : lv - 1;
    return lv == 0 || t >= lv;
}

// Carve one wave's buffers (capacity CAP entries) from base.
template <int CAP, int S>
__device__ __forceinline__ Bufs carve_bufs(unsigned char* base) {
    Bufs bf;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base + off;
        off += (bytes + 7) & ~size_t(7);
        return p;
    };
    for (int i = 0; i < 2; ++i) {
        bf.acol[i] = reinterpret_cast<int32_t*>(take(CAP * 4));
        bf.aval[i] = reinterpret_cast<double*>(take(CAP * S));
        bf.aelig[i] = take(CAP);
    }
    bf.bcol = reinterpret_cast<int32_t*>(take(CAP * 4));
    bf.bval = reinterpret_cast<double*>(take(CAP * S));
    bf.nd = reinterpret_cast<int32_t*>(take((CAP + 1) * 4));
    bf.bdup = take(CAP);
    bf.cap = CAP;
    bf.capb = CAP;
    return bf;
}

// TIER 1: every set position; a row that overflows goes to the first
// overflow list (mark 1).  TIER 2: the rows of the first list; a row that
// overflows again goes to the second list (mark 2) for the slabs.  The
// numeric pass follows the marks the symbolic pass left.
template <typename T, bool NUMERIC, int TIER>
__global__ void __launch_bounds__((TIER == 1 ? RW_WAVES1 : RW_WAVES2) * WAVE) k_rewrite_lds(RwArgs a) {
    constexpr int S = sizeof(T);
    constexpr int CAP = TIER == 1 ? RW_CAP1 : RW_CAP2;
    constexpr int WAVES = TIER == 1 ? RW_WAVES1 : RW_WAVES2;
    constexpr int PER_WAVE = rw_wave_bytes(CAP, S);
    __shared__ __align__(16) unsigned char s_buf[WAVES * PER_WAVE];
    const int w = threadIdx.x / WAVE;
    const Bufs bf = carve_bufs<CAP, S>(s_buf + w * PER_WAVE);
    const int64_t wave = (int64_t)blockIdx.x * WAVES + w;
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    const int64_t count = TIER == 1 ? a.m : a.ctrl[0];
    for (int64_t idx = wave; idx < count; idx += nw) {
        const int32_t q = TIER == 1 ? (int32_t)idx : a.ovf[idx];
        if (TIER == 1 && row_is_noop(a, q)) {
            if (!NUMERIC && lane_id() == 0) {
                atomicAdd(&a.ctrl[1], 1);
                a.csub[q] = 0;
            }
            continue;
        }
        if (NUMERIC && a.ovf_mark[q] >= TIER) continue;
        const bool ok = rewrite_row<T, NUMERIC>(a, q, bf);
        if (!ok && !NUMERIC && lane_id() == 0) {
            if (TIER == 1) {
                const int slot = atomicAdd(&a.ctrl[0], 1);
                a.ovf[slot] = q;
                a.ovf_mark[q] = 1;
            } else {
                const int slot = atomicAdd(&a.ctrl[5], 1);
                a.ovf2[slot] = q;
                a.ovf_mark[q] = 2;
            }
        }
    }
}

// A wave's buffers at capacity cap (value size S) carved from a workspace
// slab, 8-byte aligned.
__device__ inline Bufs slab_bufs(unsigned char* base, int64_t cap, int S) {
    int64_t off = 0;
    auto take = [&](int64_t bytes) {
        unsigned char* p = base + off;
        off += (bytes + 7) & ~int64_t(7);
        return p;
    };
    Bufs bf;
    for (int i = 0; i < 2; ++i) {
        bf.acol[i] = reinterpret_cast<int32_t*>(take(cap * 4));
        bf.aval[i] = reinterpret_cast<double*>(take(cap * S));
        bf.aelig[i] = take(cap);
    }
    bf.bcol = reinterpret_cast<int32_t*>(take(cap * 4));
    bf.bval = reinterpret_cast<double*>(take(cap * S));
    bf.nd = reinterpret_cast<int32_t*>(take((cap + 1) * 4));
    bf.bdup = take(cap);
    bf.cap = (int32_t)cap;
    bf.capb = (int32_t)cap;
    return bf;
}

// Rows that overflowed the LDS capacity: same algorithm, buffers in a
// workspace slab large enough for any row (n + 1 entries).
template <typename T, bool NUMERIC>
__global__ void __launch_bounds__(WAVE) k_rewrite_slab(RwArgs a) {
    const int32_t cnt = a.ctrl[5];
    const int S = sizeof(T);
    for (int32_t s = blockIdx.x; s < cnt; s += gridDim.x) {
        const Bufs bf = slab_bufs(a.slab + (int64_t)blockIdx.x * a.slab_stride, a.slab_cap, S);
        const int32_t q = a.ovf2[s];
        if (!rewrite_row<T, NUMERIC>(a, q, bf) && lane_id() == 0) atomicExch(&a.ctrl[3], 1);
    }
}

__global__ void k_rw_check(const int32_t* rows, const int32_t* targets, int32_t m, int32_t n,
                           int32_t* err) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; q < m; q += st) {
        int32_t r = rows[q];
        bool bad = r < 0 || r >= n || (q > 0 && rows[q - 1] >= r) || (targets && targets[q] < 0);
        if (bad) atomicExch(err, 1);
    }
}

__global__ void k_rw_counts(const int32_t* rowptr, int32_t n, int32_t* counts,
                            unsigned char* rewritten) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t st = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += st) {
        counts[i] = rowptr[i + 1] - rowptr[i];
        rewritten[i] = 0;
    }
}

// Copy the rows that are not rewritten, and their right-hand sides: a
// workgroup takes 256 rows and their contiguous entries; each thread finds
// its row in an LDS map of entry -> row (binary search when the rows'
// entries exceed it).
template <typename T>
__global__ void __launch_bounds__(256) k_rw_copy(const int32_t* rowptr, const int32_t* colidx,
                                                 const T* vals, int32_t n,
                                                 const unsigned char* rewritten,
                                                 const int32_t* rowptr_out, int32_t* colidx_out,
                                                 T* vals_out, const T* B, int64_t ldb, T* Bp,
                                                 int64_t ldbp, int32_t k) {
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
        const int lo = row_of(s_ptr, nr, s_row, mapped, p);
        const int32_t i = r0 + lo;
        if (rewritten[i]) continue;
        const int32_t o = rowptr_out[i] + (p - s_ptr[lo]);
        colidx_out[o] = colidx[p];
        vals_out[o] = vals[p];
    }
    const int32_t i = r0 + (int32_t)threadIdx.x;
    if (i < r1 && !rewritten[i])
        for (int32_t q = 0; q < k; ++q) Bp[i + q * ldbp] = B[i + q * ldb];
}

struct RwWs {
    int32_t* counts;
    int32_t* csub;
    int32_t* cptr;
    unsigned char* rewritten;
    int32_t* ovf;
    int32_t* ovf2;
    unsigned char* ovf_mark;
    int32_t* ctrl;
    void* scan;
    unsigned char* slab;
    int64_t slab_stride;
    int32_t slab_cap;
};

size_t carve_rw(void* base, int32_t n, int32_t m, rwt_dtype dt, RwWs* w) {
    Carver cv(base);
    w->counts = cv.take<int32_t>((size_t)n + 1);
    w->csub = cv.take<int32_t>((size_t)m + 1);
    w->cptr = cv.take<int32_t>((size_t)m + 1);
    w->rewritten = cv.take<unsigned char>(n > 0 ? n : 1);
    w->ovf = cv.take<int32_t>(m > 0 ? m : 1);
    w->ovf2 = cv.take<int32_t>(m > 0 ? m : 1);
    w->ovf_mark = cv.take<unsigned char>(m > 0 ? m : 1);
    w->ctrl = cv.take<int32_t>(8);
    w->scan = cv.take<char>(scan_ws((int64_t)(n > m ? n : m) + 1));
    const int64_t cap = (int64_t)n + 1;
    const int64_t S = (int64_t)dtype_size(dt);
    w->slab_cap = (int32_t)cap;
    w->slab_stride = (2 * cap * (4 + S + 1) + cap * (4 + S) + (cap + 1) * 4 + cap + 256 + 255) &
                     ~int64_t(255);
    w->slab = cv.take<unsigned char>((size_t)(NSLAB * w->slab_stride));
    return cv.used();
}

RwArgs make_rw(const rwt_csr* L, const int32_t* level, const int32_t* rows, const int32_t* targets,
               int32_t m, const RwWs& w) {
    RwArgs a;
    memset(&a, 0, sizeof a);
    a.n = L->n;
    a.rowptr = L->rowptr;
    a.colidx = L->colidx;
    a.vals = L->vals;
    a.level = level;
    a.set_rows = rows;
    a.targets = targets;
    a.m = m;
    a.counts = w.counts;
    a.csub = w.csub;
    a.rewritten = w.rewritten;
    a.ovf = w.ovf;
    a.ovf2 = w.ovf2;
    a.ovf_mark = w.ovf_mark;
    a.ctrl = w.ctrl;
    a.slab = w.slab;
    a.slab_stride = w.slab_stride;
    a.slab_cap = w.slab_cap;
    return a;
}

template <typename T, bool NUMERIC>
rwt_status launch_tiers(const RwArgs& a, hipStream_t s) {
    const unsigned g1 = blocks_for((size_t)a.m, RW_WAVES1, 8192);
    hipLaunchKernelGGL((k_rewrite_lds<T, NUMERIC, 1>), dim3(g1), dim3(RW_WAVES1 * WAVE), 0, s, a);
    RWT_LAUNCHED();
    // the second tier reads its row count on the device; a grid of one
    // workgroup per compute unit covers the (few) rows that reach it
    hipLaunchKernelGGL((k_rewrite_lds<T, NUMERIC, 2>), dim3(256), dim3(RW_WAVES2 * WAVE), 0, s, a);
    RWT_LAUNCHED();
    hipLaunchKernelGGL((k_rewrite_slab<T, NUMERIC>), dim3(NSLAB), dim3(WAVE), 0, s, a);
    RWT_LAUNCHED();
    return RWT_OK;
}

template <typename T>
rwt_status launch_rows(const RwArgs& a, bool numeric, hipStream_t s) {
    if (a.m == 0) return RWT_OK;
    return numeric ? launch_tiers<T, true>(a, s) : launch_tiers<T, false>(a, s);
}

// ---------------------------------------------------------------------------
// Batched candidate rows: many matrices, many candidate row sets.  Set
// position q belongs to candidate c = the last c with cand_ptr[c] <= q, whose
// matrix is cand_mat[c].
// ---------------------------------------------------------------------------
struct BatchRwArgsDev {
    const BatchRwMat* mats;
    const int32_t* cand_ptr;
    const int32_t* cand_mat;
    int32_t C;
    const int32_t* rows;
    const int32_t* targets;
    int32_t qcap;
    int32_t* counts_q;
    int32_t* pat_ptr;
    int32_t* pat;
    int32_t pat_cap;
    int32_t slot_len;
    int32_t* bump;
    int32_t* redo;
    const int32_t* gate;
    int32_t* ovf;    // positions that overflowed the small LDS tier
    int32_t* ovf2;   // positions that overflowed the large LDS tier
    unsigned char* ovf_mark;
    int32_t* ctrl;   // [0] first overflow count, [3] too large, [4] capacity error,
                     // [7] second overflow count
    unsigned char* cand_bad;
    unsigned char* slab;
    int64_t slab_stride;
    int32_t slab_cap;
};

__device__ inline int32_t cand_of(const int32_t* cand_ptr, int32_t C, int32_t q) {
    int32_t lo = 0, hi = C - 1;   // last c with cand_ptr[c] <= q
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (cand_ptr[mid] <= q) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__device__ inline RwArgs batch_row_args(const BatchRwArgsDev& ba, int32_t q) {
    const int32_t c = cand_of(ba.cand_ptr, ba.C, q);
    const BatchRwMat& M = ba.mats[ba.cand_mat[c]];
    RwArgs a{};
    a.cand_bad_out = ba.cand_bad;
    a.cand_index = c;
    a.n = M.n;
    a.rowptr = in_global(M.rowptr);
    a.colidx = in_global(M.colidx);
    a.level = in_global(M.level);
    a.set_rows = ba.rows;
    a.targets = ba.targets;
    a.ctrl = ba.ctrl;
    a.counts_q = ba.counts_q;
    a.pat_ptr = ba.pat_ptr;
    a.pat_out = ba.pat;
    a.pat_cap = ba.pat_cap;
    a.pat_start_out = ba.pat_ptr;
    a.slot_len = ba.slot_len;
    a.bump = ba.bump;
    a.redo = ba.redo;
    a.qcap = ba.qcap;
    return a;
}

// rows left unchanged keep their own pattern
template <int QMODE>
__device__ bool batch_noop_row(const BatchRwArgsDev& ba, const RwArgs& a, int32_t q) {
    const int32_t r = a.set_rows[q];
    const int32_t lv = a.level[r];
    const int32_t t = a.targets ? a.targets[q] : lv - 1;
    if (!(lv == 0 || t >= lv)) return false;
    const int32_t rb = a.rowptr[r], len = a.rowptr[r + 1] - rb;
    if (QMODE == 1) {
        if (lane_id() == 0) ba.counts_q[q] = len;
    } else if (QMODE == 3) {
        const int64_t ob = pattern_place(a, q, len);
        if (ob < 0) return true;
        for (int32_t p = lane_id(); p < len; p += WAVE) ba.pat[ob + p] = a.colidx[rb + p];
        if (lane_id() == 0) {
            ba.counts_q[q] = len;
            ba.pat_ptr[q] = (int32_t)ob;
        }
    } else {
        const int32_t ob = ba.pat_ptr[q];
        if (ba.pat_ptr[q + 1] - ob != len || (int64_t)ob + len > ba.pat_cap) {
            if (lane_id() == 0) {
                atomicExch(&ba.ctrl[4], 1);
                ba.cand_bad[cand_of(ba.cand_ptr, ba.C, q)] = 1;
            }
            return true;
        }
        for (int32_t p = lane_id(); p < len; p += WAVE) ba.pat[ob + p] = a.colidx[rb + p];
    }
    return true;
}

// Same two LDS tiers as the single-matrix rewrite: TIER 1 over every
// candidate position, TIER 2 over the positions that overflowed it; the
// pattern pass (QMODE 2) follows the marks of the length pass (QMODE 1).
// The one-pass form (QMODE 3) marks overflows like the length pass and
// writes each pattern in the tier where it fits.
template <int QMODE, int TIER>
__global__ void __launch_bounds__((TIER == 1 ? RW_WAVES1 : RW_WAVES2) * WAVE)
    k_batch_rw_lds(BatchRwArgsDev ba) {
    constexpr int CAP = TIER == 1 ? RW_CAP1 : RW_CAP2;
    constexpr int WAVES = TIER == 1 ? RW_WAVES1 : RW_WAVES2;
    constexpr int PER_WAVE = rw_wave_bytes(CAP, 8);
    __shared__ __align__(16) unsigned char s_buf[WAVES * PER_WAVE];
    if (ba.gate && ld_relaxed(ba.gate) == 0) return;   // the one pass sufficed
    const int w = threadIdx.x / WAVE;
    const Bufs bf = carve_bufs<CAP, 8>(s_buf + w * PER_WAVE);
    const int64_t count = TIER == 1 ? min(ba.cand_ptr[ba.C], ba.qcap) : ba.ctrl[0];
    const int64_t wave = (int64_t)blockIdx.x * WAVES + w;
    const int64_t nw = (int64_t)gridDim.x * WAVES;
    for (int64_t idx = wave; idx < count; idx += nw) {
        const int32_t q = TIER == 1 ? (int32_t)idx : ba.ovf[idx];
        if (TIER == 1) {
            if (ba.cand_bad[cand_of(ba.cand_ptr, ba.C, q)]) {
                if (QMODE != 2 && lane_id() == 0) ba.counts_q[q] = 0;
                continue;
            }
        }
        const RwArgs a = batch_row_args(ba, q);
        if (TIER == 1 && batch_noop_row<QMODE>(ba, a, q)) continue;
        if (QMODE == 2 && ba.ovf_mark[q] >= TIER) continue;
        const bool ok = rewrite_row<double, false, QMODE>(a, q, bf);
        if (!ok && QMODE != 2 && lane_id() == 0) {
            if (TIER == 1) {
                const int slot = atomicAdd(&ba.ctrl[0], 1);
                ba.ovf[slot] = q;
                ba.ovf_mark[q] = 1;
            } else {
                const int slot = atomicAdd(&ba.ctrl[7], 1);
                ba.ovf2[slot] = q;
                ba.ovf_mark[q] = 2;
            }
        }
    }
}

template <int QMODE>
__global__ void __launch_bounds__(WAVE) k_batch_rw_slab(BatchRwArgsDev ba) {
    if (ba.gate && ld_relaxed(ba.gate) == 0) return;
    const int32_t cnt = ba.ctrl[7];
    const int S = 8;
    for (int32_t s = blockIdx.x; s < cnt; s += gridDim.x) {
        const Bufs bf = slab_bufs(ba.slab + (int64_t)blockIdx.x * ba.slab_stride, ba.slab_cap, S);
        const int32_t q = ba.ovf2[s];
        const RwArgs a = batch_row_args(ba, q);
        if (!rewrite_row<double, false, QMODE>(a, q, bf) && lane_id() == 0) atomicExch(&ba.ctrl[3], 1);
    }
}

}  // namespace

size_t batch_rw_slab_stride(int32_t nmax) {
    const int64_t cap = (int64_t)nmax + 1;
    return (size_t)((2 * cap * (4 + 8 + 1) + cap * (4 + 8) + (cap + 1) * 4 + cap + 256 + 255) &
                    ~int64_t(255));
}

rwt_status batch_rewrite_pass(const BatchRwArgs& h, int qmode, hipStream_t s) {
    BatchRwArgsDev ba;
    ba.mats = h.mats;
    ba.cand_ptr = h.cand_ptr;
    ba.cand_mat = h.cand_mat;
    ba.C = h.C;
    ba.rows = h.rows;
    ba.targets = h.targets;
    ba.counts_q = h.counts_q;
    ba.pat_ptr = h.pat_ptr;
    ba.pat = h.pat;
    ba.pat_cap = h.pat_cap;
    ba.slot_len = h.slot_len;
    ba.bump = h.bump;
    ba.redo = h.redo;
    ba.gate = h.gate;
    ba.ovf = h.ovf;
    ba.ovf2 = h.ovf2;
    ba.ovf_mark = h.ovf_mark;
    ba.ctrl = h.ctrl;
    ba.cand_bad = h.cand_bad;
    ba.qcap = h.qcap;
    ba.slab = h.slab;
    ba.slab_stride = h.slab_stride;
    ba.slab_cap = h.slab_cap;
    const unsigned g = blocks_for((size_t)(h.qcap > 0 ? h.qcap : 1), RW_WAVES1, 8192);
    if (qmode == 1) {
        hipLaunchKernelGGL((k_batch_rw_lds<1, 1>), dim3(g), dim3(RW_WAVES1 * WAVE), 0, s, ba);
        RWT_LAUNCHED();
        hipLaunchKernelGGL((k_batch_rw_lds<1, 2>), dim3(256), dim3(RW_WAVES2 * WAVE), 0, s, ba);
        RWT_LAUNCHED();
        hipLaunchKernelGGL(k_batch_rw_slab<1>, dim3(h.nslab), dim3(WAVE), 0, s, ba);
    } else if (qmode == 2) {
        hipLaunchKernelGGL((k_batch_rw_lds<2, 1>), dim3(g), dim3(RW_WAVES1 * WAVE), 0, s, ba);
        RWT_LAUNCHED();
        hipLaunchKernelGGL((k_batch_rw_lds<2, 2>), dim3(256), dim3(RW_WAVES2 * WAVE), 0, s, ba);
        RWT_LAUNCHED();
        hipLaunchKernelGGL(k_batch_rw_slab<2>, dim3(h.nslab), dim3(WAVE), 0, s, ba);
    } else {
        hipLaunchKernelGGL((k_batch_rw_lds<3, 1>), dim3(g), dim3(RW_WAVES1 * WAVE), 0, s, ba);
        RWT_LAUNCHED();
        hipLaunchKernelGGL((k_batch_rw_lds<3, 2>), dim3(256), dim3(RW_WAVES2 * WAVE), 0, s, ba);
        RWT_LAUNCHED();
        hipLaunchKernelGGL(k_batch_rw_slab<3>, dim3(h.nslab), dim3(WAVE), 0, s, ba);
    }
    RWT_LAUNCHED();
    return RWT_OK;
}

namespace {
}  // namespace
}  // namespace rwt

using namespace rwt;

extern "C" rwt_status rwt_rewrite_ws(const rwt_csr* L, int32_t m, size_t* h_bytes) {
    RWT_REQUIRE(L != nullptr && h_bytes != nullptr, RWT_ERR_INVALID_ARG, "null argument");
    RWT_REQUIRE(L->n >= 0 && m >= 0, RWT_ERR_INVALID_ARG, "negative size");
    RwWs w;
    *h_bytes = carve_rw(nullptr, L->n, m, L->dt, &w);
    return RWT_OK;
}

static rwt_status rw_common_checks(const rwt_csr* L, const int32_t* level, const int32_t* rows,
                                   int32_t m, void* ws, size_t ws_bytes) {
    RWT_REQUIRE(L != nullptr && level != nullptr, RWT_ERR_INVALID_ARG, "null argument");
    RWT_REQUIRE(L->n >= 0 && L->nnz >= L->n && m >= 0, RWT_ERR_INVALID_ARG, "bad sizes");
    RWT_REQUIRE(L->nnz < (int64_t(1) << 31), RWT_ERR_TOO_LARGE, "nnz must be < 2^31");
    RWT_REQUIRE(m == 0 || rows != nullptr, RWT_ERR_INVALID_ARG, "null row set");
    RWT_REQUIRE(L->dt == RWT_F64 || L->dt == RWT_F32, RWT_ERR_INVALID_ARG, "bad dtype");
    RwWs w;
    size_t need = carve_rw(nullptr, L->n, m, L->dt, &w);
    RWT_REQUIRE(ws != nullptr && ws_bytes >= need, RWT_ERR_BUFFER_TOO_SMALL,
                "rewrite workspace must hold %zu bytes", need);
    return RWT_OK;
}

extern "C" rwt_status rwt_rewrite_symbolic(const rwt_csr* L, const int32_t* d_level,
                                           const int32_t* d_set_rows, const int32_t* d_targets,
                                           int32_t m, void* d_ws, size_t ws_bytes,
                                           int32_t* d_rowptr_out, int32_t* d_cptr_out,
                                           int64_t* h_sizes, rwt_stream_t stream) {
    RWT_TRY(rw_common_checks(L, d_level, d_set_rows, m, d_ws, ws_bytes));
    RWT_REQUIRE(d_rowptr_out && d_cptr_out && h_sizes, RWT_ERR_INVALID_ARG, "null output");
    hipStream_t s = hs(stream);
    RwWs w;
    carve_rw(d_ws, L->n, m, L->dt, &w);
    RWT_TRY(validate_device(*L, L->vals != nullptr, w.ctrl, nullptr, s));
    RWT_TRY(fill_u8(w.ctrl, 8 * sizeof(int32_t), s));
    if (m > 0) {
        hipLaunchKernelGGL(k_rw_check, dim3(blocks_for(m, 256, 1024)), dim3(256), 0, s, d_set_rows,
                           d_targets, m, L->n, w.ctrl + 2);
        RWT_LAUNCHED();
        int32_t bad = 0;
        RWT_HIP(hipMemcpyAsync(&bad, w.ctrl + 2, 4, hipMemcpyDeviceToHost, s));
        RWT_HIP(hipStreamSynchronize(s));
        RWT_REQUIRE(bad == 0, RWT_ERR_BAD_ROWSET,
                    "row set must be strictly ascending rows in [0, n) with targets >= 0");
        RWT_TRY(fill_u8(w.ovf_mark, m, s));
    }
    if (L->n > 0) {
        hipLaunchKernelGGL(k_rw_counts, dim3(blocks_for(L->n, 256, 8192)), dim3(256), 0, s,
                           L->rowptr, L->n, w.counts, w.rewritten);
        RWT_LAUNCHED();
    }
    RwArgs a = make_rw(L, d_level, d_set_rows, d_targets, m, w);
    if (L->dt == RWT_F64) RWT_TRY(launch_rows<double>(a, false, s));
    else RWT_TRY(launch_rows<float>(a, false, s));
    RWT_TRY(scan_exclusive(w.counts, d_rowptr_out, L->n, w.scan, s));
    // the substitution offsets stay in the workspace too: the numeric call
    // (same workspace, untouched in between) reads them from there
    RWT_TRY(scan_exclusive(w.csub, w.cptr, m, w.scan, s));
    RWT_HIP(hipMemcpyAsync(d_cptr_out, w.cptr, sizeof(int32_t) * ((size_t)m + 1),
                           hipMemcpyDeviceToDevice, s));
    int32_t tail[2] = {0, 0};
    int32_t hc[8];
    RWT_HIP(hipMemcpyAsync(&tail[0], d_rowptr_out + L->n, 4, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipMemcpyAsync(&tail[1], d_cptr_out + m, 4, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipMemcpyAsync(hc, w.ctrl, sizeof hc, hipMemcpyDeviceToHost, s));
    RWT_HIP(hipStreamSynchronize(s));
    RWT_REQUIRE(hc[3] == 0, RWT_ERR_TOO_LARGE, "a rewritten row exceeded the workspace capacity");
    h_sizes[0] = tail[0];
    h_sizes[1] = tail[1];
    h_sizes[2] = hc[1];
    return RWT_OK;
}

extern "C" rwt_status rwt_rewrite_numeric(const rwt_csr* L, const int32_t* d_level,
                                          const int32_t* d_set_rows, const int32_t* d_targets,
                                          int32_t m, const void* d_B, int32_t k, int64_t ldb,
                                          const rwt_csr* Lp, void* d_Bp, int64_t ldbp,
                                          int32_t* d_crow, int32_t* d_ccol, void* d_cval,
                                          void* d_ws, size_t ws_bytes, rwt_stream_t stream) {
    RWT_TRY(rw_common_checks(L, d_level, d_set_rows, m, d_ws, ws_bytes));
    RWT_REQUIRE(L->vals != nullptr, RWT_ERR_INVALID_ARG, "values required");
    RWT_REQUIRE(Lp != nullptr && Lp->rowptr && (Lp->nnz == 0 || (Lp->colidx && Lp->vals)),
                RWT_ERR_INVALID_ARG, "null output matrix");
    RWT_REQUIRE(Lp->n == L->n && Lp->dt == L->dt, RWT_ERR_INVALID_ARG, "output matrix mismatch");
    RWT_REQUIRE(k >= 0 && (k == 0 || L->n == 0 || (d_B && d_Bp && ldb >= L->n && ldbp >= L->n)),
                RWT_ERR_INVALID_ARG, "bad right-hand side block");
    RWT_REQUIRE(k == 0 || d_B != d_Bp, RWT_ERR_INVALID_ARG, "B' may not alias B");
    hipStream_t s = hs(stream);
    RwWs w;
    carve_rw(d_ws, L->n, m, L->dt, &w);
    RwArgs a = make_rw(L, d_level, d_set_rows, d_targets, m, w);
    a.rowptr_out = Lp->rowptr;
    a.colidx_out = const_cast<int32_t*>(Lp->colidx);
    a.vals_out = const_cast<void*>(Lp->vals);
    a.B = d_B;
    a.ldb = ldb;
    a.Bp = d_Bp;
    a.ldbp = ldbp;
    a.k = k;
    a.crow = d_crow;
    a.ccol = d_ccol;
    a.cval = d_cval;
    RWT_REQUIRE((d_crow && d_ccol && d_cval) || (!d_crow && !d_ccol && !d_cval),
                RWT_ERR_INVALID_ARG, "multiplier arrays must be all given or all NULL");
    // offsets of each row's substitutions: the symbolic call left them in
    // the workspace
    a.cptr = w.cptr;
    if (L->n > 0) {
        const unsigned g = (unsigned)((L->n + 255) / 256);
        if (L->dt == RWT_F64)
            hipLaunchKernelGGL(k_rw_copy<double>, dim3(g), dim3(256), 0, s, L->rowptr, L->colidx,
                               static_cast<const double*>(L->vals), L->n, w.rewritten, Lp->rowptr,
                               a.colidx_out, static_cast<double*>(a.vals_out),
                               static_cast<const double*>(d_B), ldb, static_cast<double*>(d_Bp),
                               ldbp, k);
        else
            hipLaunchKernelGGL(k_rw_copy<float>, dim3(g), dim3(256), 0, s, L->rowptr, L->colidx,
                               static_cast<const float*>(L->vals), L->n, w.rewritten, Lp->rowptr,
                               a.colidx_out, static_cast<float*>(a.vals_out),
                               static_cast<const float*>(d_B), ldb, static_cast<float*>(d_Bp),
                               ldbp, k);
        RWT_LAUNCHED();
    }
    if (L->dt == RWT_F64) RWT_TRY(launch_rows<double>(a, true, s));
    else RWT_TRY(launch_rows<float>(a, true, s));
    return RWT_OK;
}
