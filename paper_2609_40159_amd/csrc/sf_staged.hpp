// Sync-free row block with helper waves (the default block body of the
// single-matrix solve).
//
// The plain block body (sf_block) spends most of each level step waiting
// for the one global load that brings in a dependency from an earlier
// block, although that value was usually published steps before.  Here the
// workgroup's waves split the work:
//   compute waves (the first 128 lanes) solve the rows of each step from
//     LDS only: x of rows in the block, and a staged copy of everything a
//     row needs (its descriptor, its lanes' first entries, and the x values
//     of those entries when they lie outside the block);
//   helper waves (the other lanes) run a three-stage prefetch pipeline one
//     to three steps ahead -- row descriptors, then column index and
//     diagonal, then the matrix value and the outside x value -- write the
//     stage for the next step into a ring of LDS slots, and publish the
//     previous step's x values to HBM.
// A staged outside value can still be the not-ready sentinel (its producer
// had not published it when the helper loaded it); the compute lane then
// waits for it in HBM.  Where that is the rule -- a block whose producers
// run only just ahead of it, as along the planes of a 3D grid -- the
// helper's load only lengthens its own step, which the compute waves wait
// for; with stage_x off the helper stages the sentinel instead and the
// compute lane always loads the value itself.  The plan times both.  Rows of a step beyond the staged ones, and each
// row's entries beyond its lanes' first, use direct loads as in sf_block.
#pragma once

#include "sf_block.hpp"

namespace rwt {

constexpr int SF_COMPUTE_LANES = 128;   // waves 0 and 1 of a 256-lane workgroup
constexpr int SF_STAGE_SLOTS = 3;

template <typename T>
struct SfRow {
    int32_t i, pb, pe, pad;
    T diag;
};
template <typename T, int KT>
struct SfLane {
    int32_t j, pad;
    T v;
    T x[KT];
};
// helper ring entry: first-entry column, value position and row diagonal
// (the diagonal kept as double: one layout for both value types)
struct SfEnt2 {
    int32_t j, m;
    double diag;
};

// LDS of the stage ring for G lanes per row
template <typename T, int KT>
__host__ __device__ constexpr int sf_slot_bytes_t(int G) {
    return (int)(((SF_COMPUTE_LANES / G) * sizeof(SfRow<T>) +
                  SF_COMPUTE_LANES * sizeof(SfLane<T, KT>) + 15) & ~size_t(15));
}
// stage slots plus the helper's descriptor ring (3 x 128 int4) and entry
// ring (2 x 128 SfEnt2)
inline int sf_stage_bytes(int G, int KT, int s) {
    const int slot = s == 8 ? (KT == 1 ? sf_slot_bytes_t<double, 1>(G) : sf_slot_bytes_t<double, 4>(G))
                            : (KT == 1 ? sf_slot_bytes_t<float, 1>(G) : sf_slot_bytes_t<float, 4>(G));
    return SF_STAGE_SLOTS * slot + 3 * SF_COMPUTE_LANES * 16 + 2 * SF_COMPUTE_LANES * 16;
}
// offset of the stage ring: after the x area and the step starts
__host__ __device__ inline int sf_stage_offset(int rows, int k, int s) {
    return sf_x_bytes(rows, k, s) + (((rows + 1) * 4 + 15) & ~15);
}

template <typename T, bool TRANS, int KT>
__device__ __forceinline__ void sf_block_staged(const SfBlockArgs& b, unsigned char* s_raw) {
    const int k = b.k;   // columns of this chain, 1..KT
    const int32_t r0 = b.r0, r1 = b.r1, sb = b.sb, ns = b.ns;
    constexpr int S = (int)sizeof(T);
    T* xs = reinterpret_cast<T*>(s_raw);
    int32_t* sp = reinterpret_cast<int32_t*>(s_raw + sf_x_bytes(b.lds_rows, k, S));
    unsigned char* stage = s_raw + sf_stage_offset(b.lds_rows, k, S);
    const T* vals = static_cast<const T*>(b.vals);
    const T* Bg = static_cast<const T*>(b.B);
    T* X = static_cast<T*>(b.X);
    const int32_t* idx = TRANS ? b.crow : b.colidx;
    const int G = b.lanes;
    const int SR = SF_COMPUTE_LANES / G;        // staged rows per step
    const int slot_bytes = sf_slot_bytes_t<T, KT>(G);
    const bool helper = threadIdx.x >= SF_COMPUTE_LANES;
    const int cl = helper ? (int)threadIdx.x - SF_COMPUTE_LANES : (int)threadIdx.x;
    const int r = cl / G;                        // row of the step this lane stages / solves
    const int gl = cl & (G - 1);
    int32_t* err = b.err;
    auto rows_of = [&](int slot) {
        return reinterpret_cast<SfRow<T>*>(stage + slot * slot_bytes);
    };
    auto lanes_of = [&](int slot) {
        return reinterpret_cast<SfLane<T, KT>*>(stage + slot * slot_bytes + SR * sizeof(SfRow<T>));
    };
    auto is_local = [&](int32_t j) { return TRANS ? (j < r1) : (j >= r0); };
    auto step_beg = [&](int u) { return sp[TRANS ? ns - 1 - u : u]; };
    auto step_cnt = [&](int u) {
        const int st = TRANS ? ns - 1 - u : u;
        return sp[st + 1] - sp[st];
    };

    for (int32_t u = threadIdx.x; u <= ns; u += blockDim.x) sp[u] = b.step_pos[sb + u] - r0;
    {
        const int32_t nr = r1 - r0;
        for (int32_t e = threadIdx.x; e < nr * k; e += blockDim.x) {
            const int32_t q = e / nr, i = e - q * nr;
            xs[i * k + q] = Bg[r0 + i + (int64_t)q * b.ldb];
        }
    }
    __syncthreads();

    if (helper) {
        // Three-stage prefetch through per-lane LDS rings, one step per
        // stage: descriptors of step u+4, entries (column, value position,
        // diagonal) of step u+3 and outside x values of step u+2 are issued
        // in step u and consumed in step u+1, after a whole step in flight.
        // Every load is issued unconditionally (clamped to a valid element
        // when idle) so the compiler's in-order wait counts stay exact and
        // the loads of one step never wait for the next step's.
        int4* dring = reinterpret_cast<int4*>(stage + SF_STAGE_SLOTS * slot_bytes);   // [3][128]
        SfEnt2* ering = reinterpret_cast<SfEnt2*>(dring + 3 * SF_COMPUTE_LANES);   // [2][128]
        auto desc_load = [&](int u) {   // row r's descriptor of step u, or x = -1
            const int uc = u < ns ? u : ns - 1;
            const bool act = u < ns && r < SR && r < step_cnt(uc);
            const int4 v = b.desc[r0 + (act ? step_beg(uc) + r : 0)];
            return act ? v : make_int4(-1, 0, 0, 0);
        };
        struct EntL {
            int32_t j, m;
            T diag;
        };
        auto ent_load = [&](const int4& d) {   // this lane's first entry of a row
            const int32_t p = d.y + gl;
            const bool ok = d.x >= 0 && p < d.z;
            const int32_t pc = ok ? p : 0;
            const int32_t j = idx[pc];
            const int32_t m = TRANS ? b.cmap[pc] : pc;
            const T dg = vals[d.x >= 0 ? d.w : 0];
            return EntL{ok ? j : -1, m, dg};
        };
        struct XL {
            T v;
            T x[KT];
        };
        const bool stage_x = b.stage_x != 0;
        auto x_load = [&](const SfEnt2& e) {   // value and (staged) outside x of that entry
            XL o;
            const bool ok = e.j >= 0;
            o.v = vals[ok ? e.m : 0];
            if (stage_x) {
                const bool far = ok && !is_local(e.j);
                const int32_t jc = far ? e.j : 0;
#pragma unroll
                for (int q = 0; q < KT; ++q) {
                    const int qc = (KT == 1 || q < k) ? q : 0;
                    const T xv = ld_relaxed(&X[jc + (int64_t)qc * b.ldx]);
                    o.x[q] = far ? xv : T(0);
                }
            } else {
#pragma unroll
                for (int q = 0; q < KT; ++q) o.x[q] = sentinel_value<T>();   // loaded when used
            }
            return o;
        };
        auto fill_slot = [&](int u, const XL& xl) {   // stage of step u, for the compute waves
            const int4 d = dring[(u % 3) * SF_COMPUTE_LANES + cl];
            const SfEnt2 e = ering[(u % 2) * SF_COMPUTE_LANES + cl];
            SfLane<T, KT> ln;
            ln.j = d.x >= 0 ? e.j : -1;
            ln.pad = 0;
            ln.v = xl.v;
#pragma unroll
            for (int q = 0; q < KT; ++q) ln.x[q] = xl.x[q];
            const int slot = u % SF_STAGE_SLOTS;
            lanes_of(slot)[cl] = ln;
            if (gl == 0) rows_of(slot)[r] = SfRow<T>{d.x, d.y, d.z, 0, (T)e.diag};
        };
        auto put_ent = [&](int u, const EntL& el) {
            ering[(u % 2) * SF_COMPUTE_LANES + cl] = SfEnt2{el.j, el.m, (double)el.diag};
        };
        // prime: rings hold descriptors of steps 0..2 and entries of 0..1,
        // slot 0 is complete, and the loads of the next stages are in flight
        for (int u = 0; u < 3; ++u) dring[u * SF_COMPUTE_LANES + cl] = desc_load(u);
        for (int u = 0; u < 2; ++u) put_ent(u, ent_load(dring[u * SF_COMPUTE_LANES + cl]));
        fill_slot(0, x_load(ering[cl]));
        int4 dv = desc_load(3);
        EntL ev = ent_load(dring[2 * SF_COMPUTE_LANES + cl]);
        XL xv = x_load(ering[SF_COMPUTE_LANES + cl]);
        lds_barrier();
        for (int32_t u = 0; u < ns; ++u) {
            // consume what was issued one step ago
            dring[((u + 3) % 3) * SF_COMPUTE_LANES + cl] = dv;
            put_ent(u + 2, ev);
            fill_slot(u + 1, xv);
            // issue the next stages (the rings just written feed them)
            dv = desc_load(u + 4);
            ev = ent_load(dring[((u + 3) % 3) * SF_COMPUTE_LANES + cl]);
            xv = x_load(ering[((u + 2) % 2) * SF_COMPUTE_LANES + cl]);
            lds_barrier();
        }
    } else {
        lds_barrier();
        for (int32_t u = 0; u < ns; ++u) {
            const int slot = u % SF_STAGE_SLOTS;
            const int32_t cnt = step_cnt(u);
            const bool act = r < cnt && r < SR;
            SfRow<T> row{0, 0, 0, 0, T(1)};
            T acc[KT];
#pragma unroll
            for (int q = 0; q < KT; ++q) acc[q] = T(0);
            if (act) {
                row = rows_of(slot)[r];
                const SfLane<T, KT> ln = lanes_of(slot)[cl];
                if (ln.j >= 0) {
                    const bool local = is_local(ln.j);
#pragma unroll
                    for (int q = 0; q < KT; ++q) {
                        if (KT == 1 || q < k) {
                            T xj = local ? xs[(ln.j - r0) * k + q] : ln.x[q];
                            if (!local && is_sentinel(xj))
                                xj = wait_value(&X[ln.j + (int64_t)q * b.ldx], err, b.ticks);
                            acc[q] = ln.v * xj;
                        }
                    }
                }
            }
            // entries beyond the lanes' first: direct loads
            for (int32_t p = row.pb + gl + G; act && p < row.pe; p += G) {
                const int32_t j = idx[p];
                const T v = TRANS ? vals[b.cmap[p]] : vals[p];
                const bool local = is_local(j);
#pragma unroll
                for (int q = 0; q < KT; ++q)
                    if (KT == 1 || q < k)
                        acc[q] += v * (local ? xs[(j - r0) * k + q]
                                             : wait_value(&X[j + (int64_t)q * b.ldx], err, b.ticks));
            }
#pragma unroll
            for (int q = 0; q < KT; ++q) acc[q] = group_sum(acc[q], G);
            if (act && gl == 0) {
#pragma unroll
                for (int q = 0; q < KT; ++q)
                    if (KT == 1 || q < k) {
                        T* xi = &xs[(row.i - r0) * k + q];
                        const T xv = (*xi - acc[q]) / row.diag;
                        *xi = xv;
                        if (row.i != b.hold_row) st_relaxed(&X[row.i + (int64_t)q * b.ldx], xv);
                    }
            }
            // rows of this step beyond the staged ones: direct loads, and
            // published here
            const int32_t beg = step_beg(u);
            for (int32_t base = SR; base < cnt; base += SR) {
                const int32_t rr = base + r;
                const bool a2 = rr < cnt;
                int32_t i = r0, pb = 0, pe = 0, dpos = 0;
                if (a2) {
                    const int4 v = b.desc[r0 + beg + rr];
                    i = v.x;
                    pb = v.y;
                    pe = v.z;
                    dpos = v.w;
                }
                T a2c[KT];
#pragma unroll
                for (int q = 0; q < KT; ++q) a2c[q] = T(0);
                for (int32_t p = pb + gl; a2 && p < pe; p += G) {
                    const int32_t j = idx[p];
                    const T v = TRANS ? vals[b.cmap[p]] : vals[p];
                    const bool local = is_local(j);
#pragma unroll
                    for (int q = 0; q < KT; ++q)
                        if (KT == 1 || q < k)
                            a2c[q] += v * (local ? xs[(j - r0) * k + q]
                                                 : wait_value(&X[j + (int64_t)q * b.ldx], err, b.ticks));
                }
#pragma unroll
                for (int q = 0; q < KT; ++q) a2c[q] = group_sum(a2c[q], G);
                if (a2 && gl == 0) {
                    const T dg = vals[dpos];
#pragma unroll
                    for (int q = 0; q < KT; ++q)
                        if (KT == 1 || q < k) {
                            T* xi = &xs[(i - r0) * k + q];
                            const T xv = (*xi - a2c[q]) / dg;
                            *xi = xv;
                            if (i != b.hold_row) st_relaxed(&X[i + (int64_t)q * b.ldx], xv);
                        }
                }
            }
            lds_barrier();
        }
    }
    __syncthreads();
}

}  // namespace rwt
