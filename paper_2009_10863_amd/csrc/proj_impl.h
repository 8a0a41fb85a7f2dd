// Kernels of Fischer's projection guess (§2).
//
// Two ways of bounding the history (template flag VF_QR):
//   classic (Algorithm 1): when the history is full, restart from the new
//     solution;
//   rolling QR (Algorithm 2): when the history is full, drop the oldest
//     solution: delete the first column of R (raw solutions = X R), return
//     R to triangular form with Givens rotations of neighbouring rows and
//     rotate the columns of X and B alongside, then add the new solution.
// Two inner products (template flag VF_L2):
//   A (default): X^T A X = I, B = A X, guess x0 = X (X^T b);
//   l2 (the paper's own form): B^T B = I, guess x0 = X (B^T b).
//
// Columns are stored unnormalised with a per-column FP64 scale kept in the
// device state (true column j = scale[j] * stored column j), so that the
// normalisation of a new column, which needs its norm, does not cost an
// extra pass over the data.  Every decision (restart, drop, accept / reject)
// is taken on the device.
//
// The rolling drop costs no pass of its own.  The rotated basis is
// X' = X W^T (first d-1 columns), W the product of the rotations, so inner
// products with X' are W times inner products with X: the apply and reorth
// kernels work on the old columns and the finishing kernels rotate the
// small coefficient vectors.  The Gram-Schmidt write kernel then reads every
// old column once, writes the rotated columns back in place and the new
// orthogonalised pair into the last slot.
//
// Each reduction is split in two launches: a streaming kernel that writes
// one row of partial sums per workgroup, and a one-workgroup finishing
// kernel (proj_fin) that sums the rows in a fixed order and updates the
// state.  Nothing synchronises across workgroups inside a kernel, so no
// device-wide cache write-back or invalidation is needed mid-kernel.
//
// Streaming kernels and algorithmic bytes per unknown (s = stored element
// size, d the current number of columns, C = X for the A inner product and
// C = B for l2):
//   proj_dots      P_j = C_j^T b                      reads d s + 8
//   proj_combine   x0 = sum_j gamma_j X_j             reads d s, writes 8
//   proj_apply     w = A x (or the caller's A x),     reads 8 (+8), d s; writes 8
//                  c1 = C^T w, nu0^2 = x^T w (w^T w);
//                  restart: X_1 <- x, B_1 <- w        reads 8 (+8); writes 2 s
//   proj_reorth    c2 = C^T (w - B c1)                reads 2 d s + 8 (l2: d s + 8)
//   proj_gs_write  x'' = x - X c, w'' = w - B c,      reads 2 d s + 16; writes 2 s
//                  nu^2 = x''^T w'' (w''^T w''), store in slot d
//                  rolling drop (d = M): also rotates  reads 2 M s + 16; writes 2 M s
#pragma once

#include "common.h"
#include "launch.h"
#include "march.h"

namespace lg {

enum { VF_QR = 1, VF_L2 = 2 };

struct ProjArgs {
    const void *X;
    const void *B;
    void *Xw;                // writable views of the same arrays
    void *Bw;
    double *w;
    double *part;
    ProjState *st;
    int64_t N, ld;
    int M;
};

template <int DT>
__device__ __forceinline__ const void *colp(const void *base, int64_t ld, int j) {
    return reinterpret_cast<const typename Elem<DT>::T *>(base) + (int64_t)j * ld;
}
template <int DT>
__device__ __forceinline__ void *colw(void *base, int64_t ld, int j) {
    return reinterpret_cast<typename Elem<DT>::T *>(base) + (int64_t)j * ld;
}

// The update starts a new history: empty, or (classic) full.  With the
// rolling variant and M = 1, dropping the only column and adding the new
// one is the same as a restart.
template <int VF>
__device__ __forceinline__ bool proj_restart(int d, int M) {
    if constexpr ((VF & VF_QR) != 0) return d == 0 || M == 1;
    else return d == 0 || d >= M;
}
// largest number of columns the Gram-Schmidt kernels see
template <int VF>
constexpr int gs_max() {
    return (VF & VF_QR) ? GUESS_MAX_M : GUESS_MAX_M - 1;
}
// the columns inner products are taken with
template <int VF>
__device__ __forceinline__ const void *dot_cols(const ProjArgs &a) {
    return (VF & VF_L2) ? a.B : a.X;
}

// FP16 storage has a narrow range, so a new FP16 pair (x, b) is stored
// multiplied by 2^e with max(|x|, |b|) 2^e in [2^14, 2^15): the magnitudes of
// the raw pair at a restart, of the pair after the first Gram-Schmidt pass
// otherwise (reduced alongside that pass; the second pass changes them only
// by rounding).  Wider formats store the pair as it is (e = 0).  Either way
// the column's FP64 scale is 1 / (nu 2^e).
template <int DT>
constexpr bool scaled_store() {
    return DT == GUESS_F16;
}
__device__ __forceinline__ double absmax2(double a, double b) { return nanmax(fabs(a), fabs(b)); }

// ------------------------------------------------------------------ form
template <int DT, int VF>
LG_REDUCE_KERNEL void proj_dots_kernel(ProjArgs a, const double *__restrict__ b) {
    __shared__ double lds[kLdsDoubles];
    const int d = a.st->d;
    const void *C = dot_cols<VF>(a);
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    dispatch_d<1, GUESS_MAX_M>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double acc[D];
#pragma unroll
        for (int j = 0; j < D; ++j) acc[j] = 0.0;
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
            const V4 bv = load4<GUESS_F64>(b, c);
            V4 xv[D];
#pragma unroll
            for (int j = 0; j < D; ++j) xv[j] = load4<DT>(colp<DT>(C, a.ld, j), c);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(xv[j].v[e], bv.v[e], acc[j]);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
#pragma unroll
            for (int j = 0; j < D; ++j)
                acc[j] = __builtin_fma(load1<DT>(colp<DT>(C, a.ld, j), i), b[i], acc[j]);
        }
        block_partials<D>(acc, a.part, lds);
    });
}

template <int DT>
__global__ __launch_bounds__(kBlock) void proj_combine_kernel(ProjArgs a, double *__restrict__ x0) {
    const int d = a.st->d;
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    dispatch_d<0, GUESS_MAX_M>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double g[D > 0 ? D : 1];
#pragma unroll
        for (int j = 0; j < D; ++j) g[j] = a.st->gamma[j];
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
            V4 acc{{0.0, 0.0, 0.0, 0.0}};
            if constexpr (D > 0) {
                V4 xv[D];
#pragma unroll
                for (int j = 0; j < D; ++j) xv[j] = load4<DT>(colp<DT>(a.X, a.ld, j), c);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc.v[e] = g[0] * xv[0].v[e];
#pragma unroll
                for (int j = 1; j < D; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc.v[e] = __builtin_fma(g[j], xv[j].v[e], acc.v[e]);
            }
            store4<GUESS_F64>(x0, c, acc);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) acc = __builtin_fma(g[j], load1<DT>(colp<DT>(a.X, a.ld, j), i), acc);
            x0[i] = acc;
        }
    });
}

// ------------------------------------------------------------------ update
template <int DT, int VF, bool VAR, bool HAVE_AX, bool AL>
LG_REDUCE_KERNEL void proj_apply_kernel(ProjArgs a, Grid g, const double *__restrict__ x,
                                        const double *__restrict__ Ax) {
    __shared__ double lds[kLdsDoubles];
    constexpr bool L2 = (VF & VF_L2) != 0;
    const int d = a.st->d;
    const int64_t nc = nchunks(a.N);
    const ChunkRange cr = xcd_range(nc);
    const int rem = tail_count(a.N);
    // x and A x for one chunk (the stencil also returns its centre values)
    auto xw4 = [&](int64_t c, V4 &xv) -> V4 {
        if constexpr (HAVE_AX) {
            xv = load4<GUESS_F64>(x, c);
            return load4<GUESS_F64>(Ax, c);
        } else {
            R4 uc;
            const R4 r = apply4g<VAR, AL>(x, g, c, uc);
            xv = V4{{uc.v[0], uc.v[1], uc.v[2], uc.v[3]}};
            return V4{{r.v[0], r.v[1], r.v[2], r.v[3]}};
        }
    };
    auto xw1 = [&](int64_t i) -> double {
        if constexpr (HAVE_AX) return Ax[i];
        else return apply_pt<VAR>(VecU{x}, g, i);
    };
    if (proj_restart<VF>(d, a.M)) {
        // restart: slot 1 <- x, B slot 1 <- A x; partial nu0^2 = x^T A x (l2: |A x|^2).
        // FP16: the exponent of the stored pair needs max(|x|, |A x|) first, so this pass
        // writes w = A x and reduces the max; the Gram-Schmidt write kernel stores the pair.
        constexpr bool SC = scaled_store<DT>();
        double acc[SC ? 2 : 1];
#pragma unroll
        for (int j = 0; j < (SC ? 2 : 1); ++j) acc[j] = 0.0;
        for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
            V4 xv;
            const V4 wv = xw4(c, xv);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[0] = __builtin_fma(L2 ? wv.v[e] : xv.v[e], wv.v[e], acc[0]);
            if constexpr (SC) {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[SC ? 1 : 0] = nanmax(acc[SC ? 1 : 0], absmax2(xv.v[e], wv.v[e]));
                if constexpr (!HAVE_AX) store4<GUESS_F64>(a.w, c, wv);
            } else {
                store4<DT>(a.Xw, c, xv);
                store4<DT>(a.Bw, c, wv);
            }
        }
        if (blockIdx.x == 0 && threadIdx.x < rem) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            const double wv = xw1(i);
            acc[0] = __builtin_fma(L2 ? wv : x[i], wv, acc[0]);
            if constexpr (SC) {
                acc[SC ? 1 : 0] = nanmax(acc[SC ? 1 : 0], absmax2(x[i], wv));
                if constexpr (!HAVE_AX) a.w[i] = wv;
            } else {
                store1<DT>(a.Xw, i, x[i]);
                store1<DT>(a.Bw, i, wv);
            }
        }
        block_partials<SC ? 2 : 1, 1>(acc, a.part, lds);
        return;
    }
    const void *C = dot_cols<VF>(a);
    dispatch_d<1, gs_max<VF>()>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int ND = D + 1;
        double acc[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j) acc[j] = 0.0;
        for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
            V4 xc[D];
#pragma unroll
            for (int j = 0; j < D; ++j) xc[j] = load4<DT>(colp<DT>(C, a.ld, j), c);
            V4 xv;
            const V4 wv = xw4(c, xv);
            if constexpr (!HAVE_AX) store4<GUESS_F64>(a.w, c, wv);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[D] = __builtin_fma(L2 ? wv.v[e] : xv.v[e], wv.v[e], acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(xc[j].v[e], wv.v[e], acc[j]);
        }
        if (blockIdx.x == 0 && threadIdx.x < rem) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            const double wv = xw1(i);
            if constexpr (!HAVE_AX) a.w[i] = wv;
            acc[D] = __builtin_fma(L2 ? wv : x[i], wv, acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j) acc[j] = __builtin_fma(load1<DT>(colp<DT>(C, a.ld, j), i), wv, acc[j]);
        }
        block_partials<ND>(acc, a.part, lds);
    });
}

// proj_apply in the traversal of march.h (constant coefficient, library
// operator, grids it applies to): same per-chunk work, bit-identical w.
template <int DT, int VF, bool VAR>
LG_REDUCE_KERNEL void proj_apply_march_kernel(ProjArgs a, Grid g, March m, const double *__restrict__ x) {
    __shared__ double lds[kLdsDoubles];
    constexpr bool L2 = (VF & VF_L2) != 0;
    const int d = a.st->d;
    if (proj_restart<VF>(d, a.M)) {
        constexpr bool SC = scaled_store<DT>();
        double acc[SC ? 2 : 1];
#pragma unroll
        for (int j = 0; j < (SC ? 2 : 1); ++j) acc[j] = 0.0;
        march_sweep<VAR>(g, m, VecU{x}, [&](int64_t c, int64_t, const R2 &pa, const R2 &pb, const R4 &au) {
            const V4 xv{{pa.v[0], pa.v[1], pb.v[0], pb.v[1]}};
            const V4 wv{{au.v[0], au.v[1], au.v[2], au.v[3]}};
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[0] = __builtin_fma(L2 ? wv.v[e] : xv.v[e], wv.v[e], acc[0]);
            if constexpr (SC) {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[SC ? 1 : 0] = nanmax(acc[SC ? 1 : 0], absmax2(xv.v[e], wv.v[e]));
                store4<GUESS_F64>(a.w, c, wv);
            } else {
                store4<DT>(a.Xw, c, xv);
                store4<DT>(a.Bw, c, wv);
            }
        });
        block_partials<SC ? 2 : 1, 1>(acc, a.part, lds);
        return;
    }
    const void *C = dot_cols<VF>(a);
    dispatch_d<1, gs_max<VF>()>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int ND = D + 1;
        double acc[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j) acc[j] = 0.0;
        // the stored columns of the chunk, fetched one plane ahead
        struct Cols {
            V4 v[D];
        };
        auto pf = [&](int64_t c) {
            Cols cl;
#pragma unroll
            for (int j = 0; j < D; ++j) cl.v[j] = load4<DT>(colp<DT>(C, a.ld, j), c);
            return cl;
        };
        march_sweep_pf<VAR>(g, m, VecU{x}, pf, [&](int64_t c, int64_t, const R2 &pa, const R2 &pb, const R4 &au,
                                                    const Cols &cl) {
            const V4 *xc = cl.v;
            const V4 xv{{pa.v[0], pa.v[1], pb.v[0], pb.v[1]}};
            const V4 wv{{au.v[0], au.v[1], au.v[2], au.v[3]}};
            store4<GUESS_F64>(a.w, c, wv);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[D] = __builtin_fma(L2 ? wv.v[e] : xv.v[e], wv.v[e], acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(xc[j].v[e], wv.v[e], acc[j]);
        });
        block_partials<ND>(acc, a.part, lds);
    });
}

template <int DT, int VF>
LG_REDUCE_KERNEL void proj_reorth_kernel(ProjArgs a, const double *__restrict__ x, const double *__restrict__ w) {
    __shared__ double lds[kLdsDoubles];
    constexpr bool L2 = (VF & VF_L2) != 0;
    constexpr bool EST = scaled_store<DT>();   // also reduce max(|x'|, |w'|), x' = x - X c1
    constexpr bool NEEDX = !L2 || EST;
    if (a.st->mode != 0) return;
    const int d = a.st->d;
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    dispatch_d<1, gs_max<VF>()>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int ND = EST ? D + 1 : D;
        double cs[D], acc[ND];
#pragma unroll
        for (int j = 0; j < D; ++j) cs[j] = a.st->cs[j];
#pragma unroll
        for (int j = 0; j < ND; ++j) acc[j] = 0.0;
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
            V4 bc[D], xc[NEEDX ? D : 1];
#pragma unroll
            for (int j = 0; j < D; ++j) bc[j] = load4<DT>(colp<DT>(a.B, a.ld, j), c);
            if constexpr (NEEDX) {
#pragma unroll
                for (int j = 0; j < D; ++j) xc[j] = load4<DT>(colp<DT>(a.X, a.ld, j), c);
            }
            V4 wv = load4<GUESS_F64>(w, c);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) wv.v[e] = __builtin_fma(-cs[j], bc[j].v[e], wv.v[e]);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[j] = __builtin_fma(L2 ? bc[j].v[e] : xc[NEEDX ? j : 0].v[e], wv.v[e], acc[j]);
            if constexpr (EST) {
                V4 xv = load4<GUESS_F64>(x, c);
#pragma unroll
                for (int j = 0; j < D; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) xv.v[e] = __builtin_fma(-cs[j], xc[NEEDX ? j : 0].v[e], xv.v[e]);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[ND - 1] = nanmax(acc[ND - 1], absmax2(xv.v[e], wv.v[e]));
            }
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            double wv = w[i], xv = x[i];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                wv = __builtin_fma(-cs[j], load1<DT>(colp<DT>(a.B, a.ld, j), i), wv);
                if constexpr (EST) xv = __builtin_fma(-cs[j], load1<DT>(colp<DT>(a.X, a.ld, j), i), xv);
            }
#pragma unroll
            for (int j = 0; j < D; ++j)
                acc[j] = __builtin_fma(load1<DT>(colp<DT>(L2 ? a.B : a.X, a.ld, j), i), wv, acc[j]);
            if constexpr (EST) acc[ND - 1] = nanmax(acc[ND - 1], absmax2(xv, wv));
        }
        block_partials<ND, D>(acc, a.part, lds);
    });
}

// Rolling drop, one array (X or B) of one chunk: subtract the projection
// from v, rotate the D old columns in place (slot i <- rotated column i,
// i < D-1) and store v in slot D-1.  rot[i] = {a, b, e, f} in stored units:
// new_i = a t_i + b S_{i+1}, t_{i+1} = e t_i + f S_{i+1}, t_0 = S_0.  With MX
// the magnitudes of the values written into slot i are max-reduced into mx[i]
// (FP16: the rotated pairs' largest stored magnitudes).
template <int DT, int D, bool MX>
__device__ __forceinline__ void rotate_chunk(const void *S, void *Sw, int64_t ld, int64_t c, const double (&cs)[D],
                                             const double (&rot)[D - 1][4], double pw, V4 &v, double (&mx)[D]) {
    V4 col[D];
#pragma unroll
    for (int j = 0; j < D; ++j) col[j] = load4<DT>(colp<DT>(S, ld, j), c);
#pragma unroll
    for (int j = 0; j < D; ++j)
#pragma unroll
        for (int e = 0; e < 4; ++e) v.v[e] = __builtin_fma(-cs[j], col[j].v[e], v.v[e]);
    V4 t = col[0];
#pragma unroll
    for (int i = 0; i < D - 1; ++i) {
        V4 nw;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            nw.v[e] = __builtin_fma(rot[i][1], col[i + 1].v[e], rot[i][0] * t.v[e]);
            t.v[e] = __builtin_fma(rot[i][3], col[i + 1].v[e], rot[i][2] * t.v[e]);
            if constexpr (MX) mx[i] = nanmax(mx[i], fabs(nw.v[e]));
        }
        store4<DT>(colw<DT>(Sw, ld, i), c, nw);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        v.v[e] *= pw;
        if constexpr (MX) mx[D - 1] = nanmax(mx[D - 1], fabs(v.v[e]));
    }
    store4<DT>(colw<DT>(Sw, ld, D - 1), c, v);
}

template <int DT, int D, bool MX>
__device__ __forceinline__ double rotate_one(const void *S, void *Sw, int64_t ld, int64_t i, const double (&cs)[D],
                                             const double (&rot)[D - 1][4], double pw, double v, double (&mx)[D]) {
    double col[D];
#pragma unroll
    for (int j = 0; j < D; ++j) col[j] = load1<DT>(colp<DT>(S, ld, j), i);
#pragma unroll
    for (int j = 0; j < D; ++j) v = __builtin_fma(-cs[j], col[j], v);
    double t = col[0];
#pragma unroll
    for (int q = 0; q < D - 1; ++q) {
        const double nw = __builtin_fma(rot[q][1], col[q + 1], rot[q][0] * t);
        t = __builtin_fma(rot[q][3], col[q + 1], rot[q][2] * t);
        if constexpr (MX) mx[q] = nanmax(mx[q], fabs(nw));
        store1<DT>(colw<DT>(Sw, ld, q), i, nw);
    }
    v *= pw;
    if constexpr (MX) mx[D - 1] = nanmax(mx[D - 1], fabs(v));
    store1<DT>(colw<DT>(Sw, ld, D - 1), i, v);
    return v;
}

template <int DT, int VF>
LG_REDUCE_KERNEL void proj_gs_write_kernel(ProjArgs a, const double *__restrict__ x,
                                           const double *__restrict__ w) {
    __shared__ double lds[kLdsDoubles];
    constexpr bool L2 = (VF & VF_L2) != 0;
    constexpr bool SC = scaled_store<DT>();
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    if (a.st->mode != 0) {
        // FP16 restart: store the raw pair (x, A x) times the exponent found by the apply pass
        if constexpr (SC) {
            if (a.st->mode != 1 || a.st->d != 1) return;
            const double pw = a.st->pow2;
            for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
                V4 xv = load4<GUESS_F64>(x, c);
                V4 wv = load4<GUESS_F64>(w, c);
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xv.v[e] *= pw;
                    wv.v[e] *= pw;
                }
                store4<DT>(a.Xw, c, xv);
                store4<DT>(a.Bw, c, wv);
            }
            if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
                const int64_t i = tail_start(a.N) + threadIdx.x;
                store1<DT>(a.Xw, i, x[i] * pw);
                store1<DT>(a.Bw, i, w[i] * pw);
            }
        }
        return;
    }
    const int d = a.st->d;
    if constexpr ((VF & VF_QR) != 0) {
        if (d == a.M) {
            dispatch_d<2, GUESS_MAX_M>(d, [&](auto Dc) {
                constexpr int D = decltype(Dc)::value;
                double cs[D], rot[D - 1][4];
#pragma unroll
                for (int j = 0; j < D; ++j) cs[j] = a.st->cs[j];
#pragma unroll
                for (int i = 0; i < D - 1; ++i)
#pragma unroll
                    for (int q = 0; q < 4; ++q) rot[i][q] = a.st->rot[i][q];
                const double pw = SC ? a.st->pow2 : 1.0;
                // acc[0]: nu^2 of the new pair; FP16 also the largest stored magnitude of
                // the new pair (acc[1]) and of rotated pair i (acc[2 + i])
                double acc[SC ? D + 1 : 1], mx[D];
#pragma unroll
                for (int j = 0; j < (SC ? D + 1 : 1); ++j) acc[j] = 0.0;
#pragma unroll
                for (int j = 0; j < D; ++j) mx[j] = 0.0;
                for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
                    V4 xv = load4<GUESS_F64>(x, c);
                    V4 wv = load4<GUESS_F64>(w, c);
                    rotate_chunk<DT, D, SC>(a.X, a.Xw, a.ld, c, cs, rot, pw, xv, mx);
                    rotate_chunk<DT, D, SC>(a.B, a.Bw, a.ld, c, cs, rot, pw, wv, mx);
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc[0] = __builtin_fma(L2 ? wv.v[e] : xv.v[e], wv.v[e], acc[0]);
                }
                if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
                    const int64_t i = tail_start(a.N) + threadIdx.x;
                    const double xv = rotate_one<DT, D, SC>(a.X, a.Xw, a.ld, i, cs, rot, pw, x[i], mx);
                    const double wv = rotate_one<DT, D, SC>(a.B, a.Bw, a.ld, i, cs, rot, pw, w[i], mx);
                    acc[0] = __builtin_fma(L2 ? wv : xv, wv, acc[0]);
                }
                if constexpr (SC) {
                    acc[SC ? 1 : 0] = mx[D - 1];
#pragma unroll
                    for (int i = 0; i < D - 1; ++i) acc[SC ? 2 + i : 0] = mx[i];
                }
                block_partials<SC ? D + 1 : 1, 1>(acc, a.part, lds);
            });
            return;
        }
    }
    dispatch_d<1, GUESS_MAX_M - 1>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double cs[D];
#pragma unroll
        for (int j = 0; j < D; ++j) cs[j] = a.st->cs[j];
        void *Xd = colw<DT>(a.Xw, a.ld, D);
        void *Bd = colw<DT>(a.Bw, a.ld, D);
        const double pw = SC ? a.st->pow2 : 1.0;
        // acc[0]: nu^2 of the new pair; FP16 also its largest stored magnitude (acc[1])
        double acc[SC ? 2 : 1];
#pragma unroll
        for (int j = 0; j < (SC ? 2 : 1); ++j) acc[j] = 0.0;
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
            V4 xc[D], bc[D];
#pragma unroll
            for (int j = 0; j < D; ++j) xc[j] = load4<DT>(colp<DT>(a.X, a.ld, j), c);
#pragma unroll
            for (int j = 0; j < D; ++j) bc[j] = load4<DT>(colp<DT>(a.B, a.ld, j), c);
            V4 xv = load4<GUESS_F64>(x, c);
            V4 wv = load4<GUESS_F64>(w, c);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    xv.v[e] = __builtin_fma(-cs[j], xc[j].v[e], xv.v[e]);
                    wv.v[e] = __builtin_fma(-cs[j], bc[j].v[e], wv.v[e]);
                }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                xv.v[e] *= pw;
                wv.v[e] *= pw;
                acc[0] = __builtin_fma(L2 ? wv.v[e] : xv.v[e], wv.v[e], acc[0]);
                if constexpr (SC) acc[SC ? 1 : 0] = nanmax(acc[SC ? 1 : 0], absmax2(xv.v[e], wv.v[e]));
            }
            store4<DT>(Xd, c, xv);
            store4<DT>(Bd, c, wv);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            double xv = x[i], wv = w[i];
#pragma unroll
            for (int j = 0; j < D; ++j) {
                xv = __builtin_fma(-cs[j], load1<DT>(colp<DT>(a.X, a.ld, j), i), xv);
                wv = __builtin_fma(-cs[j], load1<DT>(colp<DT>(a.B, a.ld, j), i), wv);
            }
            xv *= pw;
            wv *= pw;
            acc[0] = __builtin_fma(L2 ? wv : xv, wv, acc[0]);
            if constexpr (SC) acc[SC ? 1 : 0] = nanmax(acc[SC ? 1 : 0], absmax2(xv, wv));
            store1<DT>(Xd, i, xv);
            store1<DT>(Bd, i, wv);
        }
        block_partials<SC ? 2 : 1, 1>(acc, a.part, lds);
    });
}

// ------------------------------------------------------------------ finishing kernels
// One workgroup: sum the nb partial rows of the preceding streaming kernel
// and take the step's decisions.
enum { FIN_DOTS = 0, FIN_APPLY = 1, FIN_REORTH = 2, FIN_GS = 3 };

// Coefficients in the rotated basis from inner products p with the old
// columns (true units): q = W p, keep q[0 .. D-2] (the last row of the
// rotated factor is dropped).
template <int D>
__device__ __forceinline__ void rot_forward(const double *gc, const double *gs, double (&q)[D]) {
#pragma unroll
    for (int i = 0; i < D - 1; ++i) {
        const double q0 = q[i], q1 = q[i + 1];
        q[i] = gc[i] * q0 + gs[i] * q1;
        q[i + 1] = -gs[i] * q0 + gc[i] * q1;
    }
}
// Old-basis coefficients of X' y: W^T [y; 0].
template <int D>
__device__ __forceinline__ void rot_backward(const double *gc, const double *gs, double (&y)[D]) {
    y[D - 1] = 0.0;
#pragma unroll
    for (int i = D - 2; i >= 0; --i) {
        const double y0 = y[i], y1 = y[i + 1];
        y[i] = gc[i] * y0 - gs[i] * y1;
        y[i + 1] = gs[i] * y0 + gc[i] * y1;
    }
}

// Rolling drop, first half (all threads of the workgroup take part): the
// Givens rotations that return R(:, 2:M) to triangular form, the rotated
// factor (written back to st->R, last row and column cleared), and the
// per-slot rotation coefficients in stored units for proj_gs_write.
// A rotated slot keeps its scale, except in FP16, where slot i gets the
// scale 2^-15 (|c_i| t_i + |s_i| mu_{i+1}) with t_0 = mu_0,
// t_{i+1} = |s_i| t_i + |c_i| mu_{i+1} (mu_j the largest true magnitude of
// stored pair j): a bound on the rotated pair's largest magnitude, so that
// no stored value exceeds 2^15.  The new scales take effect at the end of
// the update (proj_fin after proj_gs_write); until then the coefficients
// of the update refer to the old stored columns.
template <int DT>
__device__ __forceinline__ void qr_drop_plan(ProjState *st, int M) {
    __shared__ double H[GUESS_MAX_M][GUESS_MAX_M + 1];
    __shared__ double gcl[GUESS_MAX_M], gsl[GUESS_MAX_M];
    const int t = threadIdx.x;
    if (t < M * (M - 1)) {
        const int i = t / (M - 1), j = t % (M - 1);
        H[i][j] = st->R[i][j + 1];
    }
    __syncthreads();
    for (int i = 0; i < M - 1; ++i) {
        if (t == 0) {
            const double a = H[i][i], b = H[i + 1][i];
            const double r = hypot(a, b);
            const double sg = a >= 0.0 ? 1.0 : -1.0;
            const double c = fabs(a) / r, s = sg * b / r;
            gcl[i] = c;
            gsl[i] = s;
            st->gc[i] = c;
            st->gs[i] = s;
            H[i][i] = sg * r;
            H[i + 1][i] = 0.0;
        }
        __syncthreads();
        if (t > i && t < M - 1) {
            const double c = gcl[i], s = gsl[i];
            const double h0 = H[i][t], h1 = H[i + 1][t];
            H[i][t] = c * h0 + s * h1;
            H[i + 1][t] = -s * h0 + c * h1;
        }
        __syncthreads();
    }
    if (t < M * M) {
        const int i = t / M, j = t % M;
        st->R[i][j] = (i < M - 1 && j < M - 1 && j >= i) ? H[i][j] : 0.0;
    }
    __shared__ double nsc[GUESS_MAX_M];
    if (t == 0) {
        double tt = scaled_store<DT>() ? st->mu[0] : 0.0;
        for (int i = 0; i < M - 1; ++i) {
            if constexpr (scaled_store<DT>()) {
                const double ac = fabs(gcl[i]), as = fabs(gsl[i]), mn = st->mu[i + 1];
                nsc[i] = ldexp(ac * tt + as * mn, -15);
                tt = as * tt + ac * mn;
            } else {
                nsc[i] = st->scale[i];
            }
            st->nscale[i] = nsc[i];
        }
    }
    __syncthreads();
    if (t < M - 1) {
        const double c = gcl[t], s = gsl[t];
        const double si = st->scale[t], sn = st->scale[t + 1], sp = nsc[t];
        st->rot[t][0] = c * (si / sp);
        st->rot[t][1] = s * (sn / sp);
        st->rot[t][2] = -s * (si / sn);
        st->rot[t][3] = c;
    }
}

// End of an update that orthogonalised a new pair (slot d, or d - 1 after a
// rolling drop): nsq = nu^2 2^{2e} of the stored pair, mx its largest stored
// magnitude before rounding (FP16).  Accept iff nu > eps_rel nu0; the new
// column's scale is 1 / (nu 2^e) and column d of R holds its coefficients.
template <int DT>
__device__ __forceinline__ void gs_accept(ProjState *st, int d, bool drop, double nsq, double mx) {
    const int slot = drop ? d - 1 : d;     // the new pair's column
    const double pw = scaled_store<DT>() ? st->pow2 : 1.0;   // the pair was stored multiplied by pw
    const double nu = sqrt(nsq) / pw;      // NaN when rounding made it negative
    const bool fin = isfinite(nu);
    const bool ok = fin && nu > st->eps_rel * st->nu0;
    // new column of the factor: raw x = X c + nu x~
    if (ok && (int)threadIdx.x < slot) st->R[threadIdx.x][slot] = st->c[threadIdx.x];
    if (threadIdx.x == 0) {
        st->nusq = nsq / (pw * pw);
        st->nu = nu;
        st->last_accepted = ok ? 1 : 0;
        if (!fin) st->nonfinite = 1;
        if (ok) {
            st->scale[slot] = 1.0 / (nu * pw);
            if constexpr (scaled_store<DT>()) st->mu[slot] = st->scale[slot] * f16_rounded(mx);
            st->R[slot][slot] = nu;
            st->d = slot + 1;
        } else {
            st->rejects += 1;
            st->d = slot;
        }
    }
}

template <int KIND, int VF, int DT>
__global__ __launch_bounds__(kBlock) void proj_fin_kernel(ProjArgs a, int nb) {
    __shared__ double lds[kLdsDoubles];
    ProjState *st = a.st;
    const int d = st->d;
    if constexpr (KIND == FIN_DOTS) {
        if (threadIdx.x == 0) st->form_d = d;
        dispatch_d<1, GUESS_MAX_M>(d, [&](auto Dc) {
            constexpr int D = decltype(Dc)::value;
            double tot[D];
            final_sums<D>(a.part, nb, tot, lds);
            if (threadIdx.x < D) {
                const double sc = st->scale[threadIdx.x];
                // alpha_j = sc (C_j^T b); x0 = sum_j alpha_j sc X_j
                st->gamma[threadIdx.x] = sc * (sc * tot[threadIdx.x]);
            }
        });
    } else if constexpr (KIND == FIN_APPLY) {
        if (proj_restart<VF>(d, a.M)) {
            constexpr bool SC = scaled_store<DT>();
            double tot[SC ? 2 : 1];
            final_sums<SC ? 2 : 1, 1>(a.part, nb, tot, lds);
            if (threadIdx.x == 0) {
                const double nu0 = sqrt(tot[0]);
                const bool ok = isfinite(nu0) && nu0 > 0.0;
                // FP16: the raw pair is stored times 2^e (by proj_gs_write), e from max(|x|, |A x|)
                const double pw = SC ? ldexp(1.0, f16_scale_exp(tot[SC ? 1 : 0])) : 1.0;
                st->pow2 = pw;
                st->upd_d = d;
                st->nu0sq = tot[0];
                st->nu0 = nu0;
                st->nu = nu0;
                st->mode = 1;
                st->drop = 0;
                if ((VF & VF_QR) != 0 && d > 0) st->drops += 1;
                else st->restarts += 1;
                st->last_accepted = ok ? 1 : 0;
                if (!isfinite(nu0)) st->nonfinite = 1;
                st->scale[0] = ok ? 1.0 / (nu0 * pw) : 0.0;
                if constexpr (SC) st->mu[0] = ok ? st->scale[0] * f16_rounded(tot[SC ? 1 : 0] * pw) : 0.0;
                st->R[0][0] = ok ? nu0 : 0.0;
                st->d = ok ? 1 : 0;
            }
            return;
        }
        const bool drop = (VF & VF_QR) != 0 && d == a.M;
        if (drop) qr_drop_plan<DT>(st, a.M);
        dispatch_d<1, gs_max<VF>()>(d, [&](auto Dc) {
            constexpr int D = decltype(Dc)::value;
            double tot[D + 1];
            final_sums<D + 1>(a.part, nb, tot, lds);
            if (drop) {
                if constexpr (D >= 2) {
                    if (threadIdx.x == 0) {
                        double q[D];
#pragma unroll
                        for (int j = 0; j < D; ++j) q[j] = st->scale[j] * tot[j];
                        rot_forward<D>(st->gc, st->gs, q);
#pragma unroll
                        for (int j = 0; j < D - 1; ++j) st->c[j] = q[j];
                        rot_backward<D>(st->gc, st->gs, q);
#pragma unroll
                        for (int j = 0; j < D; ++j) st->cs[j] = q[j] * st->scale[j];
                    }
                }
            } else if (threadIdx.x < D) {
                const double sc = st->scale[threadIdx.x];
                const double cj = sc * tot[threadIdx.x];        // <column j, x>, column of unit norm
                st->c[threadIdx.x] = cj;
                st->cs[threadIdx.x] = cj * sc;
            }
            if (threadIdx.x == 0) {
                st->upd_d = D;
                st->nu0sq = tot[D];
                st->nu0 = sqrt(tot[D]);
                st->mode = 0;
                st->drop = drop ? 1 : 0;
                if (drop) st->drops += 1;
            }
        });
    } else if constexpr (KIND == FIN_REORTH) {
        if (st->mode != 0) return;
        const bool drop = (VF & VF_QR) != 0 && st->drop != 0;
        dispatch_d<1, gs_max<VF>()>(d, [&](auto Dc) {
            constexpr int D = decltype(Dc)::value;
            constexpr int ND = scaled_store<DT>() ? D + 1 : D;
            double tot[ND];
            final_sums<ND, D>(a.part, nb, tot, lds);
            if (drop) {
                if constexpr (D >= 2) {
                    if (threadIdx.x == 0) {
                        double q[D];
#pragma unroll
                        for (int j = 0; j < D; ++j) q[j] = st->scale[j] * tot[j];
                        rot_forward<D>(st->gc, st->gs, q);
#pragma unroll
                        for (int j = 0; j < D - 1; ++j) q[j] += st->c[j];
#pragma unroll
                        for (int j = 0; j < D - 1; ++j) st->c[j] = q[j];
                        rot_backward<D>(st->gc, st->gs, q);
#pragma unroll
                        for (int j = 0; j < D; ++j) st->cs[j] = q[j] * st->scale[j];
                    }
                }
            } else if (threadIdx.x < D) {
                const double sc = st->scale[threadIdx.x];
                const double cj = st->c[threadIdx.x] + sc * tot[threadIdx.x];
                st->c[threadIdx.x] = cj;
                st->cs[threadIdx.x] = cj * sc;
            }
            if constexpr (scaled_store<DT>()) {
                // the new pair is stored times 2^e, e from its largest magnitude after the
                // first Gram-Schmidt pass
                if (threadIdx.x == 0) st->pow2 = ldexp(1.0, f16_scale_exp(tot[ND - 1]));
            }
        });
    } else {
        if (st->mode != 0 || d < 1 || d > a.M) return;
        const bool drop = (VF & VF_QR) != 0 && st->drop != 0;
        if (!drop && d >= a.M) return;
        if constexpr (scaled_store<DT>()) {
            if ((VF & VF_QR) != 0 && drop) {
                dispatch_d<2, GUESS_MAX_M>(d, [&](auto Dc) {
                    constexpr int D = decltype(Dc)::value;
                    double tot[D + 1];
                    final_sums<D + 1, 1>(a.part, nb, tot, lds);
                    gs_accept<DT>(st, d, true, tot[0], tot[1]);
                    // the rotated slots take their new scales
                    if (threadIdx.x < D - 1) {
                        const double sp = st->nscale[threadIdx.x];
                        st->scale[threadIdx.x] = sp;
                        st->mu[threadIdx.x] = sp * f16_rounded(tot[2 + threadIdx.x]);
                    }
                });
                return;
            }
            double tot[2];
            final_sums<2, 1>(a.part, nb, tot, lds);
            gs_accept<DT>(st, d, drop, tot[0], tot[1]);
        } else {
            double tot[1];
            final_sums<1>(a.part, nb, tot, lds);
            gs_accept<DT>(st, d, drop, tot[0], 0.0);
        }
    }
}

// ------------------------------------------------------------------ per-format launchers
inline ProjArgs make_args(const ProjBufs &p) {
    ProjArgs a;
    a.X = p.X;
    a.B = p.B;
    a.Xw = p.X;
    a.Bw = p.B;
    a.w = p.w;
    a.part = p.part;
    a.st = p.st;
    a.N = p.N;
    a.ld = p.ld;
    a.M = p.M;
    return a;
}

template <int DT, int VF>
void proj_form_dt(const ProjBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev) {
    const ProjArgs a = make_args(p);
    const int gr = stream_grid(nchunks(a.N), reduce_blocks());
    klaunch(ev, 0, proj_dots_kernel<DT, VF>, gr, kBlock, s, a, b);
    klaunch(ev, 1, proj_fin_kernel<FIN_DOTS, VF, DT>, 1, kBlock, s, a, gr);
    klaunch_sh(ev, 2, proj_combine_kernel<DT>, stream_grid(nchunks(a.N), grid_cap()), kBlock, gather_lds(), s, a, x0);
}

template <int DT, int VF>
void proj_update_dt(const ProjBufs &p, const Grid *g, const double *x, const double *Ax, hipStream_t s,
                    KEvents *ev) {
    const ProjArgs a = make_args(p);
    const int gr = stream_grid(nchunks(a.N), reduce_blocks());
    const Grid gg = g ? *g : Grid{};
    int ga = gr;   // partial rows written by the apply kernel
    if (!Ax && march_ok(*g) && march_enabled()) {
        const int wgs = g->kx ? resident_wgs<proj_apply_march_kernel<DT, VF, true>>()
                              : resident_wgs<proj_apply_march_kernel<DT, VF, false>>();
        const March m = make_march(*g, wgs);
        ga = march_grid(m);
        if (g->kx) klaunch(ev, 0, proj_apply_march_kernel<DT, VF, true>, ga, kBlock, s, a, gg, m, x);
        else klaunch(ev, 0, proj_apply_march_kernel<DT, VF, false>, ga, kBlock, s, a, gg, m, x);
    } else if (Ax) {
        klaunch(ev, 0, proj_apply_kernel<DT, VF, false, true, true>, gr, kBlock, s, a, gg, x, Ax);
    } else if (g->kx) {
        if (g->aligned) klaunch(ev, 0, proj_apply_kernel<DT, VF, true, false, true>, gr, kBlock, s, a, gg, x, Ax);
        else klaunch(ev, 0, proj_apply_kernel<DT, VF, true, false, false>, gr, kBlock, s, a, gg, x, Ax);
    } else {
        if (g->aligned) klaunch(ev, 0, proj_apply_kernel<DT, VF, false, false, true>, gr, kBlock, s, a, gg, x, Ax);
        else klaunch(ev, 0, proj_apply_kernel<DT, VF, false, false, false>, gr, kBlock, s, a, gg, x, Ax);
    }
    klaunch(ev, 1, proj_fin_kernel<FIN_APPLY, VF, DT>, 1, kBlock, s, a, ga);
    const double *w = Ax ? Ax : a.w;
    klaunch(ev, 2, proj_reorth_kernel<DT, VF>, gr, kBlock, s, a, x, w);
    klaunch(ev, 3, proj_fin_kernel<FIN_REORTH, VF, DT>, 1, kBlock, s, a, gr);
    // The write pass stores two columns: one chunk per thread, so that no loop iteration waits
    // on the stores of the one before (partial rows: at most 2 per workgroup, M + 1 for an FP16
    // rolling drop, within the buffer's capacity).
    const int ndw = (scaled_store<DT>() && (VF & VF_QR) != 0) ? a.M + 1 : 2;
    int wcap = kPartialDoubles / ndw;
    if (write_blocks() > 0 && write_blocks() < wcap) wcap = write_blocks();
    const int gw = stream_grid(nchunks(a.N), wcap);
    klaunch(ev, 4, proj_gs_write_kernel<DT, VF>, gw, kBlock, s, a, x, w);
    klaunch(ev, 5, proj_fin_kernel<FIN_GS, VF, DT>, 1, kBlock, s, a, gw);
}

}  // namespace lg
