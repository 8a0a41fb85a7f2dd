// Kernels of Fischer's projection guess, classic restart variant (§2,
// Algorithm 1), in A-orthonormal form: X^T A X = I, B = A X, guess
// x0 = X (X^T b).
//
// Columns are stored unnormalised with a per-column FP64 scale kept in the
// device state (true column j = scale[j] * stored column j), so that the
// normalisation of a new column, which needs its norm, does not cost an
// extra pass over the data.  Every decision (restart, accept / reject) is
// taken on the device.
//
// Each reduction is split in two launches: a streaming kernel that writes
// one row of partial sums per workgroup, and a one-workgroup finishing
// kernel (proj_fin) that sums the rows in a fixed order and updates the
// state.  Nothing synchronises across workgroups inside a kernel, so no
// device-wide cache write-back or invalidation is needed mid-kernel.
//
// Streaming kernels and algorithmic bytes per unknown (s = stored element
// size, d the current number of columns):
//   proj_dots      P_j = X_j^T b                      reads d s + 8
//   proj_combine   x0 = sum_j gamma_j X_j             reads d s, writes 8
//   proj_apply     w = A x (or the caller's A x),     reads 8 (+8), d s; writes 8
//                  c1 = X^T w, nu0^2 = x^T w;
//                  restart: X_1 <- x, B_1 <- w        reads 8 (+8); writes 2 s
//   proj_reorth    c2 = X^T (w - B c1)                reads 2 d s + 8
//   proj_gs_write  x'' = x - X c, w'' = w - B c,      reads 2 d s + 16; writes 2 s
//                  nu^2 = x''^T w'', store in slot d
#pragma once

#include "common.h"
#include "launch.h"

namespace lg {

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

__device__ __forceinline__ bool proj_restart(const ProjState *st, int M) {
    const int d = st->d;
    return d == 0 || d >= M;
}

// ------------------------------------------------------------------ form
template <int DT>
LG_REDUCE_KERNEL void proj_dots_kernel(ProjArgs a, const double *__restrict__ b) {
    __shared__ double lds[kLdsDoubles];
    const int d = a.st->d;
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
            for (int j = 0; j < D; ++j) xv[j] = load4<DT>(colp<DT>(a.X, a.ld, j), c);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(xv[j].v[e], bv.v[e], acc[j]);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
#pragma unroll
            for (int j = 0; j < D; ++j)
                acc[j] = __builtin_fma(load1<DT>(colp<DT>(a.X, a.ld, j), i), b[i], acc[j]);
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
template <int DT, bool VAR, bool HAVE_AX, bool AL>
LG_REDUCE_KERNEL void proj_apply_kernel(ProjArgs a, Grid g, const double *__restrict__ x,
                                        const double *__restrict__ Ax) {
    __shared__ double lds[kLdsDoubles];
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
    if (d == 0 || d >= a.M) {
        // restart: slot 1 <- x, B slot 1 <- A x; partial nu0^2 = x^T A x
        double acc[1] = {0.0};
        for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
            V4 xv;
            const V4 wv = xw4(c, xv);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[0] = __builtin_fma(xv.v[e], wv.v[e], acc[0]);
            store4<DT>(a.Xw, c, xv);
            store4<DT>(a.Bw, c, wv);
        }
        if (blockIdx.x == 0 && threadIdx.x < rem) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            const double wv = xw1(i);
            acc[0] = __builtin_fma(x[i], wv, acc[0]);
            store1<DT>(a.Xw, i, x[i]);
            store1<DT>(a.Bw, i, wv);
        }
        block_partials<1>(acc, a.part, lds);
        return;
    }
    dispatch_d<1, GUESS_MAX_M - 1>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        constexpr int ND = D + 1;
        double acc[ND];
#pragma unroll
        for (int j = 0; j < ND; ++j) acc[j] = 0.0;
        for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
            V4 xc[D];
#pragma unroll
            for (int j = 0; j < D; ++j) xc[j] = load4<DT>(colp<DT>(a.X, a.ld, j), c);
            V4 xv;
            const V4 wv = xw4(c, xv);
            if constexpr (!HAVE_AX) store4<GUESS_F64>(a.w, c, wv);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[D] = __builtin_fma(xv.v[e], wv.v[e], acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(xc[j].v[e], wv.v[e], acc[j]);
        }
        if (blockIdx.x == 0 && threadIdx.x < rem) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            const double wv = xw1(i);
            if constexpr (!HAVE_AX) a.w[i] = wv;
            acc[D] = __builtin_fma(x[i], wv, acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j) acc[j] = __builtin_fma(load1<DT>(colp<DT>(a.X, a.ld, j), i), wv, acc[j]);
        }
        block_partials<ND>(acc, a.part, lds);
    });
}

template <int DT>
LG_REDUCE_KERNEL void proj_reorth_kernel(ProjArgs a, const double *__restrict__ w) {
    __shared__ double lds[kLdsDoubles];
    if (a.st->mode != 0) return;
    const int d = a.st->d;
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    dispatch_d<1, GUESS_MAX_M - 1>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double cs[D], acc[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            cs[j] = a.st->cs[j];
            acc[j] = 0.0;
        }
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
            V4 bc[D], xc[D];
#pragma unroll
            for (int j = 0; j < D; ++j) bc[j] = load4<DT>(colp<DT>(a.B, a.ld, j), c);
#pragma unroll
            for (int j = 0; j < D; ++j) xc[j] = load4<DT>(colp<DT>(a.X, a.ld, j), c);
            V4 wv = load4<GUESS_F64>(w, c);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) wv.v[e] = __builtin_fma(-cs[j], bc[j].v[e], wv.v[e]);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(xc[j].v[e], wv.v[e], acc[j]);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            double wv = w[i];
#pragma unroll
            for (int j = 0; j < D; ++j) wv = __builtin_fma(-cs[j], load1<DT>(colp<DT>(a.B, a.ld, j), i), wv);
#pragma unroll
            for (int j = 0; j < D; ++j) acc[j] = __builtin_fma(load1<DT>(colp<DT>(a.X, a.ld, j), i), wv, acc[j]);
        }
        block_partials<D>(acc, a.part, lds);
    });
}

template <int DT>
LG_REDUCE_KERNEL void proj_gs_write_kernel(ProjArgs a, const double *__restrict__ x,
                                           const double *__restrict__ w) {
    __shared__ double lds[kLdsDoubles];
    if (a.st->mode != 0) return;
    const int d = a.st->d;
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    dispatch_d<1, GUESS_MAX_M - 1>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double cs[D];
#pragma unroll
        for (int j = 0; j < D; ++j) cs[j] = a.st->cs[j];
        void *Xd = colw<DT>(a.Xw, a.ld, D);
        void *Bd = colw<DT>(a.Bw, a.ld, D);
        double acc[1] = {0.0};
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
            for (int e = 0; e < 4; ++e) acc[0] = __builtin_fma(xv.v[e], wv.v[e], acc[0]);
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
            acc[0] = __builtin_fma(xv, wv, acc[0]);
            store1<DT>(Xd, i, xv);
            store1<DT>(Bd, i, wv);
        }
        block_partials<1>(acc, a.part, lds);
    });
}

// ------------------------------------------------------------------ finishing kernels
// One workgroup: sum the nb partial rows of the preceding streaming kernel
// and take the step's decisions.
enum { FIN_DOTS = 0, FIN_APPLY = 1, FIN_REORTH = 2, FIN_GS = 3 };

template <int KIND>
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
                // alpha_j = sc (X_j^T b); x0 = sum_j alpha_j sc X_j
                st->gamma[threadIdx.x] = sc * (sc * tot[threadIdx.x]);
            }
        });
    } else if constexpr (KIND == FIN_APPLY) {
        if (d == 0 || d >= a.M) {
            double tot[1];
            final_sums<1>(a.part, nb, tot, lds);
            if (threadIdx.x == 0) {
                const double nu0 = sqrt(tot[0]);
                const bool ok = isfinite(nu0) && nu0 > 0.0;
                st->upd_d = d;
                st->nu0sq = tot[0];
                st->nu0 = nu0;
                st->nu = nu0;
                st->mode = 1;
                st->restarts += 1;
                st->last_accepted = ok ? 1 : 0;
                if (!isfinite(nu0)) st->nonfinite = 1;
                st->scale[0] = ok ? 1.0 / nu0 : 0.0;
                st->d = ok ? 1 : 0;
            }
            return;
        }
        dispatch_d<1, GUESS_MAX_M - 1>(d, [&](auto Dc) {
            constexpr int D = decltype(Dc)::value;
            double tot[D + 1];
            final_sums<D + 1>(a.part, nb, tot, lds);
            if (threadIdx.x < D) {
                const double sc = st->scale[threadIdx.x];
                const double cj = sc * tot[threadIdx.x];        // <X_j, A x>, X_j of unit A-norm
                st->c[threadIdx.x] = cj;
                st->cs[threadIdx.x] = cj * sc;
            }
            if (threadIdx.x == 0) {
                st->upd_d = D;
                st->nu0sq = tot[D];
                st->nu0 = sqrt(tot[D]);
                st->mode = 0;
            }
        });
    } else if constexpr (KIND == FIN_REORTH) {
        if (st->mode != 0) return;
        dispatch_d<1, GUESS_MAX_M - 1>(d, [&](auto Dc) {
            constexpr int D = decltype(Dc)::value;
            double tot[D];
            final_sums<D>(a.part, nb, tot, lds);
            if (threadIdx.x < D) {
                const double sc = st->scale[threadIdx.x];
                const double cj = st->c[threadIdx.x] + sc * tot[threadIdx.x];
                st->c[threadIdx.x] = cj;
                st->cs[threadIdx.x] = cj * sc;
            }
        });
    } else {
        if (st->mode != 0 || d < 1 || d >= a.M) return;
        double tot[1];
        final_sums<1>(a.part, nb, tot, lds);
        if (threadIdx.x == 0) {
            const double nu = sqrt(tot[0]);      // NaN when rounding made it negative
            const bool fin = isfinite(nu);
            const bool ok = fin && nu > st->eps_rel * st->nu0;
            st->nusq = tot[0];
            st->nu = nu;
            st->last_accepted = ok ? 1 : 0;
            if (!fin) st->nonfinite = 1;
            if (ok) {
                st->scale[d] = 1.0 / nu;
                st->d = d + 1;
            } else {
                st->rejects += 1;
            }
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

template <int DT>
void proj_form_dt(const ProjBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev) {
    const ProjArgs a = make_args(p);
    const int gr = stream_grid(nchunks(a.N), reduce_blocks());
    klaunch(ev, 0, proj_dots_kernel<DT>, gr, kBlock, s, a, b);
    klaunch(ev, 1, proj_fin_kernel<FIN_DOTS>, 1, kBlock, s, a, gr);
    klaunch(ev, 2, proj_combine_kernel<DT>, stream_grid(nchunks(a.N), grid_cap()), kBlock, s, a, x0);
}

template <int DT>
void proj_update_dt(const ProjBufs &p, const Grid *g, const double *x, const double *Ax, hipStream_t s,
                    KEvents *ev) {
    const ProjArgs a = make_args(p);
    const int gr = stream_grid(nchunks(a.N), reduce_blocks());
    const Grid gg = g ? *g : Grid{};
    if (Ax) {
        klaunch(ev, 0, proj_apply_kernel<DT, false, true, true>, gr, kBlock, s, a, gg, x, Ax);
    } else if (g->kx) {
        if (g->aligned) klaunch(ev, 0, proj_apply_kernel<DT, true, false, true>, gr, kBlock, s, a, gg, x, Ax);
        else klaunch(ev, 0, proj_apply_kernel<DT, true, false, false>, gr, kBlock, s, a, gg, x, Ax);
    } else {
        if (g->aligned) klaunch(ev, 0, proj_apply_kernel<DT, false, false, true>, gr, kBlock, s, a, gg, x, Ax);
        else klaunch(ev, 0, proj_apply_kernel<DT, false, false, false>, gr, kBlock, s, a, gg, x, Ax);
    }
    klaunch(ev, 1, proj_fin_kernel<FIN_APPLY>, 1, kBlock, s, a, gr);
    const double *w = Ax ? Ax : a.w;
    klaunch(ev, 2, proj_reorth_kernel<DT>, gr, kBlock, s, a, w);
    klaunch(ev, 3, proj_fin_kernel<FIN_REORTH>, 1, kBlock, s, a, gr);
    klaunch(ev, 4, proj_gs_write_kernel<DT>, gr, kBlock, s, a, x, w);
    klaunch(ev, 5, proj_fin_kernel<FIN_GS>, 1, kBlock, s, a, gr);
}

}  // namespace lg
