// Matrix-free 7-point operator and Jacobi-preconditioned CG (§5.3).
//
// PCG keeps its scalars (rho, alpha, beta, residual norms, iteration count,
// convergence flag) on the device: each reduction kernel's last workgroup
// finishes the dot products in a fixed order and updates them, and every
// kernel returns at once when the solve has converged or broken down.  The
// host therefore enqueues iterations in batches and only reads the state
// between batches; the iteration count is still exact.
//
// Algorithmic bytes per unknown and iteration (constant coefficient):
//   pcg_q     q = A p, p^T q                 reads 8, writes 8
//   pcg_xr    x += a p, r -= a q, r^T r,     reads 32, writes 16
//             r^T z with z = D^{-1} r
//   pcg_p     p = D^{-1} r + b p             reads 16, writes 8
// (variable coefficient: + 6 face values per unknown in pcg_q, and the
// reciprocal diagonal in pcg_xr and pcg_p.)
#include "common.h"
#include "launch.h"

namespace lg {

// ------------------------------------------------------------------ setup
// Face coefficient 2 a b / (a + b) of two nodal values (evaluated as
// ((2a) b) / (a + b)); a is the node with the lower index along the axis.
__device__ __forceinline__ double harmonic(double a, double b) {
#pragma clang fp contract(off)
    return ((2.0 * a) * b) / (a + b);
}

__global__ void build_faces_kernel(Grid g, const double *__restrict__ kappa, double *kx, double *ky,
                                   double *kz) {
    // kappa on (nx+2)(ny+2)(nz+2) nodes, x fastest; interior node (i,j,l) is padded (i+1,j+1,l+1)
    const int64_t mx = g.nx + 2, mxy = mx * (g.ny + 2);
    auto K = [&](int64_t pi, int64_t pj, int64_t pl) { return kappa[pl * mxy + pj * mx + pi]; };
    const int64_t nfx = (int64_t)(g.nx + 1) * g.ny * g.nz;
    const int64_t nfy = (int64_t)g.nx * (g.ny + 1) * g.nz;
    const int64_t nfz = (int64_t)g.nx * g.ny * (g.nz + 1);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nfx + nfy + nfz; t += stride) {
        if (t < nfx) {
            const int64_t f = t % (g.nx + 1), r = t / (g.nx + 1);
            const int64_t j = r % g.ny, l = r / g.ny;
            kx[t] = harmonic(K(f, j + 1, l + 1), K(f + 1, j + 1, l + 1));
        } else if (t < nfx + nfy) {
            const int64_t u = t - nfx;
            const int64_t i = u % g.nx, r = u / g.nx;
            const int64_t f = r % (g.ny + 1), l = r / (g.ny + 1);
            ky[u] = harmonic(K(i + 1, f, l + 1), K(i + 1, f + 1, l + 1));
        } else {
            const int64_t u = t - nfx - nfy;
            const int64_t i = u % g.nx, r = u / g.nx;
            const int64_t j = r % g.ny, f = r / g.ny;
            kz[u] = harmonic(K(i + 1, j + 1, f), K(i + 1, j + 1, f + 1));
        }
    }
}

__global__ void build_dinv_kernel(Grid g, double *dinv) {
#pragma clang fp contract(off)
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < g.n; p += stride) {
        int i, j, l;
        coords(g, p, i, j, l);
        const int64_t rx = ((int64_t)l * g.ny + j) * (g.nx + 1) + i;
        const int64_t ry = ((int64_t)l * (g.ny + 1) + j) * g.nx + i;
        double s = g.kx[rx] + g.kx[rx + 1];
        s = s + g.ky[ry];
        s = s + g.ky[ry + g.nx];
        s = s + g.kz[p];
        s = s + g.kz[p + g.nxy];
        const double dg = g.c * s + g.shift;
        dinv[p] = 1.0 / dg;
    }
}

int launch_build_faces(Grid &g, const double *kappa, double *kx, double *ky, double *kz, double *dinv,
                       hipStream_t s) {
    build_faces_kernel<<<1024, kBlock, 0, s>>>(g, kappa, kx, ky, kz);
    g.kx = kx;
    g.ky = ky;
    g.kz = kz;
    build_dinv_kernel<<<1024, kBlock, 0, s>>>(g, dinv);
    g.dinv = dinv;
    return GUESS_OK;
}

// ------------------------------------------------------------------ apply
template <bool VAR>
__global__ __launch_bounds__(kBlock) void op_apply_kernel(Grid g, const double *__restrict__ x,
                                                          double *__restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < g.n; p += stride) {
        int i, j, l;
        coords(g, p, i, j, l);
        y[p] = apply_at<VAR>(x, g, i, j, l, p);
    }
}

int launch_op_apply(const Grid &g, const double *x, double *y, hipStream_t s) {
    const int grid = stream_grid(g.n, grid_cap());
    if (g.kx) op_apply_kernel<true><<<grid, kBlock, 0, s>>>(g, x, y);
    else op_apply_kernel<false><<<grid, kBlock, 0, s>>>(g, x, y);
    return GUESS_OK;
}

// ------------------------------------------------------------------ PCG
int pcg_grid(const Grid &g) { return stream_grid(g.n, reduce_blocks()); }

__device__ __forceinline__ bool pcg_done(const PcgState *st) { return st->converged | st->breakdown; }

// r = b - A x, p = z = D^{-1} r; sums r^T r, r^T z, b^T b.
template <bool VAR>
__global__ __launch_bounds__(kBlock) void pcg_init_kernel(Grid g, const double *__restrict__ b,
                                                          const double *__restrict__ x,
                                                          double *__restrict__ r, double *__restrict__ p,
                                                          double *part, PcgState *st, double rtol) {
    __shared__ double lds[kLdsDoubles];
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < g.n; q += stride) {
        int i, j, l;
        coords(g, q, i, j, l);
        const double bq = b[q];
        const double rq = bq - apply_at<VAR>(x, g, i, j, l, q);
        const double zq = dinv_at<VAR>(g, q) * rq;
        r[q] = rq;
        p[q] = zq;
        acc[0] = __builtin_fma(rq, rq, acc[0]);
        acc[1] = __builtin_fma(rq, zq, acc[1]);
        acc[2] = __builtin_fma(bq, bq, acc[2]);
    }
    block_partials<3>(acc, part, lds);
    if (last_block(&st->ticket[0])) {
        double tot[3];
        final_sums<3>(part, gridDim.x, tot, lds);
        if (threadIdx.x == 0) {
            st->rr = tot[0];
            st->rr0 = tot[0];
            st->rho = tot[1];
            st->bb = tot[2];
            st->it = 0;
            st->breakdown = 0;
            const double rn = sqrt(tot[0]);
            if (st->rule == GUESS_STOP_RHS) {
                st->thresh = rtol * sqrt(tot[2]);
                st->converged = rn <= st->thresh;
            } else {
                st->thresh = rtol * fmax(rn, 1.0);
                st->converged = rn < st->thresh;
            }
        }
    }
}

// q = A p; alpha = rho / p^T q.
template <bool VAR>
__global__ __launch_bounds__(kBlock) void pcg_q_kernel(Grid g, const double *__restrict__ p,
                                                       double *__restrict__ q, double *part,
                                                       PcgState *st) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done(st)) return;
    double acc[1] = {0.0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < g.n; t += stride) {
        int i, j, l;
        coords(g, t, i, j, l);
        const double qt = apply_at<VAR>(p, g, i, j, l, t);
        q[t] = qt;
        acc[0] = __builtin_fma(p[t], qt, acc[0]);
    }
    block_partials<1>(acc, part, lds);
    if (last_block(&st->ticket[1])) {
        double tot[1];
        final_sums<1>(part, gridDim.x, tot, lds);
        if (threadIdx.x == 0) {
            const double pq = tot[0];
            if (!(pq > 0.0) || !isfinite(pq)) {
                st->breakdown = 1;
                st->it += 1;
            } else {
                st->alpha = st->rho / pq;
            }
        }
    }
}

// x += alpha p; r -= alpha q; sums r^T r and r^T z (z = D^{-1} r); stop test; beta.
template <bool VAR>
__global__ __launch_bounds__(kBlock) void pcg_xr_kernel(Grid g, double *__restrict__ x,
                                                        double *__restrict__ r,
                                                        const double *__restrict__ p,
                                                        const double *__restrict__ q, double *part,
                                                        PcgState *st) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done(st)) return;
    const double alpha = st->alpha;
    double acc[2] = {0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < g.n; t += stride) {
        x[t] = __builtin_fma(alpha, p[t], x[t]);
        const double rt = __builtin_fma(-alpha, q[t], r[t]);
        r[t] = rt;
        const double zt = dinv_at<VAR>(g, t) * rt;
        acc[0] = __builtin_fma(rt, rt, acc[0]);
        acc[1] = __builtin_fma(rt, zt, acc[1]);
    }
    block_partials<2>(acc, part, lds);
    if (last_block(&st->ticket[2])) {
        double tot[2];
        final_sums<2>(part, gridDim.x, tot, lds);
        if (threadIdx.x == 0) {
            st->it += 1;
            st->rr = tot[0];
            const double rn = sqrt(tot[0]);
            const bool stop = st->rule == GUESS_STOP_RHS ? (rn <= st->thresh) : (rn < st->thresh);
            if (stop) {
                st->converged = 1;
            } else {
                st->beta = tot[1] / st->rho;
                st->rho = tot[1];
            }
        }
    }
}

// p = D^{-1} r + beta p.
template <bool VAR>
__global__ __launch_bounds__(kBlock) void pcg_p_kernel(Grid g, const double *__restrict__ r,
                                                       double *__restrict__ p, const PcgState *st) {
    if (pcg_done(st)) return;
    const double beta = st->beta;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < g.n; t += stride)
        p[t] = __builtin_fma(beta, p[t], dinv_at<VAR>(g, t) * r[t]);
}

int launch_pcg_init(const Grid &g, const double *b, const double *x, double *r, double *p, double *part,
                    PcgState *st, double rtol, int rule, hipStream_t s) {
    (void)rule;
    const int gr = pcg_grid(g);
    if (g.kx) pcg_init_kernel<true><<<gr, kBlock, 0, s>>>(g, b, x, r, p, part, st, rtol);
    else pcg_init_kernel<false><<<gr, kBlock, 0, s>>>(g, b, x, r, p, part, st, rtol);
    return GUESS_OK;
}

int launch_pcg_iter(const Grid &g, double *x, double *r, double *p, double *q, double *part, PcgState *st,
                    hipStream_t s) {
    const int gr = pcg_grid(g);
    const int gs = stream_grid(g.n, grid_cap());
    if (g.kx) {
        pcg_q_kernel<true><<<gr, kBlock, 0, s>>>(g, p, q, part, st);
        pcg_xr_kernel<true><<<gr, kBlock, 0, s>>>(g, x, r, p, q, part, st);
        pcg_p_kernel<true><<<gs, kBlock, 0, s>>>(g, r, p, st);
    } else {
        pcg_q_kernel<false><<<gr, kBlock, 0, s>>>(g, p, q, part, st);
        pcg_xr_kernel<false><<<gr, kBlock, 0, s>>>(g, x, r, p, q, part, st);
        pcg_p_kernel<false><<<gs, kBlock, 0, s>>>(g, r, p, st);
    }
    return GUESS_OK;
}

}  // namespace lg
