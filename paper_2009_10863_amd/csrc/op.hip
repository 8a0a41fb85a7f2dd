// Matrix-free 7-point operator: variable-coefficient setup (face
// coefficients, reciprocal diagonal) and y = A x (16 bytes per unknown).
#include "common.h"
#include "launch.h"
#include "march.h"

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
// Every kernel below handles 4 consecutive unknowns per thread and step
// (32-byte accesses); N mod 4 trailing unknowns go through the point form.
static __device__ __forceinline__ V4 toV(const R4 &r) { return V4{{r.v[0], r.v[1], r.v[2], r.v[3]}}; }

template <bool VAR, bool AL>
__global__ __launch_bounds__(kBlock) void op_apply_kernel(Grid g, const double *__restrict__ x,
                                                          double *__restrict__ y) {
    const ChunkRange cr = xcd_range(nchunks(g.n));
    for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
        R4 uc;
        store4<GUESS_F64>(y, c, toV(apply4g<VAR, AL>(x, g, c, uc)));
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(g.n)) {
        const int64_t p = tail_start(g.n) + threadIdx.x;
        y[p] = apply_pt<VAR>(VecU{x}, g, p);
    }
}

template <bool VAR>
__global__ __launch_bounds__(kBlock) void op_apply_march_kernel(Grid g, March m, const double *__restrict__ x,
                                                                double *__restrict__ y) {
    march_sweep<VAR>(g, m, VecU{x}, [&](int64_t c, int64_t, const R2 &, const R2 &, const R4 &au) {
        store4<GUESS_F64>(y, c, toV(au));
    });
}

template <bool VAR>
static void op_apply_v(const Grid &g, const double *x, double *y, hipStream_t s) {
    if (march_ok(g) && march_enabled()) {
        const int wgs = resident_wgs<op_apply_march_kernel<VAR>>();
        const March m = make_march(g, wgs);
        op_apply_march_kernel<VAR><<<march_grid(m), kBlock, 0, s>>>(g, m, x, y);
        return;
    }
    const int grid = stream_grid(nchunks(g.n), reduce_blocks());
    if (g.aligned) op_apply_kernel<VAR, true><<<grid, kBlock, 0, s>>>(g, x, y);
    else op_apply_kernel<VAR, false><<<grid, kBlock, 0, s>>>(g, x, y);
}

int launch_op_apply(const Grid &g, const double *x, double *y, hipStream_t s) {
    if (g.kx) op_apply_v<true>(g, x, y, s);
    else op_apply_v<false>(g, x, y, s);
    return GUESS_OK;
}

}  // namespace lg
