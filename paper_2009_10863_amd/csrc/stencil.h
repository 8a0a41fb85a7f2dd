// 7-point Helmholtz operators, evaluated point by point on the device.
//
// Constant coefficient:  (Au)_i = c (6 u_i - sum_nb u_nb) + s u_i
// Variable coefficient:  (Au)_i = c sum_faces k_f (u_i - u_nb) + s u_i
// (finite-difference replacement of the paper's spectral-element operator,
// §5; the paper's method only needs a matrix-free SPD operator).
//
// The evaluation order is fixed -- neighbours west, east, south, north,
// bottom, top, summed left to right, no fused multiply-add, then
// c * s + shift * u -- so that the result is reproducible bit for bit by any
// implementation that follows the same definition.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lg {

struct Grid {
    int nx, ny, nz;
    int64_t nxy, n;
    double c, shift;        // c = 1/h^2
    const double *kx;       // variable coefficient faces, or nullptr
    const double *ky;
    const double *kz;
    const double *dinv;     // reciprocal diagonal (variable coefficient only)
    double dinv_const;      // reciprocal diagonal (constant coefficient)
};

__device__ __forceinline__ double apply_const_at(const double *__restrict__ u, const Grid &g,
                                                 int i, int j, int l, int64_t p) {
#pragma clang fp contract(off)
    const double uc = u[p];
    double s = 6.0 * uc;
    s = s - (i > 0 ? u[p - 1] : 0.0);
    s = s - (i < g.nx - 1 ? u[p + 1] : 0.0);
    s = s - (j > 0 ? u[p - g.nx] : 0.0);
    s = s - (j < g.ny - 1 ? u[p + g.nx] : 0.0);
    s = s - (l > 0 ? u[p - g.nxy] : 0.0);
    s = s - (l < g.nz - 1 ? u[p + g.nxy] : 0.0);
    const double a = g.c * s;
    const double b = g.shift * uc;
    return a + b;
}

// Face arrays (x fastest):
//   kx: (nz, ny, nx+1)  face f along x at row (j, l) is kx[(l*ny + j)*(nx+1) + f]
//   ky: (nz, ny+1, nx)  ky[(l*(ny+1) + f)*nx + i]
//   kz: (nz+1, ny, nx)  kz[(f*ny + j)*nx + i]
// The west face of node i is f = i, the east face f = i + 1 (likewise y, z).
__device__ __forceinline__ double apply_var_at(const double *__restrict__ u, const Grid &g,
                                               int i, int j, int l, int64_t p) {
#pragma clang fp contract(off)
    const double uc = u[p];
    const int64_t rx = ((int64_t)l * g.ny + j) * (g.nx + 1) + i;
    const int64_t ry = ((int64_t)l * (g.ny + 1) + j) * g.nx + i;
    const int64_t rz = ((int64_t)l * g.ny + j) * g.nx + i;
    const double uw = i > 0 ? u[p - 1] : 0.0;
    const double ue = i < g.nx - 1 ? u[p + 1] : 0.0;
    const double us = j > 0 ? u[p - g.nx] : 0.0;
    const double un = j < g.ny - 1 ? u[p + g.nx] : 0.0;
    const double ub = l > 0 ? u[p - g.nxy] : 0.0;
    const double ut = l < g.nz - 1 ? u[p + g.nxy] : 0.0;
    double s = g.kx[rx] * (uc - uw);
    s = s + g.kx[rx + 1] * (uc - ue);
    s = s + g.ky[ry] * (uc - us);
    s = s + g.ky[ry + g.nx] * (uc - un);
    s = s + g.kz[rz] * (uc - ub);
    s = s + g.kz[rz + g.nxy] * (uc - ut);
    const double a = g.c * s;
    const double b = g.shift * uc;
    return a + b;
}

template <bool VAR>
__device__ __forceinline__ double apply_at(const double *__restrict__ u, const Grid &g,
                                           int i, int j, int l, int64_t p) {
    if constexpr (VAR) return apply_var_at(u, g, i, j, l, p);
    else return apply_const_at(u, g, i, j, l, p);
}

template <bool VAR>
__device__ __forceinline__ double dinv_at(const Grid &g, int64_t p) {
    if constexpr (VAR) return g.dinv[p];
    else return g.dinv_const;
}

__device__ __forceinline__ void coords(const Grid &g, int64_t p, int &i, int &j, int &l) {
    l = (int)(p / g.nxy);
    const int64_t r = p - (int64_t)l * g.nxy;
    j = (int)(r / g.nx);
    i = (int)(r - (int64_t)j * g.nx);
}

}  // namespace lg
