// 7-point Helmholtz operators, evaluated on the device.
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
//
// Two evaluation shapes:
//   apply_pt    one unknown (any grid; ragged tails)
//   apply4      one chunk: the two element pairs (p0, p0+1), (p0+128,
//               p0+129) of the tiling in common.h.  With nx even each pair
//               lies in one grid row: centre, south, north, bottom and top
//               values arrive as 16-byte loads, the west / east neighbours of
//               the pair as two scalar loads.  Odd nx falls back to the point
//               form for each of the four unknowns.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lg {

// Division by a fixed 32-bit divisor d >= 1 for numerators n < 2^31:
// q = (umulhi(n, m) + n) >> s with s = ceil(log2 d), m = floor(2^32 (2^s - d) / d) + 1.
struct FastDiv {
    uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t s = 0;
    while ((1ull << s) < d) ++s;
    const uint64_t m = ((1ull << 32) * ((1ull << s) - d)) / d + 1;
    return FastDiv{d, (uint32_t)m, s};
}

__device__ __forceinline__ uint32_t fdiv(const FastDiv &f, uint32_t n) {
    return (__umulhi(n, f.m) + n) >> f.s;
}

struct Grid {
    int nx, ny, nz;
    int64_t nxy, n;
    double c, shift;        // c = 1/h^2
    const double *kx;       // variable coefficient faces, or nullptr
    const double *ky;
    const double *kz;
    const double *dinv;     // reciprocal diagonal (variable coefficient only)
    double dinv_const;      // reciprocal diagonal (constant coefficient)
    FastDiv fnx, fny;       // division by nx and ny
    int aligned;            // nx % 2 == 0: every element pair of a chunk lies in one grid row
};

__device__ __forceinline__ void coords(const Grid &g, int64_t p, int &i, int &j, int &l) {
    const uint32_t r = fdiv(g.fnx, (uint32_t)p);      // row index l * ny + j
    i = (int)((uint32_t)p - r * (uint32_t)g.nx);
    const uint32_t q = fdiv(g.fny, r);
    j = (int)(r - q * (uint32_t)g.ny);
    l = (int)q;
}

// Point form.  U(q) returns the value of the operand at flat index q.
template <class U>
__device__ __forceinline__ double apply_const_pt(U u, const Grid &g, int i, int j, int l, int64_t p) {
#pragma clang fp contract(off)
    const double uc = u(p);
    double s = 6.0 * uc;
    s = s - (i > 0 ? u(p - 1) : 0.0);
    s = s - (i < g.nx - 1 ? u(p + 1) : 0.0);
    s = s - (j > 0 ? u(p - g.nx) : 0.0);
    s = s - (j < g.ny - 1 ? u(p + g.nx) : 0.0);
    s = s - (l > 0 ? u(p - g.nxy) : 0.0);
    s = s - (l < g.nz - 1 ? u(p + g.nxy) : 0.0);
    const double a = g.c * s;
    const double b = g.shift * uc;
    return a + b;
}

// Face arrays (x fastest):
//   kx: (nz, ny, nx+1)  face f along x at row (j, l) is kx[(l*ny + j)*(nx+1) + f]
//   ky: (nz, ny+1, nx)  ky[(l*(ny+1) + f)*nx + i]
//   kz: (nz+1, ny, nx)  kz[(f*ny + j)*nx + i]
// The west face of node i is f = i, the east face f = i + 1 (likewise y, z).
template <class U>
__device__ __forceinline__ double apply_var_pt(U u, const Grid &g, int i, int j, int l, int64_t p) {
#pragma clang fp contract(off)
    const double uc = u(p);
    const int64_t rx = ((int64_t)l * g.ny + j) * (g.nx + 1) + i;
    const int64_t ry = ((int64_t)l * (g.ny + 1) + j) * g.nx + i;
    const int64_t rz = ((int64_t)l * g.ny + j) * g.nx + i;
    const double uw = i > 0 ? u(p - 1) : 0.0;
    const double ue = i < g.nx - 1 ? u(p + 1) : 0.0;
    const double us = j > 0 ? u(p - g.nx) : 0.0;
    const double un = j < g.ny - 1 ? u(p + g.nx) : 0.0;
    const double ub = l > 0 ? u(p - g.nxy) : 0.0;
    const double ut = l < g.nz - 1 ? u(p + g.nxy) : 0.0;
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

template <bool VAR, class U>
__device__ __forceinline__ double apply_pt(U u, const Grid &g, int i, int j, int l, int64_t p) {
    if constexpr (VAR) return apply_var_pt(u, g, i, j, l, p);
    else return apply_const_pt(u, g, i, j, l, p);
}

template <bool VAR, class U>
__device__ __forceinline__ double apply_pt(U u, const Grid &g, int64_t p) {
    int i, j, l;
    coords(g, p, i, j, l);
    return apply_pt<VAR>(u, g, i, j, l, p);
}

template <bool VAR>
__device__ __forceinline__ double dinv_at(const Grid &g, int64_t p) {
    if constexpr (VAR) return g.dinv[p];
    else return g.dinv_const;
}

// ---------------------------------------------------------------- chunk form
typedef double dv2 __attribute__((ext_vector_type(2)));

struct R2 {
    double v[2];
};
struct R4 {
    double v[4];
};

__device__ __forceinline__ R2 ld2(const double *__restrict__ u, int64_t p0) {
    const dv2 a = *reinterpret_cast<const dv2 *>(u + p0);
    return R2{{a.x, a.y}};
}

// Operand access: u(q) gives one value, u.two(q) the values q, q+1 (q even).
struct VecU {
    const double *__restrict__ u;
    __device__ __forceinline__ double operator()(int64_t q) const { return u[q]; }
    __device__ __forceinline__ R2 two(int64_t q) const { return ld2(u, q); }
};

// A u at p0, p0+1 (p0 even, nx even: one grid row).  Also returns the centre values.
// Every load is unconditional -- a neighbour outside the grid is read at the
// centre's address and replaced by 0 afterwards -- so that the wave issues
// all of its loads back to back instead of waiting around each branch.
template <bool VAR, class U>
__device__ __forceinline__ R2 apply2(U u, const Grid &g, int64_t p0, R2 &uc) {
#pragma clang fp contract(off)
    int i0, j, l;
    coords(g, p0, i0, j, l);
    const bool hw = i0 > 0, he = i0 + 2 < g.nx, hs = j > 0, hn = j < g.ny - 1, hb = l > 0,
               ht = l < g.nz - 1;
    uc = u.two(p0);
    const double uw0 = u(hw ? p0 - 1 : p0);
    const double ue0 = u(he ? p0 + 2 : p0);
    const R2 us0 = u.two(hs ? p0 - g.nx : p0);
    const R2 un0 = u.two(hn ? p0 + g.nx : p0);
    const R2 ub0 = u.two(hb ? p0 - g.nxy : p0);
    const R2 ut0 = u.two(ht ? p0 + g.nxy : p0);
    const double uw = hw ? uw0 : 0.0;
    const double ue = he ? ue0 : 0.0;
    R2 us, un, ub, ut;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        us.v[e] = hs ? us0.v[e] : 0.0;
        un.v[e] = hn ? un0.v[e] : 0.0;
        ub.v[e] = hb ? ub0.v[e] : 0.0;
        ut.v[e] = ht ? ut0.v[e] : 0.0;
    }
    R2 r;
    if constexpr (!VAR) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const double w = e == 0 ? uw : uc.v[0];
            const double ea = e == 1 ? ue : uc.v[1];
            double s = 6.0 * uc.v[e];
            s = s - w;
            s = s - ea;
            s = s - us.v[e];
            s = s - un.v[e];
            s = s - ub.v[e];
            s = s - ut.v[e];
            const double a = g.c * s;
            const double b = g.shift * uc.v[e];
            r.v[e] = a + b;
        }
    } else {
        const int64_t rx = ((int64_t)l * g.ny + j) * (g.nx + 1) + i0;
        const int64_t ry = ((int64_t)l * (g.ny + 1) + j) * g.nx + i0;
        const double kx0 = g.kx[rx], kx1 = g.kx[rx + 1], kx2 = g.kx[rx + 2];
        const R2 ks = ld2(g.ky, ry), kn = ld2(g.ky, ry + g.nx);
        const R2 kb = ld2(g.kz, p0), kt = ld2(g.kz, p0 + g.nxy);
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const double w = e == 0 ? uw : uc.v[0];
            const double ea = e == 1 ? ue : uc.v[1];
            const double x = uc.v[e];
            double s = (e == 0 ? kx0 : kx1) * (x - w);
            s = s + (e == 0 ? kx1 : kx2) * (x - ea);
            s = s + ks.v[e] * (x - us.v[e]);
            s = s + kn.v[e] * (x - un.v[e]);
            s = s + kb.v[e] * (x - ub.v[e]);
            s = s + kt.v[e] * (x - ut.v[e]);
            const double a = g.c * s;
            const double b = g.shift * x;
            r.v[e] = a + b;
        }
    }
    return r;
}

// A u on chunk c (see common.h); uc receives the centre values.
template <bool VAR, bool AL, class U>
__device__ __forceinline__ R4 apply4g(U u, const Grid &g, int64_t c, R4 &uc) {
    const int64_t p0 = ((c >> 6) << 8) + ((c & 63) << 1);
    R4 r;
    if constexpr (AL) {
        R2 c0, c1;
        const R2 r0 = apply2<VAR>(u, g, p0, c0);
        const R2 r1 = apply2<VAR>(u, g, p0 + 128, c1);
        uc = R4{{c0.v[0], c0.v[1], c1.v[0], c1.v[1]}};
        r = R4{{r0.v[0], r0.v[1], r1.v[0], r1.v[1]}};
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t p = p0 + (e & 1) + (e >> 1) * 128;
            uc.v[e] = u(p);
            r.v[e] = apply_pt<VAR>(u, g, p);
        }
    }
    return r;
}

template <bool VAR, bool AL>
__device__ __forceinline__ R4 apply4g(const double *__restrict__ u, const Grid &g, int64_t c, R4 &uc) {
    return apply4g<VAR, AL>(VecU{u}, g, c, uc);
}

}  // namespace lg
