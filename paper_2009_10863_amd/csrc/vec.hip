// Generic FP64 vector kernels (multi-dot, combination, copy) and the
// plane-wave right-hand-side generator of the synthetic workloads.
#include <cstdlib>

#include "common.h"
#include "launch.h"

namespace lg {

constexpr int kMaxVecK = 64;

struct CombArgs {
    double c[kMaxVecK];
};

// out[k] = <V_k, y> for K <= 64 vectors, 8 at a time so that the
// accumulators stay in registers; deterministic two-stage reduction (partial
// sums per workgroup, then one workgroup sums them in a fixed order).
__global__ __launch_bounds__(kBlock) void multidot8_kernel(int64_t N, int K0, int KN,
                                                           const double *__restrict__ V,
                                                           const double *__restrict__ y, double *part) {
    // partial sums of up to 8 dot products (vectors K0 .. K0+KN-1) per workgroup
    double acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N; t += stride) {
        const double yt = y[t];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (k < KN) acc[k] = __builtin_fma(V[(int64_t)(K0 + k) * N + t], yt, acc[k]);
    }
    __shared__ double lds[kLdsDoubles];
    block_partials<8>(acc, part, lds);
}

__global__ __launch_bounds__(kBlock) void multidot_final_kernel(int nb, int K0, int KN, const double *part,
                                                                double *out) {
    __shared__ double lds[kLdsDoubles];
    double tot[8];
    final_sums<8>(part, nb, tot, lds);
    if (threadIdx.x < KN) out[K0 + threadIdx.x] = tot[threadIdx.x];
}

int launch_multidot(int64_t N, int K, const double *V, const double *y, double *part, double *out_dev,
                    hipStream_t s) {
    if (K < 1 || K > kMaxVecK) return GUESS_EINVAL;
    const int gr = stream_grid(N, reduce_blocks());
    for (int k0 = 0; k0 < K; k0 += 8) {
        const int kn = K - k0 < 8 ? K - k0 : 8;
        multidot8_kernel<<<gr, kBlock, 0, s>>>(N, k0, kn, V, y, part);
        multidot_final_kernel<<<1, kBlock, 0, s>>>(gr, k0, kn, part, out_dev);
    }
    return GUESS_OK;
}

__global__ __launch_bounds__(kBlock) void combine_kernel(int64_t N, int K, const double *__restrict__ V,
                                                         CombArgs a, double *__restrict__ y) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < N; t += stride) {
        double acc = a.c[0] * V[t];
        for (int k = 1; k < K; ++k) acc = __builtin_fma(a.c[k], V[(int64_t)k * N + t], acc);
        y[t] = acc;
    }
}

int launch_combine(int64_t N, int K, const double *V, const double *c, double *y, hipStream_t s) {
    if (K < 1 || K > kMaxVecK) return GUESS_EINVAL;
    CombArgs a{};
    for (int k = 0; k < K; ++k) a.c[k] = c[k];
    combine_kernel<<<stream_grid(N, grid_cap()), kBlock, 0, s>>>(N, K, V, a, y);
    return GUESS_OK;
}

// Plain copy with 16-byte accesses (the roofline reference kernel).
__global__ __launch_bounds__(kBlock) void copy_kernel(const d2 *__restrict__ src, d2 *__restrict__ dst,
                                                      int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < n16; t += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + t), dst + t);
}

__global__ void copy_tail_kernel(const unsigned char *src, unsigned char *dst, int64_t off, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[off + t] = src[off + t];
}

int launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 > 0)
        copy_kernel<<<stream_grid(n16, grid_cap()), kBlock, 0, s>>>((const d2 *)src, (d2 *)dst, n16);
    const int64_t tail = (int64_t)(bytes - (size_t)n16 * 16);
    if (tail > 0)
        copy_tail_kernel<<<1, 64, 0, s>>>((const unsigned char *)src, (unsigned char *)dst, n16 * 16, tail);
    return GUESS_OK;
}

// Read-only and write-only references with the same 16-byte non-temporal
// accesses as the copy.  Each thread keeps U accesses in flight per step
// (elements t, t + S, ..., t + (U-1) S of a grid-stride loop of stride U S,
// S = threads in the grid), which a kernel streaming several vectors gets
// from its several streams.  The read kernel sums what it streams (one
// partial per workgroup into out, so no load can be dropped); the write
// kernel fills with a constant.  Grid and U: see launch_read / launch_write.
template <int U>
__global__ __launch_bounds__(kBlock) void read_kernel(const d2 *__restrict__ src, int64_t n16,
                                                      double *__restrict__ out) {
    __shared__ double lds[kLdsDoubles];
    const int64_t S = (int64_t)gridDim.x * kBlock;
    double acc[1] = {0.0};
    double part[U];
#pragma unroll
    for (int u = 0; u < U; ++u) part[u] = 0.0;
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; t + (U - 1) * S < n16; t += U * S) {
        d2 v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = __builtin_nontemporal_load(src + t + u * S);
#pragma unroll
        for (int u = 0; u < U; ++u) part[u] += v[u].x + v[u].y;
    }
    for (; t < n16; t += S) {
        const d2 v = __builtin_nontemporal_load(src + t);
        part[0] += v.x + v.y;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[0] += part[u];
    block_partials<1>(acc, out, lds);
}

// The same read traffic as K separate vectors: `src` taken as K equal
// segments, each thread reading element t of every segment per step of a
// grid-stride loop (the access pattern of a pass that streams K vectors).
template <int K>
__global__ __launch_bounds__(kBlock) void read_streams_kernel(const d2 *__restrict__ src, int64_t seg,
                                                              double *__restrict__ out) {
    __shared__ double lds[kLdsDoubles];
    const int64_t S = (int64_t)gridDim.x * kBlock;
    double acc[1] = {0.0};
    double part[K];
#pragma unroll
    for (int k = 0; k < K; ++k) part[k] = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x; t < seg; t += S) {
        d2 v[K];
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = __builtin_nontemporal_load(src + k * seg + t);
#pragma unroll
        for (int k = 0; k < K; ++k) part[k] += v[k].x + v[k].y;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) acc[0] += part[k];
    block_partials<1>(acc, out, lds);
}

template <int U>
__global__ __launch_bounds__(kBlock) void write_kernel(d2 *__restrict__ dst, int64_t n16, double v) {
    const int64_t S = (int64_t)gridDim.x * kBlock;
    const d2 w{v, v};
    int64_t t = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (; t + (U - 1) * S < n16; t += U * S) {
#pragma unroll
        for (int u = 0; u < U; ++u) __builtin_nontemporal_store(w, dst + t + u * S);
    }
    for (; t < n16; t += S) __builtin_nontemporal_store(w, dst + t);
}

// Launch shapes: the read kernel runs kMaxPartialBlocks workgroups with one
// access in flight per thread and step, the write kernel one workgroup per
// 256 accesses (no loop).  Measured on MI355X over 512 .. 2^20 workgroups and
// 1 .. 8 accesses per step (1 GiB): reads peaked at 6.87 TB/s with about
// 2048 x 256 accesses in flight (twice as many fell to 5.5 TB/s), writes at
// 6.5-6.6 TB/s with the full grid (4.2-5.6 TB/s with 512-65536 workgroups
// looping).  LIBGUESS_ROOF_GRID (workgroups; the read kernel's partial rows
// cap it at kMaxPartialBlocks) and LIBGUESS_ROOF_UNROLL (1, 2, 4 or 8)
// override the shape, for measurements.
static int roof_env(const char *name, int dflt) {
    const char *v = std::getenv(name);
    return (v && *v) ? std::atoi(v) : dflt;
}

int launch_read(const void *src, size_t bytes, double *out, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 <= 0) return GUESS_OK;
    int grid = roof_env("LIBGUESS_ROOF_GRID", kMaxPartialBlocks);
    grid = grid < 1 ? 1 : (grid > kMaxPartialBlocks ? kMaxPartialBlocks : grid);
    grid = stream_grid(n16, grid);
    const d2 *p = (const d2 *)src;
    switch (roof_env("LIBGUESS_ROOF_UNROLL", 1)) {
        case 2: read_kernel<2><<<grid, kBlock, 0, s>>>(p, n16, out); break;
        case 4: read_kernel<4><<<grid, kBlock, 0, s>>>(p, n16, out); break;
        case 8: read_kernel<8><<<grid, kBlock, 0, s>>>(p, n16, out); break;
        default: read_kernel<1><<<grid, kBlock, 0, s>>>(p, n16, out); break;
    }
    return GUESS_OK;
}

// Sixteen streams (the second Gram-Schmidt pass at d = 7 reads 2d + 2) on the
// reduction grid of the guess kernels.
constexpr int kRoofStreams = 16;

int launch_read_streams(const void *src, size_t bytes, double *out, hipStream_t s) {
    const int64_t seg = (int64_t)(bytes / 16) / kRoofStreams;
    if (seg <= 0) return GUESS_OK;
    int grid = roof_env("LIBGUESS_ROOF_GRID", reduce_blocks());
    grid = grid < 1 ? 1 : (grid > kMaxPartialBlocks ? kMaxPartialBlocks : grid);
    grid = stream_grid(seg, grid);
    read_streams_kernel<kRoofStreams><<<grid, kBlock, 0, s>>>((const d2 *)src, seg, out);
    return GUESS_OK;
}

int launch_write(void *dst, size_t bytes, hipStream_t s) {
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 <= 0) return GUESS_OK;
    int grid = roof_env("LIBGUESS_ROOF_GRID", grid_cap());
    grid = stream_grid(n16, grid < 1 ? 1 : grid);
    d2 *p = (d2 *)dst;
    switch (roof_env("LIBGUESS_ROOF_UNROLL", 1)) {
        case 2: write_kernel<2><<<grid, kBlock, 0, s>>>(p, n16, 1.0); break;
        case 4: write_kernel<4><<<grid, kBlock, 0, s>>>(p, n16, 1.0); break;
        case 8: write_kernel<8><<<grid, kBlock, 0, s>>>(p, n16, 1.0); break;
        default: write_kernel<1><<<grid, kBlock, 0, s>>>(p, n16, 1.0); break;
    }
    return GUESS_OK;
}

// b_i = sum_k amp_k Re(ex_k(i) ey_k(j) ez_k(l)) with per-axis complex tables
// ex_k(i) = exp(1i (2 pi kx_k x_i + theta_k)), ey_k(j) = exp(1i 2 pi ky_k y_j),
// ez_k(l) = exp(1i 2 pi kz_k z_l); tables are laid out [k][i] (re, im).
struct AmpArgs {
    double a[kMaxVecK];
};

__global__ __launch_bounds__(kBlock) void plane_wave_kernel(int n, int K, const d2 *__restrict__ tx,
                                                            const d2 *__restrict__ ty,
                                                            const d2 *__restrict__ tz, AmpArgs amp,
                                                            double *__restrict__ b) {
    const int64_t N = (int64_t)n * n * n;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += stride) {
        const int i = (int)(p % n);
        const int j = (int)((p / n) % n);
        const int l = (int)(p / ((int64_t)n * n));
        double acc = 0.0;
        for (int k = 0; k < K; ++k) {
            const d2 ex = tx[(int64_t)k * n + i], ey = ty[(int64_t)k * n + j], ez = tz[(int64_t)k * n + l];
            const double ur = ex.x * ey.x - ex.y * ey.y;
            const double ui = ex.x * ey.y + ex.y * ey.x;
            const double re = ur * ez.x - ui * ez.y;
            acc = __builtin_fma(amp.a[k], re, acc);
        }
        b[p] = acc;
    }
}

int launch_plane_wave_rhs(int n, int K, const double *tabx, const double *taby, const double *tabz,
                          const double *amp, double *b, hipStream_t s) {
    if (K < 1 || K > kMaxVecK) return GUESS_EINVAL;
    AmpArgs a{};
    for (int k = 0; k < K; ++k) a.a[k] = amp[k];
    const int64_t N = (int64_t)n * n * n;
    plane_wave_kernel<<<stream_grid(N, grid_cap()), kBlock, 0, s>>>(n, K, (const d2 *)tabx, (const d2 *)taby,
                                                                    (const d2 *)tabz, a, b);
    return GUESS_OK;
}

// Moving Gaussian source: per-axis tables g_a(i) = exp(-(x_i - c_a)^2 / (2 sigma^2)),
// x_i = (i + 1) / (n + 1), then b = amp * (g_x(i) * (g_y(j) * g_z(l))).
__global__ void gaussian_tables_kernel(int n, double cx, double cy, double cz, double inv2s2, double *tab) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3 * n) return;
    const int axis = t / n, i = t - axis * n;
    const double x = (i + 1) * (1.0 / (n + 1));
    const double c = axis == 0 ? cx : (axis == 1 ? cy : cz);
    const double d = x - c;
    tab[t] = exp(-(d * d) * inv2s2);
}

__global__ __launch_bounds__(kBlock) void gaussian_rhs_kernel(int n, const double *__restrict__ tab, double amp,
                                                             double *__restrict__ b) {
    const int64_t N = (int64_t)n * n * n;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t p = (int64_t)blockIdx.x * kBlock + threadIdx.x; p < N; p += stride) {
        const int i = (int)(p % n);
        const int j = (int)((p / n) % n);
        const int l = (int)(p / ((int64_t)n * n));
        b[p] = amp * (tab[i] * (tab[n + j] * tab[2 * n + l]));
    }
}

int launch_gaussian_rhs(int n, const double *center, double sigma, double amp, double *tab, double *b,
                        hipStream_t s) {
    const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
    gaussian_tables_kernel<<<(3 * n + 255) / 256, 256, 0, s>>>(n, center[0], center[1], center[2], inv2s2, tab);
    const int64_t N = (int64_t)n * n * n;
    gaussian_rhs_kernel<<<stream_grid(N, grid_cap()), kBlock, 0, s>>>(n, tab, amp, b);
    return GUESS_OK;
}

}  // namespace lg
