// Device-side building blocks shared by the libguess kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "libguess.h"

namespace lg {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64s)

// Reduction kernels stream several vectors per step: allow up to 128 VGPRs
// (4 waves per SIMD) so that every load of a step is in flight at once.
#ifndef LG_WAVES_MIN
#define LG_WAVES_MIN 1
#endif
#ifndef LG_WAVES_MAX
#define LG_WAVES_MAX 4
#endif
#define LG_REDUCE_KERNEL \
    __global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(LG_WAVES_MIN, LG_WAVES_MAX)))
constexpr int kWaves = kBlock / 64;
constexpr int kMaxPartialBlocks = 2048;
constexpr int kMaxDots = 2 * GUESS_MAX_M + 4;
constexpr int kPartialDoubles = kMaxPartialBlocks * kMaxDots;   // capacity of a partial-row buffer

// ------------------------------------------------------------------ storage types
// DT: GUESS_F64 / F32 / F16 / BF16.  Stored element type and conversions.
template <int DT> struct Elem;
template <> struct Elem<GUESS_F64> { using T = double; };
template <> struct Elem<GUESS_F32> { using T = float; };
template <> struct Elem<GUESS_F16> { using T = _Float16; };
template <> struct Elem<GUESS_BF16> { using T = uint16_t; };

// FP32 -> BF16 bits, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_bits_to_f32(uint16_t b) {
    return __uint_as_float(((uint32_t)b) << 16);
}

// Round an FP64 value into storage format DT (two-step FP64 -> FP32 -> DT).
template <int DT> __device__ __forceinline__ typename Elem<DT>::T to_store(double v);
template <> __device__ __forceinline__ double to_store<GUESS_F64>(double v) { return v; }
template <> __device__ __forceinline__ float to_store<GUESS_F32>(double v) { return (float)v; }
template <> __device__ __forceinline__ _Float16 to_store<GUESS_F16>(double v) {
    // The FP32 value is made opaque so that the compiler cannot merge the two
    // conversions into one direct FP64 -> FP16 rounding (which differs from
    // the two-step rounding when the FP32 value lands on an FP16 midpoint).
    // Not volatile: the empty asm has no side effects, so it does not hold
    // back the scheduling of the loads and stores around it.
    float f = (float)v;
    asm("" : "+v"(f));
    return (_Float16)f;
}
template <> __device__ __forceinline__ uint16_t to_store<GUESS_BF16>(double v) {
    return f32_to_bf16_bits((float)v);
}

// Widen a stored element to FP32 / FP64 (exact).
template <int DT> __device__ __forceinline__ float to_f32(typename Elem<DT>::T v);
template <> __device__ __forceinline__ float to_f32<GUESS_F32>(float v) { return v; }
template <> __device__ __forceinline__ float to_f32<GUESS_F16>(_Float16 v) { return (float)v; }
template <> __device__ __forceinline__ float to_f32<GUESS_BF16>(uint16_t v) {
    return bf16_bits_to_f32(v);
}
template <int DT> __device__ __forceinline__ double to_f64(typename Elem<DT>::T v) {
    return (double)to_f32<DT>(v);
}
template <> __device__ __forceinline__ double to_f64<GUESS_F64>(double v) { return v; }

// ------------------------------------------------------------------ work split
// Vectors are processed in tiles of 256 consecutive elements, one tile per
// wave and step.  Lane L of the wave owns the element pairs (2L, 2L+1) and
// (128+2L, 129+2L) of the tile -- its "chunk" -- so that every load or store
// instruction of the wave covers one contiguous range (1 KiB for FP64).
// Elements past the last full tile (N mod 256 of them) form the ragged tail
// and are handled one per thread by workgroup 0.
__host__ __device__ __forceinline__ int64_t nchunks(int64_t N) { return (N >> 8) << 6; }
__host__ __device__ __forceinline__ int64_t tail_start(int64_t N) { return (N >> 8) << 8; }
__host__ __device__ __forceinline__ int tail_count(int64_t N) { return (int)(N & 255); }
// first element of chunk c's first pair; the second pair starts 128 later
__device__ __forceinline__ int64_t chunk_elem(int64_t c) { return ((c >> 6) << 8) + ((c & 63) << 1); }

// XCD-aware split for stencil kernels.  Workgroups are dealt to the 8 XCDs
// round-robin (workgroup b runs on XCD b mod 8), and each XCD has its own
// L2.  Giving XCD k one contiguous eighth of the chunks (a z-slab of the
// grid) that its workgroups sweep together keeps the z-1 / z+1 planes a
// stencil reads in that XCD's L2 instead of another XCD's.
constexpr int kXcds = 8;
struct ChunkRange {
    int64_t begin, end, step;
};
__device__ __forceinline__ ChunkRange xcd_range(int64_t nc) {
    const int g = gridDim.x;
    if (g % kXcds != 0) return ChunkRange{(int64_t)blockIdx.x * 256 + threadIdx.x, nc, (int64_t)g * 256};
    const int xcd = blockIdx.x % kXcds, local = blockIdx.x / kXcds, per = g / kXcds;
    const int64_t span = (nc + kXcds * 64 - 1) / (kXcds * 64) * 64;   // multiple of a wave's 64 chunks
    const int64_t b = (int64_t)xcd * span;
    const int64_t e = b + span < nc ? b + span : nc;
    return ChunkRange{b + (int64_t)local * 256 + threadIdx.x, e, (int64_t)per * 256};
}

typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f2 __attribute__((ext_vector_type(2)));
typedef _Float16 h2 __attribute__((ext_vector_type(2)));

// The 4 values of a chunk, in the order (2L, 2L+1, 128+2L, 129+2L).
struct V4 { double v[4]; };
struct F4 { float v[4]; };

template <int DT> struct Pair;
template <> struct Pair<GUESS_F64> { using T = d2; };
template <> struct Pair<GUESS_F32> { using T = f2; };
template <> struct Pair<GUESS_F16> { using T = h2; };
template <> struct Pair<GUESS_BF16> { using T = uint32_t; };

template <int DT>
__device__ __forceinline__ typename Pair<DT>::T ldpair(const void *p, int64_t e) {
    using T = typename Pair<DT>::T;
    return __builtin_nontemporal_load(reinterpret_cast<const T *>(p) + (e >> 1));
}
template <int DT>
__device__ __forceinline__ void stpair(void *p, int64_t e, typename Pair<DT>::T v) {
    using T = typename Pair<DT>::T;
    __builtin_nontemporal_store(v, reinterpret_cast<T *>(p) + (e >> 1));
}

template <int DT> __device__ __forceinline__ void widen2(typename Pair<DT>::T v, float &a, float &b);
template <> __device__ __forceinline__ void widen2<GUESS_F32>(f2 v, float &a, float &b) { a = v.x; b = v.y; }
template <> __device__ __forceinline__ void widen2<GUESS_F16>(h2 v, float &a, float &b) {
    a = (float)v.x;
    b = (float)v.y;
}
template <> __device__ __forceinline__ void widen2<GUESS_BF16>(uint32_t v, float &a, float &b) {
    a = __uint_as_float(v << 16);
    b = __uint_as_float(v & 0xffff0000u);
}

template <int DT>
__device__ __forceinline__ V4 load4(const void *p, int64_t c) {
    const int64_t e = chunk_elem(c);
    if constexpr (DT == GUESS_F64) {
        const d2 a = ldpair<DT>(p, e), b = ldpair<DT>(p, e + 128);
        return V4{{a.x, a.y, b.x, b.y}};
    } else {
        float a0, a1, b0, b1;
        widen2<DT>(ldpair<DT>(p, e), a0, a1);
        widen2<DT>(ldpair<DT>(p, e + 128), b0, b1);
        return V4{{(double)a0, (double)a1, (double)b0, (double)b1}};
    }
}

// FP32 view of a chunk of reduced-precision storage (FP32-accumulating kernels).
template <int DT>
__device__ __forceinline__ F4 load4f(const void *p, int64_t c) {
    const int64_t e = chunk_elem(c);
    F4 r;
    widen2<DT>(ldpair<DT>(p, e), r.v[0], r.v[1]);
    widen2<DT>(ldpair<DT>(p, e + 128), r.v[2], r.v[3]);
    return r;
}

template <int DT>
__device__ __forceinline__ typename Pair<DT>::T narrow2(double a, double b) {
    if constexpr (DT == GUESS_F64) return d2{a, b};
    else if constexpr (DT == GUESS_F32) return f2{(float)a, (float)b};
    else if constexpr (DT == GUESS_F16) return h2{to_store<GUESS_F16>(a), to_store<GUESS_F16>(b)};
    else return (uint32_t)to_store<GUESS_BF16>(a) | ((uint32_t)to_store<GUESS_BF16>(b) << 16);
}

template <int DT>
__device__ __forceinline__ void store4(void *p, int64_t c, const V4 &x) {
    const int64_t e = chunk_elem(c);
    stpair<DT>(p, e, narrow2<DT>(x.v[0], x.v[1]));
    stpair<DT>(p, e + 128, narrow2<DT>(x.v[2], x.v[3]));
}

// Scalar element access (ragged tails).
template <int DT> __device__ __forceinline__ double load1(const void *p, int64_t i) {
    return to_f64<DT>(reinterpret_cast<const typename Elem<DT>::T *>(p)[i]);
}
template <int DT> __device__ __forceinline__ void store1(void *p, int64_t i, double v) {
    reinterpret_cast<typename Elem<DT>::T *>(p)[i] = to_store<DT>(v);
}

// ------------------------------------------------------------------ reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// LDS scratch that a kernel passes to the reduction helpers below.
constexpr int kLdsDoubles = kWaves * kMaxDots + kMaxDots;

// Largest of two magnitudes, NaN-propagating (a NaN anywhere gives NaN).
__device__ __forceinline__ double nanmax(double a, double b) { return (a != a || a > b) ? a : b; }
__device__ __forceinline__ double wave_nanmax(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = nanmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Reduce ND per-thread values over the workgroup -- values j < NS by sum,
// the others (magnitudes) by NaN-propagating max; thread j < ND of the
// block writes the block's result for value j to part[blockIdx.x * ND + j].
// The order of additions is fixed, so results do not depend on timing.
template <int ND, int NS = ND>
__device__ __forceinline__ void block_partials(const double (&v)[ND], double *part, double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        double s = j < NS ? wave_sum(v[j]) : wave_nanmax(v[j]);
        if (lane == 0) lds[wave * ND + j] = s;
    }
    __syncthreads();
    if (threadIdx.x < ND) {
        const bool sum = (int)threadIdx.x < NS;
        double s = lds[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s = sum ? s + lds[w * ND + threadIdx.x] : nanmax(s, lds[w * ND + threadIdx.x]);
        part[(int64_t)blockIdx.x * ND + threadIdx.x] = s;
    }
    __syncthreads();
}

// Result for value j over nb partial rows (written by an earlier kernel),
// summed (j < NS) or max-reduced (j >= NS) in a fixed order (thread t takes
// rows t, t+256, ...; then a fixed tree), so every workgroup that calls it
// obtains identical totals.  Every thread of the workgroup receives all ND
// results.
template <int ND, int NS = ND>
__device__ __forceinline__ void final_sums(const double *part, int nb, double (&tot)[ND],
                                           double *lds) {
    double v[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) v[j] = 0.0;
    int r = threadIdx.x;
    // four rows in flight per thread, combined in row order
    for (; r + 3 * kBlock < nb; r += 4 * kBlock) {
        double x[4][ND];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < ND; ++j) x[q][j] = __builtin_nontemporal_load(part + (int64_t)(r + q * kBlock) * ND + j);
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < ND; ++j) v[j] = j < NS ? v[j] + x[q][j] : nanmax(v[j], x[q][j]);
    }
    for (; r < nb; r += kBlock) {
        const double *row = part + (int64_t)r * ND;
#pragma unroll
        for (int j = 0; j < ND; ++j) {
            const double x = __builtin_nontemporal_load(row + j);
            v[j] = j < NS ? v[j] + x : nanmax(v[j], x);
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        double s = j < NS ? wave_sum(v[j]) : wave_nanmax(v[j]);
        if (lane == 0) lds[wave * ND + j] = s;
    }
    __syncthreads();
    double *out = lds + kWaves * kMaxDots;
    if (threadIdx.x < ND) {
        const bool sum = (int)threadIdx.x < NS;
        double s = lds[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s = sum ? s + lds[w * ND + threadIdx.x] : nanmax(s, lds[w * ND + threadIdx.x]);
        out[threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ND; ++j) tot[j] = out[j];
}

// Power-of-two exponent e that brings a largest magnitude m into
// [2^14, 2^15) (FP16 storage: the stored values of a vector then stay well
// inside FP16's normal range and cannot overflow).  m = f 2^E, f in
// [0.5, 1), gives e = 15 - E, clamped to [-100, 100]; zero or non-finite m
// gives 0.
constexpr int kF16ExpClamp = 100;
__host__ __device__ __forceinline__ int f16_scale_exp(double m) {
    if (!(m > 0.0) || !(m <= 1.7976931348623157e308)) return 0;
    int E = 0;
    (void)frexp(m, &E);
    int e = 15 - E;
    return e < -kF16ExpClamp ? -kF16ExpClamp : (e > kF16ExpClamp ? kF16ExpClamp : e);
}

// Value an FP64 magnitude takes once stored in FP16 (two-step rounding),
// widened back to FP64.
__device__ __forceinline__ double f16_rounded(double v) { return to_f64<GUESS_F16>(to_store<GUESS_F16>(v)); }

// Call f(std::integral_constant<int, D>) for the runtime value d in [LO, HI].
template <int LO, int HI, class F>
__device__ __forceinline__ void dispatch_d(int d, F &&f) {
    if constexpr (LO <= HI) {
        if (d == LO) {
            f(std::integral_constant<int, LO>{});
            return;
        }
        dispatch_d<LO + 1, HI>(d, f);
    }
}

// ------------------------------------------------------------------ launch shapes
// Grid for a grid-stride streaming loop over `chunks` work items.
inline int stream_grid(int64_t chunks, int cap) {
    int64_t g = (chunks + kBlock - 1) / kBlock;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

}  // namespace lg
