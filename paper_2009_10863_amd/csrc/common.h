// Device-side building blocks shared by the libguess kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "libguess.h"

namespace lg {

constexpr int kBlock = 256;          // threads per workgroup (4 wave64s)
constexpr int kWaves = kBlock / 64;
constexpr int kMaxPartialBlocks = 2048;
constexpr int kMaxDots = 2 * GUESS_MAX_M + 4;

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
    return (_Float16)(float)v;
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

// ------------------------------------------------------------------ 4-wide access
// Every streaming kernel moves 4 consecutive elements per thread and step:
// 32 B of FP64, 16 B of FP32, 8 B of FP16/BF16.  Pointers are 16-B aligned.
typedef double d2 __attribute__((ext_vector_type(2)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u2 __attribute__((ext_vector_type(2)));

struct V4 { double v[4]; };

template <int DT> __device__ __forceinline__ V4 load4(const void *p, int64_t c);
template <> __device__ __forceinline__ V4 load4<GUESS_F64>(const void *p, int64_t c) {
    const d2 *q = reinterpret_cast<const d2 *>(p) + 2 * c;
    d2 a = __builtin_nontemporal_load(q), b = __builtin_nontemporal_load(q + 1);
    return V4{{a.x, a.y, b.x, b.y}};
}
template <> __device__ __forceinline__ V4 load4<GUESS_F32>(const void *p, int64_t c) {
    f4 a = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p) + c);
    return V4{{(double)a.x, (double)a.y, (double)a.z, (double)a.w}};
}
template <> __device__ __forceinline__ V4 load4<GUESS_F16>(const void *p, int64_t c) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    h4 a = __builtin_nontemporal_load(reinterpret_cast<const h4 *>(p) + c);
    return V4{{(double)(float)a.x, (double)(float)a.y, (double)(float)a.z, (double)(float)a.w}};
}
template <> __device__ __forceinline__ V4 load4<GUESS_BF16>(const void *p, int64_t c) {
    u2 a = __builtin_nontemporal_load(reinterpret_cast<const u2 *>(p) + c);
    return V4{{(double)__uint_as_float(a.x << 16), (double)__uint_as_float(a.x & 0xffff0000u),
               (double)__uint_as_float(a.y << 16), (double)__uint_as_float(a.y & 0xffff0000u)}};
}

// FP32 view of 4 stored elements (for FP32-accumulating kernels).
struct F4 { float v[4]; };
template <int DT> __device__ __forceinline__ F4 load4f(const void *p, int64_t c);
template <> __device__ __forceinline__ F4 load4f<GUESS_F32>(const void *p, int64_t c) {
    f4 a = __builtin_nontemporal_load(reinterpret_cast<const f4 *>(p) + c);
    return F4{{a.x, a.y, a.z, a.w}};
}
template <> __device__ __forceinline__ F4 load4f<GUESS_F16>(const void *p, int64_t c) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    h4 a = __builtin_nontemporal_load(reinterpret_cast<const h4 *>(p) + c);
    return F4{{(float)a.x, (float)a.y, (float)a.z, (float)a.w}};
}
template <> __device__ __forceinline__ F4 load4f<GUESS_BF16>(const void *p, int64_t c) {
    u2 a = __builtin_nontemporal_load(reinterpret_cast<const u2 *>(p) + c);
    return F4{{__uint_as_float(a.x << 16), __uint_as_float(a.x & 0xffff0000u),
               __uint_as_float(a.y << 16), __uint_as_float(a.y & 0xffff0000u)}};
}

template <int DT> __device__ __forceinline__ void store4(void *p, int64_t c, const V4 &x);
template <> __device__ __forceinline__ void store4<GUESS_F64>(void *p, int64_t c, const V4 &x) {
    d2 *q = reinterpret_cast<d2 *>(p) + 2 * c;
    d2 a = {x.v[0], x.v[1]}, b = {x.v[2], x.v[3]};
    __builtin_nontemporal_store(a, q);
    __builtin_nontemporal_store(b, q + 1);
}
template <> __device__ __forceinline__ void store4<GUESS_F32>(void *p, int64_t c, const V4 &x) {
    f4 a = {(float)x.v[0], (float)x.v[1], (float)x.v[2], (float)x.v[3]};
    __builtin_nontemporal_store(a, reinterpret_cast<f4 *>(p) + c);
}
template <> __device__ __forceinline__ void store4<GUESS_F16>(void *p, int64_t c, const V4 &x) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    h4 a = {to_store<GUESS_F16>(x.v[0]), to_store<GUESS_F16>(x.v[1]),
            to_store<GUESS_F16>(x.v[2]), to_store<GUESS_F16>(x.v[3])};
    __builtin_nontemporal_store(a, reinterpret_cast<h4 *>(p) + c);
}
template <> __device__ __forceinline__ void store4<GUESS_BF16>(void *p, int64_t c, const V4 &x) {
    u2 a;
    a.x = (uint32_t)to_store<GUESS_BF16>(x.v[0]) | ((uint32_t)to_store<GUESS_BF16>(x.v[1]) << 16);
    a.y = (uint32_t)to_store<GUESS_BF16>(x.v[2]) | ((uint32_t)to_store<GUESS_BF16>(x.v[3]) << 16);
    __builtin_nontemporal_store(a, reinterpret_cast<u2 *>(p) + c);
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

// Sum ND per-thread values over the workgroup; thread j < ND of the block
// writes the block's total of value j to part[blockIdx.x * ND + j].
// The order of additions is fixed, so results do not depend on timing.
template <int ND>
__device__ __forceinline__ void block_partials(const double (&v)[ND], double *part, double *lds) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        double s = wave_sum(v[j]);
        if (lane == 0) lds[wave * ND + j] = s;
    }
    __syncthreads();
    if (threadIdx.x < ND) {
        double s = lds[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s += lds[w * ND + threadIdx.x];
        part[(int64_t)blockIdx.x * ND + threadIdx.x] = s;
    }
    __syncthreads();
}

// True in exactly one workgroup: the last to arrive.  All partial results
// written before the call by every workgroup are visible to it afterwards.
// The last workgroup re-arms the ticket for the next launch.
__device__ __forceinline__ bool last_block(unsigned int *ticket) {
    __shared__ int is_last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned int t = atomicAdd(ticket, 1u);
        is_last = (t == gridDim.x - 1);
        if (is_last) atomicExch(ticket, 0u);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last != 0;
}

// In the last workgroup: total of value j over all nb partial rows, summed in
// a fixed order (thread t takes rows t, t+256, ...; then a fixed tree).
// Every thread of the workgroup receives all ND totals.
template <int ND>
__device__ __forceinline__ void final_sums(const double *part, int nb, double (&tot)[ND],
                                           double *lds) {
    double v[ND];
#pragma unroll
    for (int j = 0; j < ND; ++j) v[j] = 0.0;
    for (int r = threadIdx.x; r < nb; r += kBlock) {
        const double *row = part + (int64_t)r * ND;
#pragma unroll
        for (int j = 0; j < ND; ++j) v[j] += __builtin_nontemporal_load(row + j);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int j = 0; j < ND; ++j) {
        double s = wave_sum(v[j]);
        if (lane == 0) lds[wave * ND + j] = s;
    }
    __syncthreads();
    double *out = lds + kWaves * kMaxDots;
    if (threadIdx.x < ND) {
        double s = lds[threadIdx.x];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) s += lds[w * ND + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < ND; ++j) tot[j] = out[j];
}

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
