// Polynomial-extrapolation guess kernels (§3, eq. ExtrapExpn).
//
// extrap_form:  x0 = sum_{j<k} beta_j h_j, h_0 the oldest stored solution.
//   One pass over the k ring slots and one FP64 store: (k s + 8) bytes per
//   unknown, s the stored element size.  Each thread streams 4 consecutive
//   unknowns of every slot (all k loads issued before the FMA chain), with
//   non-temporal hints since nothing is reused.  FP64 history accumulates in
//   FP64; FP32/FP16/BF16 history is widened and accumulated in FP32.  An FP16
//   slot holds round(2^e x) with its own exponent e, so its weight enters the
//   FP32 sum as beta_j 2^-e (exact: a power of two).
// ring_store:   slot <- round(x): 8 + s bytes per unknown.  FP16 slots store
//   round(2^e x), e from max |x| (max |x| 2^e in [2^14, 2^15)): the store
//   tries the previous slot's exponent while reducing max |x|, and a second
//   kernel re-stores the slot (another 8 + s bytes per unknown) only when
//   the exponent of this solution differs -- rarely, for a slowly varying
//   sequence.
#include "common.h"
#include "launch.h"

namespace lg {

struct ExtrapArgs {
    const void *slot[GUESS_MAX_M];
    double beta[GUESS_MAX_M];
    const RingState *rs;      // FP16: per-slot exponents
    int sidx[GUESS_MAX_M];    // FP16: physical slot index of slot[j]
};

// Weight of slot j in the FP32 accumulation.
template <int DT>
__device__ __forceinline__ float fp32_weight(const ExtrapArgs &a, int j) {
    if constexpr (DT == GUESS_F16) return (float)ldexp(a.beta[j], -a.rs->exps[a.sidx[j]]);
    else return (float)a.beta[j];
}

template <int DT, int K>
__global__ __launch_bounds__(kBlock) void extrap_form_kernel(ExtrapArgs a, double *__restrict__ x0,
                                                             int64_t N) {
    const int64_t nc = nchunks(N);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    float bw[DT == GUESS_F64 ? 1 : K];
    if constexpr (DT != GUESS_F64) {
#pragma unroll
        for (int j = 0; j < K; ++j) bw[j] = fp32_weight<DT>(a, j);
    }
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
        if constexpr (DT == GUESS_F64) {
            V4 h[K];
#pragma unroll
            for (int j = 0; j < K; ++j) h[j] = load4<DT>(a.slot[j], c);
            V4 acc;
#pragma unroll
            for (int e = 0; e < 4; ++e) acc.v[e] = a.beta[0] * h[0].v[e];
#pragma unroll
            for (int j = 1; j < K; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc.v[e] = __builtin_fma(a.beta[j], h[j].v[e], acc.v[e]);
            store4<GUESS_F64>(x0, c, acc);
        } else {
            F4 h[K];
#pragma unroll
            for (int j = 0; j < K; ++j) h[j] = load4f<DT>(a.slot[j], c);
            float acc[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[e] = bw[0] * h[0].v[e];
#pragma unroll
            for (int j = 1; j < K; ++j) {
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[e] = __builtin_fmaf(bw[j], h[j].v[e], acc[e]);
            }
            V4 out{{(double)acc[0], (double)acc[1], (double)acc[2], (double)acc[3]}};
            store4<GUESS_F64>(x0, c, out);
        }
    }
    // ragged tail (the N mod 256 unknowns past the last full tile), same arithmetic
    const int rem = tail_count(N);
    if (blockIdx.x == 0 && threadIdx.x < rem) {
        const int64_t i = tail_start(N) + threadIdx.x;
        if constexpr (DT == GUESS_F64) {
            double acc = a.beta[0] * load1<DT>(a.slot[0], i);
            for (int j = 1; j < K; ++j) acc = __builtin_fma(a.beta[j], load1<DT>(a.slot[j], i), acc);
            x0[i] = acc;
        } else {
            float acc = bw[0] * (float)load1<DT>(a.slot[0], i);
            for (int j = 1; j < K; ++j) acc = __builtin_fmaf(bw[j], (float)load1<DT>(a.slot[j], i), acc);
            x0[i] = (double)acc;
        }
    }
}

template <int DT>
__global__ __launch_bounds__(kBlock) void ring_store_kernel(const double *__restrict__ x,
                                                            void *__restrict__ slot, int64_t N) {
    const int64_t nc = nchunks(N);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride)
        store4<DT>(slot, c, load4<GUESS_F64>(x, c));
    const int rem = tail_count(N);
    if (blockIdx.x == 0 && threadIdx.x < rem) {
        const int64_t i = tail_start(N) + threadIdx.x;
        store1<DT>(slot, i, x[i]);
    }
}

// slot <- round(2^e x) over the whole vector; returns this thread's max |x|
__device__ __forceinline__ double f16_scaled_store(const double *__restrict__ x, void *__restrict__ slot,
                                                   int64_t N, int e) {
    const int64_t nc = nchunks(N);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const double pw = ldexp(1.0, e);
    double mx = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
        V4 v = load4<GUESS_F64>(x, c);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            mx = nanmax(mx, fabs(v.v[q]));
            v.v[q] *= pw;
        }
        store4<GUESS_F16>(slot, c, v);
    }
    const int rem = tail_count(N);
    if (blockIdx.x == 0 && threadIdx.x < rem) {
        const int64_t i = tail_start(N) + threadIdx.x;
        mx = nanmax(mx, fabs(x[i]));
        store1<GUESS_F16>(slot, i, x[i] * pw);
    }
    return mx;
}

// FP16 store, first kernel: the previous store's exponent, max |x| reduced
// into rs->maxbits[gen] (non-negative doubles order like their bit patterns,
// a NaN above everything, so an integer max of the bits is the NaN-propagating
// max).  rs->maxbits[gen] is zero on entry: the previous store cleared it.
__global__ __launch_bounds__(kBlock) void ring_store_f16_kernel(const double *__restrict__ x,
                                                                void *__restrict__ slot, int64_t N,
                                                                RingState *rs, int gen) {
    __shared__ double wmax[kWaves];
    const int e = rs->e_guess;
    const double mx = wave_nanmax(f16_scaled_store(x, slot, N, e));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) m = nanmax(m, wmax[w]);
        // the running maximum only grows: a workgroup whose maximum does not exceed a value it
        // reads there has nothing to add (a stale read costs one atomic, never a wrong result)
        const unsigned long long mb = (unsigned long long)__double_as_longlong(m);
        if (mb > __hip_atomic_load(&rs->maxbits[gen], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
            atomicMax(&rs->maxbits[gen], mb);
        if (blockIdx.x == 0) {
            rs->e_used[gen] = e;
            rs->maxbits[gen ^ 1] = 0ull;   // the next store's accumulator
        }
    }
}

// FP16 store, second kernel: the exponent of this solution; the slot is
// written again only when it differs from the one the first kernel used.
__global__ __launch_bounds__(kBlock) void ring_fix_f16_kernel(const double *__restrict__ x,
                                                              void *__restrict__ slot, int64_t N,
                                                              RingState *rs, int gen, int sidx) {
    const int e = f16_scale_exp(__longlong_as_double((long long)rs->maxbits[gen]));
    const int eu = rs->e_used[gen];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        rs->exps[sidx] = e;
        rs->e_guess = e;
        rs->last_fixed = e != eu ? 1 : 0;
        if (e != eu) rs->fixes += 1;
    }
    if (e == eu) return;
    (void)f16_scaled_store(x, slot, N, e);
}

__global__ __launch_bounds__(kBlock) void fill_zero_kernel(double *__restrict__ x, int64_t N) {
    const int64_t nc = nchunks(N);
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    const V4 z{{0.0, 0.0, 0.0, 0.0}};
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride)
        store4<GUESS_F64>(x, c, z);
    const int rem = tail_count(N);
    if (blockIdx.x == 0 && threadIdx.x < rem) x[tail_start(N) + threadIdx.x] = 0.0;
}

template <int DT>
__global__ __launch_bounds__(kBlock) void widen_kernel(const void *__restrict__ src, double scale,
                                                       double *__restrict__ out, int64_t N) {
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < N; i += stride)
        out[i] = scale * load1<DT>(src, i);
}

int launch_widen(int dtype, const void *src, double scale, double *out, int64_t N, hipStream_t s) {
    const int grid = stream_grid(N, grid_cap());
    switch (dtype) {
        case GUESS_F64: widen_kernel<GUESS_F64><<<grid, kBlock, 0, s>>>(src, scale, out, N); break;
        case GUESS_F32: widen_kernel<GUESS_F32><<<grid, kBlock, 0, s>>>(src, scale, out, N); break;
        case GUESS_F16: widen_kernel<GUESS_F16><<<grid, kBlock, 0, s>>>(src, scale, out, N); break;
        case GUESS_BF16: widen_kernel<GUESS_BF16><<<grid, kBlock, 0, s>>>(src, scale, out, N); break;
        default: return GUESS_EINVAL;
    }
    return GUESS_OK;
}

template <int DT, int K>
static void run_form(const ExtrapArgs &a, double *x0, int64_t N, int grid, hipStream_t s, KEvents *ev) {
    klaunch_sh(ev, 0, extrap_form_kernel<DT, K>, grid, kBlock, gather_lds(), s, a, x0, N);
}

template <int DT>
static int form_dt(int k, const ExtrapArgs &a, double *x0, int64_t N, int grid, hipStream_t s, KEvents *ev) {
    switch (k) {
#define LG_K(KK) case KK: run_form<DT, KK>(a, x0, N, grid, s, ev); break;
        LG_K(1) LG_K(2) LG_K(3) LG_K(4) LG_K(5) LG_K(6) LG_K(7) LG_K(8)
        LG_K(9) LG_K(10) LG_K(11) LG_K(12) LG_K(13) LG_K(14) LG_K(15) LG_K(16)
#undef LG_K
        default: return GUESS_EINVAL;
    }
    return GUESS_OK;
}

int launch_extrap_form(int dtype, int k, const void *const *slots, const double *beta, double *x0,
                       int64_t N, hipStream_t s, KEvents *ev, const RingState *rs, const int *slot_index) {
    if (k < 1 || k > GUESS_MAX_M) return GUESS_EINVAL;
    if (dtype == GUESS_F16 && (!rs || !slot_index)) return GUESS_EINVAL;
    ExtrapArgs a{};
    a.rs = rs;
    for (int j = 0; j < k; ++j) {
        a.slot[j] = slots[j];
        a.beta[j] = beta[j];
        a.sidx[j] = slot_index ? slot_index[j] : 0;
    }
    const int grid = stream_grid(nchunks(N), grid_cap());
    switch (dtype) {
        case GUESS_F64: return form_dt<GUESS_F64>(k, a, x0, N, grid, s, ev);
        case GUESS_F32: return form_dt<GUESS_F32>(k, a, x0, N, grid, s, ev);
        case GUESS_F16: return form_dt<GUESS_F16>(k, a, x0, N, grid, s, ev);
        case GUESS_BF16: return form_dt<GUESS_BF16>(k, a, x0, N, grid, s, ev);
    }
    return GUESS_EINVAL;
}

int launch_ring_store(int dtype, const double *x, void *slot, int64_t N, hipStream_t s, KEvents *ev,
                      RingState *rs, int slot_index, int gen) {
    const int grid = stream_grid(nchunks(N), grid_cap());
    switch (dtype) {
        case GUESS_F64: klaunch(ev, 0, ring_store_kernel<GUESS_F64>, grid, kBlock, s, x, slot, N); break;
        case GUESS_F32: klaunch(ev, 0, ring_store_kernel<GUESS_F32>, grid, kBlock, s, x, slot, N); break;
        case GUESS_F16:
            if (!rs || (gen != 0 && gen != 1)) return GUESS_EINVAL;
            // one atomic max per workgroup, all on one word: the reduction grid keeps them few
            // (one per workgroup of the full grid took the store from 30 to 190 us at 256^3)
            klaunch(ev, 0, ring_store_f16_kernel, stream_grid(nchunks(N), reduce_blocks()), kBlock, s, x, slot, N,
                    rs, gen);
            klaunch(ev, 1, ring_fix_f16_kernel, grid, kBlock, s, x, slot, N, rs, gen, slot_index);
            break;
        case GUESS_BF16: klaunch(ev, 0, ring_store_kernel<GUESS_BF16>, grid, kBlock, s, x, slot, N); break;
        default: return GUESS_EINVAL;
    }
    return GUESS_OK;
}

int launch_fill_zero(double *x, int64_t N, hipStream_t s) {
    fill_zero_kernel<<<stream_grid(nchunks(N), grid_cap()), kBlock, 0, s>>>(x, N);
    return GUESS_OK;
}

}  // namespace lg
