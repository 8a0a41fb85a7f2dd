// Projection guess through the Gram matrix of the stored raw solutions (§2).
//
// The guess of §2 is the A-norm-optimal combination of the stored
// solutions W.  Algorithms 1 and 2 reach it through an A-orthonormal basis
// built by Gram-Schmidt; in exact arithmetic the same guess is
// x0 = W y with G y = W^T b, G = W^T A W, and the rejection test's norm is
// nu^2 = w^T A w - g^T G^{-1} g, g = W^T A w (the Schur complement of the
// extended Gram matrix).  This form stores the solutions themselves, rounded
// to the storage format (FP16: round(2^e x), e from max |x|), and keeps G
// and its Cholesky factor L (G = L L^T) in FP64 on the device, A applied to
// each stored vector: the guess is then the A-norm-optimal combination of
// what is stored, with no normalised column whose rounding near-dependence
// could magnify.  The history is bounded like Algorithms 1 and 2: classic
// restarts or the rolling window (drop the oldest solution).  X = W L^-T is
// the A-orthonormal basis of the Gram-Schmidt forms, and L^T is their factor
// R (raw solutions = X R).
//
// Columns live in M physical slots; perm[j] is the slot of the j-th oldest
// solution, so a rolling drop moves no data.  Kernels (bytes per unknown,
// s the stored element size, d the number of stored solutions):
//   raw_store   slot <- round(2^e x) (e: the previous store's exponent)     8 + s
//   raw_fix     FP16: the slot again with this solution's exponent when it  0 or 8 + s
//               differs (max |x| is reduced by raw_store)
//   raw_apply   A w on the stored vector (z-marching or chunk stencil),     (d + 1) s
//               fused with g = W^T A w and w^T A w
//   raw_fin     one workgroup: restart / drop, Schur complement with L, accept, G and L
//   raw_dots    c = W^T b                                                   d s + 8
//   raw_solve   one workgroup: G y = c through L
//   raw_combine x0 = W y                                                    d s + 8
#pragma once

#include "common.h"
#include "launch.h"
#include "march.h"

namespace lg {

struct RawArgs {
    void *W;                 // M slots of N elements of the storage type
    double *part;
    RawState *st;
    int64_t N, ld;
    int M, qr;
};

template <int DT>
__device__ __forceinline__ typename Elem<DT>::T *slotp(void *W, int64_t ld, int s) {
    return reinterpret_cast<typename Elem<DT>::T *>(W) + (int64_t)s * ld;
}

// Slot the new solution goes to: a full history restarts (classic) or drops
// its oldest solution (rolling), and either way the new vector takes the
// oldest one's slot; otherwise the next free slot.
__device__ __forceinline__ int raw_new_slot(const RawState *st, int M) {
    const int d = st->d;
    return d >= M ? st->perm[0] : st->perm[d];
}

// Stored vector as a stencil operand (values in stored units, widened to
// FP64; ordinary cached loads, since neighbouring rows and planes re-read).
template <int DT>
struct StoredU {
    const typename Elem<DT>::T *__restrict__ w;
    __device__ __forceinline__ double operator()(int64_t q) const { return to_f64<DT>(w[q]); }
    __device__ __forceinline__ R2 two(int64_t q) const {
        using P = typename Pair<DT>::T;
        const P v = *reinterpret_cast<const P *>(w + q);
        if constexpr (DT == GUESS_F64) {
            return R2{{v.x, v.y}};
        } else {
            float a, b;
            widen2<DT>(v, a, b);
            return R2{{(double)a, (double)b}};
        }
    }
};

// ------------------------------------------------------------------ store
// slot <- round(2^e x) over the whole vector; returns this thread's max |x|.
template <int DT>
__device__ __forceinline__ double raw_store_pass(const double *__restrict__ x, void *slot, int64_t N, int e) {
    const int64_t nc = nchunks(N), stride = (int64_t)gridDim.x * kBlock;
    const double pw = ldexp(1.0, e);
    double mx = 0.0;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
        V4 v = load4<GUESS_F64>(x, c);
        if constexpr (DT == GUESS_F16) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                mx = nanmax(mx, fabs(v.v[q]));
                v.v[q] *= pw;
            }
        }
        store4<DT>(slot, c, v);
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(N)) {
        const int64_t i = tail_start(N) + threadIdx.x;
        if constexpr (DT == GUESS_F16) mx = nanmax(mx, fabs(x[i]));
        store1<DT>(slot, i, DT == GUESS_F16 ? x[i] * pw : x[i]);
    }
    return mx;
}

template <int DT>
__global__ __launch_bounds__(kBlock) void raw_store_kernel(RawArgs a, const double *__restrict__ x) {
    __shared__ double wmax[kWaves];
    RawState *st = a.st;
    const int s = raw_new_slot(st, a.M);
    const int e = DT == GUESS_F16 ? st->e_guess : 0;
    const double mx = raw_store_pass<DT>(x, slotp<DT>(a.W, a.ld, s), a.N, e);
    if constexpr (DT == GUESS_F16) {
        // max |x| into st->maxbits (non-negative doubles order like their bit patterns, a NaN
        // above everything); raw_fin cleared it at the end of the previous update
        const double m = wave_nanmax(mx);
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = m;
        __syncthreads();
        if (threadIdx.x == 0) {
            double t = wmax[0];
#pragma unroll
            for (int w = 1; w < kWaves; ++w) t = nanmax(t, wmax[w]);
            // the running maximum only grows (see the ring store): skip what cannot raise it
            const unsigned long long tb = (unsigned long long)__double_as_longlong(t);
            if (tb > __hip_atomic_load(&st->maxbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                atomicMax(&st->maxbits, tb);
            if (blockIdx.x == 0) st->e_used = e;
        }
    }
}

// FP16 only: this solution's exponent; the slot is stored again only when it
// differs from the exponent raw_store used.
template <int DT>
__global__ __launch_bounds__(kBlock) void raw_fix_kernel(RawArgs a, const double *__restrict__ x) {
    RawState *st = a.st;
    const int s = raw_new_slot(st, a.M);
    const int e = f16_scale_exp(__longlong_as_double((long long)st->maxbits));
    const int eu = st->e_used;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->new_exp = e;
        st->e_guess = e;
        st->fixed = e != eu ? 1 : 0;
    }
    if (e == eu) return;
    (void)raw_store_pass<GUESS_F16>(x, slotp<GUESS_F16>(a.W, a.ld, s), a.N, e);
}

// ------------------------------------------------------------------ apply + Gram row
// Partial rows: tot[j] = W_j^T (A w) for the d stored solutions (stored
// units), tot[d] = w^T A w.  A full history (d = M) has no Gram row: the
// classic variant restarts, and the rolling one drops the oldest solution,
// whose slot the new vector already occupies, so the row is taken with the
// M - 1 others.
template <int DT, bool VAR, bool AL>
LG_REDUCE_KERNEL void raw_apply_kernel(RawArgs a, Grid g) {
    __shared__ double lds[kLdsDoubles];
    const RawState *st = a.st;
    const int d = st->d;
    const bool full = d >= a.M;
    const int first = full ? 1 : 0;                       // rolling: skip the dropped oldest slot
    const int nd = full ? (a.qr ? a.M - 1 : 0) : d;       // columns of the Gram row
    const int s = raw_new_slot(st, a.M);
    const StoredU<DT> u{slotp<DT>(a.W, a.ld, s)};
    const int64_t nc = nchunks(a.N);
    const ChunkRange cr = xcd_range(nc);
    dispatch_d<0, GUESS_MAX_M - 1>(nd, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        const typename Elem<DT>::T *col[D > 0 ? D : 1];
#pragma unroll
        for (int j = 0; j < D; ++j) col[j] = slotp<DT>(a.W, a.ld, st->perm[first + j]);
        double acc[D + 1];
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] = 0.0;
        for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
            V4 wc[D > 0 ? D : 1];
#pragma unroll
            for (int j = 0; j < D; ++j) wc[j] = load4<DT>(col[j], c);
            R4 uc;
            const R4 aw = apply4g<VAR, AL>(u, g, c, uc);
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[D] = __builtin_fma(uc.v[e], aw.v[e], acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(wc[j].v[e], aw.v[e], acc[j]);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            const double awi = apply_pt<VAR>(u, g, i);
            acc[D] = __builtin_fma(u(i), awi, acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j) acc[j] = __builtin_fma(to_f64<DT>(col[j][i]), awi, acc[j]);
        }
        block_partials<D + 1>(acc, a.part, lds);
    });
}

// Same work in the z-marching traversal (grids it applies to).
template <int DT, bool VAR>
LG_REDUCE_KERNEL void raw_apply_march_kernel(RawArgs a, Grid g, March m) {
    __shared__ double lds[kLdsDoubles];
    const RawState *st = a.st;
    const int d = st->d;
    const bool full = d >= a.M;
    const int first = full ? 1 : 0;
    const int nd = full ? (a.qr ? a.M - 1 : 0) : d;
    const int s = raw_new_slot(st, a.M);
    const StoredU<DT> u{slotp<DT>(a.W, a.ld, s)};
    dispatch_d<0, GUESS_MAX_M - 1>(nd, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        const typename Elem<DT>::T *col[D > 0 ? D : 1];
#pragma unroll
        for (int j = 0; j < D; ++j) col[j] = slotp<DT>(a.W, a.ld, st->perm[first + j]);
        double acc[D + 1];
#pragma unroll
        for (int j = 0; j <= D; ++j) acc[j] = 0.0;
        // the Gram row's columns at the chunk, fetched one plane ahead
        struct Cols {
            V4 v[D > 0 ? D : 1];
        };
        auto pf = [&](int64_t c) {
            Cols cl;
#pragma unroll
            for (int j = 0; j < D; ++j) cl.v[j] = load4<DT>(col[j], c);
            return cl;
        };
        march_sweep_pf<VAR>(g, m, u, pf, [&](int64_t c, int64_t, const R2 &pa, const R2 &pb, const R4 &aw,
                                             const Cols &cl) {
            const V4 *wc = cl.v;
            const double uv[4] = {pa.v[0], pa.v[1], pb.v[0], pb.v[1]};
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[D] = __builtin_fma(uv[e], aw.v[e], acc[D]);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(wc[j].v[e], aw.v[e], acc[j]);
        });
        block_partials<D + 1>(acc, a.part, lds);
    });
}

// ------------------------------------------------------------------ small dense algebra (one thread)
// Cholesky factor of the leading n x n block of G into L (lower); false if
// G is not numerically positive definite.
__device__ __forceinline__ bool raw_cholesky(const double (&G)[GUESS_MAX_M][GUESS_MAX_M],
                                             double (&L)[GUESS_MAX_M][GUESS_MAX_M], int n) {
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = G[i][j];
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.0) || !isfinite(s)) return false;
                L[i][i] = sqrt(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
        for (int j = i + 1; j < GUESS_MAX_M; ++j) L[i][j] = 0.0;
    }
    return true;
}

// z = L^{-1} g (forward substitution over the leading n rows).
__device__ __forceinline__ void raw_forward(const double (&L)[GUESS_MAX_M][GUESS_MAX_M], const double *g,
                                            double *z, int n) {
    for (int i = 0; i < n; ++i) {
        double s = g[i];
        for (int k = 0; k < i; ++k) s -= L[i][k] * z[k];
        z[i] = s / L[i][i];
    }
}

// y = L^{-T} z (back substitution).
__device__ __forceinline__ void raw_backward(const double (&L)[GUESS_MAX_M][GUESS_MAX_M], const double *z,
                                             double *y, int n) {
    for (int i = n - 1; i >= 0; --i) {
        double s = z[i];
        for (int k = i + 1; k < n; ++k) s -= L[k][i] * y[k];
        y[i] = s / L[i][i];
    }
}

// End of an update: sums of the raw_apply rows, then the decisions.
template <int DT>
__global__ __launch_bounds__(kBlock) void raw_fin_kernel(RawArgs a, int nb) {
    __shared__ double lds[kLdsDoubles];
    RawState *st = a.st;
    const int d = st->d, M = a.M;
    const bool full = d >= M;
    const int nd = full ? (a.qr ? M - 1 : 0) : d;
    dispatch_d<0, GUESS_MAX_M - 1>(nd, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double tot[D + 1];
        final_sums<D + 1>(a.part, nb, tot, lds);
        if (threadIdx.x != 0) return;
        const int slot = raw_new_slot(st, M);
        const int e = DT == GUESS_F16 ? st->new_exp : 0;
        const double sw = ldexp(1.0, -e);
        int dd = d;
        if (full) {
            if (a.qr) {
                // drop the oldest solution: its slot (holding the new vector) moves to the end
                for (int j = 0; j < M - 1; ++j) st->perm[j] = st->perm[j + 1];
                st->perm[M - 1] = slot;
                for (int i = 0; i < M - 1; ++i)
                    for (int j = 0; j < M - 1; ++j) st->G[i][j] = st->G[i + 1][j + 1];
                dd = M - 1;
                st->drops += 1;
                if (!raw_cholesky(st->G, st->L, dd)) dd = 0;   // cannot happen for an SPD G
            } else {
                dd = 0;
                st->restarts += 1;
            }
        } else if (d == 0) {
            st->restarts += 1;
        }
        // the Gram row in true units (the new vector stands for sw * stored, column j for
        // 2^-e_j * stored)
        double gr[GUESS_MAX_M], z[GUESS_MAX_M];
#pragma unroll
        for (int j = 0; j < D; ++j) gr[j] = tot[j] * sw * ldexp(1.0, -st->exps[st->perm[j]]);
        const double s0 = tot[D] * sw * sw;
        const double nu0 = sqrt(s0);          // NaN when rounding made it negative
        double nu;
        bool ok;
        if (dd == 0) {
            nu = nu0;
            ok = isfinite(nu0) && nu0 > 0.0;
        } else {
            raw_forward(st->L, gr, z, dd);
            double zz = 0.0;
            for (int j = 0; j < dd; ++j) zz = __builtin_fma(z[j], z[j], zz);
            nu = sqrt(s0 - zz);
            ok = isfinite(nu) && nu > st->eps_rel * nu0;
        }
        st->upd_d = d;
        st->nu0 = nu0;
        st->nu = nu;
        st->last_accepted = ok ? 1 : 0;
        if (!isfinite(nu)) st->nonfinite = 1;
        if (ok) {
            for (int j = 0; j < dd; ++j) {
                st->G[dd][j] = gr[j];
                st->G[j][dd] = gr[j];
                st->L[dd][j] = z[j];
                st->L[j][dd] = 0.0;
            }
            st->G[dd][dd] = s0;
            st->L[dd][dd] = nu;
            st->perm[dd] = slot;
            st->exps[slot] = e;
            st->d = dd + 1;
        } else {
            if (dd > 0 || d > 0) st->rejects += 1;
            st->d = dd;
        }
        st->maxbits = 0ull;      // the next store's accumulator
    });
}

// ------------------------------------------------------------------ guess
template <int DT>
LG_REDUCE_KERNEL void raw_dots_kernel(RawArgs a, const double *__restrict__ b) {
    __shared__ double lds[kLdsDoubles];
    const RawState *st = a.st;
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    dispatch_d<1, GUESS_MAX_M>(st->d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        const void *col[D];
#pragma unroll
        for (int j = 0; j < D; ++j) col[j] = slotp<DT>(a.W, a.ld, st->perm[j]);
        double acc[D];
#pragma unroll
        for (int j = 0; j < D; ++j) acc[j] = 0.0;
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
            const V4 bv = load4<GUESS_F64>(b, c);
            V4 wv[D];
#pragma unroll
            for (int j = 0; j < D; ++j) wv[j] = load4<DT>(col[j], c);
#pragma unroll
            for (int j = 0; j < D; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[j] = __builtin_fma(wv[j].v[e], bv.v[e], acc[j]);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
#pragma unroll
            for (int j = 0; j < D; ++j) acc[j] = __builtin_fma(load1<DT>(col[j], i), b[i], acc[j]);
        }
        block_partials<D>(acc, a.part, lds);
    });
}

// G y = c through L; gamma_j multiplies stored column j (its 2^-e folded in).
template <int DT>
__global__ __launch_bounds__(kBlock) void raw_solve_kernel(RawArgs a, int nb) {
    __shared__ double lds[kLdsDoubles];
    RawState *st = a.st;
    const int d = st->d;
    if (threadIdx.x == 0) st->form_d = d;
    dispatch_d<1, GUESS_MAX_M>(d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        double tot[D];
        final_sums<D>(a.part, nb, tot, lds);
        if (threadIdx.x != 0) return;
        double c[GUESS_MAX_M], z[GUESS_MAX_M], y[GUESS_MAX_M];
#pragma unroll
        for (int j = 0; j < D; ++j) c[j] = tot[j] * ldexp(1.0, -st->exps[st->perm[j]]);
        raw_forward(st->L, c, z, D);
        raw_backward(st->L, z, y, D);
#pragma unroll
        for (int j = 0; j < D; ++j) st->gamma[j] = y[j] * ldexp(1.0, -st->exps[st->perm[j]]);
    });
}

template <int DT>
__global__ __launch_bounds__(kBlock) void raw_combine_kernel(RawArgs a, double *__restrict__ x0) {
    const RawState *st = a.st;
    const int64_t nc = nchunks(a.N), stride = (int64_t)gridDim.x * kBlock;
    dispatch_d<0, GUESS_MAX_M>(st->d, [&](auto Dc) {
        constexpr int D = decltype(Dc)::value;
        const void *col[D > 0 ? D : 1];
        double gm[D > 0 ? D : 1];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            col[j] = slotp<DT>(a.W, a.ld, st->perm[j]);
            gm[j] = st->gamma[j];
        }
        for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
            V4 acc{{0.0, 0.0, 0.0, 0.0}};
            if constexpr (D > 0) {
                V4 wv[D];
#pragma unroll
                for (int j = 0; j < D; ++j) wv[j] = load4<DT>(col[j], c);
#pragma unroll
                for (int e = 0; e < 4; ++e) acc.v[e] = gm[0] * wv[0].v[e];
#pragma unroll
                for (int j = 1; j < D; ++j)
#pragma unroll
                    for (int e = 0; e < 4; ++e) acc.v[e] = __builtin_fma(gm[j], wv[j].v[e], acc.v[e]);
            }
            store4<GUESS_F64>(x0, c, acc);
        }
        if (blockIdx.x == 0 && threadIdx.x < tail_count(a.N)) {
            const int64_t i = tail_start(a.N) + threadIdx.x;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) acc = __builtin_fma(gm[j], load1<DT>(col[j], i), acc);
            x0[i] = acc;
        }
    });
}

// ------------------------------------------------------------------ launchers
inline RawArgs make_raw_args(const RawBufs &p) {
    return RawArgs{p.W, p.part, p.st, p.N, p.ld, p.M, p.qr};
}

template <int DT>
void raw_form_dt(const RawBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev) {
    const RawArgs a = make_raw_args(p);
    const int gr = stream_grid(nchunks(a.N), reduce_blocks());
    klaunch(ev, 0, raw_dots_kernel<DT>, gr, kBlock, s, a, b);
    klaunch(ev, 1, raw_solve_kernel<DT>, 1, kBlock, s, a, gr);
    klaunch_sh(ev, 2, raw_combine_kernel<DT>, stream_grid(nchunks(a.N), grid_cap()), kBlock, gather_lds(), s, a, x0);
}

template <int DT>
void raw_update_dt(const RawBufs &p, const Grid &g, const double *x, hipStream_t s, KEvents *ev) {
    const RawArgs a = make_raw_args(p);
    const int gs = stream_grid(nchunks(a.N), grid_cap());
    int k = 0;
    // FP16: one atomic max per workgroup on one word, so the store runs on the reduction grid
    klaunch(ev, k++, raw_store_kernel<DT>, DT == GUESS_F16 ? stream_grid(nchunks(a.N), reduce_blocks()) : gs, kBlock,
            s, a, x);
    if constexpr (DT == GUESS_F16) klaunch(ev, k++, raw_fix_kernel<DT>, gs, kBlock, s, a, x);
    int ga = stream_grid(nchunks(a.N), reduce_blocks());
    // 2-byte formats: the chunk form (256^3, FP16 / BF16: 47 against 64 us in the z-march, whose
    // plane-by-plane latency a 2-byte operand does not hide); FP32: the z-march (within 5 %)
    if (march_ok(g) && march_enabled() && (DT == GUESS_F32 || raw_march())) {
        const int wgs = g.kx ? resident_wgs<raw_apply_march_kernel<DT, true>>()
                             : resident_wgs<raw_apply_march_kernel<DT, false>>();
        const March m = make_march(g, wgs);
        ga = march_grid(m);
        if (g.kx) klaunch(ev, k++, raw_apply_march_kernel<DT, true>, ga, kBlock, s, a, g, m);
        else klaunch(ev, k++, raw_apply_march_kernel<DT, false>, ga, kBlock, s, a, g, m);
    } else if (g.kx) {
        if (g.aligned) klaunch(ev, k++, raw_apply_kernel<DT, true, true>, ga, kBlock, s, a, g);
        else klaunch(ev, k++, raw_apply_kernel<DT, true, false>, ga, kBlock, s, a, g);
    } else {
        if (g.aligned) klaunch(ev, k++, raw_apply_kernel<DT, false, true>, ga, kBlock, s, a, g);
        else klaunch(ev, k++, raw_apply_kernel<DT, false, false>, ga, kBlock, s, a, g);
    }
    klaunch(ev, k++, raw_fin_kernel<DT>, 1, kBlock, s, a, ga);
}

}  // namespace lg
