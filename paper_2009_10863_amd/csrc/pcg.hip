// Jacobi-preconditioned conjugate gradients (§5.3) on the 7-point operator.
//
// PCG keeps its scalars (rho, alpha, thresholds, iteration count,
// convergence flag) on the device, and every kernel returns at once when the
// solve has converged or broken down.  The host therefore enqueues
// iterations in batches and only reads the state between batches; the
// iteration count is still exact.
//
// A kernel returns early only on what an earlier kernel decided: the
// convergence flag holds the iteration whose stop test passed, so the
// workgroups of that same pcg_a launch -- including any that start after
// workgroup 0 has written the flag -- all still apply their share of the
// last x update.
//
// This translation unit is compiled with the max-ILP instruction scheduler:
// the search-direction stencil issues ~30 loads per chunk, and grouping them
// measured 6 % faster per iteration than the default schedule at 256^3.
#include "common.h"
#include "launch.h"
#include "march.h"

namespace lg {

static __device__ __forceinline__ V4 toV(const R4 &r) { return V4{{r.v[0], r.v[1], r.v[2], r.v[3]}}; }

// ------------------------------------------------------------------ PCG
// Two streaming kernels per iteration k (1-based), both with one row of
// partial sums per workgroup.  Every workgroup of the next kernel sums the
// previous kernel's rows itself, in the same fixed order, so all of them see
// identical scalars without any cross-workgroup synchronisation.
//
//   pcg_a(k): from rows (r^T r, r^T z, b^T b) of r_{k-1}: stop test (k = 1:
//             also the threshold); for k > 1 first x += alpha_{k-1} p_{k-1}
//             (the update of the previous iteration, deferred to the pass
//             that reads p_{k-1} anyway); rho_k = r^T z; beta = rho_k /
//             rho_{k-1}; p_k = z + beta p_{k-1} formed on the fly at the
//             stencil points (z = D^{-1} r), stored, and q = A p_k;
//             rows: p_k^T q.
//   pcg_b(k): alpha = rho_k / p_k^T q; r -= alpha q; rows: (r^T r, r^T z, 0).
//   pcg_finish: after the last iteration, the pending x update if any.
// Per iteration: reads r, p_{k-1}, x (pcg_a, 24 B/unknown), r, q (pcg_b,
// 16 B); writes x, p_k, q, r (32 B): 72 B per unknown (constant
// coefficient).  p_k and p_{k-1} live in two buffers used alternately.
// x receives exactly the same FMAs as in the textbook order.
int pcg_grid(const Grid &g) { return stream_grid(nchunks(g.n), reduce_blocks()); }

// Solve over before iteration k's pcg_a (stopped at an earlier iteration)...
__device__ __forceinline__ bool pcg_done_before_a(const PcgState *st, int k) {
    return st->breakdown || (st->converged != 0 && st->converged < k);
}
// ... and before iteration k's pcg_b (stopped at iteration k or earlier).
__device__ __forceinline__ bool pcg_done_before_b(const PcgState *st, int k) {
    return st->breakdown || (st->converged != 0 && st->converged <= k);
}

template <bool VAR>
__device__ __forceinline__ V4 dinv4(const Grid &g, int64_t c) {
    if constexpr (VAR) return load4<GUESS_F64>(g.dinv, c);
    else return V4{{g.dinv_const, g.dinv_const, g.dinv_const, g.dinv_const}};
}

// The next search direction as a stencil operand: p = D^{-1} r + beta p_old
// (first iteration: p = D^{-1} r), evaluated wherever the stencil reads it.
template <bool VAR>
struct PNext {
    const double *__restrict__ r;
    const double *__restrict__ pold;
    const double *__restrict__ dinv;
    double dconst, beta;
    bool first;
    // p_old is read even in the first iteration (and then ignored by the
    // select), so that no load sits behind a branch
    __device__ __forceinline__ double operator()(int64_t q) const {
        const double z = (VAR ? dinv[q] : dconst) * r[q];
        const double pq = __builtin_fma(beta, pold[q], z);
        return first ? z : pq;
    }
    __device__ __forceinline__ R2 two(int64_t q) const {
        const R2 rv = ld2(r, q);
        const R2 pv = ld2(pold, q);
        R2 dv;
        if constexpr (VAR) dv = ld2(dinv, q);
        else dv = R2{{dconst, dconst}};
        R2 out;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const double z = dv.v[e] * rv.v[e];
            const double pq = __builtin_fma(beta, pv.v[e], z);
            out.v[e] = first ? z : pq;
        }
        return out;
    }
};

// r = b - A x; rows (r^T r, r^T D^{-1} r, b^T b).
template <bool VAR, bool AL>
LG_REDUCE_KERNEL void pcg_init_kernel(Grid g, const double *__restrict__ b, const double *__restrict__ x,
                                      double *__restrict__ r, double *part) {
    __shared__ double lds[kLdsDoubles];
    double acc[3] = {0.0, 0.0, 0.0};
    const ChunkRange cr = xcd_range(nchunks(g.n));
    for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
        R4 uc;
        const R4 ax = apply4g<VAR, AL>(x, g, c, uc);
        const V4 bv = load4<GUESS_F64>(b, c), dv = dinv4<VAR>(g, c);
        V4 rv;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            rv.v[e] = bv.v[e] - ax.v[e];
            acc[0] = __builtin_fma(rv.v[e], rv.v[e], acc[0]);
            acc[1] = __builtin_fma(rv.v[e], dv.v[e] * rv.v[e], acc[1]);
            acc[2] = __builtin_fma(bv.v[e], bv.v[e], acc[2]);
        }
        store4<GUESS_F64>(r, c, rv);
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(g.n)) {
        const int64_t q = tail_start(g.n) + threadIdx.x;
        const double rq = b[q] - apply_pt<VAR>(VecU{x}, g, q);
        r[q] = rq;
        acc[0] = __builtin_fma(rq, rq, acc[0]);
        acc[1] = __builtin_fma(rq, dinv_at<VAR>(g, q) * rq, acc[1]);
        acc[2] = __builtin_fma(b[q], b[q], acc[2]);
    }
    block_partials<3>(acc, part, lds);
}

// Start of iteration k, shared by both forms of pcg_a: the stop test on the
// rows of r_{k-1} (nb rows of part_b) and beta.  Returns false when the
// solve stops here.
__device__ __forceinline__ bool pcg_a_begin(const double *part_b, int nb, PcgState *st, int k, double rtol,
                                            double *lds, double &beta) {
    double tot[3];
    final_sums<3>(part_b, nb, tot, lds);
    const double rr = tot[0], rz = tot[1];
    const double rn = sqrt(rr);
    double thresh;
    if (k == 1) thresh = st->rule == GUESS_STOP_RHS ? rtol * sqrt(tot[2]) : rtol * fmax(rn, 1.0);
    else thresh = st->thresh;
    const bool stop = st->rule == GUESS_STOP_RHS ? (rn <= thresh) : (rn < thresh);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (k == 1) {
            st->thresh = thresh;
            st->bb = tot[2];
            st->rr0 = rr;
        }
        st->rr = rr;
        if (stop) {
            st->converged = k;
            st->it = k - 1;
        } else {
            st->rho[k & 1] = rz;
        }
    }
    if (stop) return false;
    beta = k == 1 ? 0.0 : rz / st->rho[(k - 1) & 1];
    return true;
}

// The deferred x updates over the whole vector: x += a1 p1, then (TWO)
// x += a2 p2, the older iteration first (the stop in pcg_a, and pcg_finish).
template <bool TWO>
__device__ __forceinline__ void x_update_all(const Grid &g, double *__restrict__ x, const double *__restrict__ p1,
                                             double a1, const double *__restrict__ p2, double a2) {
    const int64_t nc = nchunks(g.n), stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
        V4 xv = load4<GUESS_F64>(x, c);
        const V4 pv = load4<GUESS_F64>(p1, c);
#pragma unroll
        for (int e = 0; e < 4; ++e) xv.v[e] = __builtin_fma(a1, pv.v[e], xv.v[e]);
        if constexpr (TWO) {
            const V4 pw = load4<GUESS_F64>(p2, c);
#pragma unroll
            for (int e = 0; e < 4; ++e) xv.v[e] = __builtin_fma(a2, pw.v[e], xv.v[e]);
        }
        store4<GUESS_F64>(x, c, xv);
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(g.n)) {
        const int64_t t = tail_start(g.n) + threadIdx.x;
        double xt = __builtin_fma(a1, p1[t], x[t]);
        if constexpr (TWO) xt = __builtin_fma(a2, p2[t], xt);
        x[t] = xt;
    }
}

// Iteration k's start in both forms of pcg_a when the solve stops there:
// apply what x still lacks (the updates of iterations k-2 and k-1 for odd
// k >= 3, of k-1 for even k, nothing for k = 1).
template <bool XU>
__device__ __forceinline__ void x_update_at_stop(const Grid &g, double *x, const double *pold2, const double *pold,
                                                 PcgState *st, int k) {
    if constexpr (XU) {
        x_update_all<true>(g, x, pold2, st->alpha[k & 1], pold, st->alpha[(k - 1) & 1]);
    } else if (k > 1) {
        x_update_all<false>(g, x, pold, st->alpha[(k - 1) & 1], nullptr, 0.0);
        if (blockIdx.x == 0 && threadIdx.x == 0) st->x_pending = 0;
    }
}

// XU (odd k >= 3): x += alpha_{k-2} p_{k-2}, then += alpha_{k-1} p_{k-1}, on the
// way; other iterations leave x alone, so x is read and written every other
// iteration.
template <bool VAR, bool AL, bool XU>
LG_REDUCE_KERNEL void pcg_a_kernel(Grid g, double *__restrict__ x, const double *__restrict__ r,
                                   const double *__restrict__ pold, const double *__restrict__ pold2,
                                   double *__restrict__ pnew, double *__restrict__ q, const double *part_b, int nb_b,
                                   double *part_a, PcgState *st, int k, double rtol) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done_before_a(st, k)) return;
    double beta;
    const double a1 = XU ? st->alpha[k & 1] : 0.0, a2 = XU ? st->alpha[(k - 1) & 1] : 0.0;
    if (XU && blockIdx.x == 0 && threadIdx.x == 0) st->x_pending = 0;
    if (!pcg_a_begin(part_b, nb_b, st, k, rtol, lds, beta)) {
        x_update_at_stop<XU>(g, x, pold2, pold, st, k);
        return;
    }
    const bool first = k == 1;
    const PNext<VAR> pn{r, pold, g.dinv, g.dinv_const, beta, first};
    double acc[1] = {0.0};
    const ChunkRange cr = xcd_range(nchunks(g.n));
    for (int64_t c = cr.begin; c < cr.end; c += cr.step) {
        R4 pc;
        const R4 qv = apply4g<VAR, AL>(pn, g, c, pc);
        store4<GUESS_F64>(pnew, c, toV(pc));
        store4<GUESS_F64>(q, c, toV(qv));
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[0] = __builtin_fma(pc.v[e], qv.v[e], acc[0]);
        if constexpr (XU) {
            V4 xv = load4<GUESS_F64>(x, c);
            const V4 pv = load4<GUESS_F64>(pold2, c), pw = load4<GUESS_F64>(pold, c);
#pragma unroll
            for (int e = 0; e < 4; ++e) xv.v[e] = __builtin_fma(a2, pw.v[e], __builtin_fma(a1, pv.v[e], xv.v[e]));
            store4<GUESS_F64>(x, c, xv);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(g.n)) {
        const int64_t t = tail_start(g.n) + threadIdx.x;
        const double pt = pn(t);
        const double qt = apply_pt<VAR>(pn, g, t);
        if (XU) x[t] = __builtin_fma(a2, pold[t], __builtin_fma(a1, pold2[t], x[t]));
        pnew[t] = pt;
        q[t] = qt;
        acc[0] = __builtin_fma(pt, qt, acc[0]);
    }
    block_partials<1>(acc, part_a, lds);
}

// ------------------------------------------------------------------ z-marching pcg_a
// Same arithmetic as pcg_a_kernel in the traversal of march.h (constant
// coefficient): p and q are bit-identical to the chunk form.
template <bool VAR, bool XU>
LG_REDUCE_KERNEL void pcg_a_march_kernel(Grid g, March m, double *__restrict__ x, const double *__restrict__ r,
                                         const double *__restrict__ pold, const double *__restrict__ pold2,
                                         double *__restrict__ pnew, double *__restrict__ q, const double *part_b,
                                         int nb_b, double *part_a, PcgState *st, int k, double rtol) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done_before_a(st, k)) return;
    double beta;
    const double a1 = XU ? st->alpha[k & 1] : 0.0, a2 = XU ? st->alpha[(k - 1) & 1] : 0.0;
    if (XU && blockIdx.x == 0 && threadIdx.x == 0) st->x_pending = 0;
    if (!pcg_a_begin(part_b, nb_b, st, k, rtol, lds, beta)) {
        x_update_at_stop<XU>(g, x, pold2, pold, st, k);
        return;
    }
    const bool first = k == 1;
    const PNext<VAR> pn{r, pold, g.dinv, g.dinv_const, beta, first};
    double acc[1] = {0.0};
    // x, p_{k-2} and p_{k-1} of the chunk, fetched one plane ahead for the deferred updates
    struct XP {
        V4 x, p1, p2;
    };
    auto pf = [&](int64_t c) {
        XP v{};
        if constexpr (XU) {
            v.x = load4<GUESS_F64>(x, c);
            v.p1 = load4<GUESS_F64>(pold2, c);
            v.p2 = load4<GUESS_F64>(pold, c);
        }
        return v;
    };
    march_sweep_pf<VAR>(g, m, pn, pf, [&](int64_t c, int64_t e, const R2 &pa, const R2 &pb, const R4 &qv, const XP &xp) {
        if constexpr (XU) {
            // deferred x += alpha_{k-2} p_{k-2}, then += alpha_{k-1} p_{k-1}, on this chunk
            V4 xv = xp.x;
#pragma unroll
            for (int i = 0; i < 4; ++i) xv.v[i] = __builtin_fma(a2, xp.p2.v[i], __builtin_fma(a1, xp.p1.v[i], xv.v[i]));
            store4<GUESS_F64>(x, c, xv);
        }
        store4<GUESS_F64>(pnew, c, V4{{pa.v[0], pa.v[1], pb.v[0], pb.v[1]}});
        store4<GUESS_F64>(q, c, toV(qv));
        acc[0] = __builtin_fma(pa.v[0], qv.v[0], acc[0]);
        acc[0] = __builtin_fma(pa.v[1], qv.v[1], acc[0]);
        acc[0] = __builtin_fma(pb.v[0], qv.v[2], acc[0]);
        acc[0] = __builtin_fma(pb.v[1], qv.v[3], acc[0]);
        (void)e;
    });
    block_partials<1>(acc, part_a, lds);
}

// r = b - A x in the traversal of march.h; rows (r^T r, r^T D^{-1} r, b^T b).
template <bool VAR>
LG_REDUCE_KERNEL void pcg_init_march_kernel(Grid g, March m, const double *__restrict__ b,
                                            const double *__restrict__ x, double *__restrict__ r, double *part) {
    __shared__ double lds[kLdsDoubles];
    double acc[3] = {0.0, 0.0, 0.0};
    struct BD {
        V4 b, d;
    };
    auto pf = [&](int64_t c) { return BD{load4<GUESS_F64>(b, c), dinv4<VAR>(g, c)}; };
    march_sweep_pf<VAR>(g, m, VecU{x}, pf, [&](int64_t c, int64_t, const R2 &, const R2 &, const R4 &ax, const BD &bd) {
        const V4 &bv = bd.b, &dv = bd.d;
        V4 rv;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            rv.v[e] = bv.v[e] - ax.v[e];
            acc[0] = __builtin_fma(rv.v[e], rv.v[e], acc[0]);
            acc[1] = __builtin_fma(rv.v[e], dv.v[e] * rv.v[e], acc[1]);
            acc[2] = __builtin_fma(bv.v[e], bv.v[e], acc[2]);
        }
        store4<GUESS_F64>(r, c, rv);
    });
    block_partials<3>(acc, part, lds);
}

template <bool VAR>
LG_REDUCE_KERNEL void pcg_b_kernel(Grid g, double *__restrict__ r, const double *__restrict__ q,
                                   const double *part_a, int nb_a, double *part_b, PcgState *st, int k) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done_before_b(st, k)) return;
    double tot[1];
    final_sums<1>(part_a, nb_a, tot, lds);
    const double pq = tot[0];
    if (!(pq > 0.0) || !isfinite(pq)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->breakdown = 1;
            st->it = k;
        }
        return;
    }
    const double alpha = st->rho[k & 1] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->alpha[k & 1] = alpha;
        st->x_last = k;
        st->x_pending = 1;
    }
    double acc[3] = {0.0, 0.0, 0.0};
    const int64_t nc = nchunks(g.n), stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
        V4 rv = load4<GUESS_F64>(r, c);
        const V4 qv = load4<GUESS_F64>(q, c), dv = dinv4<VAR>(g, c);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            rv.v[e] = __builtin_fma(-alpha, qv.v[e], rv.v[e]);
            acc[0] = __builtin_fma(rv.v[e], rv.v[e], acc[0]);
            acc[1] = __builtin_fma(rv.v[e], dv.v[e] * rv.v[e], acc[1]);
        }
        store4<GUESS_F64>(r, c, rv);
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(g.n)) {
        const int64_t t = tail_start(g.n) + threadIdx.x;
        const double rt = __builtin_fma(-alpha, q[t], r[t]);
        r[t] = rt;
        acc[0] = __builtin_fma(rt, rt, acc[0]);
        acc[1] = __builtin_fma(rt, dinv_at<VAR>(g, t) * rt, acc[1]);
    }
    block_partials<3>(acc, part_b, lds);
}

int launch_pcg_init(const Grid &g, const double *b, const double *x, double *r, double *part_b, hipStream_t s) {
    const int gr = pcg_grid(g);
    if (march_ok(g) && march_enabled()) {
        // same number of partial rows as the chunk form (the consumers expect
        // gr); the items are split over all gr workgroups
        const March m = make_march(g, gr);
        if (g.kx) pcg_init_march_kernel<true><<<gr, kBlock, 0, s>>>(g, m, b, x, r, part_b);
        else pcg_init_march_kernel<false><<<gr, kBlock, 0, s>>>(g, m, b, x, r, part_b);
        return GUESS_OK;
    }
    if (g.kx) {
        if (g.aligned) pcg_init_kernel<true, true><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
        else pcg_init_kernel<true, false><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
    } else {
        if (g.aligned) pcg_init_kernel<false, true><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
        else pcg_init_kernel<false, false><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
    }
    return GUESS_OK;
}

template <bool VAR, bool AL, bool XU>
static void pcg_iter_x(const Grid &g, double *x, double *r, double *const p[3], double *q, double *part_a,
                       double *part_b, PcgState *st, int k, double rtol, hipStream_t s) {
    const int gr = pcg_grid(g);
    double *pnew = p[k % 3];
    const double *pold = p[(k - 1) % 3], *pold2 = p[(k + 1) % 3];    // p_{k-1}, p_{k-2}
    int ga = gr;
    if (AL && march_ok(g) && march_enabled()) {
        const int wgs = resident_wgs<pcg_a_march_kernel<VAR, XU>>();
        const March m = make_march(g, wgs);
        ga = march_grid(m);
        pcg_a_march_kernel<VAR, XU><<<ga, kBlock, 0, s>>>(g, m, x, r, pold, pold2, pnew, q, part_b, gr, part_a, st,
                                                          k, rtol);
    } else {
        pcg_a_kernel<VAR, AL, XU><<<gr, kBlock, 0, s>>>(g, x, r, pold, pold2, pnew, q, part_b, gr, part_a, st, k,
                                                        rtol);
    }
    pcg_b_kernel<VAR><<<gr, kBlock, 0, s>>>(g, r, q, part_a, ga, part_b, st, k);
}

template <bool VAR, bool AL>
static void pcg_iter_v(const Grid &g, double *x, double *r, double *const p[3], double *q, double *part_a,
                       double *part_b, PcgState *st, int k, double rtol, hipStream_t s) {
    if ((k & 1) && k >= 3) pcg_iter_x<VAR, AL, true>(g, x, r, p, q, part_a, part_b, st, k, rtol, s);
    else pcg_iter_x<VAR, AL, false>(g, x, r, p, q, part_a, part_b, st, k, rtol, s);
}

int launch_pcg_iter(const Grid &g, double *x, double *r, double *const p[3], double *q, double *part_a,
                    double *part_b, PcgState *st, int k, double rtol, hipStream_t s) {
    if (g.kx) {
        if (g.aligned) pcg_iter_v<true, true>(g, x, r, p, q, part_a, part_b, st, k, rtol, s);
        else pcg_iter_v<true, false>(g, x, r, p, q, part_a, part_b, st, k, rtol, s);
    } else {
        if (g.aligned) pcg_iter_v<false, true>(g, x, r, p, q, part_a, part_b, st, k, rtol, s);
        else pcg_iter_v<false, false>(g, x, r, p, q, part_a, part_b, st, k, rtol, s);
    }
    return GUESS_OK;
}

// Convergence check after the last allowed iteration (pcg_a without the update).
__global__ __launch_bounds__(kBlock) void pcg_check_kernel(const double *part_b, int nb, PcgState *st, int k,
                                                           double rtol) {
    __shared__ double lds[kLdsDoubles];
    if (st->converged != 0 || st->breakdown) return;
    double tot[3];
    final_sums<3>(part_b, nb, tot, lds);
    if (threadIdx.x == 0) {
        const double rn = sqrt(tot[0]);
        double thresh = st->thresh;
        if (k == 1) thresh = st->rule == GUESS_STOP_RHS ? rtol * sqrt(tot[2]) : rtol * fmax(rn, 1.0);
        const bool stop = st->rule == GUESS_STOP_RHS ? (rn <= thresh) : (rn < thresh);
        st->rr = tot[0];
        if (k == 1) {
            st->bb = tot[2];
            st->rr0 = tot[0];
        }
        if (stop) {
            st->converged = k;
            st->it = k - 1;
        }
    }
}

int launch_pcg_check(const Grid &g, const double *part_b, PcgState *st, int k, double rtol, hipStream_t s) {
    pcg_check_kernel<<<1, kBlock, 0, s>>>(part_b, pcg_grid(g), st, k, rtol);
    return GUESS_OK;
}

// The x updates that no later pcg_a applied: those of the last completed
// iteration L and, for even L, of L-1 (odd iterations apply the two before them).
__global__ __launch_bounds__(kBlock) void pcg_finish_kernel(Grid g, double *x, const double *p0, const double *p1,
                                                            const double *p2, PcgState *st) {
    if (!st->x_pending) return;
    const int L = st->x_last;
    const double *p[3] = {p0, p1, p2};
    if (L % 2 == 0) x_update_all<true>(g, x, p[(L - 1) % 3], st->alpha[(L - 1) & 1], p[L % 3], st->alpha[L & 1]);
    else x_update_all<false>(g, x, p[L % 3], st->alpha[L & 1], nullptr, 0.0);
}

int launch_pcg_finish(const Grid &g, double *x, double *const p[3], PcgState *st, hipStream_t s) {
    pcg_finish_kernel<<<stream_grid(nchunks(g.n) > 0 ? nchunks(g.n) : 1, grid_cap()), kBlock, 0, s>>>(
        g, x, p[0], p[1], p[2], st);
    return GUESS_OK;
}

}  // namespace lg
