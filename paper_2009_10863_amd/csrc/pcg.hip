// Jacobi-preconditioned conjugate gradients (§5.3) on the 7-point operator.
//
// PCG keeps its scalars (rho, alpha, thresholds, iteration count,
// convergence flag) on the device, and every kernel returns at once when the
// solve has converged or broken down.  The host therefore enqueues
// iterations in batches and only reads the state between batches; the
// iteration count is still exact.
//
// This translation unit is compiled with the max-ILP instruction scheduler:
// the search-direction stencil issues ~30 loads per chunk, and grouping them
// measured 6 % faster per iteration than the default schedule at 256^3.
#include "common.h"
#include "launch.h"

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

__device__ __forceinline__ bool pcg_done(const PcgState *st) { return st->converged | st->breakdown; }

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
            st->converged = 1;
            st->it = k - 1;
        } else {
            st->rho[k & 1] = rz;
        }
    }
    if (stop) return false;
    beta = k == 1 ? 0.0 : rz / st->rho[(k - 1) & 1];
    return true;
}

// x += alpha p over the whole vector (the deferred update when the solve
// stops in pcg_a, and pcg_finish).
__device__ __forceinline__ void x_update_all(const Grid &g, double *__restrict__ x, const double *__restrict__ p,
                                             double alpha) {
    const int64_t nc = nchunks(g.n), stride = (int64_t)gridDim.x * kBlock;
    for (int64_t c = (int64_t)blockIdx.x * kBlock + threadIdx.x; c < nc; c += stride) {
        V4 xv = load4<GUESS_F64>(x, c);
        const V4 pv = load4<GUESS_F64>(p, c);
#pragma unroll
        for (int e = 0; e < 4; ++e) xv.v[e] = __builtin_fma(alpha, pv.v[e], xv.v[e]);
        store4<GUESS_F64>(x, c, xv);
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(g.n)) {
        const int64_t t = tail_start(g.n) + threadIdx.x;
        x[t] = __builtin_fma(alpha, p[t], x[t]);
    }
}

template <bool VAR, bool AL>
LG_REDUCE_KERNEL void pcg_a_kernel(Grid g, double *__restrict__ x, const double *__restrict__ r,
                                   const double *__restrict__ pold, double *__restrict__ pnew,
                                   double *__restrict__ q, const double *part_b, int nb_b, double *part_a,
                                   PcgState *st, int k, double rtol) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done(st)) return;
    double beta;
    const double alpha = k > 1 ? st->alpha : 0.0;   // alpha_{k-1}
    if (k > 1 && blockIdx.x == 0 && threadIdx.x == 0) st->x_pending = 0;
    if (!pcg_a_begin(part_b, nb_b, st, k, rtol, lds, beta)) {
        if (k > 1) x_update_all(g, x, pold, alpha);
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
        if (!first) {
            V4 xv = load4<GUESS_F64>(x, c);
            const V4 pv = load4<GUESS_F64>(pold, c);
#pragma unroll
            for (int e = 0; e < 4; ++e) xv.v[e] = __builtin_fma(alpha, pv.v[e], xv.v[e]);
            store4<GUESS_F64>(x, c, xv);
        }
    }
    if (blockIdx.x == 0 && threadIdx.x < tail_count(g.n)) {
        const int64_t t = tail_start(g.n) + threadIdx.x;
        const double pt = pn(t);
        const double qt = apply_pt<VAR>(pn, g, t);
        if (!first) x[t] = __builtin_fma(alpha, pold[t], x[t]);
        pnew[t] = pt;
        q[t] = qt;
        acc[0] = __builtin_fma(pt, qt, acc[0]);
    }
    block_partials<1>(acc, part_a, lds);
}

// ------------------------------------------------------------------ z-marching pcg_a
// Same arithmetic as pcg_a_kernel, different traversal (constant
// coefficient; every z-plane a whole number of 4-tile groups).  A wave owns
// one 256-element tile of a z-plane and sweeps it through a range of
// planes, keeping the search direction of planes z-1, z, z+1 in registers:
// per step it loads r and p_old once for plane z+1 and for the rows y-1,
// y+1, and takes the x-neighbours from the adjacent lanes (the tile's first
// and last element from one extra load when the tile does not start or end
// a grid row).  The 7-point values, their order and rounding are those of
// the chunk form, so p and q are bit-identical to it.
struct March {
    int tp;      // 256-element tiles per z-plane
    int zlen;    // planes per work item
    int items;   // tp * number of plane ranges
};

static bool march_ok(const Grid &g) {
    return !g.kx && g.aligned && g.nxy % 256 == 0 && (g.nxy / 256) % kWaves == 0;
}

static March make_march(const Grid &g) {
    March m;
    m.tp = (int)(g.nxy / 256);
    // about 1024 workgroups of kWaves items each
    int nr = (1024 * kWaves) / m.tp;
    nr = nr < 1 ? 1 : (nr > g.nz ? g.nz : nr);
    m.zlen = (g.nz + nr - 1) / nr;
    nr = (g.nz + m.zlen - 1) / m.zlen;
    m.items = m.tp * nr;
    return m;
}

static int march_grid(const March &m) {
    const int wg = (m.items + kWaves - 1) / kWaves;
    return wg < kMaxPartialBlocks ? wg : kMaxPartialBlocks;
}

__device__ __forceinline__ R2 sel2(bool keep, const R2 &v) {
    return R2{{keep ? v.v[0] : 0.0, keep ? v.v[1] : 0.0}};
}

// q at one element: fixed order west, east, south, north, bottom, top.
__device__ __forceinline__ double q_const(const Grid &g, double uc, double w, double e, double s_, double n,
                                          double b, double t) {
#pragma clang fp contract(off)
    double s = 6.0 * uc;
    s = s - w;
    s = s - e;
    s = s - s_;
    s = s - n;
    s = s - b;
    s = s - t;
    const double a = g.c * s;
    const double bb = g.shift * uc;
    return a + bb;
}

LG_REDUCE_KERNEL void pcg_a_march_kernel(Grid g, March m, double *__restrict__ x, const double *__restrict__ r,
                                         const double *__restrict__ pold, double *__restrict__ pnew,
                                         double *__restrict__ q, const double *part_b, int nb_b, double *part_a,
                                         PcgState *st, int k, double rtol) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done(st)) return;
    double beta;
    const double alpha = k > 1 ? st->alpha : 0.0;   // alpha_{k-1}
    if (k > 1 && blockIdx.x == 0 && threadIdx.x == 0) st->x_pending = 0;
    if (!pcg_a_begin(part_b, nb_b, st, k, rtol, lds, beta)) {
        if (k > 1) x_update_all(g, x, pold, alpha);
        return;
    }
    const bool first = k == 1;
    const PNext<false> pn{r, pold, nullptr, g.dinv_const, beta, first};
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // consecutive logical workgroups (neighbouring tiles) on one XCD
    const int nwg = gridDim.x;
    const int lb = nwg % kXcds == 0 ? (int)(blockIdx.x % kXcds) * (nwg / kXcds) + (int)(blockIdx.x / kXcds)
                                    : (int)blockIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int64_t nxy = g.nxy;
    double acc[1] = {0.0};
    for (int item = lb * kWaves + wave; item < m.items; item += nwg * kWaves) {
        const int tau = item % m.tp, zr = item / m.tp;
        const int z0 = zr * m.zlen;
        const int z1 = z0 + m.zlen < nz ? z0 + m.zlen : nz;
        const int64_t offa = (int64_t)tau * 256 + 2 * lane, offb = offa + 128;
        const uint32_t ja = fdiv(g.fnx, (uint32_t)offa), jb = fdiv(g.fnx, (uint32_t)offb);
        const int ia = (int)((uint32_t)offa - ja * (uint32_t)nx), ib = (int)((uint32_t)offb - jb * (uint32_t)nx);
        const bool hwa = ia > 0, hea = ia + 2 < nx, hwb = ib > 0, heb = ib + 2 < nx;
        const bool hsa = ja > 0, hna = (int)ja < ny - 1, hsb = jb > 0, hnb = (int)jb < ny - 1;
        // plane z0 - 1 (bottom neighbours of the first plane) and plane z0
        int64_t ea = (int64_t)z0 * nxy + offa;
        const int64_t eprev = z0 > 0 ? ea - nxy : ea;
        R2 pa_prev = sel2(z0 > 0, pn.two(eprev)), pb_prev = sel2(z0 > 0, pn.two(eprev + 128));
        R2 pa = pn.two(ea), pb = pn.two(ea + 128);
        for (int z = z0; z < z1; ++z, ea += nxy) {
            const bool ht = z + 1 < nz;
            const int64_t enext = ht ? ea + nxy : ea;
            const R2 pa_next = sel2(ht, pn.two(enext)), pb_next = sel2(ht, pn.two(enext + 128));
            const R2 sa = sel2(hsa, pn.two(hsa ? ea - nx : ea)), na = sel2(hna, pn.two(hna ? ea + nx : ea));
            const R2 sb = sel2(hsb, pn.two(hsb ? ea + 128 - nx : ea + 128));
            const R2 nb = sel2(hnb, pn.two(hnb ? ea + 128 + nx : ea + 128));
            // x-neighbours across lanes; the tile's outer neighbours by load
            double ew = 0.0, ee = 0.0;
            if (lane == 0 && hwa) ew = pn(ea - 1);
            if (lane == 63 && heb) ee = pn(ea + 256 - 2 * 63);
            const double wa_ = __shfl(pa.v[1], (lane + 63) & 63, 64);
            const double wb_ = __shfl(pb.v[1], (lane + 63) & 63, 64);
            const double ea_ = __shfl(pa.v[0], (lane + 1) & 63, 64);
            const double eb_ = __shfl(pb.v[0], (lane + 1) & 63, 64);
            const double wa = hwa ? (lane > 0 ? wa_ : ew) : 0.0;
            const double wb = hwb ? (lane > 0 ? wb_ : wa_) : 0.0;
            const double eaa = hea ? (lane < 63 ? ea_ : eb_) : 0.0;
            const double ebb = heb ? (lane < 63 ? eb_ : ee) : 0.0;
            R4 qv;
            qv.v[0] = q_const(g, pa.v[0], wa, pa.v[1], sa.v[0], na.v[0], pa_prev.v[0], pa_next.v[0]);
            qv.v[1] = q_const(g, pa.v[1], pa.v[0], eaa, sa.v[1], na.v[1], pa_prev.v[1], pa_next.v[1]);
            qv.v[2] = q_const(g, pb.v[0], wb, pb.v[1], sb.v[0], nb.v[0], pb_prev.v[0], pb_next.v[0]);
            qv.v[3] = q_const(g, pb.v[1], pb.v[0], ebb, sb.v[1], nb.v[1], pb_prev.v[1], pb_next.v[1]);
            if (!first) {
                // deferred x += alpha_{k-1} p_{k-1} on this plane's pairs
                const R2 xa = ld2(x, ea), xb = ld2(x, ea + 128);
                const R2 oa = ld2(pold, ea), ob = ld2(pold, ea + 128);
                __builtin_nontemporal_store(d2{__builtin_fma(alpha, oa.v[0], xa.v[0]), __builtin_fma(alpha, oa.v[1], xa.v[1])},
                                            reinterpret_cast<d2 *>(x + ea));
                __builtin_nontemporal_store(d2{__builtin_fma(alpha, ob.v[0], xb.v[0]), __builtin_fma(alpha, ob.v[1], xb.v[1])},
                                            reinterpret_cast<d2 *>(x + ea + 128));
            }
            __builtin_nontemporal_store(d2{pa.v[0], pa.v[1]}, reinterpret_cast<d2 *>(pnew + ea));
            __builtin_nontemporal_store(d2{pb.v[0], pb.v[1]}, reinterpret_cast<d2 *>(pnew + ea + 128));
            __builtin_nontemporal_store(d2{qv.v[0], qv.v[1]}, reinterpret_cast<d2 *>(q + ea));
            __builtin_nontemporal_store(d2{qv.v[2], qv.v[3]}, reinterpret_cast<d2 *>(q + ea + 128));
            acc[0] = __builtin_fma(pa.v[0], qv.v[0], acc[0]);
            acc[0] = __builtin_fma(pa.v[1], qv.v[1], acc[0]);
            acc[0] = __builtin_fma(pb.v[0], qv.v[2], acc[0]);
            acc[0] = __builtin_fma(pb.v[1], qv.v[3], acc[0]);
            pa_prev = pa;
            pb_prev = pb;
            pa = pa_next;
            pb = pb_next;
        }
    }
    block_partials<1>(acc, part_a, lds);
}

template <bool VAR>
LG_REDUCE_KERNEL void pcg_b_kernel(Grid g, double *__restrict__ r, const double *__restrict__ q,
                                   const double *part_a, int nb_a, double *part_b, PcgState *st, int k) {
    __shared__ double lds[kLdsDoubles];
    if (pcg_done(st)) return;
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
        st->alpha = alpha;
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
    if (g.kx) {
        if (g.aligned) pcg_init_kernel<true, true><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
        else pcg_init_kernel<true, false><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
    } else {
        if (g.aligned) pcg_init_kernel<false, true><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
        else pcg_init_kernel<false, false><<<gr, kBlock, 0, s>>>(g, b, x, r, part_b);
    }
    return GUESS_OK;
}

template <bool VAR, bool AL>
static void pcg_iter_v(const Grid &g, double *x, double *r, double *const p[2], double *q, double *part_a,
                       double *part_b, PcgState *st, int k, double rtol, hipStream_t s) {
    const int gr = pcg_grid(g);
    double *pnew = p[k & 1];
    const double *pold = p[(k - 1) & 1];
    int ga = gr;
    if (!VAR && AL && march_ok(g) && march_enabled()) {
        const March m = make_march(g);
        ga = march_grid(m);
        pcg_a_march_kernel<<<ga, kBlock, 0, s>>>(g, m, x, r, pold, pnew, q, part_b, gr, part_a, st, k, rtol);
    } else {
        pcg_a_kernel<VAR, AL><<<gr, kBlock, 0, s>>>(g, x, r, pold, pnew, q, part_b, gr, part_a, st, k, rtol);
    }
    pcg_b_kernel<VAR><<<gr, kBlock, 0, s>>>(g, r, q, part_a, ga, part_b, st, k);
}

int launch_pcg_iter(const Grid &g, double *x, double *r, double *const p[2], double *q, double *part_a,
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
    if (pcg_done(st)) return;
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
            st->converged = 1;
            st->it = k - 1;
        }
    }
}

int launch_pcg_check(const Grid &g, const double *part_b, PcgState *st, int k, double rtol, hipStream_t s) {
    pcg_check_kernel<<<1, kBlock, 0, s>>>(part_b, pcg_grid(g), st, k, rtol);
    return GUESS_OK;
}

// The x update of the last completed iteration when no later pcg_a applied it.
__global__ __launch_bounds__(kBlock) void pcg_finish_kernel(Grid g, double *x, const double *p, PcgState *st) {
    if (!st->x_pending) return;
    x_update_all(g, x, p, st->alpha);
}

int launch_pcg_finish(const Grid &g, double *x, const double *p, PcgState *st, hipStream_t s) {
    pcg_finish_kernel<<<stream_grid(nchunks(g.n) > 0 ? nchunks(g.n) : 1, grid_cap()), kBlock, 0, s>>>(g, x, p, st);
    return GUESS_OK;
}

}  // namespace lg
