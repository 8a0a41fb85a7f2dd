// z-marching traversal for the 7-point stencils.
//
// Applies where every z-plane is a whole number of 4-tile groups (nx even,
// nx*ny a multiple of 1024).  A wave owns one 256-element tile of a z-plane
// (the same lane layout as the chunk form of common.h: lane L holds the
// pairs (2L, 2L+1) and (128+2L, 129+2L)) and sweeps it through a range of
// planes, keeping the operand of planes z-1, z, z+1 in registers.  Per plane
// it loads the operand once for plane z+1 and for the rows y-1, y+1, and
// takes the x-neighbours from the adjacent lanes; only the tile's first and
// last element may need one extra load (when the tile does not start or end
// a grid row).  The four workgroup waves own four consecutive tiles, and
// consecutive workgroups are placed on one XCD, so the y-neighbour rows are
// mostly read from that XCD's L2.
//
// Each point is evaluated with the fixed order of the chunk form (west,
// east, south, north, bottom, top, no contraction, then c*s + shift*u), so
// results are bit-identical to it; only the traversal differs.
#pragma once

#include <atomic>

#include "common.h"
#include "stencil.h"

namespace lg {

struct March {
    int tp;      // 256-element tiles per z-plane
    int nr;      // z ranges: range r covers planes [r*nz/nr, (r+1)*nz/nr)
    int items;   // tp * nr work items (one tile over one z range)
};

inline bool march_ok(const Grid &g) {
    return g.aligned && g.nxy % 256 == 0 && (g.nxy / 256) % kWaves == 0;
}

// LIBGUESS_MARCH_NR > 0 forces the number of z ranges (for measurements).
int march_nr_override();

// Work split: one work item (one tile over one z range) per wave.  A range
// of about kMarchPlanes planes amortises the start of a sweep (two planes
// loaded before the first result); more ranges are taken where that leaves
// resident workgroup slots (`wgs`) empty, fewer where the workgroups would
// exceed the partial-row capacity.  A plane too large for that capacity
// makes the waves loop over several items.  (Measured on 256^3 and 384^3:
// ranges of 16 planes or fewer, or splits that put several items on some
// waves, cost up to 30 % in the stencil kernels.)
constexpr int kMarchPlanes = 21;

inline March make_march(const Grid &g, int wgs) {
    March m;
    m.tp = (int)(g.nxy / 256);
    auto nwg = [&](int nr) { return ((int64_t)m.tp * nr + kWaves - 1) / kWaves; };
    const int64_t fill = wgs < kMaxPartialBlocks ? (wgs < 1 ? 1 : wgs) : kMaxPartialBlocks;
    int nr = (g.nz + kMarchPlanes / 2) / kMarchPlanes;
    if (nr < 1) nr = 1;
    while (nr < g.nz && nwg(nr) < fill) ++nr;
    while (nr > 1 && nwg(nr) > kMaxPartialBlocks) --nr;
    const int forced = march_nr_override();
    if (forced > 0) nr = forced < g.nz ? forced : g.nz;
    m.nr = nr;
    m.items = m.tp * nr;
    return m;
}

// Workgroups of kernel K (kBlock threads each) that are resident on the
// device at once: the runtime's occupancy per CU times the CU count, queried
// on first use (every device here is the same part).  LIBGUESS_MARCH_WGS
// overrides it (for measurements).
int march_wgs_override();

template <auto K>
int resident_wgs() {
    static std::atomic<int> cached{0};
    int n = cached.load(std::memory_order_relaxed);
    if (n > 0) return n;
    n = march_wgs_override();
    if (n <= 0) {
        int dev = 0, cus = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, K, kBlock, 0) != hipSuccess || per < 1) per = 4;
        n = per * cus;
    }
    cached.store(n, std::memory_order_relaxed);
    return n;
}

// Workgroups to launch: one per kWaves items, within the partial-row capacity.
inline int march_grid(const March &m) {
    const int n = (m.items + kWaves - 1) / kWaves;
    return n < kMaxPartialBlocks ? n : kMaxPartialBlocks;
}

__device__ __forceinline__ R2 sel2(bool keep, const R2 &v) {
    return R2{{keep ? v.v[0] : 0.0, keep ? v.v[1] : 0.0}};
}

// (A u) at one element: fixed order west, east, south, north, bottom, top.
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

// (A u) at one element, variable coefficient: faces west, east, south,
// north, bottom, top in this order, then c*s + shift*u.
__device__ __forceinline__ double q_var(const Grid &g, double uc, double kw, double w, double ke, double e,
                                        double ks, double s_, double kn, double n, double kb, double b, double kt,
                                        double t) {
#pragma clang fp contract(off)
    double s = kw * (uc - w);
    s = s + ke * (uc - e);
    s = s + ks * (uc - s_);
    s = s + kn * (uc - n);
    s = s + kb * (uc - b);
    s = s + kt * (uc - t);
    const double a = g.c * s;
    const double bb = g.shift * uc;
    return a + bb;
}

// Sweep the wave's work items.  U: operand access (u(q), u.two(q) as in
// stencil.h).  pf(c) loads whatever the chunk's work needs besides the
// stencil (other vectors at chunk c) and returns it; f(c, e, ua, ub, au, pre)
// is called once per chunk with its chunk index c (as in common.h), the flat
// index e of its first pair, the centre values of both pairs, A u at the
// chunk's four elements and pf's result for that chunk.  The sweep issues
// pf for plane z+1 together with that plane's operand loads, one plane ahead
// of f, so that those loads overlap the current plane's work.  VAR: variable
// coefficient (face arrays of the Grid; the z-faces shared by consecutive
// planes are loaded once).
template <bool VAR, class U, class PF, class F>
__device__ __forceinline__ void march_sweep_pf(const Grid &g, const March &m, const U &u, PF &&pf, F &&f) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nwg = gridDim.x;
    const int lb = nwg % kXcds == 0 ? (int)(blockIdx.x % kXcds) * (nwg / kXcds) + (int)(blockIdx.x / kXcds)
                                    : (int)blockIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int64_t nxy = g.nxy;
    const int64_t cstep = (int64_t)m.tp * 64;     // chunks per plane
    for (int item = lb * kWaves + wave; item < m.items; item += nwg * kWaves) {
        const int tau = item % m.tp, zr = item / m.tp;
        const int z0 = (int)((int64_t)zr * nz / m.nr);
        const int z1 = (int)((int64_t)(zr + 1) * nz / m.nr);
        const int64_t offa = (int64_t)tau * 256 + 2 * lane, offb = offa + 128;
        const uint32_t ja = fdiv(g.fnx, (uint32_t)offa), jb = fdiv(g.fnx, (uint32_t)offb);
        const int ia = (int)((uint32_t)offa - ja * (uint32_t)nx), ib = (int)((uint32_t)offb - jb * (uint32_t)nx);
        const bool hwa = ia > 0, hea = ia + 2 < nx, hwb = ib > 0, heb = ib + 2 < nx;
        const bool hsa = ja > 0, hna = (int)ja < ny - 1, hsb = jb > 0, hnb = (int)jb < ny - 1;
        int64_t ea = (int64_t)z0 * nxy + offa;
        int64_t c = ((int64_t)z0 * m.tp + tau) * 64 + lane;
        const int64_t eprev = z0 > 0 ? ea - nxy : ea;
        R2 pa_prev = sel2(z0 > 0, u.two(eprev)), pb_prev = sel2(z0 > 0, u.two(eprev + 128));
        R2 pa = u.two(ea), pb = u.two(ea + 128);
        auto pre = pf(c);
        // bottom z-faces of plane z0 (face index f = z: kz[(f*ny + j)*nx + i] = kz[e])
        R2 kba{{0.0, 0.0}}, kbb{{0.0, 0.0}};
        if constexpr (VAR) {
            kba = ld2(g.kz, ea);
            kbb = ld2(g.kz, ea + 128);
        }
        for (int z = z0; z < z1; ++z, ea += nxy, c += cstep) {
            const bool ht = z + 1 < nz;
            const int64_t enext = ht ? ea + nxy : ea;
            const R2 pa_next = sel2(ht, u.two(enext)), pb_next = sel2(ht, u.two(enext + 128));
            // the next plane's other data (the current chunk again on the range's last plane,
            // so every load stays inside the vectors)
            const auto pre_next = pf(z + 1 < z1 ? c + cstep : c);
            const R2 sa = sel2(hsa, u.two(hsa ? ea - nx : ea)), na = sel2(hna, u.two(hna ? ea + nx : ea));
            const R2 sb = sel2(hsb, u.two(hsb ? ea + 128 - nx : ea + 128));
            const R2 nb = sel2(hnb, u.two(hnb ? ea + 128 + nx : ea + 128));
            // x-neighbours across lanes; the tile's outer neighbours by load
            double ew = 0.0, ee = 0.0;
            if (lane == 0 && hwa) ew = u(ea - 1);
            if (lane == 63 && heb) ee = u(ea + 256 - 2 * 63);
            const double wa_ = __shfl(pa.v[1], (lane + 63) & 63, 64);
            const double wb_ = __shfl(pb.v[1], (lane + 63) & 63, 64);
            const double ea_ = __shfl(pa.v[0], (lane + 1) & 63, 64);
            const double eb_ = __shfl(pb.v[0], (lane + 1) & 63, 64);
            const double wa = hwa ? (lane > 0 ? wa_ : ew) : 0.0;
            const double wb = hwb ? (lane > 0 ? wb_ : wa_) : 0.0;
            const double eaa = hea ? (lane < 63 ? ea_ : eb_) : 0.0;
            const double ebb = heb ? (lane < 63 ? eb_ : ee) : 0.0;
            R4 au;
            if constexpr (!VAR) {
                au.v[0] = q_const(g, pa.v[0], wa, pa.v[1], sa.v[0], na.v[0], pa_prev.v[0], pa_next.v[0]);
                au.v[1] = q_const(g, pa.v[1], pa.v[0], eaa, sa.v[1], na.v[1], pa_prev.v[1], pa_next.v[1]);
                au.v[2] = q_const(g, pb.v[0], wb, pb.v[1], sb.v[0], nb.v[0], pb_prev.v[0], pb_next.v[0]);
                au.v[3] = q_const(g, pb.v[1], pb.v[0], ebb, sb.v[1], nb.v[1], pb_prev.v[1], pb_next.v[1]);
            } else {
                // x-faces of each pair's row (nx+1 per row), y-faces south / north, z-faces top
                const int64_t rxa = ((int64_t)z * ny + ja) * (nx + 1) + ia;
                const int64_t rxb = ((int64_t)z * ny + jb) * (nx + 1) + ib;
                const int64_t rya = ((int64_t)z * (ny + 1) + ja) * nx + ia;
                const int64_t ryb = ((int64_t)z * (ny + 1) + jb) * nx + ib;
                const double xa0 = g.kx[rxa], xa1 = g.kx[rxa + 1], xa2 = g.kx[rxa + 2];
                const double xb0 = g.kx[rxb], xb1 = g.kx[rxb + 1], xb2 = g.kx[rxb + 2];
                const R2 ksa = ld2(g.ky, rya), kna = ld2(g.ky, rya + nx);
                const R2 ksb = ld2(g.ky, ryb), knb = ld2(g.ky, ryb + nx);
                const R2 kta = ld2(g.kz, ea + nxy), ktb = ld2(g.kz, ea + 128 + nxy);
                au.v[0] = q_var(g, pa.v[0], xa0, wa, xa1, pa.v[1], ksa.v[0], sa.v[0], kna.v[0], na.v[0], kba.v[0],
                                pa_prev.v[0], kta.v[0], pa_next.v[0]);
                au.v[1] = q_var(g, pa.v[1], xa1, pa.v[0], xa2, eaa, ksa.v[1], sa.v[1], kna.v[1], na.v[1], kba.v[1],
                                pa_prev.v[1], kta.v[1], pa_next.v[1]);
                au.v[2] = q_var(g, pb.v[0], xb0, wb, xb1, pb.v[1], ksb.v[0], sb.v[0], knb.v[0], nb.v[0], kbb.v[0],
                                pb_prev.v[0], ktb.v[0], pb_next.v[0]);
                au.v[3] = q_var(g, pb.v[1], xb1, pb.v[0], xb2, ebb, ksb.v[1], sb.v[1], knb.v[1], nb.v[1], kbb.v[1],
                                pb_prev.v[1], ktb.v[1], pb_next.v[1]);
                kba = kta;
                kbb = ktb;
            }
            f(c, ea, pa, pb, au, pre);
            pre = pre_next;
            pa_prev = pa;
            pb_prev = pb;
            pa = pa_next;
            pb = pb_next;
        }
    }
}

// The sweep without other data: f(c, e, ua, ub, au).
template <bool VAR, class U, class F>
__device__ __forceinline__ void march_sweep(const Grid &g, const March &m, const U &u, F &&f) {
    march_sweep_pf<VAR>(g, m, u, [](int64_t) { return 0; },
                        [&](int64_t c, int64_t e, const R2 &pa, const R2 &pb, const R4 &au, int) { f(c, e, pa, pb, au); });
}

}  // namespace lg
