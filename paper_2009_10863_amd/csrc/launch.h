// Host-side launchers of the libguess kernels (one translation unit per family).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "libguess.h"
#include "stencil.h"

namespace lg {

// Optional per-kernel timing: with events, the i-th kernel of a launcher is
// dispatched through hipExtLaunchKernel, whose dispatch packet itself stamps
// start[i] and stop[i], so the measured time is the kernel's own run time.
struct KEvents {
    hipEvent_t start[8], stop[8];
    int count;          // kernels launched (set by the launcher)
};

template <typename... Args, typename F = void (*)(Args...)>
inline void klaunch_sh(KEvents *ev, int i, F f, int grid, int block, size_t shmem, hipStream_t s, Args... args) {
    if (ev) {
        hipExtLaunchKernelGGL(f, dim3(grid), dim3(block), shmem, s, ev->start[i], ev->stop[i], 0, args...);
        ev->count = i + 1;
    } else {
        hipLaunchKernelGGL(f, dim3(grid), dim3(block), shmem, s, args...);
    }
}
template <typename... Args, typename F = void (*)(Args...)>
inline void klaunch(KEvents *ev, int i, F f, int grid, int block, hipStream_t s, Args... args) {
    klaunch_sh<Args...>(ev, i, f, grid, block, 0, s, args...);
}

// Device-resident state of a projection history.  Decisions (restart,
// accept / reject) are taken on the device, so a sequence of guess_form /
// guess_update calls never waits for the host.
struct ProjState {
    int d;                  // columns in the history
    int mode;               // 1 while the current update is a restart
    int last_accepted;
    int restarts;
    int rejects;
    int nonfinite;          // sticky
    int M;
    int form_d;             // columns used by the last guess (written by proj_combine)
    int upd_d;              // columns at the start of the last update (written by proj_apply)
    int drop;               // rolling variant: the current update drops the oldest column
    int drops;              // rolling variant: drops so far
    int pad;
    double eps_rel;
    double nu0sq, nusq, nu0, nu;
    double pow2;            // power of two the current update's new pair is stored multiplied by
    double scale[GUESS_MAX_M];   // column j of X (and B) = scale[j] * stored column j
    double gamma[GUESS_MAX_M];   // guess: x0 = sum_j gamma[j] * stored X_j
    double c[GUESS_MAX_M];       // update: Gram-Schmidt coefficients (true units)
    double cs[GUESS_MAX_M];      // update: coefficients of the stored columns
    double R[GUESS_MAX_M][GUESS_MAX_M];  // raw solutions of the history = X R (upper triangular)
    double gc[GUESS_MAX_M], gs[GUESS_MAX_M];  // rolling drop: Givens rotations (c, s)
    double rot[GUESS_MAX_M][4];  // rolling drop: the rotations in stored units, per slot
    // FP16 storage only:
    double mu[GUESS_MAX_M];      // largest true magnitude of stored pair j (X_j and B_j together)
    double nscale[GUESS_MAX_M];  // rolling drop: scale of each rotated slot, committed by the update's end
};

// Device-resident state of an FP16 extrapolation ring: every slot holds
// round(2^e x) with its own exponent e (from max |x|).  A store first tries
// the exponent of the previous store, reduces max |x| alongside, and a
// second kernel re-stores the slot only when the exponent differs.
struct RingState {
    unsigned long long maxbits[2];  // bits of max |x| of the store in flight (two, alternating)
    int e_used[2];                  // exponent each in-flight store was written with
    int e_guess;                    // exponent the next store tries
    int last_fixed;                 // the last update re-stored its slot
    int fixes;                      // re-stores so far
    int pad;
    int exps[GUESS_MAX_M + 1];      // exponent of each physical slot
};

// Device-resident state of a PCG solve (rho of iteration k in rho[k & 1]).
struct PcgState {
    double rho[2];
    double alpha[2];        // alpha_k of iteration k at [k & 1]
    double rr, bb, rr0, thresh;
    int it;
    int converged;          // 0, or the iteration k whose stop test (on r_{k-1}) passed
    int breakdown, rule;
    int x_last;             // last completed iteration (alpha_k known)
    int x_pending;          // x still lacks the updates of x_last and, if x_last is even, x_last - 1
};

// ---- extrapolation (extrap.hip)
int launch_extrap_form(int dtype, int k, const void *const *slots, const double *beta,
                       double *x0, int64_t N, hipStream_t s, KEvents *ev = nullptr,
                       const RingState *rs = nullptr, const int *slot_index = nullptr);
int launch_ring_store(int dtype, const double *x, void *slot, int64_t N, hipStream_t s,
                      KEvents *ev = nullptr, RingState *rs = nullptr, int slot_index = 0, int gen = 0);
int launch_fill_zero(double *x, int64_t N, hipStream_t s);
int launch_widen(int dtype, const void *src, double scale, double *out, int64_t N, hipStream_t s);

// Device-resident state of a raw-solution projection history (rawproj_impl.h):
// the stored solutions' slots, their Gram matrix G = W^T A W and its Cholesky
// factor L (FP64, oldest solution first), FP16 exponents.
struct RawState {
    int d;                       // stored solutions
    int last_accepted, restarts, rejects, nonfinite, drops, form_d, upd_d;
    int perm[GUESS_MAX_M];       // slot of the j-th oldest stored solution
    int exps[GUESS_MAX_M];       // FP16: exponent of each slot (stored = round(2^e x)); else 0
    int e_guess;                 // FP16: exponent the next store tries first
    int e_used;                  // FP16: exponent the store of this update used
    int new_exp;                 // FP16: exponent of this update's solution
    int fixed;                   // FP16: this update stored its slot twice
    unsigned long long maxbits;  // FP16: bits of max |x| of the store in flight
    double eps_rel, nu0, nu;
    double G[GUESS_MAX_M][GUESS_MAX_M];
    double L[GUESS_MAX_M][GUESS_MAX_M];
    double gamma[GUESS_MAX_M];   // guess: x0 = sum_j gamma[j] * stored column perm[j]
};

struct RawBufs {
    void *W;                 // M slots of N elements of the storage type
    double *part;            // per-workgroup partial sums
    RawState *st;
    int64_t N, ld;
    int M, qr, dtype;
};
int launch_raw_form(const RawBufs &p, const double *b, double *x0, hipStream_t s, KEvents *ev = nullptr);
int launch_raw_update(const RawBufs &p, const Grid &g, const double *x, hipStream_t s, KEvents *ev = nullptr);

// ---- projection (proj.hip)
struct ProjBufs {
    void *X;                 // M stored columns of X, each N elements of the storage type
    void *B;                 // M stored columns of B = A X
    double *w;               // FP64 scratch N (A x of the current update)
    double *part;            // per-workgroup partial sums
    ProjState *st;           // device state
    int64_t N, ld;           // ld: elements between consecutive columns
    int M, dtype;
    int vf;                  // variant flags: 1 rolling QR, 2 l2 inner product
};
int launch_proj_form(const ProjBufs &p, const double *b, double *x0, hipStream_t s,
                     KEvents *ev = nullptr);
int launch_proj_update(const ProjBufs &p, const Grid *g, const double *x, const double *Ax,
                       hipStream_t s, KEvents *ev = nullptr);

// ---- operator and PCG (op.hip)
int launch_build_faces(Grid &g, const double *kappa, double *kx, double *ky, double *kz,
                       double *dinv, hipStream_t s);
int launch_op_apply(const Grid &g, const double *x, double *y, hipStream_t s);
int launch_pcg_init(const Grid &g, const double *b, const double *x, double *r, double *part_b,
                    hipStream_t s);
int launch_pcg_iter(const Grid &g, double *x, double *r, double *const p[3], double *q, double *part_a,
                    double *part_b, PcgState *st, int k, double rtol, hipStream_t s);
int launch_pcg_check(const Grid &g, const double *part_b, PcgState *st, int k, double rtol, hipStream_t s);
int launch_pcg_finish(const Grid &g, double *x, double *const p[3], PcgState *st, hipStream_t s);
int pcg_grid(const Grid &g);

// ---- vectors and workload (vec.hip)
int launch_multidot(int64_t N, int K, const double *V, const double *y, double *part,
                    double *out_dev, hipStream_t s);
int launch_combine(int64_t N, int K, const double *V, const double *c, double *y, hipStream_t s);
int launch_copy(void *dst, const void *src, size_t bytes, hipStream_t s);
int launch_read(const void *src, size_t bytes, double *out, hipStream_t s);
int launch_read_streams(const void *src, size_t bytes, double *out, hipStream_t s);
int launch_write(void *dst, size_t bytes, hipStream_t s);
int launch_plane_wave_rhs(int n, int K, const double *tabx, const double *taby,
                          const double *tabz, const double *amp, double *b, hipStream_t s);
int launch_gaussian_rhs(int n, const double *center, double sigma, double amp, double *tab, double *b,
                        hipStream_t s);

// grid-size knob for the streaming kernels (LIBGUESS_GRID_CAP, default below)
int grid_cap();
// workgroups of the Gram-Schmidt write pass (LIBGUESS_WRITE_BLOCKS; 0: one chunk per thread)
int write_blocks();
// LDS bytes reserved (unused) by each workgroup of the kernels that combine many stored
// vectors into one (extrapolation, projection combination), which caps how many of their
// workgroups a CU holds at once (LIBGUESS_GATHER_LDS, default 65536: two per CU)
int gather_lds();
// the raw-solution projection's operator apply in the z-marching form also for 2-byte formats
// (LIBGUESS_RAW_MARCH, default 0; FP32 always marches)
bool raw_march();
int reduce_blocks();
bool march_enabled();

}  // namespace lg
