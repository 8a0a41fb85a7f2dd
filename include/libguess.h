/*
 * libguess -- initial guesses for sequences of SPD linear solves, MI355X (gfx950).
 *
 * Method: A. P. Austin, N. Chalmers, T. Warburton, "Initial Guesses for
 * Sequences of Linear Systems in a GPU-Accelerated Incompressible Flow
 * Solver" (2020).  The guess methods are:
 *
 *   - stabilized least-squares polynomial extrapolation (§3.2, eq.
 *     LSQRCoeffs; the guess is the fixed combination of eq. ExtrapExpn),
 *     with the previous-solution guess as its M = 1 case (§3.1);
 *   - sparse extrapolation (§3.3, eq. CPQRCoeffs): m+1 of the M stored
 *     solutions, chosen by column-pivoted QR;
 *   - Fischer's projection (§2), with the history bounded by restarts
 *     (classic, Algorithm 1) or by a rolling window kept with a QR update
 *     (Algorithm 2).  By default in A-orthonormal form: the history keeps X
 *     with X^T A X = I and B = A X and the guess is X (X^T b); optionally in
 *     the paper's l2 form: B^T B = I and the guess is X (B^T b).  Each update
 *     applies A once and runs twice-iterated classical Gram-Schmidt.
 *
 * around a matrix-free 7-point Helmholtz / variable-coefficient operator
 * and a Jacobi-preconditioned CG (§5.3) that measures the guesses by the iterations they save.
 *
 * Conventions (every entry point):
 *   - Vectors are FP64, length N, on the device of the calling thread's
 *     current HIP device, owned by the caller.  The library never frees or
 *     retains caller memory beyond the call.
 *   - Grids are n_x x n_y x n_z interior nodes, flattened with x fastest;
 *     boundary values are the Dirichlet value 0 and are not stored.
 *   - Work is enqueued on the stream bound to the context or operator
 *     (NULL = the null stream).  guess_form, guess_update and op_apply return
 *     without a host synchronisation; pcg_solve and guess_get_info
 *     synchronise that stream.
 *   - Every function returns a status code (GUESS_OK = 0 or a negative
 *     error); no C++ exception crosses the boundary.  guess_last_error()
 *     gives a message for the calling thread's last failure.
 *   - A context or operator must not be used from two threads at once;
 *     distinct contexts are independent.
 */
#ifndef LIBGUESS_H
#define LIBGUESS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct guess_ctx *guess_t;
typedef struct guess_op *guess_op_t;

/* guess methods */
enum {
    GUESS_ZERO = 0,   /* x0 = 0                                                    */
    GUESS_LAST = 1,   /* x0 = previous solution (extrapolation with M = 1, §3.1)    */
    GUESS_EXTRAP = 2, /* least-squares extrapolation of degree m over M solutions  */
    GUESS_PROJ = 3,   /* A-orthonormal projection, classic restart (§2, Alg. 1)     */
    GUESS_SPEXTRAP = 4, /* sparse extrapolation: m+1 of M solutions chosen by
                           column-pivoted QR (§3.3, eq. CPQRCoeffs)               */
    GUESS_PROJ_QR = 5,  /* projection, rolling window with QR update (§2, Alg. 2) */
    GUESS_PROJ_RAW = 6, /* projection through the Gram matrix of the stored raw
                           solutions, classic restarts (guess_update)             */
    GUESS_PROJ_RAW_QR = 7 /* the same with the rolling window (drop the oldest)      */
};

/* projection inner product */
enum {
    GUESS_INNER_A = 0,  /* X^T A X = I, x0 = X (X^T b): minimises the A-norm error       */
    GUESS_INNER_L2 = 1  /* B^T B = I, x0 = X (B^T b): minimises ||b - A x0||_2 (§2)      */
};

/* storage format of the history vectors */
enum { GUESS_F64 = 0, GUESS_F32 = 1, GUESS_F16 = 2, GUESS_BF16 = 3 };

/* status codes */
enum {
    GUESS_OK = 0,
    GUESS_EINVAL = -1,      /* invalid argument                        */
    GUESS_ENOMEM = -2,      /* device allocation failed                */
    GUESS_EHIP = -3,        /* HIP runtime error                       */
    GUESS_ENOTCONV = -4,    /* pcg_solve: maxit reached                */
    GUESS_EBREAKDOWN = -5,  /* pcg_solve: p^T A p <= 0 or not finite  */
    GUESS_ENONFINITE = -6   /* non-finite value where one is required  */
};

/* PCG stopping rules (§6.4) */
enum {
    GUESS_STOP_RHS = 0,       /* ||r|| <= rtol ||b||                                   */
    GUESS_STOP_INITRESID = 1  /* ||r|| <  rtol max(||r0||, 1): the paper's default rule */
};

/* ------------------------------------------------------------------ operator */

/*
 * The operator replaces the paper's spectral-element discretisation of §5
 * (whose mesh and solver are not part of the guess method): a 7-point
 * finite-difference Helmholtz / variable-coefficient operator, symmetric
 * positive definite, so every guess method and the PCG of §5.3 apply as
 * stated.  Create the operator A on an nx x ny x nz grid of interior nodes:
 *   kappa == NULL:  (Au)_i = inv_h2 (6 u_i - sum_nb u_nb) + shift u_i
 *   kappa != NULL:  (Au)_i = inv_h2 sum_faces k_f (u_i - u_nb) + shift u_i,
 *                   k_f = 2 k_i k_nb / (k_i + k_nb),
 * with kappa a device array of nodal values on all (nx+2)(ny+2)(nz+2) nodes
 * (boundary included, x fastest), read once here and not retained (its size
 * cannot be checked here: a shorter array is read past its end).  For the
 * unit cube with n^3 interior nodes inv_h2 = (n+1)^2.  Neighbour order and
 * rounding are fixed: west, east, south, north, bottom, top, summed left to
 * right without fused multiply-add, then inv_h2 * s + shift * u.
 * Requires nx, ny, nz >= 1, inv_h2 > 0, shift >= 0; EINVAL otherwise.
 */
int guess_op_create(int nx, int ny, int nz, double inv_h2, double shift,
                    const double *kappa, guess_op_t *out);
void guess_op_destroy(guess_op_t A);
/* Bind a hipStream_t (passed as void*) to the operator and its PCG. */
int guess_op_set_stream(guess_op_t A, void *stream);
/* Number of unknowns nx*ny*nz. */
int64_t guess_op_size(guess_op_t A);

/* y = A x (the operator above, evaluated in the fixed order stated there).
 * x and y are device vectors of guess_op_size(A) doubles, 16-byte aligned,
 * and must not alias (EINVAL).  Enqueued on the operator's stream. */
int op_apply(guess_op_t A, const double *x, double *y);

/*
 * Jacobi-preconditioned CG (§5.3) for A x = b.  x holds the initial guess on
 * entry and the solution on exit.  Stops when the recurrence residual meets
 * the rule (GUESS_STOP_RHS or GUESS_STOP_INITRESID) with tolerance rtol, the
 * test also applied before the first iteration (a guess that already meets
 * it costs 0 iterations).  On return *iters = number of operator
 * applications in the loop, *relres = ||r|| / ||b|| (||r|| when b = 0).
 * Returns GUESS_OK, GUESS_ENOTCONV (maxit reached; x holds the last iterate)
 * or GUESS_EBREAKDOWN.  iters / relres may be NULL.  Synchronises the stream.
 */
int pcg_solve(guess_op_t A, const double *b, double *x, double rtol, int maxit,
              int *iters, double *relres);
int pcg_solve_ex(guess_op_t A, const double *b, double *x, double rtol, int maxit,
                 int stop_rule, int *iters, double *relres);

/* ------------------------------------------------------------------ guesses */

typedef struct guess_opts {
    int64_t N;          /* vector length, >= 1                                      */
    int M;              /* history size, 1 <= M <= GUESS_MAX_M                      */
    int method;         /* GUESS_ZERO / LAST / EXTRAP / PROJ / SPEXTRAP / PROJ_QR    */
    int degree;         /* EXTRAP, SPEXTRAP: polynomial degree m, 0 <= m <= M - 1    */
    int dtype;          /* storage format of the history (GUESS_F64 ...)             */
    double eps_rel;     /* PROJ: reject if nu <= eps_rel * nu0; <= 0 selects the default
                           of the storage format: 1e-6 (F64), 1e-4 (F32), 1e-2 (F16, BF16),
                           which grows with its unit roundoff; PROJ_RAW: 1e-6          */
    guess_op_t op;      /* PROJ: operator applied in guess_update when Ax == NULL    */
    void *stream;       /* hipStream_t; NULL = null stream                           */
    int inner;          /* PROJ, PROJ_QR: GUESS_INNER_A (default) or GUESS_INNER_L2  */
    void *workspace;    /* NULL, or caller device memory, 256-byte aligned, that holds the
                           history and scratch (guess_workspace_bytes); the library then
                           allocates no device memory for the context and never frees it */
    size_t workspace_bytes;
} guess_opts;

#define GUESS_MAX_M 16

/*
 * Create a context with FP64 history, eps_rel = 1e-6, no operator, the null
 * stream.  LAST forces M = 1.  Returns NULL on failure (see guess_last_error).
 * The history bound M is the paper's M (§2, Algorithms 1 and 2; §3.2, the M
 * solutions the extrapolation fits), the degree its m (§3.2).  The rejection
 * threshold reads the paper's absolute epsilon of §2 (which depends on the
 * solver's stopping criterion) as relative: a new solution is kept iff its
 * A-norm after Gram-Schmidt exceeds eps_rel times its A-norm before, so the
 * test does not depend on the scale of the solutions.
 */
guess_t guess_create(int64_t N, int M, int method, int degree);
/* As guess_create with every option of guess_opts (storage format, eps_rel,
 * operator, stream, inner product, caller workspace).  *out receives the
 * context, or NULL with a status: EINVAL for a bad option (the checks are
 * listed with guess_opts), ENOMEM when a device allocation fails. */
int guess_create_ex(const guess_opts *o, guess_t *out);
void guess_destroy(guess_t g);
int guess_set_stream(guess_t g, void *stream);
int guess_set_op(guess_t g, guess_op_t A);
/* Device bytes the history and scratch of such a context occupy (the size a
 * caller workspace must have; buffers inside it are 256-byte aligned).  An
 * FP64 extrapolation ring has M + 1 slots (see guess_next_slot). */
size_t guess_workspace_bytes(int64_t N, int M, int method, int dtype);

/*
 * Form the initial guess x0 for right-hand side b.
 *   EXTRAP / LAST: x0 = sum_j beta_j h_j over the k stored solutions, oldest
 *     first (eq. ExtrapExpn), with beta the least-squares weights of degree
 *     min(m, k-1) over k nodes (warm-up while k < M); x0 = 0 when k = 0.
 *     b is not read and may be NULL.  x0 may alias the caller's solve buffer.
 *   SPEXTRAP: as EXTRAP with the sparse weights of guess_spextrap_weights;
 *     only the m+1 solutions with a nonzero weight are read.
 *   PROJ, PROJ_QR: x0 = X (X^T b) (l2: X (B^T b)), x0 = 0 when the
 *     history is empty.  b is required and must not alias x0.
 *   ZERO: x0 = 0.
 * FP64 history accumulates in FP64; reduced-precision history is read,
 * widened and accumulated in FP32 (extrapolation) or FP64 (projection).
 */
int guess_form(guess_t g, const double *b, double *x0);

/*
 * Raw-solution projection (GUESS_PROJ_RAW, GUESS_PROJ_RAW_QR).  The guess of
 * §2 -- the A-norm-optimal combination of the stored solutions -- computed
 * from the stored solutions W themselves and their Gram matrix G = W^T A W
 * (FP64, with its Cholesky factor L, on the device) instead of an
 * A-orthonormal basis: x0 = W y with G y = W^T b; a new solution w (rounded
 * to the storage format; FP16 as round(2^e x) with e from max |x|) is kept iff
 * nu > eps_rel * nu0, nu^2 = w^T A w - g^T G^{-1} g, g = W^T A w, nu0^2 = w^T A w
 * (the A-norm of its part outside the stored span, and its own).  In exact
 * arithmetic the guesses and decisions are those of Algorithm 1 (classic
 * restarts) and Algorithm 2 (rolling window); the basis X = W L^-T, and
 * guess_proj_factor returns L^T (raw solutions = X R).  A reduced-precision
 * history keeps the exact projection onto the vectors actually stored, with no
 * normalised column whose rounding near-dependence could magnify; it needs
 * the bound operator (applied once per update, to the stored vector) and
 * takes no Ax.  Reduced-precision storage only (FP32, FP16, BF16; EINVAL for
 * FP64): in FP64 the Schur complement of nearly dependent exact solutions is
 * accurate only to u cond(G) w^T A w, far above eps_rel^2 w^T A w, while a
 * rounded history's own rounding keeps G's condition moderate.  Default
 * eps_rel 1e-6.  Bytes per unknown: guess 2 (d s + 8); update 8 + (d + 2) s
 * (FP16: 8 + s more when a solution's exponent differs from the previous one).
 */

/*
 * Add the solution x of the latest solve to the history (§2: the update of
 * Algorithms 1 and 2; §3.2: the extrapolation keeps the last M solutions).
 * x (and Ax) are device vectors of N doubles, 16-byte aligned, owned by the
 * caller and only read.
 *   EXTRAP / LAST: x is rounded to the storage format into the next ring slot;
 *     when x is that slot (guess_next_slot) nothing is copied.
 *   PROJ: Ax = A x if the caller has it (Ax = b is allowed, then
 *     X^T A X = I holds only to the solve tolerance); Ax == NULL makes the
 *     library apply the bound operator once (EINVAL if none is bound).
 *     Restart when the history is empty or full (slot 1 <- x / ||x||_A;
 *     Algorithm 1's restart step); otherwise two classical Gram-Schmidt
 *     passes in the A inner product (Algorithm 1's orthogonalisation),
 *     then the new pair is kept iff nu > eps_rel * nu0 (nu, nu0 the A-norms
 *     after / before orthogonalisation).  The decision is taken on the
 *     device; a non-finite nu rejects the vector and sets a sticky flag.
 *   PROJ_QR: as PROJ, except that a full history (d = M) drops its oldest
 *     solution instead of restarting: the factor R of raw solutions = X R
 *     loses its first column and Givens rotations of neighbouring rows make
 *     it triangular again (rotation of a over b: c = |a|/r, s = sign(a) b/r,
 *     r = sqrt(a^2 + b^2), sign(0) = 1); the columns of X and B are rotated
 *     alike, then the new solution is orthogonalised as above.  With M = 1
 *     every update replaces the single column.
 *   GUESS_INNER_L2: inner products b_j^T b~ and norms ||b~||_2 in place of
 *     the A inner product and A-norm.
 *   ZERO: nothing.
 */
int guess_update(guess_t g, const double *x, const double *Ax);

/*
 * Solving in place (§4: extrapolation then moves (M+1) N values per step and
 * the update copies nothing).  An FP64 extrapolation ring (EXTRAP, LAST,
 * SPEXTRAP) keeps one slot more than M: the slot the next update writes,
 * which no guess reads.  *slot receives its device address (N doubles);
 * the caller may form the guess into it, solve there, and pass it to
 * guess_update, which then only advances the ring.  The address changes
 * with every update.  EINVAL for other methods or storage formats.
 */
int guess_next_slot(guess_t g, double **slot);

typedef struct guess_info {
    int64_t N;
    int method, dtype, M, degree;
    int count;          /* EXTRAP/LAST: stored solutions (<= M); PROJ: columns d      */
    int head;           /* EXTRAP/LAST: ring slot the next update writes (of M + 1
                           slots for FP64 history, M otherwise)                       */
    int last_accepted;  /* PROJ: 1 if the last update stored its vector                */
    int restarts;       /* PROJ: restarts so far                                       */
    int rejects;        /* PROJ: rejected vectors so far                               */
    int nonfinite;      /* sticky: a non-finite norm or value was met                  */
    double nu, nu0;     /* PROJ: last A-norms after / before Gram-Schmidt             */
    double form_bytes;  /* algorithmic HBM bytes of the last guess_form                */
    double update_bytes;/* algorithmic HBM bytes of the last guess_update              */
    int drops;          /* PROJ_QR: oldest-solution drops so far                       */
    int inner;          /* PROJ, PROJ_QR: GUESS_INNER_A / GUESS_INNER_L2               */
    double eps_rel;     /* PROJ, PROJ_QR: rejection threshold in use                   */
} guess_info;

/* Snapshot of the context state.  Synchronises the context's stream. */
int guess_get_info(guess_t g, guess_info *info);
/* Empty the history (EXTRAP: count = 0; PROJ: d = 0). */
int guess_reset(guess_t g);

/*
 * Least-squares extrapolation weights of degree m over k equispaced
 * solutions (§3.2, eq. LSQRCoeffs), computed on the host in FP64 with a
 * Legendre basis and Householder QR.  beta[0] multiplies the oldest
 * solution.  Requires 1 <= k <= GUESS_MAX_M, 0 <= m <= k - 1.
 */
int guess_extrap_weights(int m, int k, double *beta);

/*
 * Sparse extrapolation weights (§3.3, eq. CPQRCoeffs): column-pivoted QR of
 * V^T (Legendre basis on the nodes of §3.2) selects m+1 of the k stored
 * solutions; their weights make the scheme exact for polynomials of degree
 * <= m (eq. PolyExactness) and the other k-m-1 weights are exactly 0.
 * Pivot norms within a relative 1e-10 of the largest count as tied and the
 * oldest tied solution is taken.  Host-only, FP64; beta[0] multiplies the
 * oldest solution.  Requires 1 <= k <= GUESS_MAX_M, 0 <= m <= k - 1.
 */
int guess_spextrap_weights(int m, int k, double *beta);

/* Copy stored history vector j (PROJ: column j of X (which = 0) or B
 * (which = 1), scale applied; EXTRAP and PROJ_RAW: j-th oldest stored
 * solution (which = 0), FP16 slots descaled) into the FP64 device vector
 * out.  For tests and checkpoints; synchronises. */
int guess_history_get(guess_t g, int which, int j, double *out);

/*
 * The same vector as the storage format holds it: out receives the stored
 * values widened to FP64 without any scale, *scale (host) the FP64 factor
 * that turns them into the true values.  Reduced-precision storage (the
 * paper fixes no precision; the reading is the library's): a projection
 * column is the stored pair round(2^e x''), round(2^e b'') with scale
 * 1 / (nu 2^e) -- in exact arithmetic the normalised column of §2's update
 * step -- e = 0 except for FP16, where max |stored| lies in [2^14, 2^15);
 * an FP16 extrapolation slot holds round(2^e x) with scale 2^-e; other
 * slots have scale 1.  Same indices and errors as guess_history_get
 * (GUESS_EINVAL for an index out of range or a method without history);
 * out is a device vector of N doubles owned by the caller.  Synchronises.
 */
int guess_history_raw(guess_t g, int which, int j, double *out, double *scale);

/*
 * PROJ, PROJ_QR: the triangular factor of the history, raw solutions = X R
 * (§2, Algorithm 2; kept for both variants), with X the true columns.  The
 * raw solutions are the accepted ones since the last restart (classic) or
 * the window of the last d accepted ones (rolling).  Writes *d and the d x d
 * factor row-major into R (room for GUESS_MAX_M^2 values, host memory).
 * PROJ_RAW, PROJ_RAW_QR: R = L^T, L the Cholesky factor of the stored
 * solutions' Gram matrix (the same R in exact arithmetic, the stored vectors
 * being the raw solutions).  Synchronises the context's stream.
 */
int guess_proj_factor(guess_t g, double *R, int *d);

/*
 * Per-kernel timing (tracing aid).  With profiling enabled every kernel that
 * guess_form / guess_update launch for this context is dispatched with a
 * start and a stop event stamped by the dispatch itself (hipExtLaunchKernel),
 * so each time is the kernel's own run time.
 * guess_kernel_times waits for the most recent such call and returns the
 * device time of each of its kernels in launch order (ms[0..*n-1]):
 *   EXTRAP/LAST form: extrap_form;  update: ring_store
 *   PROJ form: proj_dots, proj_fin, proj_combine;  update: proj_apply,
 *   proj_fin, proj_reorth, proj_fin, proj_gs_write, proj_fin (proj_fin: the
 *   one-workgroup finishing step of a reduction; reorth, gs_write and their
 *   finishing steps return at once after a restart)
 * *n = 0 when profiling is off or the last call launched no kernel.
 */
int guess_profile(guess_t g, int enable);
int guess_kernel_times(guess_t g, double *ms, int max, int *n);

/* ------------------------------------------------------------------ workload */

/*
 * Right-hand side of a plane-wave workload on an n^3 unit-cube grid:
 *   b_i = sum_k a_k cos(2 pi (kx_k x + ky_k y + kz_k z) + theta_k)
 * at interior node (x, y, z) = (i, j, l) / (n + 1).  kvec: host int array
 * 3K (kx, ky, kz per mode); theta, amp: host arrays of K doubles.  b is a
 * device vector of n^3 doubles.  K <= 64.  Enqueued on `stream`.  The
 * per-axis tables are kept per host thread; a call with other modes first
 * waits for the previous call's kernel.
 */
int workload_plane_wave_rhs(int n, int K, const int *kvec, const double *theta,
                            const double *amp, double *b, void *stream);

/*
 * Synthetic right-hand side whose solutions are not confined to a fixed
 * low-dimensional space: a Gaussian source at `center` (host array of 3
 * coordinates in the unit cube) of width sigma > 0,
 *   b_i = amp * (g_x(i) * (g_y(j) * g_z(l))),  g_a(i) = exp(-(x_i - c_a)^2 / (2 sigma^2)),
 * x_i = (i + 1) / (n + 1), on the n^3 interior nodes, x fastest.  b is a
 * device vector of n^3 doubles; a small per-thread table buffer is kept
 * between calls (a call on another stream than the previous one first waits
 * for that call's kernels).  Enqueued on `stream`; EINVAL for bad arguments.
 */
int workload_gaussian_rhs(int n, const double *center, double sigma, double amp, double *b, void *stream);

/* ------------------------------------------------------------------ vectors */

/* out[k] = <v_k, y> for K device vectors v_k = V + k * N (K <= 64), FP64;
 * deterministic two-stage reduction; out is a host array.  Synchronises. */
int vec_multidot(int64_t N, int K, const double *V, const double *y, double *out,
                 void *stream);
/*
 * vec_multidot for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, kernels and results (bit for bit) as vec_multidot, but the
 * reduction's scratch (the partial rows and the results) is a static device
 * array of the library, 128.5 KiB per GPU, held until the process ends; no
 * hipMalloc / hipFree / allocating routine is called.  K above 64 is
 * rejected (GUESS_EINVAL): the scratch holds 64 results.  Every call on one
 * GPU shares that GPU's array, so calls that overlap on one GPU (other
 * streams or host threads) race; the library serialises only the one-time
 * lookup of the array's device address.  out is a host array of K doubles.
 * Synchronises.
 */
int vec_multidot_noalloc(int64_t N, int K, const double *V, const double *y, double *out,
                         void *stream);
/* y = sum_k c_k v_k (c host array of K doubles, V as above). */
int vec_combine(int64_t N, int K, const double *V, const double *c, double *y,
                void *stream);

/* ------------------------------------------------------------------ misc */

const char *guess_strerror(int code);
const char *guess_last_error(void);
/* Plain device copy dst <- src of `bytes` bytes with a hand-written kernel
 * (bandwidth reference for the roofline). */
int guess_copy_kernel(void *dst, const void *src, size_t bytes, void *stream);

/* Bandwidth references of the roofline (§6.2 of the paper judges each
 * kernel against a measured copy; a read roof and a write roof say how much
 * of a kernel's reads and writes HBM can carry): the same 16-byte
 * non-temporal accesses as the guess kernels.
 *   GUESS_ROOF_COPY:  guess_copy_kernel (bytes read and bytes written);
 *   GUESS_ROOF_READ:  reads `bytes` of src (multiple of 16 counted) and
 *                     writes one FP64 partial sum per workgroup into dst,
 *                     which must hold 2048 doubles (16 KiB);
 *   GUESS_ROOF_WRITE: writes `bytes` of dst (src unused, may be NULL);
 *   GUESS_ROOF_READ_STREAMS: as GUESS_ROOF_READ, with src read as 16 equal
 *                     segments streamed side by side (the pattern of a pass
 *                     over 16 vectors); bytes / 16 rounded down to a
 *                     multiple of 16 elements are read.
 * Device pointers, 16-byte aligned; EINVAL otherwise or for another mode. */
enum { GUESS_ROOF_COPY = 0, GUESS_ROOF_READ = 1, GUESS_ROOF_WRITE = 2, GUESS_ROOF_READ_STREAMS = 3 };
int guess_roof_kernel(int mode, void *dst, const void *src, size_t bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* LIBGUESS_H */
