// libguess C ABI: contexts, operators, PCG driver and the host-side
// least-squares weight solver.  Every device step runs in the kernels of
// extrap.hip, proj.hip, op.hip and vec.hip; this file only allocates,
// validates arguments, keeps host-side bookkeeping and launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "launch.h"
#include "libguess.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string &msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(GUESS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define LG_HIP(expr)                                   \
    do {                                               \
        hipError_t e_ = (expr);                        \
        if (e_ != hipSuccess) return hip_fail(e_, #expr); \
    } while (0)

#define LG_TRY(expr)                \
    do {                            \
        int r_ = (expr);            \
        if (r_ != GUESS_OK) return r_; \
    } while (0)

int check_launch(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, what);
    return GUESS_OK;
}

int esize(int dtype) {
    switch (dtype) {
        case GUESS_F64: return 8;
        case GUESS_F32: return 4;
        case GUESS_F16: return 2;
        case GUESS_BF16: return 2;
    }
    return 0;
}

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Stride between stored columns / ring slots: a multiple of 128 elements, so
// every column starts 256-byte aligned for every storage format.
int64_t col_stride(int64_t N) { return (N + 127) / 128 * 128; }

int env_int(const char *name, int dflt) {
    const char *v = std::getenv(name);
    if (!v || !*v) return dflt;
    return std::atoi(v);
}

}  // namespace

namespace lg {

int grid_cap() {
    static const int v = [] {
        int x = env_int("LIBGUESS_GRID_CAP", 1 << 20);
        return x < 1 ? 1 : x;
    }();
    return v;
}

int write_blocks() {
    static const int v = [] {
        int x = env_int("LIBGUESS_WRITE_BLOCKS", 0);
        return x < 0 ? 0 : x;
    }();
    return v;
}

bool raw_march() {
    static const bool v = env_int("LIBGUESS_RAW_MARCH", 0) != 0;
    return v;
}

int gather_lds() {
    static const int v = [] {
        int x = env_int("LIBGUESS_GATHER_LDS", 65536);
        return x < 0 ? 0 : (x > 65536 ? 65536 : x);
    }();
    return v;
}

int reduce_blocks() {
    static const int v = [] {
        int x = env_int("LIBGUESS_REDUCE_BLOCKS", 1024);
        if (x < 1) x = 1;
        if (x > kMaxPartialBlocks) x = kMaxPartialBlocks;
        return x;
    }();
    return v;
}

// LIBGUESS_MARCH=0 selects the chunk form of PCG's stencil kernel everywhere
// (for comparisons); the default uses the z-marching form where it applies.
bool march_enabled() {
    static const bool v = env_int("LIBGUESS_MARCH", 1) != 0;
    return v;
}

int march_wgs_override() {
    static const int v = env_int("LIBGUESS_MARCH_WGS", 0);
    return v;
}

int march_nr_override() {
    static const int v = env_int("LIBGUESS_MARCH_NR", 0);
    return v;
}

}  // namespace lg

// ====================================================================== operator
struct guess_op {
    lg::Grid g{};
    hipStream_t stream = nullptr;
    double *kx = nullptr, *ky = nullptr, *kz = nullptr, *dinv = nullptr;
    double *r = nullptr, *p[3] = {nullptr, nullptr, nullptr}, *q = nullptr;   // p_k in p[k % 3]
    double *part_a = nullptr, *part_b = nullptr;  // per-workgroup partial sums of the two PCG kernels
    lg::PcgState *st = nullptr;
    lg::PcgState *host_st = nullptr;  // pinned
};

static void op_free(guess_op *A) {
    if (!A) return;
    for (void *ptr : {(void *)A->kx, (void *)A->ky, (void *)A->kz, (void *)A->dinv, (void *)A->r,
                      (void *)A->p[0], (void *)A->p[1], (void *)A->p[2], (void *)A->q, (void *)A->part_a, (void *)A->part_b,
                      (void *)A->st})
        if (ptr) (void)hipFree(ptr);
    if (A->host_st) (void)hipHostFree(A->host_st);
    delete A;
}

extern "C" int guess_op_create(int nx, int ny, int nz, double inv_h2, double shift, const double *kappa,
                               guess_op_t *out) {
    if (!out) return fail(GUESS_EINVAL, "guess_op_create: out is NULL");
    *out = nullptr;
    if (nx < 1 || ny < 1 || nz < 1) return fail(GUESS_EINVAL, "guess_op_create: grid sizes must be >= 1");
    if (!(inv_h2 > 0.0) || !(shift >= 0.0) || !std::isfinite(inv_h2) || !std::isfinite(shift))
        return fail(GUESS_EINVAL, "guess_op_create: need inv_h2 > 0 and shift >= 0");
    const int64_t n = (int64_t)nx * ny * nz;
    if (n >= ((int64_t)1 << 31)) return fail(GUESS_EINVAL, "guess_op_create: grid too large (N >= 2^31)");
    guess_op *A = new (std::nothrow) guess_op();
    if (!A) return fail(GUESS_ENOMEM, "guess_op_create: host allocation failed");
    A->g.nx = nx;
    A->g.ny = ny;
    A->g.nz = nz;
    A->g.nxy = (int64_t)nx * ny;
    A->g.n = n;
    A->g.c = inv_h2;
    A->g.shift = shift;
    A->g.dinv_const = 1.0 / (inv_h2 * 6.0 + shift);
    A->g.fnx = lg::make_fastdiv((uint32_t)nx);
    A->g.fny = lg::make_fastdiv((uint32_t)ny);
    A->g.aligned = (nx % 2) == 0;
    auto alloc = [&](void **ptr, size_t bytes) -> int {
        hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(GUESS_ENOMEM, "guess_op_create: device allocation failed");
        }
        return GUESS_OK;
    };
    int rc = GUESS_OK;
    if (rc == GUESS_OK) rc = alloc((void **)&A->r, n * 8);
    if (rc == GUESS_OK) rc = alloc((void **)&A->p[0], n * 8);
    if (rc == GUESS_OK) rc = alloc((void **)&A->p[1], n * 8);
    if (rc == GUESS_OK) rc = alloc((void **)&A->p[2], n * 8);
    if (rc == GUESS_OK) rc = alloc((void **)&A->q, n * 8);
    if (rc == GUESS_OK) rc = alloc((void **)&A->part_a, sizeof(double) * lg::kMaxPartialBlocks);
    if (rc == GUESS_OK) rc = alloc((void **)&A->part_b, sizeof(double) * lg::kMaxPartialBlocks * 3);
    if (rc == GUESS_OK) rc = alloc((void **)&A->st, sizeof(lg::PcgState));
    if (rc == GUESS_OK && hipHostMalloc((void **)&A->host_st, sizeof(lg::PcgState), hipHostMallocDefault) != hipSuccess)
        rc = fail(GUESS_ENOMEM, "guess_op_create: pinned allocation failed");
    if (rc == GUESS_OK) {
        lg::PcgState z{};
        if (hipMemcpy(A->st, &z, sizeof z, hipMemcpyHostToDevice) != hipSuccess)
            rc = fail(GUESS_EHIP, "guess_op_create: state upload failed");
    }
    if (rc == GUESS_OK && kappa) {
        const int64_t nfx = (int64_t)(nx + 1) * ny * nz, nfy = (int64_t)nx * (ny + 1) * nz,
                      nfz = (int64_t)nx * ny * (nz + 1);
        rc = alloc((void **)&A->kx, nfx * 8);
        if (rc == GUESS_OK) rc = alloc((void **)&A->ky, nfy * 8);
        if (rc == GUESS_OK) rc = alloc((void **)&A->kz, nfz * 8);
        if (rc == GUESS_OK) rc = alloc((void **)&A->dinv, n * 8);
        if (rc == GUESS_OK) {
            lg::launch_build_faces(A->g, kappa, A->kx, A->ky, A->kz, A->dinv, nullptr);
            rc = check_launch("build_faces");
            if (rc == GUESS_OK && hipDeviceSynchronize() != hipSuccess)
                rc = fail(GUESS_EHIP, "guess_op_create: face construction failed");
        }
    }
    if (rc != GUESS_OK) {
        op_free(A);
        return rc;
    }
    *out = A;
    return GUESS_OK;
}

extern "C" void guess_op_destroy(guess_op_t A) { op_free(A); }

extern "C" int guess_op_set_stream(guess_op_t A, void *stream) {
    if (!A) return fail(GUESS_EINVAL, "guess_op_set_stream: NULL operator");
    A->stream = (hipStream_t)stream;
    return GUESS_OK;
}

extern "C" int64_t guess_op_size(guess_op_t A) { return A ? A->g.n : 0; }

extern "C" int op_apply(guess_op_t A, const double *x, double *y) {
    if (!A || !x || !y) return fail(GUESS_EINVAL, "op_apply: NULL argument");
    if (x == y) return fail(GUESS_EINVAL, "op_apply: x and y must not alias");
    if (!aligned16(x) || !aligned16(y)) return fail(GUESS_EINVAL, "op_apply: vectors must be 16-byte aligned");
    lg::launch_op_apply(A->g, x, y, A->stream);
    return check_launch("op_apply");
}

extern "C" int pcg_solve_ex(guess_op_t A, const double *b, double *x, double rtol, int maxit, int stop_rule,
                            int *iters, double *relres) {
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    if (!A || !b || !x) return fail(GUESS_EINVAL, "pcg_solve: NULL argument");
    if (b == x) return fail(GUESS_EINVAL, "pcg_solve: b and x must not alias");
    if (!aligned16(b) || !aligned16(x)) return fail(GUESS_EINVAL, "pcg_solve: vectors must be 16-byte aligned");
    if (!(rtol >= 0.0) || maxit < 0) return fail(GUESS_EINVAL, "pcg_solve: need rtol >= 0 and maxit >= 0");
    if (stop_rule != GUESS_STOP_RHS && stop_rule != GUESS_STOP_INITRESID)
        return fail(GUESS_EINVAL, "pcg_solve: unknown stopping rule");
    hipStream_t s = A->stream;
    lg::PcgState init{};
    init.rule = stop_rule;
    *A->host_st = init;
    LG_HIP(hipMemcpyAsync(A->st, A->host_st, sizeof init, hipMemcpyHostToDevice, s));
    lg::launch_pcg_init(A->g, b, x, A->r, A->part_b, s);
    LG_TRY(check_launch("pcg_init"));
    auto read_state = [&]() -> int {
        LG_HIP(hipMemcpyAsync(A->host_st, A->st, sizeof(lg::PcgState), hipMemcpyDeviceToHost, s));
        LG_HIP(hipStreamSynchronize(s));
        return GUESS_OK;
    };
    // Iteration k's first kernel also runs the stop test on r_{k-1}, so the
    // test after the last allowed iteration is a separate check.  Iterations
    // are enqueued in batches; kernels of a batch return at once after
    // convergence, so the count stays exact.  Batches grow with the
    // iteration count so that short solves do not pay for long batches.
    int k = 1;
    while (k <= maxit) {
        int chunk = k <= 4 ? 2 : (k <= 32 ? 4 : (k <= 128 ? 8 : 16));
        if (chunk > maxit - k + 1) chunk = maxit - k + 1;
        for (int c = 0; c < chunk; ++c, ++k)
            lg::launch_pcg_iter(A->g, x, A->r, A->p, A->q, A->part_a, A->part_b, A->st, k, rtol, s);
        LG_TRY(check_launch("pcg_iter"));
        LG_TRY(read_state());
        if (A->host_st->converged | A->host_st->breakdown) break;
    }
    if (!(A->host_st->converged | A->host_st->breakdown)) {
        lg::launch_pcg_check(A->g, A->part_b, A->st, k, rtol, s);
        LG_TRY(check_launch("pcg_check"));
    }
    // the x updates of the last iterations unless a later pcg_a applied them
    // (a no-op on the device when nothing is pending)
    if (k > 1) {
        lg::launch_pcg_finish(A->g, x, A->p, A->st, s);
        LG_TRY(check_launch("pcg_finish"));
    }
    LG_TRY(read_state());
    const lg::PcgState &st = *A->host_st;
    const int its = (st.converged | st.breakdown) ? st.it : maxit;
    if (iters) *iters = its;
    if (relres) *relres = st.bb > 0.0 ? std::sqrt(st.rr) / std::sqrt(st.bb) : std::sqrt(st.rr);
    if (st.converged) return GUESS_OK;
    if (st.breakdown) return fail(GUESS_EBREAKDOWN, "pcg_solve: breakdown (p^T A p <= 0 or not finite)");
    return fail(GUESS_ENOTCONV, "pcg_solve: maxit reached");
}

extern "C" int pcg_solve(guess_op_t A, const double *b, double *x, double rtol, int maxit, int *iters,
                         double *relres) {
    return pcg_solve_ex(A, b, x, rtol, maxit, GUESS_STOP_RHS, iters, relres);
}

// ====================================================================== weights
// Least-squares extrapolation weights beta = V (V^T V)^{-1} v (§3.2) with a
// Legendre basis on the nodes t_i = -1 + (i-1) h, h = 2/(k-1), evaluated at
// t = 1 + h.  With V = Q R (Householder), beta = Q R^{-T} v.
extern "C" int guess_extrap_weights(int m, int k, double *beta) {
    if (!beta) return fail(GUESS_EINVAL, "guess_extrap_weights: beta is NULL");
    if (k < 1 || k > GUESS_MAX_M || m < 0 || m > k - 1)
        return fail(GUESS_EINVAL, "guess_extrap_weights: need 1 <= k <= 16 and 0 <= m <= k-1");
    if (k == 1) {
        beta[0] = 1.0;
        return GUESS_OK;
    }
    const int n = m + 1;
    const double h = 2.0 / (k - 1);
    double V[GUESS_MAX_M][GUESS_MAX_M];  // V[i][j] = P_j(t_i)
    double v[GUESS_MAX_M];
    auto legendre = [&](double t, double *P) {
        P[0] = 1.0;
        if (n > 1) P[1] = t;
        for (int j = 1; j + 1 < n; ++j) P[j + 1] = ((2 * j + 1) * t * P[j] - j * P[j - 1]) / (j + 1);
    };
    for (int i = 0; i < k; ++i) legendre(-1.0 + i * h, V[i]);
    legendre(1.0 + h, v);
    // Householder QR: reflector c acts on rows c..k-1; u[c] stores its vector.
    double u[GUESS_MAX_M][GUESS_MAX_M];
    double R[GUESS_MAX_M][GUESS_MAX_M];
    for (int c = 0; c < n; ++c) {
        double nrm = 0.0;
        for (int i = c; i < k; ++i) nrm += V[i][c] * V[i][c];
        nrm = std::sqrt(nrm);
        const double alpha = V[c][c] > 0 ? -nrm : nrm;
        for (int i = 0; i < k; ++i) u[c][i] = 0.0;
        for (int i = c; i < k; ++i) u[c][i] = V[i][c];
        u[c][c] -= alpha;
        double un = 0.0;
        for (int i = c; i < k; ++i) un += u[c][i] * u[c][i];
        un = std::sqrt(un);
        if (un > 0)
            for (int i = c; i < k; ++i) u[c][i] /= un;
        for (int j = c; j < n; ++j) {
            double dot = 0.0;
            for (int i = c; i < k; ++i) dot += u[c][i] * V[i][j];
            for (int i = c; i < k; ++i) V[i][j] -= 2.0 * u[c][i] * dot;
        }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) R[i][j] = j >= i ? V[i][j] : 0.0;
    // R^T y = v (forward substitution)
    double z[GUESS_MAX_M];
    for (int i = 0; i < k; ++i) z[i] = 0.0;
    for (int i = 0; i < n; ++i) {
        double s = v[i];
        for (int j = 0; j < i; ++j) s -= R[j][i] * z[j];
        z[i] = s / R[i][i];
    }
    // beta = H_0 H_1 ... H_{n-1} [y; 0]
    for (int c = n - 1; c >= 0; --c) {
        double dot = 0.0;
        for (int i = c; i < k; ++i) dot += u[c][i] * z[i];
        for (int i = c; i < k; ++i) z[i] -= 2.0 * u[c][i] * dot;
    }
    for (int i = 0; i < k; ++i) beta[i] = z[i];
    return GUESS_OK;
}

// Sparse extrapolation weights (§3.3, eq. CPQRCoeffs).  Column-pivoted QR
// of V^T (Legendre basis, nodes as above) picks m+1 history nodes: each
// pivot is the node whose column has the largest component orthogonal to
// the nodes already taken (modified Gram-Schmidt here).  Norms within a
// relative 1e-10 of the maximum count as equal and the oldest such node
// wins: the first-maximum rule, made insensitive to the rounding that
// separates the exact ties the symmetric nodes produce.  Given the nodes S,
// the weights solve (V_S)^T beta_S = v, i.e. they are the Lagrange weights
// of the interpolant through S evaluated at the new node.
extern "C" int guess_spextrap_weights(int m, int k, double *beta) {
    if (!beta) return fail(GUESS_EINVAL, "guess_spextrap_weights: beta is NULL");
    if (k < 1 || k > GUESS_MAX_M || m < 0 || m > k - 1)
        return fail(GUESS_EINVAL, "guess_spextrap_weights: need 1 <= k <= 16 and 0 <= m <= k-1");
    for (int i = 0; i < k; ++i) beta[i] = 0.0;
    if (k == 1) {
        beta[0] = 1.0;
        return GUESS_OK;
    }
    const int n = m + 1;
    const double h = 2.0 / (k - 1);
    double t[GUESS_MAX_M];
    double C[GUESS_MAX_M][GUESS_MAX_M];  // C[i] = column i of V^T, then its residual
    for (int i = 0; i < k; ++i) {
        t[i] = -1.0 + i * h;
        C[i][0] = 1.0;
        if (n > 1) C[i][1] = t[i];
        for (int j = 1; j + 1 < n; ++j) C[i][j + 1] = ((2 * j + 1) * t[i] * C[i][j] - j * C[i][j - 1]) / (j + 1);
    }
    bool taken[GUESS_MAX_M] = {};
    int S[GUESS_MAX_M];
    for (int p = 0; p < n; ++p) {
        double nn[GUESS_MAX_M], mx = 0.0;
        for (int i = 0; i < k; ++i) {
            nn[i] = 0.0;
            if (taken[i]) continue;
            for (int j = 0; j < n; ++j) nn[i] += C[i][j] * C[i][j];
            mx = nn[i] > mx ? nn[i] : mx;
        }
        if (!(mx > 0.0)) return fail(GUESS_EINVAL, "guess_spextrap_weights: rank-deficient basis");
        int piv = -1;
        for (int i = 0; i < k && piv < 0; ++i)
            if (!taken[i] && nn[i] >= mx * (1.0 - 1e-10)) piv = i;
        taken[piv] = true;
        S[p] = piv;
        double q[GUESS_MAX_M];
        const double qn = std::sqrt(nn[piv]);
        for (int j = 0; j < n; ++j) q[j] = C[piv][j] / qn;
        for (int i = 0; i < k; ++i) {
            if (taken[i]) continue;
            double dot = 0.0;
            for (int j = 0; j < n; ++j) dot += q[j] * C[i][j];
            for (int j = 0; j < n; ++j) C[i][j] -= dot * q[j];
        }
    }
    // In units of h the nodes are the integers 0..k-1 and the new node is k,
    // so each weight is a ratio of integer products: exact in 64 bits
    // (|numerator| <= 16^15), reduced, then one rounding to FP64.
    for (int a = 0; a < n; ++a) {
        int64_t num = 1, den = 1;
        for (int b = 0; b < n; ++b) {
            if (b == a) continue;
            num *= (int64_t)(k - S[b]);
            den *= (int64_t)(S[a] - S[b]);
            const int64_t g = std::gcd(num < 0 ? -num : num, den < 0 ? -den : den);
            num /= g;
            den /= g;
        }
        beta[S[a]] = (double)num / (double)den;
    }
    return GUESS_OK;
}

// ====================================================================== context
struct guess_ctx {
    int64_t N = 0, ld = 0;
    int M = 1, method = GUESS_ZERO, degree = 0, dtype = GUESS_F64, es = 8;
    int inner = GUESS_INNER_A, vf = 0;   // projection: inner product, kernel variant flags
    bool external = false;               // device buffers carved from the caller's workspace
    double eps_rel = 1e-6;
    guess_op_t op = nullptr;
    hipStream_t stream = nullptr;
    // extrapolation ring: `slots` physical slots for M logical ones; an FP64
    // ring keeps one spare, the slot the next update writes, which the guess
    // never reads (so a caller may form the guess into it and solve in place)
    void *ring = nullptr;
    int count = 0, head = 0, slots = 1;
    lg::RingState *rs = nullptr, *host_rs = nullptr;   // FP16 ring: per-slot exponents (device)
    int gen = 0;                                         // FP16 ring: stores so far, mod 2
    double beta[GUESS_MAX_M + 1][GUESS_MAX_M][GUESS_MAX_M] = {};  // [k][m][i]
    bool have_beta[GUESS_MAX_M + 1][GUESS_MAX_M] = {};
    // projection
    void *X = nullptr, *B = nullptr;
    double *w = nullptr, *part = nullptr;
    lg::ProjState *st = nullptr, *host_st = nullptr;
    int last_update_ax = 0;
    // raw-solution projection: stored solutions in X, FP64 Gram matrix and factor in rst
    lg::RawState *rst = nullptr, *host_rst = nullptr;
    // bookkeeping
    double form_bytes = 0.0, update_bytes = 0.0;
    // optional per-kernel timing of the most recent form / update call
    bool prof = false;
    lg::KEvents kev{};
};

static void ctx_free(guess_ctx *g) {
    if (!g) return;
    if (g->prof)
        for (int i = 0; i < 8; ++i) {
            (void)hipEventDestroy(g->kev.start[i]);
            (void)hipEventDestroy(g->kev.stop[i]);
        }
    if (!g->external)
        for (void *ptr : {g->ring, g->X, g->B, (void *)g->w, (void *)g->part, (void *)g->st, (void *)g->rs,
                          (void *)g->rst})
            if (ptr) (void)hipFree(ptr);
    if (g->host_st) (void)hipHostFree(g->host_st);
    if (g->host_rst) (void)hipHostFree(g->host_rst);
    if (g->host_rs) (void)hipHostFree(g->host_rs);
    delete g;
}

static bool ring_method(int method) {
    return method == GUESS_LAST || method == GUESS_EXTRAP || method == GUESS_SPEXTRAP;
}
static bool proj_method(int method) { return method == GUESS_PROJ || method == GUESS_PROJ_QR; }
static bool raw_method(int method) { return method == GUESS_PROJ_RAW || method == GUESS_PROJ_RAW_QR; }

// Device buffers of a context, in carving order; every one starts 256-byte
// aligned (sizes rounded up to 256 bytes).
static size_t round256(size_t b) { return (b + 255) / 256 * 256; }

static int ctx_buffers(int64_t N, int M, int method, int dtype, size_t sizes[6]) {
    for (int i = 0; i < 6; ++i) sizes[i] = 0;   // ring, X, B, w, part, state
    const int es = esize(dtype);
    if (N < 1 || M < 1 || es == 0) return 0;
    const size_t col = (size_t)col_stride(N) * es;
    const int spare = dtype == GUESS_F64 ? 1 : 0;
    if (method == GUESS_LAST) sizes[0] = col * (1 + spare);
    else if (ring_method(method)) sizes[0] = col * (M + spare);
    if (ring_method(method) && dtype == GUESS_F16) sizes[5] = round256(sizeof(lg::RingState));
    else if (proj_method(method)) {
        sizes[1] = col * M;
        sizes[2] = col * M;
        sizes[3] = round256((size_t)N * 8);
        sizes[4] = round256(sizeof(double) * lg::kMaxPartialBlocks * lg::kMaxDots);
        sizes[5] = round256(sizeof(lg::ProjState));
    } else if (raw_method(method)) {
        sizes[1] = col * M;
        sizes[4] = round256(sizeof(double) * lg::kMaxPartialBlocks * lg::kMaxDots);
        sizes[5] = round256(sizeof(lg::RawState));
    }
    return 1;
}

extern "C" size_t guess_workspace_bytes(int64_t N, int M, int method, int dtype) {
    if (method == GUESS_LAST) M = 1;
    size_t sizes[6];
    ctx_buffers(N, M, method, dtype, sizes);
    size_t t = 0;
    for (size_t b : sizes) t += b;
    return t;
}

// FP16 ring: every exponent 0, both max accumulators clear.
static int ring_upload_state(guess_ctx *g) {
    *g->host_rs = lg::RingState{};
    LG_HIP(hipMemcpyAsync(g->rs, g->host_rs, sizeof(lg::RingState), hipMemcpyHostToDevice, g->stream));
    LG_HIP(hipStreamSynchronize(g->stream));
    return GUESS_OK;
}

static int ring_read_state(guess_ctx *g) {
    LG_HIP(hipMemcpyAsync(g->host_rs, g->rs, sizeof(lg::RingState), hipMemcpyDeviceToHost, g->stream));
    LG_HIP(hipStreamSynchronize(g->stream));
    return GUESS_OK;
}

// Raw-solution projection: empty history, slots in order.
static int raw_upload_state(guess_ctx *g) {
    lg::RawState s{};
    for (int j = 0; j < GUESS_MAX_M; ++j) s.perm[j] = j;
    s.eps_rel = g->eps_rel;
    *g->host_rst = s;
    LG_HIP(hipMemcpyAsync(g->rst, g->host_rst, sizeof s, hipMemcpyHostToDevice, g->stream));
    LG_HIP(hipStreamSynchronize(g->stream));
    return GUESS_OK;
}

static int raw_read_state(guess_ctx *g) {
    LG_HIP(hipMemcpyAsync(g->host_rst, g->rst, sizeof(lg::RawState), hipMemcpyDeviceToHost, g->stream));
    LG_HIP(hipStreamSynchronize(g->stream));
    return GUESS_OK;
}

static int proj_upload_state(guess_ctx *g) {
    lg::ProjState s{};
    s.M = g->M;
    s.eps_rel = g->eps_rel;
    s.pow2 = 1.0;
    *g->host_st = s;
    LG_HIP(hipMemcpyAsync(g->st, g->host_st, sizeof s, hipMemcpyHostToDevice, g->stream));
    LG_HIP(hipStreamSynchronize(g->stream));
    return GUESS_OK;
}

// Rejection threshold when the caller gives none.  Rounding a stored column
// to the storage format adds noise of relative size u_s, which the
// normalisation of a column accepted with ratio nu/nu0 amplifies by nu0/nu;
// the default therefore grows with the format's unit roundoff (the values
// are the best of 1e-6 ... 1e-1 on the plane-wave sequences at 256^3).
static double default_eps_rel(int dtype, int method) {
    // the raw-solution form takes rounding into its Gram matrix; one threshold fits every format
    if (method == GUESS_PROJ_RAW || method == GUESS_PROJ_RAW_QR) return 1e-6;
    switch (dtype) {
        case GUESS_F32: return 1e-4;
        case GUESS_F16:
        case GUESS_BF16: return 1e-2;
        default: return 1e-6;
    }
}

extern "C" int guess_create_ex(const guess_opts *o, guess_t *out) {
    if (!o || !out) return fail(GUESS_EINVAL, "guess_create_ex: NULL argument");
    *out = nullptr;
    int M = o->M;
    if (o->method == GUESS_LAST) M = 1;
    if (o->N < 1) return fail(GUESS_EINVAL, "guess_create: need N >= 1");
    if (o->method < GUESS_ZERO || o->method > GUESS_PROJ_RAW_QR) return fail(GUESS_EINVAL, "guess_create: unknown method");
    if (o->method != GUESS_ZERO && (M < 1 || M > GUESS_MAX_M))
        return fail(GUESS_EINVAL, "guess_create: need 1 <= M <= 16");
    const int degree = o->method == GUESS_LAST ? 0 : o->degree;
    if ((o->method == GUESS_EXTRAP || o->method == GUESS_SPEXTRAP) && (degree < 0 || degree > M - 1))
        return fail(GUESS_EINVAL, "guess_create: need 0 <= degree <= M-1");
    if (esize(o->dtype) == 0) return fail(GUESS_EINVAL, "guess_create: unknown dtype");
    // In FP64 the Schur complement nu^2 = w^T A w - g^T G^{-1} g of nearly dependent exact
    // solutions is accurate only to u cond(G) w^T A w, far above eps_rel^2 w^T A w; the
    // Gram-Schmidt forms (PROJ, PROJ_QR) compute nu from the remainder itself.
    if ((o->method == GUESS_PROJ_RAW || o->method == GUESS_PROJ_RAW_QR) && o->dtype == GUESS_F64)
        return fail(GUESS_EINVAL, "guess_create: the raw-solution projection is for reduced-precision histories; "
                                  "FP64 histories use GUESS_PROJ / GUESS_PROJ_QR");
    if (o->inner != GUESS_INNER_A && o->inner != GUESS_INNER_L2)
        return fail(GUESS_EINVAL, "guess_create: unknown inner product");
    if (o->op && o->op->g.n != o->N) return fail(GUESS_EINVAL, "guess_create: operator size differs from N");
    guess_ctx *g = new (std::nothrow) guess_ctx();
    if (!g) return fail(GUESS_ENOMEM, "guess_create: host allocation failed");
    g->N = o->N;
    g->ld = col_stride(o->N);
    g->M = o->method == GUESS_ZERO ? 0 : M;
    g->method = o->method;
    g->degree = degree;
    g->dtype = o->dtype;
    g->es = esize(o->dtype);
    g->eps_rel = o->eps_rel > 0.0 ? o->eps_rel : default_eps_rel(o->dtype, o->method);
    g->inner = o->inner;
    g->vf = (o->method == GUESS_PROJ_QR ? 1 : 0) | (o->inner == GUESS_INNER_L2 ? 2 : 0);
    g->op = o->op;
    g->stream = (hipStream_t)o->stream;
    const size_t col = (size_t)g->ld * g->es;
    // caller workspace: carve the buffers in the order of ctx_buffers
    size_t sizes[6];
    ctx_buffers(o->N, g->M > 0 ? g->M : 1, o->method, o->dtype, sizes);
    char *carve = nullptr;
    if (o->workspace) {
        size_t need = 0;
        for (size_t b : sizes) need += b;
        if (((uintptr_t)o->workspace & 255u) != 0 || o->workspace_bytes < need) {
            delete g;
            return fail(GUESS_EINVAL, "guess_create: workspace must be 256-byte aligned and hold " +
                                          std::to_string(need) + " bytes");
        }
        carve = (char *)o->workspace;
        g->external = true;
    }
    auto alloc = [&](void **ptr, size_t bytes) -> int {
        if (carve) {
            *ptr = carve;
            carve += round256(bytes);
            return GUESS_OK;
        }
        hipError_t e = hipMalloc(ptr, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(GUESS_ENOMEM, "guess_create: device allocation of " + std::to_string(bytes) +
                                          " bytes failed");
        }
        return GUESS_OK;
    };
    int rc = GUESS_OK;
    if (ring_method(g->method)) {
        g->slots = g->M + (g->dtype == GUESS_F64 ? 1 : 0);
        rc = alloc(&g->ring, col * g->slots);
        if (rc == GUESS_OK && g->dtype == GUESS_F16) {
            rc = alloc((void **)&g->rs, sizeof(lg::RingState));
            if (rc == GUESS_OK && hipHostMalloc((void **)&g->host_rs, sizeof(lg::RingState), hipHostMallocDefault) != hipSuccess)
                rc = fail(GUESS_ENOMEM, "guess_create: pinned allocation failed");
            if (rc == GUESS_OK) rc = ring_upload_state(g);
        }
    } else if (proj_method(g->method)) {
        rc = alloc(&g->X, col * g->M);
        if (rc == GUESS_OK) rc = alloc(&g->B, col * g->M);
        if (rc == GUESS_OK) rc = alloc((void **)&g->w, (size_t)g->N * 8);
        if (rc == GUESS_OK) rc = alloc((void **)&g->part, sizeof(double) * lg::kMaxPartialBlocks * lg::kMaxDots);
        if (rc == GUESS_OK) rc = alloc((void **)&g->st, sizeof(lg::ProjState));
        if (rc == GUESS_OK && hipHostMalloc((void **)&g->host_st, sizeof(lg::ProjState), hipHostMallocDefault) != hipSuccess)
            rc = fail(GUESS_ENOMEM, "guess_create: pinned allocation failed");
        if (rc == GUESS_OK) rc = proj_upload_state(g);
    } else if (raw_method(g->method)) {
        rc = alloc(&g->X, col * g->M);
        if (rc == GUESS_OK) rc = alloc((void **)&g->part, sizeof(double) * lg::kMaxPartialBlocks * lg::kMaxDots);
        if (rc == GUESS_OK) rc = alloc((void **)&g->rst, sizeof(lg::RawState));
        if (rc == GUESS_OK && hipHostMalloc((void **)&g->host_rst, sizeof(lg::RawState), hipHostMallocDefault) != hipSuccess)
            rc = fail(GUESS_ENOMEM, "guess_create: pinned allocation failed");
        if (rc == GUESS_OK) rc = raw_upload_state(g);
    }
    if (rc != GUESS_OK) {
        ctx_free(g);
        return rc;
    }
    *out = g;
    return GUESS_OK;
}

extern "C" guess_t guess_create(int64_t N, int M, int method, int degree) {
    guess_opts o{};
    o.N = N;
    o.M = M;
    o.method = method;
    o.degree = degree;
    o.dtype = GUESS_F64;
    o.eps_rel = 1e-6;
    guess_t g = nullptr;
    if (guess_create_ex(&o, &g) != GUESS_OK) return nullptr;
    return g;
}

extern "C" void guess_destroy(guess_t g) { ctx_free(g); }

extern "C" int guess_set_stream(guess_t g, void *stream) {
    if (!g) return fail(GUESS_EINVAL, "guess_set_stream: NULL context");
    g->stream = (hipStream_t)stream;
    return GUESS_OK;
}

extern "C" int guess_set_op(guess_t g, guess_op_t A) {
    if (!g) return fail(GUESS_EINVAL, "guess_set_op: NULL context");
    if (A && A->g.n != g->N) return fail(GUESS_EINVAL, "guess_set_op: operator size differs from N");
    g->op = A;
    return GUESS_OK;
}

static int ring_weights(guess_ctx *g, int m, int k, const double **out) {
    if (!g->have_beta[k][m]) {
        if (g->method == GUESS_SPEXTRAP) LG_TRY(guess_spextrap_weights(m, k, g->beta[k][m]));
        else LG_TRY(guess_extrap_weights(m, k, g->beta[k][m]));
        g->have_beta[k][m] = true;
    }
    *out = g->beta[k][m];
    return GUESS_OK;
}

static lg::RawBufs raw_bufs(guess_ctx *g) {
    lg::RawBufs p;
    p.W = g->X;
    p.part = g->part;
    p.st = g->rst;
    p.N = g->N;
    p.ld = g->ld;
    p.M = g->M;
    p.qr = g->method == GUESS_PROJ_RAW_QR ? 1 : 0;
    p.dtype = g->dtype;
    return p;
}

static lg::ProjBufs proj_bufs(guess_ctx *g) {
    lg::ProjBufs p;
    p.X = g->X;
    p.B = g->B;
    p.w = g->w;
    p.part = g->part;
    p.st = g->st;
    p.N = g->N;
    p.ld = g->ld;
    p.M = g->M;
    p.dtype = g->dtype;
    p.vf = g->vf;
    return p;
}

extern "C" int guess_form(guess_t g, const double *b, double *x0) {
    if (!g || !x0) return fail(GUESS_EINVAL, "guess_form: NULL argument");
    g->kev.count = 0;
    if (!aligned16(x0)) return fail(GUESS_EINVAL, "guess_form: x0 must be 16-byte aligned");
    const int64_t N = g->N;
    switch (g->method) {
        case GUESS_ZERO:
            lg::launch_fill_zero(x0, N, g->stream);
            g->form_bytes = 8.0 * N;
            return check_launch("guess_form");
        case GUESS_LAST:
        case GUESS_EXTRAP:
        case GUESS_SPEXTRAP: {
            const int k = g->count;
            if (k == 0) {
                lg::launch_fill_zero(x0, N, g->stream);
                g->form_bytes = 8.0 * N;
                return check_launch("guess_form");
            }
            const int m = g->degree < k - 1 ? g->degree : k - 1;
            const double *beta;
            LG_TRY(ring_weights(g, m, k, &beta));
            // stored solutions with a nonzero weight, oldest first (all of them
            // for least-squares weights, m+1 for the sparse scheme)
            const void *slots[GUESS_MAX_M];
            double w[GUESS_MAX_M];
            int sidx[GUESS_MAX_M];
            int nz = 0;
            const int oldest = ((g->head - k) % g->slots + g->slots) % g->slots;
            for (int j = 0; j < k; ++j) {
                if (g->method == GUESS_SPEXTRAP && beta[j] == 0.0) continue;
                sidx[nz] = (oldest + j) % g->slots;
                slots[nz] = (const char *)g->ring + (size_t)sidx[nz] * g->ld * g->es;
                w[nz++] = beta[j];
            }
            LG_TRY(lg::launch_extrap_form(g->dtype, nz, slots, w, x0, N, g->stream, g->prof ? &g->kev : nullptr,
                                          g->rs, sidx));
            g->form_bytes = (double)N * (nz * g->es + 8);
            return check_launch("guess_form");
        }
        case GUESS_PROJ:
        case GUESS_PROJ_QR: {
            if (!b) return fail(GUESS_EINVAL, "guess_form: projection needs b");
            if (b == x0) return fail(GUESS_EINVAL, "guess_form: b and x0 must not alias");
            if (!aligned16(b)) return fail(GUESS_EINVAL, "guess_form: b must be 16-byte aligned");
            LG_TRY(lg::launch_proj_form(proj_bufs(g), b, x0, g->stream, g->prof ? &g->kev : nullptr));
            g->form_bytes = -1.0;  // known after the device reports d
            return check_launch("guess_form");
        }
        case GUESS_PROJ_RAW:
        case GUESS_PROJ_RAW_QR: {
            if (!b) return fail(GUESS_EINVAL, "guess_form: projection needs b");
            if (b == x0) return fail(GUESS_EINVAL, "guess_form: b and x0 must not alias");
            if (!aligned16(b)) return fail(GUESS_EINVAL, "guess_form: b must be 16-byte aligned");
            LG_TRY(lg::launch_raw_form(raw_bufs(g), b, x0, g->stream, g->prof ? &g->kev : nullptr));
            g->form_bytes = -1.0;
            return check_launch("guess_form");
        }
    }
    return fail(GUESS_EINVAL, "guess_form: bad method");
}

extern "C" int guess_update(guess_t g, const double *x, const double *Ax) {
    if (!g || !x) return fail(GUESS_EINVAL, "guess_update: NULL argument");
    g->kev.count = 0;
    if (!aligned16(x) || (Ax && !aligned16(Ax))) return fail(GUESS_EINVAL, "guess_update: vectors must be 16-byte aligned");
    const int64_t N = g->N;
    switch (g->method) {
        case GUESS_ZERO:
            g->update_bytes = 0.0;
            return GUESS_OK;
        case GUESS_LAST:
        case GUESS_EXTRAP:
        case GUESS_SPEXTRAP: {
            void *slot = (char *)g->ring + (size_t)g->head * g->ld * g->es;
            // a solution computed in the spare slot itself is already stored (§4: no copy
            // when the solver works in place)
            const bool in_place = (const void *)x == slot;
            if (!in_place) {
                LG_TRY(lg::launch_ring_store(g->dtype, x, slot, N, g->stream, g->prof ? &g->kev : nullptr, g->rs,
                                             g->head, g->gen));
                g->gen ^= 1;
            }
            g->head = (g->head + 1) % g->slots;
            if (g->count < g->M) ++g->count;
            g->update_bytes = in_place ? 0.0 : (double)N * (8 + g->es);
            return in_place ? GUESS_OK : check_launch("guess_update");
        }
        case GUESS_PROJ:
        case GUESS_PROJ_QR: {
            if (!Ax && !g->op) return fail(GUESS_EINVAL, "guess_update: projection needs Ax or an operator");
            if (Ax == x) return fail(GUESS_EINVAL, "guess_update: Ax must not alias x");
            LG_TRY(lg::launch_proj_update(proj_bufs(g), g->op ? &g->op->g : nullptr, x, Ax, g->stream,
                                          g->prof ? &g->kev : nullptr));
            g->last_update_ax = Ax != nullptr;
            g->update_bytes = -1.0;
            return check_launch("guess_update");
        }
        case GUESS_PROJ_RAW:
        case GUESS_PROJ_RAW_QR: {
            if (!g->op) return fail(GUESS_EINVAL, "guess_update: the raw-solution projection needs an operator");
            if (Ax) return fail(GUESS_EINVAL, "guess_update: the raw-solution projection applies A to the stored "
                                              "vector itself; pass Ax = NULL");
            LG_TRY(lg::launch_raw_update(raw_bufs(g), g->op->g, x, g->stream, g->prof ? &g->kev : nullptr));
            g->update_bytes = -1.0;
            return check_launch("guess_update");
        }
    }
    return fail(GUESS_EINVAL, "guess_update: bad method");
}

extern "C" int guess_next_slot(guess_t g, double **slot) {
    if (!g || !slot) return fail(GUESS_EINVAL, "guess_next_slot: NULL argument");
    *slot = nullptr;
    if (!ring_method(g->method) || g->dtype != GUESS_F64)
        return fail(GUESS_EINVAL, "guess_next_slot: needs an extrapolation context with FP64 history");
    *slot = (double *)((char *)g->ring + (size_t)g->head * g->ld * g->es);
    return GUESS_OK;
}

extern "C" int guess_get_info(guess_t g, guess_info *info) {
    if (!g || !info) return fail(GUESS_EINVAL, "guess_get_info: NULL argument");
    std::memset(info, 0, sizeof *info);
    info->N = g->N;
    info->method = g->method;
    info->dtype = g->dtype;
    info->M = g->M;
    info->degree = g->degree;
    info->form_bytes = g->form_bytes;
    info->update_bytes = g->update_bytes;
    info->inner = g->inner;
    info->eps_rel = g->eps_rel;
    if (proj_method(g->method)) {
        LG_HIP(hipMemcpyAsync(g->host_st, g->st, sizeof(lg::ProjState), hipMemcpyDeviceToHost, g->stream));
        LG_HIP(hipStreamSynchronize(g->stream));
        const lg::ProjState &s = *g->host_st;
        info->count = s.d;
        info->last_accepted = s.last_accepted;
        info->restarts = s.restarts;
        info->rejects = s.rejects;
        info->nonfinite = s.nonfinite;
        info->nu = s.nu;
        info->nu0 = s.nu0;
        info->drops = s.drops;
        const double N = (double)g->N, es = g->es;
        if (g->form_bytes < 0) info->form_bytes = 2.0 * N * (s.form_d * es + 8.0) - (s.form_d == 0 ? N * 8.0 : 0.0);
        if (g->update_bytes < 0) {
            // apply 16 + d s; reorth 2 d s + 8 (l2: d s + 8; FP16, either: 2 d s + 16, as it
            // also forms x - X c1 for the exponent); write 2 d s + 16 + 2 s, or with a
            // rolling drop 4 d s + 16; restart 8 (+8) + 2 s, FP16 16 + 16 + 2 s (the apply
            // pass writes A x, or reads the caller's, and the write kernel stores the pair)
            const int d = s.upd_d;
            const bool f16 = g->dtype == GUESS_F16;
            const bool restart = d == 0 || (g->method == GUESS_PROJ_QR ? g->M == 1 : d >= g->M);
            const double reorth = f16 ? 2.0 * d * es + 16.0 : (g->inner == GUESS_INNER_L2 ? 1.0 : 2.0) * d * es + 8.0;
            if (restart && f16) info->update_bytes = N * (32.0 + 2.0 * es);
            else if (restart) info->update_bytes = N * (8.0 + 2.0 * es + (g->last_update_ax ? 8.0 : 0.0));
            else if (s.drop) info->update_bytes = N * (16.0 + d * es + reorth + 4.0 * d * es + 16.0);
            else info->update_bytes = N * (16.0 + d * es + reorth + 2.0 * d * es + 16.0 + 2.0 * es);
            // a variable-coefficient operator applied by the library also reads its face arrays
            if (!g->last_update_ax && g->op && g->op->g.kx) {
                const lg::Grid &G = g->op->g;
                info->update_bytes += 8.0 * ((double)(G.nx + 1) * G.ny * G.nz + (double)G.nx * (G.ny + 1) * G.nz +
                                             (double)G.nx * G.ny * (G.nz + 1));
            }
        }
    } else if (raw_method(g->method)) {
        LG_TRY(raw_read_state(g));
        const lg::RawState &s = *g->host_rst;
        info->count = s.d;
        info->last_accepted = s.last_accepted;
        info->restarts = s.restarts;
        info->rejects = s.rejects;
        info->nonfinite = s.nonfinite;
        info->nu = s.nu;
        info->nu0 = s.nu0;
        info->drops = s.drops;
        const double N = (double)g->N, es = g->es;
        if (g->form_bytes < 0) info->form_bytes = s.form_d == 0 ? 8.0 * N : 2.0 * N * (s.form_d * es + 8.0);
        if (g->update_bytes < 0) {
            // store 8 + s (FP16: twice when the exponent changed); apply: the stored vector and
            // the columns of the Gram row, (nd + 1) s
            const int d = s.upd_d;
            const int nd = d >= g->M ? (g->method == GUESS_PROJ_RAW_QR ? g->M - 1 : 0) : d;
            info->update_bytes = N * (8.0 + es) * (s.fixed && g->dtype == GUESS_F16 ? 2.0 : 1.0) + N * (nd + 1) * es;
            if (g->op && g->op->g.kx) {
                const lg::Grid &G = g->op->g;
                info->update_bytes += 8.0 * ((double)(G.nx + 1) * G.ny * G.nz + (double)G.nx * (G.ny + 1) * G.nz +
                                             (double)G.nx * G.ny * (G.nz + 1));
            }
        }
    } else {
        LG_HIP(hipStreamSynchronize(g->stream));
        info->count = g->count;
        info->head = g->head;
        // an FP16 store that had to be repeated with this solution's exponent moved its bytes twice
        if (g->rs && g->update_bytes > 0.0) {
            LG_TRY(ring_read_state(g));
            if (g->host_rs->last_fixed) info->update_bytes = 2.0 * g->update_bytes;
        }
    }
    return GUESS_OK;
}

extern "C" int guess_reset(guess_t g) {
    if (!g) return fail(GUESS_EINVAL, "guess_reset: NULL context");
    g->count = 0;
    g->head = 0;
    if (proj_method(g->method)) {
        LG_HIP(hipStreamSynchronize(g->stream));
        LG_HIP(hipMemcpyAsync(g->host_st, g->st, sizeof(lg::ProjState), hipMemcpyDeviceToHost, g->stream));
        LG_HIP(hipStreamSynchronize(g->stream));
        g->host_st->d = 0;
        g->host_st->mode = 0;
        g->host_st->drop = 0;
        LG_HIP(hipMemcpyAsync(g->st, g->host_st, sizeof(lg::ProjState), hipMemcpyHostToDevice, g->stream));
        LG_HIP(hipStreamSynchronize(g->stream));
    } else if (raw_method(g->method)) {
        LG_HIP(hipStreamSynchronize(g->stream));
        LG_TRY(raw_read_state(g));
        g->host_rst->d = 0;
        LG_HIP(hipMemcpyAsync(g->rst, g->host_rst, sizeof(lg::RawState), hipMemcpyHostToDevice, g->stream));
        LG_HIP(hipStreamSynchronize(g->stream));
    }
    return GUESS_OK;
}

extern "C" int guess_profile(guess_t g, int enable) {
    if (!g) return fail(GUESS_EINVAL, "guess_profile: NULL context");
    if (enable && !g->prof) {
        for (int i = 0; i < 8; ++i) {
            LG_HIP(hipEventCreate(&g->kev.start[i]));
            LG_HIP(hipEventCreate(&g->kev.stop[i]));
        }
        g->prof = true;
    } else if (!enable && g->prof) {
        LG_HIP(hipStreamSynchronize(g->stream));
        for (int i = 0; i < 8; ++i) {
            (void)hipEventDestroy(g->kev.start[i]);
            (void)hipEventDestroy(g->kev.stop[i]);
        }
        g->prof = false;
    }
    g->kev.count = 0;
    return GUESS_OK;
}

extern "C" int guess_kernel_times(guess_t g, double *ms, int max, int *n) {
    if (!g || !n || (max > 0 && !ms)) return fail(GUESS_EINVAL, "guess_kernel_times: NULL argument");
    *n = 0;
    if (!g->prof || g->kev.count == 0) return GUESS_OK;
    const int cnt = g->kev.count;
    LG_HIP(hipEventSynchronize(g->kev.stop[cnt - 1]));
    for (int i = 0; i < cnt && i < max; ++i) {
        float t = 0.0f;
        LG_HIP(hipEventElapsedTime(&t, g->kev.start[i], g->kev.stop[i]));
        ms[i] = t;
    }
    *n = cnt < max ? cnt : max;
    return GUESS_OK;
}

// Stored vector j and its FP64 scale (true values = scale * stored values).
static int history_vector(guess_t g, int which, int j, const char *fn, const void **src, double *scale) {
    if (ring_method(g->method)) {
        if (j < 0 || j >= g->count) return fail(GUESS_EINVAL, std::string(fn) + ": index out of range");
        const int slot = ((g->head - g->count) % g->slots + g->slots + j) % g->slots;
        *src = (const char *)g->ring + (size_t)slot * g->ld * g->es;
        *scale = 1.0;
        if (g->rs) {
            LG_TRY(ring_read_state(g));
            *scale = std::ldexp(1.0, -g->host_rs->exps[slot]);
        }
        return GUESS_OK;
    }
    if (raw_method(g->method)) {
        LG_TRY(raw_read_state(g));
        if (j < 0 || j >= g->host_rst->d || which != 0) return fail(GUESS_EINVAL, std::string(fn) + ": index out of range");
        const int slot = g->host_rst->perm[j];
        *src = (const char *)g->X + (size_t)slot * g->ld * g->es;
        *scale = std::ldexp(1.0, -g->host_rst->exps[slot]);
        return GUESS_OK;
    }
    if (proj_method(g->method)) {
        LG_HIP(hipMemcpyAsync(g->host_st, g->st, sizeof(lg::ProjState), hipMemcpyDeviceToHost, g->stream));
        LG_HIP(hipStreamSynchronize(g->stream));
        if (j < 0 || j >= g->host_st->d || (which != 0 && which != 1))
            return fail(GUESS_EINVAL, std::string(fn) + ": index out of range");
        *src = (const char *)(which == 0 ? g->X : g->B) + (size_t)j * g->ld * g->es;
        *scale = g->host_st->scale[j];
        return GUESS_OK;
    }
    return fail(GUESS_EINVAL, std::string(fn) + ": no history for this method");
}

extern "C" int guess_history_get(guess_t g, int which, int j, double *out) {
    if (!g || !out) return fail(GUESS_EINVAL, "guess_history_get: NULL argument");
    const void *src = nullptr;
    double scale = 1.0;
    LG_TRY(history_vector(g, which, j, "guess_history_get", &src, &scale));
    LG_TRY(lg::launch_widen(g->dtype, src, scale, out, g->N, g->stream));
    LG_TRY(check_launch("guess_history_get"));
    LG_HIP(hipStreamSynchronize(g->stream));
    return GUESS_OK;
}

extern "C" int guess_history_raw(guess_t g, int which, int j, double *out, double *scale) {
    if (!g || !out || !scale) return fail(GUESS_EINVAL, "guess_history_raw: NULL argument");
    const void *src = nullptr;
    LG_TRY(history_vector(g, which, j, "guess_history_raw", &src, scale));
    LG_TRY(lg::launch_widen(g->dtype, src, 1.0, out, g->N, g->stream));
    LG_TRY(check_launch("guess_history_raw"));
    LG_HIP(hipStreamSynchronize(g->stream));
    return GUESS_OK;
}

extern "C" int guess_proj_factor(guess_t g, double *R, int *d) {
    if (!g || !R || !d) return fail(GUESS_EINVAL, "guess_proj_factor: NULL argument");
    if (raw_method(g->method)) {
        // R = L^T: raw solutions = X R with X = W L^-T A-orthonormal
        LG_TRY(raw_read_state(g));
        const int n = g->host_rst->d;
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) R[i * n + j] = j >= i ? g->host_rst->L[j][i] : 0.0;
        *d = n;
        return GUESS_OK;
    }
    if (!proj_method(g->method)) return fail(GUESS_EINVAL, "guess_proj_factor: not a projection context");
    LG_HIP(hipMemcpyAsync(g->host_st, g->st, sizeof(lg::ProjState), hipMemcpyDeviceToHost, g->stream));
    LG_HIP(hipStreamSynchronize(g->stream));
    const int n = g->host_st->d;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) R[i * n + j] = j >= i ? g->host_st->R[i][j] : 0.0;
    *d = n;
    return GUESS_OK;
}

// ====================================================================== workload
namespace {
// The workload generators keep device tables per host thread.  A table is
// rewritten only after the kernels of the previous call that read it have
// finished: `done` is recorded after every launch, so a call on another
// stream (or with other parameters) first waits for it.
struct PlaneWaveTables {
    int n = -1, K = -1;
    std::vector<int> kvec;
    std::vector<double> theta;
    double *dev = nullptr;  // 3 tables of K*n complex values
    hipEvent_t done = nullptr;
};
thread_local PlaneWaveTables g_pw;

int record_done(hipEvent_t &ev, hipStream_t s) {
    if (!ev && hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        ev = nullptr;
        return fail(GUESS_EHIP, "workload: event creation failed");
    }
    LG_HIP(hipEventRecord(ev, s));
    return GUESS_OK;
}
}  // namespace

extern "C" int workload_plane_wave_rhs(int n, int K, const int *kvec, const double *theta, const double *amp,
                                       double *b, void *stream) {
    if (n < 1 || K < 1 || K > 64 || !kvec || !theta || !amp || !b)
        return fail(GUESS_EINVAL, "workload_plane_wave_rhs: bad argument");
    hipStream_t s = (hipStream_t)stream;
    const bool same = g_pw.dev && g_pw.n == n && g_pw.K == K &&
                      std::equal(kvec, kvec + 3 * K, g_pw.kvec.begin()) &&
                      std::equal(theta, theta + K, g_pw.theta.begin());
    if (!same) {
        if (g_pw.dev) {
            if (g_pw.done) LG_HIP(hipEventSynchronize(g_pw.done));
            (void)hipFree(g_pw.dev);
            g_pw.dev = nullptr;
        }
        std::vector<double> tab((size_t)3 * K * n * 2);
        const double two_pi = 2.0 * M_PI, h = 1.0 / (n + 1);
        for (int axis = 0; axis < 3; ++axis)
            for (int k = 0; k < K; ++k)
                for (int i = 0; i < n; ++i) {
                    double ph = two_pi * kvec[3 * k + axis] * ((i + 1) * h);
                    if (axis == 0) ph += theta[k];
                    const size_t o = (((size_t)axis * K + k) * n + i) * 2;
                    tab[o] = std::cos(ph);
                    tab[o + 1] = std::sin(ph);
                }
        if (hipMalloc((void **)&g_pw.dev, tab.size() * 8) != hipSuccess) {
            (void)hipGetLastError();
            g_pw.dev = nullptr;
            return fail(GUESS_ENOMEM, "workload_plane_wave_rhs: allocation failed");
        }
        LG_HIP(hipMemcpy(g_pw.dev, tab.data(), tab.size() * 8, hipMemcpyHostToDevice));
        g_pw.n = n;
        g_pw.K = K;
        g_pw.kvec.assign(kvec, kvec + 3 * K);
        g_pw.theta.assign(theta, theta + K);
    }
    const size_t tsz = (size_t)K * n * 2;
    LG_TRY(lg::launch_plane_wave_rhs(n, K, g_pw.dev, g_pw.dev + tsz, g_pw.dev + 2 * tsz, amp, b, s));
    LG_TRY(check_launch("workload_plane_wave_rhs"));
    return record_done(g_pw.done, s);
}

namespace {
struct GaussTables {
    int n = 0;
    double *dev = nullptr;
    hipStream_t last = nullptr;   // stream of the previous call (compared, never used)
    hipEvent_t done = nullptr;
};
thread_local GaussTables g_gauss;
}  // namespace

extern "C" int workload_gaussian_rhs(int n, const double *center, double sigma, double amp, double *b,
                                     void *stream) {
    if (n < 1 || !center || !b || !(sigma > 0.0) || !std::isfinite(sigma))
        return fail(GUESS_EINVAL, "workload_gaussian_rhs: bad argument");
    hipStream_t s = (hipStream_t)stream;
    // every call rewrites the tables: on the previous call's stream that is ordered, on another
    // stream wait for the previous call's kernels first
    if (g_gauss.done && (g_gauss.last != s || !g_gauss.dev || g_gauss.n < n))
        LG_HIP(hipEventSynchronize(g_gauss.done));
    if (!g_gauss.dev || g_gauss.n < n) {
        if (g_gauss.dev) {
            (void)hipFree(g_gauss.dev);
            g_gauss.dev = nullptr;
        }
        if (hipMalloc((void **)&g_gauss.dev, sizeof(double) * 3 * (size_t)n) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GUESS_ENOMEM, "workload_gaussian_rhs: allocation failed");
        }
        g_gauss.n = n;
    }
    LG_TRY(lg::launch_gaussian_rhs(n, center, sigma, amp, g_gauss.dev, b, s));
    LG_TRY(check_launch("workload_gaussian_rhs"));
    g_gauss.last = s;
    return record_done(g_gauss.done, s);
}

// ====================================================================== vectors
namespace {
struct VecScratch {
    double *part = nullptr, *out = nullptr;
};
thread_local VecScratch g_vec;
}  // namespace

extern "C" int vec_multidot(int64_t N, int K, const double *V, const double *y, double *out, void *stream) {
    if (N < 1 || K < 1 || K > 64 || !V || !y || !out) return fail(GUESS_EINVAL, "vec_multidot: bad argument");
    hipStream_t s = (hipStream_t)stream;
    if (!g_vec.part) {
        if (hipMalloc((void **)&g_vec.part, sizeof(double) * lg::kMaxPartialBlocks * 8) != hipSuccess ||
            hipMalloc((void **)&g_vec.out, sizeof(double) * 64) != hipSuccess) {
            (void)hipGetLastError();
            return fail(GUESS_ENOMEM, "vec_multidot: allocation failed");
        }
    }
    LG_TRY(lg::launch_multidot(N, K, V, y, g_vec.part, g_vec.out, s));
    LG_TRY(check_launch("vec_multidot"));
    LG_HIP(hipMemcpyAsync(out, g_vec.out, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    LG_HIP(hipStreamSynchronize(s));
    return GUESS_OK;
}

// ---------------------------------------------------------------------- allocation-free multi-dot
// Scratch of vec_multidot_noalloc: the partial rows of the first reduction
// stage (at most kMaxPartialBlocks rows of 8 values) followed by the K <= 64
// results.  Every value the second stage reads was written by the first stage
// of the same call, so nothing needs clearing.  Each GPU the library runs on
// holds its own copy (128.5 KiB) until the process ends, and every call on
// that GPU shares it.  In host code `scratch` only names the symbol: its
// device address on the current GPU comes from hipGetSymbolAddress.
constexpr int kNoallocPart = lg::kMaxPartialBlocks * 8;
constexpr int kNoallocK = 64;
static __device__ __align__(256) double scratch[kNoallocPart + kNoallocK];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};
}  // namespace

// Device address of the current GPU's scratch, looked up once per device with
// that device current.
static int scratch_address(double **out) {
    int dev = -1;
    LG_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GUESS_EINVAL, "vec_multidot_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        LG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(GUESS_EHIP, "vec_multidot_noalloc: no device address for the scratch array");
        g_scratch_dev[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[dev];
    return GUESS_OK;
}

extern "C" int vec_multidot_noalloc(int64_t N, int K, const double *V, const double *y, double *out,
                                    void *stream) {
    if (N < 1 || !V || !y || !out) return fail(GUESS_EINVAL, "vec_multidot_noalloc: bad argument");
    if (K < 1 || K > kNoallocK)
        return fail(GUESS_EINVAL, "vec_multidot_noalloc: K must be in 1..64 (the static scratch holds 64 results)");
    if (lg::reduce_blocks() * 8 > kNoallocPart)
        return fail(GUESS_EINVAL, "vec_multidot_noalloc: more partial rows than the static scratch holds");
    double *sp = nullptr;
    LG_TRY(scratch_address(&sp));
    hipStream_t s = (hipStream_t)stream;
    LG_TRY(lg::launch_multidot(N, K, V, y, sp, sp + kNoallocPart, s));
    LG_TRY(check_launch("vec_multidot_noalloc"));
    LG_HIP(hipMemcpyAsync(out, sp + kNoallocPart, sizeof(double) * K, hipMemcpyDeviceToHost, s));
    LG_HIP(hipStreamSynchronize(s));
    return GUESS_OK;
}

extern "C" int vec_combine(int64_t N, int K, const double *V, const double *c, double *y, void *stream) {
    if (N < 1 || K < 1 || K > 64 || !V || !c || !y) return fail(GUESS_EINVAL, "vec_combine: bad argument");
    LG_TRY(lg::launch_combine(N, K, V, c, y, (hipStream_t)stream));
    return check_launch("vec_combine");
}

extern "C" int guess_copy_kernel(void *dst, const void *src, size_t bytes, void *stream) {
    if (!dst || !src) return fail(GUESS_EINVAL, "guess_copy_kernel: NULL argument");
    if (!aligned16(dst) || !aligned16(src)) return fail(GUESS_EINVAL, "guess_copy_kernel: need 16-byte alignment");
    LG_TRY(lg::launch_copy(dst, src, bytes, (hipStream_t)stream));
    return check_launch("guess_copy_kernel");
}

extern "C" int guess_roof_kernel(int mode, void *dst, const void *src, size_t bytes, void *stream) {
    hipStream_t s = (hipStream_t)stream;
    switch (mode) {
        case GUESS_ROOF_COPY: return guess_copy_kernel(dst, src, bytes, stream);
        case GUESS_ROOF_READ:
        case GUESS_ROOF_READ_STREAMS:
            if (!dst || !src) return fail(GUESS_EINVAL, "guess_roof_kernel: NULL argument");
            if (!aligned16(src) || !aligned16(dst)) return fail(GUESS_EINVAL, "guess_roof_kernel: need 16-byte alignment");
            if (mode == GUESS_ROOF_READ) LG_TRY(lg::launch_read(src, bytes, (double *)dst, s));
            else LG_TRY(lg::launch_read_streams(src, bytes, (double *)dst, s));
            return check_launch("guess_roof_kernel");
        case GUESS_ROOF_WRITE:
            if (!dst) return fail(GUESS_EINVAL, "guess_roof_kernel: NULL argument");
            if (!aligned16(dst)) return fail(GUESS_EINVAL, "guess_roof_kernel: need 16-byte alignment");
            LG_TRY(lg::launch_write(dst, bytes, s));
            return check_launch("guess_roof_kernel");
    }
    return fail(GUESS_EINVAL, "guess_roof_kernel: unknown mode");
}

// ====================================================================== errors
extern "C" const char *guess_strerror(int code) {
    switch (code) {
        case GUESS_OK: return "success";
        case GUESS_EINVAL: return "invalid argument";
        case GUESS_ENOMEM: return "out of device memory";
        case GUESS_EHIP: return "HIP runtime error";
        case GUESS_ENOTCONV: return "PCG did not converge within maxit";
        case GUESS_EBREAKDOWN: return "PCG breakdown";
        case GUESS_ENONFINITE: return "non-finite value";
    }
    return "unknown status";
}

extern "C" const char *guess_last_error(void) { return g_err.c_str(); }
