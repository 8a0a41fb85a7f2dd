"""Polynomial extrapolation weights and guesses (oracle; test infrastructure only).

Follows §3 of the paper:

* the guess is a fixed linear combination of the last M solutions, with the
  first weight on the oldest stored solution (§3, eq. ExtrapExpn);
* naive extrapolation through all M points has the binomial weights of the
  theorem in §3.1 (eq. NaiveExtrapCoeffs);
* stabilized extrapolation fits a degree-m polynomial in the least-squares
  sense at the equispaced nodes t_i = -1 + (i-1) h, h = 2/(M-1), and evaluates
  it at t = 1 + h, giving beta^T = v^T (V^T V)^{-1} V^T (§3.2, eq. LSQRCoeffs);
* the Lebesgue constant of a scheme is the 1-norm of its weights (§6.5).

Weights are computed in exact rational arithmetic (``fractions.Fraction``),
with the monomial basis: the least-squares weights do not depend on the choice
of polynomial basis, nor on an affine change of the time variable (§3.2).
"""
from __future__ import annotations

from fractions import Fraction
from math import comb

import numpy as np


def time_nodes(M: int):
    """Equispaced history nodes and the new node (§3.2).

    For M = 1 the single history value sits at t = 0 and the new node at
    t = 1; with one point only the constant fit exists, so any placement gives
    the same weight (beta = [1], the previous-solution guess).
    """
    if M < 1:
        raise ValueError("M must be >= 1")
    if M == 1:
        return [Fraction(0)], Fraction(1)
    h = Fraction(2, M - 1)
    t = [Fraction(-1) + (i - 1) * h for i in range(1, M + 1)]
    return t, Fraction(1) + h


def _solve_exact(G, rhs):
    """Gauss-Jordan elimination on a small nonsingular rational system."""
    n = len(G)
    A = [list(G[r]) + [rhs[r]] for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        p = A[col][col]
        A[col] = [a / p for a in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [a - f * b for a, b in zip(A[r], A[col])]
    return [A[r][n] for r in range(n)]


def vandermonde(M: int, m: int):
    """V_ij = psi_j(t_i) with psi_j(t) = t^j, and v_j = psi_j(t_new) (§3.2)."""
    t, tn = time_nodes(M)
    V = [[ti ** j for j in range(m + 1)] for ti in t]
    v = [tn ** j for j in range(m + 1)]
    return V, v


def beta_ls_exact(m: int, M: int):
    """Least-squares extrapolation weights beta (length M) as Fractions.

    beta = V (V^T V)^{-1} v, i.e. beta^T = v^T (V^T V)^{-1} V^T
    (§3.2, eq. LSQRCoeffs).  Requires 0 <= m <= M - 1.
    """
    if not (0 <= m <= M - 1):
        raise ValueError("need 0 <= m <= M-1")
    V, v = vandermonde(M, m)
    G = [[sum(V[i][a] * V[i][b] for i in range(M)) for b in range(m + 1)]
         for a in range(m + 1)]
    y = _solve_exact(G, v)
    return [sum(V[i][j] * y[j] for j in range(m + 1)) for i in range(M)]


def beta_naive_exact(M: int):
    """Weights of Lagrange extrapolation through M equispaced points.

    beta_i = (-1)^(M-i) C(M, i-1), i = 1..M (§3.1, theorem, eq.
    NaiveExtrapCoeffs).
    """
    return [Fraction((-1) ** (M - i) * comb(M, i - 1)) for i in range(1, M + 1)]


def lebesgue(beta) -> Fraction:
    """Lebesgue constant Lambda = ||beta||_1 (§6.5)."""
    return sum(abs(Fraction(b)) for b in beta)


def to_f64(beta) -> np.ndarray:
    """Round exact weights to FP64 once (correct rounding of each ratio)."""
    return np.array([float(Fraction(b)) for b in beta], dtype=np.float64)


def effective_params(m: int, M: int, k: int):
    """Warm-up rule while the history holds only k < M solutions.

    The paper does not treat the start of a sequence.  Reading used here:
    with k stored solutions the guess is EXTRAP(min(m, k-1), k); k = 1 gives
    the previous solution and k = 0 gives the zero guess.  Returns (m_eff, k)
    or None for the zero guess.
    """
    k = min(k, M)
    if k <= 0:
        return None
    return min(m, k - 1), k


def form(history_oldest_first, beta) -> np.ndarray:
    """x0 = sum_i beta_i x_{n-M+i}, summed oldest first (§3, eq. ExtrapExpn)."""
    beta = np.asarray(beta, dtype=np.float64)
    if len(history_oldest_first) != len(beta):
        raise ValueError("history length and weight count differ")
    acc = beta[0] * np.asarray(history_oldest_first[0], dtype=np.float64)
    for b, x in zip(beta[1:], history_oldest_first[1:]):
        acc = acc + b * np.asarray(x, dtype=np.float64)
    return acc


class ExtrapHistory:
    """Last-M-solutions history with least-squares extrapolation (§3.2), or
    with sparse extrapolation (§3.3) when ``sparse`` is set.

    ``dtype`` selects the storage format of stored solutions (see
    ``oracle.lowprec``); the guess itself is always evaluated in FP64 from the
    stored (rounded) values, which is the exact value the GPU's FP32
    accumulation approximates.

    FP16 storage (a reading; the paper fixes no precision): a solution x is
    stored as round(2^e x) with e = lowprec.f16_scale_exp(max |x|), so the
    stored magnitudes lie below 2^15 whatever the size of the solution; the
    value it stands for is 2^-e round(2^e x).  Other formats store round(x).
    """

    def __init__(self, M: int, m: int, dtype: str = "f64", sparse: bool = False):
        if not (0 <= m <= M - 1):
            raise ValueError("need 0 <= m <= M-1")
        self.M, self.m, self.dtype, self.sparse = M, m, dtype, sparse
        self.hist = []          # oldest first, stored values (descaled) as float64 arrays
        self.exps = []          # power-of-two exponent of each stored solution (FP16; else 0)
        self._cache = {}

    def weights(self, k: int):
        p = effective_params(self.m, self.M, k)
        if p is None:
            return None
        if p not in self._cache:
            self._cache[p] = to_f64(beta_sparse_exact(*p) if self.sparse else beta_ls_exact(*p))
        return self._cache[p]

    def form(self, b=None, N=None) -> np.ndarray:
        k = len(self.hist)
        if k == 0:
            n = N if N is not None else (len(b) if b is not None else None)
            if n is None:
                raise ValueError("need N for an empty history")
            return np.zeros(n, dtype=np.float64)
        return form(self.hist, self.weights(k))

    def update(self, x) -> None:
        from .lowprec import f16_scale_exp, round_store

        x = np.asarray(x, dtype=np.float64)
        e = f16_scale_exp(float(np.max(np.abs(x)))) if self.dtype == "f16" and x.size else 0
        self.hist.append(round_store(x, self.dtype, e))
        self.exps.append(e)
        if len(self.hist) > self.M:
            self.hist.pop(0)
            self.exps.pop(0)

    def reset(self) -> None:
        self.hist = []
        self.exps = []


# ---------------------------------------------------------------- sparse extrapolation (§3.3)
def legendre_vandermonde(M: int, m: int):
    """V_ij = P_j(t_i), v_j = P_j(t_new) with Legendre polynomials P_j (§3.2).

    The paper allows any basis well behaved on [-1, 1]; the least-squares
    weights do not depend on it, but the nodes chosen by column pivoting do.
    Reading used here: Legendre, through the three-term recurrence
    (j+1) P_{j+1} = (2j+1) t P_j - j P_{j-1}, in exact arithmetic.
    """
    t, tn = time_nodes(M)

    def P(x):
        out = [Fraction(1)]
        if m >= 1:
            out.append(Fraction(x))
        for j in range(1, m):
            out.append(((2 * j + 1) * x * out[j] - j * out[j - 1]) / (j + 1))
        return out[: m + 1]

    return [P(ti) for ti in t], P(tn)


def cpqr_pivots(m: int, M: int):
    """Column order chosen by column-pivoted QR of V^T (§3.3), first m+1 pivots.

    Column pivoting takes, at each step, the column of V^T (one history node)
    whose component orthogonal to the columns already taken has the largest
    norm.  The computation is exact (rational Gram-Schmidt without
    normalisation, so no square roots); among exactly equal norms the lowest
    node index wins, the first-maximum rule of LAPACK's pivoting.  Returns
    0-based node indices in pivot order.
    """
    if not (0 <= m <= M - 1):
        raise ValueError("need 0 <= m <= M-1")
    V, _ = legendre_vandermonde(M, m)
    cols = [list(row) for row in V]          # column i of V^T = row i of V
    basis = []                               # orthogonal (unnormalised) directions taken so far
    chosen = []

    def residual(c):
        r = list(c)
        for q, qq in basis:
            f = sum(a * b for a, b in zip(r, q)) / qq
            r = [a - f * b for a, b in zip(r, q)]
        return r

    for _ in range(m + 1):
        best, best_i, best_r = None, None, None
        for i in range(M):
            if i in chosen:
                continue
            r = residual(cols[i])
            nn = sum(a * a for a in r)
            if best is None or nn > best:
                best, best_i, best_r = nn, i, r
        if best == 0:
            raise ValueError("V^T is rank deficient")
        chosen.append(best_i)
        basis.append((best_r, best))
    return chosen


def beta_sparse_exact(m: int, M: int):
    """Sparse extrapolation weights (§3.3, eq. CPQRCoeffs) as Fractions.

    With V^T P = Q R and R = [R_hat R_tilde], the weights are
    beta = P [R_hat^{-1} Q^T v; 0]: the m+1 pivot columns of V^T form the
    square block Q R_hat, so beta_hat solves (V_S)^T beta_hat = v on the
    pivot nodes S, and every other weight is zero.
    """
    S = cpqr_pivots(m, M)
    V, v = legendre_vandermonde(M, m)
    G = [[V[S[c]][r] for c in range(m + 1)] for r in range(m + 1)]     # (V_S)^T
    bh = _solve_exact(G, v)
    beta = [Fraction(0)] * M
    for c, i in enumerate(S):
        beta[i] = bh[c]
    return beta
