"""Fischer's projection guesses (oracle).

TEST INFRASTRUCTURE ONLY.

§2 of the paper keeps a history of solutions X and of right-hand sides
B = A X, guesses from the projection of b onto span B, re-orthogonalises each
new pair twice with classical Gram-Schmidt, rejects a new vector whose
projected norm is below a threshold, and bounds the history at M columns in
one of two ways:

* classic (Algorithm 1): when the history is full, discard all of it and
  start again from the new pair;
* rolling QR (Algorithm 2): keep the triangular factor R with
  [raw solutions] = X R; when the history is full, drop the oldest raw
  solution by deleting the first column of R, return the resulting upper
  Hessenberg matrix to triangular form with Givens rotations of neighbouring
  rows, and rotate the columns of X and B alongside, so that the window
  slides by one step.

Two inner products are provided:

* ``inner="A"`` (default): the A-orthonormal form for SPD A.  X^T A X = I,
  B = A X, the guess x0 = X (X^T b) minimises the A-norm error over span X;
  Gram-Schmidt coefficients are <x_j, A x~> = x_j^T b~ and the norm of a new
  vector is sqrt(x~^T b~).
* ``inner="l2"``: the paper's own form.  B^T B = I, the guess
  x0 = X (B^T b) minimises ||b - A x||_2 over span X; coefficients are
  b_j^T b~ and the norm is ||b~||_2.

Readings: the rejection test is relative, accept iff nu > eps_rel * nu0 with
nu0 the norm of the raw pair before orthogonalisation; the Givens rotation
that zeroes the subdiagonal entry b below the diagonal entry a has
c = |a| / r, s = sign(a) b / r, r = sqrt(a^2 + b^2), with sign(0) = +1, so
the new diagonal entry is sign(a) r (the listing's formulas for the rotation
are read this way).
Otherwise the steps are those of Algorithms 1 and 2 in order.
"""
from __future__ import annotations

import numpy as np


class Projection:
    def __init__(self, M: int, apply_A, eps_rel: float = 1e-6, dtype: str = "f64",
                 variant: str = "classic", inner: str = "A"):
        if M < 1:
            raise ValueError("M must be >= 1")
        if variant not in ("classic", "qr") or inner not in ("A", "l2"):
            raise ValueError("variant must be classic or qr, inner A or l2")
        self.M, self.apply_A, self.eps_rel, self.dtype = M, apply_A, eps_rel, dtype
        self.variant, self.inner = variant, inner
        self.reset()
        self.last_accepted = None
        self.last_nu = None
        self.last_nu0 = None

    # ------------------------------------------------------------ state
    def reset(self) -> None:
        self.X = []          # solution history
        self.B = []          # B = A X
        self.raw = []        # raw solutions of the window: raw = X R
        self.R = np.zeros((0, 0))
        self.ratios = []     # nu / nu0 of every column accepted since the last reset / restart
        self.drops = 0

    @property
    def d(self) -> int:
        return len(self.X)

    @property
    def amplification(self) -> float:
        """max nu0 / nu over the accepted columns (1 for an empty history).

        Rounding errors of size u in a column accepted with ratio nu/nu0 are
        amplified by nu0/nu in the normalised column (and carried into every
        column it is later rotated with), so two correct FP64 implementations
        agree on the guess only to about u times this factor.
        """
        return max([1.0] + [1.0 / r for r in self.ratios])

    def _ip(self, x, b, j):
        """Inner product of column j of the history with the pair (x, b = A x)."""
        return float(self.X[j] @ b) if self.inner == "A" else float(self.B[j] @ b)

    def _norm2(self, x, b):
        return float(x @ b) if self.inner == "A" else float(b @ b)

    def _store(self, v):
        from .lowprec import round_store

        return round_store(v, self.dtype)

    # ------------------------------------------------------------ guess
    def form(self, b) -> np.ndarray:
        """x0 = X alpha with alpha_j = <column j, b>, or 0 for an empty history."""
        b = np.asarray(b, dtype=np.float64)
        if self.d == 0:
            return np.zeros_like(b)
        alpha = [float(xj @ b) for xj in self.X] if self.inner == "A" else [float(bj @ b) for bj in self.B]
        x0 = alpha[0] * self.X[0]
        for a, xj in zip(alpha[1:], self.X[1:]):
            x0 = x0 + a * xj
        return x0

    # ------------------------------------------------------------ update
    def _drop_oldest(self):
        """Algorithm 2, QR update: delete the first column of R, restore triangular
        form with Givens rotations of rows i, i+1, rotate the columns of X and B."""
        d = self.d
        R = self.R[:, 1:].copy()                 # d x (d-1), upper Hessenberg
        X, B = list(self.X), list(self.B)
        for i in range(d - 1):
            a, b = R[i, i], R[i + 1, i]
            r = float(np.hypot(a, b))
            sg = 1.0 if a >= 0 else -1.0
            c = abs(a) / r
            s = sg * b / r
            G = np.array([[c, s], [-s, c]])
            R[i:i + 2, :] = G @ R[i:i + 2, :]
            R[i, i], R[i + 1, i] = sg * r, 0.0        # the entries the rotation fixes by construction
            X[i], X[i + 1] = c * X[i] + s * X[i + 1], -s * X[i] + c * X[i + 1]
            B[i], B[i + 1] = c * B[i] + s * B[i + 1], -s * B[i] + c * B[i + 1]
        self.R = R[: d - 1, :]
        self.X = [self._store(v) for v in X[: d - 1]]
        self.B = [self._store(v) for v in B[: d - 1]]
        self.raw = self.raw[1:]
        self.drops += 1

    def _add_first(self, x, xt, bt, nu0):
        ok = bool(np.isfinite(nu0) and nu0 > 0.0)
        if ok:
            self.X.append(self._store(xt / nu0))
            self.B.append(self._store(bt / nu0))
            self.raw.append(np.array(x, dtype=np.float64, copy=True))
            self.R = np.array([[nu0]])
            self.ratios.append(1.0)
        self.last_nu = nu0
        self.last_accepted = ok
        return ok

    def update(self, x, Ax=None) -> bool:
        """Add the new solution to the history; returns whether it was accepted."""
        xt = np.array(x, dtype=np.float64, copy=True)
        bt = self.apply_A(xt) if Ax is None else np.array(Ax, dtype=np.float64, copy=True)
        s0 = self._norm2(xt, bt)
        nu0 = float(np.sqrt(s0)) if s0 >= 0 else float("nan")
        self.last_nu0 = nu0
        if self.variant == "classic":
            if self.d == 0 or self.d >= self.M:
                self.reset()
                return self._add_first(x, xt, bt, nu0)
        else:
            if self.d == self.M:
                self._drop_oldest()
            if self.d == 0:
                return self._add_first(x, xt, bt, nu0)
        d = self.d
        ctot = np.zeros(d)
        for _ in range(2):
            c = [self._ip(xt, bt, j) for j in range(d)]
            for cj, xj, bj in zip(c, self.X, self.B):
                bt = bt - cj * bj
                xt = xt - cj * xj
            ctot += np.array(c)
        s = self._norm2(xt, bt)
        nu = float(np.sqrt(s)) if s >= 0 else float("nan")
        self.last_nu = nu
        ok = bool(np.isfinite(nu) and nu > self.eps_rel * nu0)
        if ok:
            self.X.append(self._store(xt / nu))
            self.B.append(self._store(bt / nu))
            self.raw.append(np.array(x, dtype=np.float64, copy=True))
            R = np.zeros((d + 1, d + 1))
            R[:d, :d] = self.R
            R[:d, d] = ctot
            R[d, d] = nu
            self.R = R
            self.ratios.append(nu / nu0)
        self.last_accepted = ok
        return ok


class AOrthoProjection(Projection):
    """Classic restart variant in the A inner product (Algorithm 1, A-orthonormal form)."""

    def __init__(self, M: int, apply_A, eps_rel: float = 1e-6, dtype: str = "f64"):
        super().__init__(M, apply_A, eps_rel, dtype, "classic", "A")


def brute_force_guess(S, apply_A, b) -> np.ndarray:
    """A-norm-optimal guess over span of the columns of S by normal equations.

    x = S (S^T A S)^{-1} S^T b minimises ||A^{-1} b - x||_A over span S.
    """
    S = np.asarray(S, dtype=np.float64)          # k x N (rows are vectors)
    AS = np.stack([apply_A(s) for s in S])
    G = S @ AS.T
    rhs = S @ np.asarray(b, dtype=np.float64)
    y = np.linalg.solve(G, rhs)
    return y @ S


def l2_residual_guess(S, apply_A, b) -> np.ndarray:
    """Residual-2-norm-optimal guess over span S (the paper's ell-2 form, §2).

    x = S (S^T A^T A S)^{-1} (A S)^T b minimises ||b - A x||_2 over span S.
    """
    S = np.asarray(S, dtype=np.float64)
    AS = np.stack([apply_A(s) for s in S])
    G = AS @ AS.T
    rhs = AS @ np.asarray(b, dtype=np.float64)
    y = np.linalg.solve(G, rhs)
    return y @ S
