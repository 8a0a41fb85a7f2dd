"""Fischer's projection, classic restart variant, A inner product (oracle).

TEST INFRASTRUCTURE ONLY.

§2 of the paper keeps a history of solutions X and of right-hand sides
B = A X with orthonormal B, guesses x0 = X B^T b (minimising the residual
2-norm over span X), re-orthogonalises each new pair twice with classical
Gram-Schmidt, rejects a new vector whose projected norm is below a threshold,
and discards the whole history when it is full (Algorithm 1, "classic").

Reading used here (the A-orthonormal form of the same algorithm, for SPD A):
the history satisfies X^T A X = I and B = A X, the guess is x0 = X (X^T b),
which minimises the A-norm error ||x* - x||_A over span X, the Gram-Schmidt
coefficients are A-inner products <x_j, A x~> = x_j^T b~ and the norm of a
new vector is its A-norm sqrt(x~^T b~).  The rejection test is relative:
accept iff nu > eps_rel * nu0, nu0 = ||x||_A of the raw solution.  The
algorithm is otherwise Algorithm 1 step by step.
"""
from __future__ import annotations

import numpy as np


class AOrthoProjection:
    def __init__(self, M: int, apply_A, eps_rel: float = 1e-6, dtype: str = "f64"):
        if M < 1:
            raise ValueError("M must be >= 1")
        self.M, self.apply_A, self.eps_rel, self.dtype = M, apply_A, eps_rel, dtype
        self.X = []          # A-orthonormal solution history
        self.B = []          # B = A X
        self.raw = []        # raw solutions accepted since the last restart
        self.ratios = []     # nu / nu0 of each stored column when it was accepted
        self.last_accepted = None
        self.last_nu = None
        self.last_nu0 = None

    @property
    def d(self) -> int:
        return len(self.X)

    @property
    def amplification(self) -> float:
        """max nu0 / nu over the stored columns (1 for an empty history).

        Rounding errors of size u in a column accepted with ratio nu/nu0 are
        amplified by nu0/nu in the normalised column, so two correct FP64
        implementations of this algorithm agree on the guess only to about
        u times this factor.
        """
        return max([1.0] + [1.0 / r for r in self.ratios])

    def form(self, b) -> np.ndarray:
        """x0 = X (X^T b), or 0 when the history is empty (Algorithm 1, first step)."""
        b = np.asarray(b, dtype=np.float64)
        if self.d == 0:
            return np.zeros_like(b)
        alpha = [float(xj @ b) for xj in self.X]
        x0 = alpha[0] * self.X[0]
        for a, xj in zip(alpha[1:], self.X[1:]):
            x0 = x0 + a * xj
        return x0

    def _store(self, v):
        from .lowprec import round_store

        return round_store(v, self.dtype)

    def update(self, x, Ax=None) -> bool:
        """Add the new solution to the history; returns whether it was accepted.

        Algorithm 1 after the solve: one operator application, then either a
        restart (d = 0 or d >= M) or twice-iterated classical Gram-Schmidt and
        the acceptance test.
        """
        xt = np.array(x, dtype=np.float64, copy=True)
        bt = self.apply_A(xt) if Ax is None else np.array(Ax, dtype=np.float64, copy=True)
        nu0 = float(np.sqrt(xt @ bt)) if (xt @ bt) >= 0 else float("nan")
        self.last_nu0 = nu0
        if self.d == 0 or self.d >= self.M:
            self.X, self.B, self.raw, self.ratios = [], [], [], []
            ok = np.isfinite(nu0) and nu0 > 0.0
            if ok:
                self.X.append(self._store(xt / nu0))
                self.B.append(self._store(bt / nu0))
                self.raw.append(np.array(x, dtype=np.float64, copy=True))
                self.ratios.append(1.0)
            self.last_nu = nu0
            self.last_accepted = bool(ok)
            return bool(ok)
        for _ in range(2):
            c = [float(xj @ bt) for xj in self.X]
            for cj, xj, bj in zip(c, self.X, self.B):
                bt = bt - cj * bj
                xt = xt - cj * xj
        s = float(xt @ bt)
        nu = float(np.sqrt(s)) if s >= 0 else float("nan")
        self.last_nu = nu
        ok = bool(np.isfinite(nu) and nu > self.eps_rel * nu0)
        if ok:
            self.X.append(self._store(xt / nu))
            self.B.append(self._store(bt / nu))
            self.raw.append(np.array(x, dtype=np.float64, copy=True))
            self.ratios.append(nu / nu0)
        self.last_accepted = ok
        return ok

    def reset(self) -> None:
        self.X, self.B, self.raw, self.ratios = [], [], [], []


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
