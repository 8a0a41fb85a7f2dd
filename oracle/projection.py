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

Storage (the paper fixes no precision; this reading says which numbers are
rounded to the storage format).  Column j is held as a stored pair S_j, T_j
(arrays of the storage format) and one FP64 scale sigma_j; the true columns
are X_j = sigma_j S_j and B_j = sigma_j T_j.

* A new pair (x, b) of norm nu -- the raw solution at a restart, the
  twice-orthogonalised remainder otherwise -- is stored as
  S = round(2^e x), T = round(2^e b), sigma = 1 / (nu 2^e).  In exact
  arithmetic sigma S = x / nu: the normalised column of the algorithm's update
  step; only the rounding is placed on the unnormalised remainder.
* e = 0 for FP64, FP32 and BF16.  FP16 has too narrow a range for raw
  solutions and remainders, so there e is chosen from the pair's largest
  magnitude m (lowprec.f16_scale_exp: m 2^e in [2^14, 2^15)), with m taken
  from the raw pair at a restart and from the pair after the first
  Gram-Schmidt pass otherwise (the second pass changes it only by rounding).
* Rolling drop: within one update the rotated columns are exact FP64 vectors
  (the new solution is orthogonalised against them); they are rounded when
  the update stores them.  A rotated column keeps its slot's scale, except in
  FP16, where slot i gets sigma'_i = 2^-15 (|c_i| t_i + |s_i| mu_{i+1}) with
  t_0 = mu_0, t_{i+1} = |s_i| t_i + |c_i| mu_{i+1} and mu_j the largest true
  magnitude of stored pair j: a bound on the rotated pair's largest
  magnitude, so no stored value exceeds 2^15.
Otherwise the steps are those of Algorithms 1 and 2 in order.
"""
from __future__ import annotations

import numpy as np

from .lowprec import f16_scale_exp, round_store


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
        self.last_exp = 0

    # ------------------------------------------------------------ state
    def reset(self) -> None:
        self.S = []          # stored columns of X (values of the storage format)
        self.T = []          # stored columns of B = A X
        self.sig = []        # FP64 scale of each stored pair: X_j = sig_j S_j, B_j = sig_j T_j
        self.mu = []         # largest true magnitude of each stored pair (X_j and B_j together)
        self.raw = []        # raw solutions of the window: raw = X R
        self.R = np.zeros((0, 0))
        self.ratios = []     # nu / nu0 of every column accepted since the last reset / restart
        self.drops = 0

    @property
    def d(self) -> int:
        return len(self.S)

    @property
    def X(self):
        """True columns of the solution history."""
        return [sg * v for sg, v in zip(self.sig, self.S)]

    @property
    def B(self):
        """True columns of B = A X."""
        return [sg * v for sg, v in zip(self.sig, self.T)]

    @property
    def amplification(self) -> float:
        """max nu0 / nu over the accepted columns (1 for an empty history).

        Rounding errors of size u in a column accepted with ratio nu/nu0 are
        amplified by nu0/nu in the normalised column (and carried into every
        column it is later rotated with), so two correct FP64 implementations
        agree on the guess only to about u times this factor.
        """
        return max([1.0] + [1.0 / r for r in self.ratios])

    def _ip(self, xj, bj, b):
        """Inner product of the column pair (xj, bj) with the pair (x, b = A x)."""
        return float(xj @ b) if self.inner == "A" else float(bj @ b)

    def _norm2(self, x, b):
        return float(x @ b) if self.inner == "A" else float(b @ b)

    def _exp_for(self, x, b) -> int:
        """Power-of-two exponent of a new pair: 0, or for FP16 from its largest magnitude."""
        if self.dtype != "f16":
            return 0
        return f16_scale_exp(max(float(np.max(np.abs(x))), float(np.max(np.abs(b)))))

    def _put(self, x, b, sig):
        """Append the stored pair round(x / sig), round(b / sig) with scale sig; x / sig and
        b / sig are the caller's exact FP64 vectors in stored units."""
        S = round_store(x, self.dtype)
        T = round_store(b, self.dtype)
        self.S.append(S)
        self.T.append(T)
        self.sig.append(sig)
        self.mu.append(sig * max(float(np.max(np.abs(S))), float(np.max(np.abs(T)))))

    def _put_new(self, x, b, nu, e):
        """New column of norm nu: S = round(2^e x), T = round(2^e b), sigma = 1 / (nu 2^e)."""
        self._put(np.ldexp(x, e), np.ldexp(b, e), 1.0 / float(np.ldexp(nu, e)))

    # ------------------------------------------------------------ guess
    def form(self, b) -> np.ndarray:
        """x0 = X alpha with alpha_j = <column j, b>, or 0 for an empty history."""
        b = np.asarray(b, dtype=np.float64)
        if self.d == 0:
            return np.zeros_like(b)
        X = self.X
        alpha = [float(xj @ b) for xj in X] if self.inner == "A" else [float(bj @ b) for bj in self.B]
        x0 = alpha[0] * X[0]
        for a, xj in zip(alpha[1:], X[1:]):
            x0 = x0 + a * xj
        return x0

    # ------------------------------------------------------------ update
    def _drop_oldest(self):
        """Algorithm 2, QR update: delete the first column of R, restore triangular
        form with Givens rotations of rows i, i+1, rotate the columns of X and B.

        Updates R and the raw window; returns the d-1 rotated true columns of X
        and of B (exact FP64 vectors) and the rotations (c_i, s_i)."""
        d = self.d
        R = self.R[:, 1:].copy()                 # d x (d-1), upper Hessenberg
        X, B = self.X, self.B
        rots = []
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
            rots.append((c, s))
        self.R = R[: d - 1, :]
        self.raw = self.raw[1:]
        self.drops += 1
        return X[: d - 1], B[: d - 1], rots

    def _rotated_scales(self, rots):
        """Scale of each slot after a rolling drop (see the module docstring)."""
        if self.dtype != "f16":
            return list(self.sig[: len(rots)])
        out, t = [], self.mu[0]
        for i, (c, s) in enumerate(rots):
            out.append(float(np.ldexp(abs(c) * t + abs(s) * self.mu[i + 1], -15)))
            t = abs(s) * t + abs(c) * self.mu[i + 1]
        return out

    def _restart(self, x, xt, bt, nu0):
        ok = bool(np.isfinite(nu0) and nu0 > 0.0)
        self.last_exp = 0
        if ok:
            self.last_exp = self._exp_for(xt, bt)
            self._put_new(xt, bt, nu0, self.last_exp)
            self.raw.append(np.array(x, dtype=np.float64, copy=True))
            self.R = np.array([[nu0]])
            self.ratios.append(1.0)
        self.last_nu = nu0
        self.last_accepted = ok
        return ok

    def update(self, x, Ax=None, decide=None) -> bool:
        """Add the new solution to the history; returns whether it was accepted.

        ``decide`` (True / False) replaces the rejection test by a given
        decision: a replay that compares two implementations forces the other
        side's decision where nu / nu0 sits within rounding of eps_rel.
        """
        xt = np.array(x, dtype=np.float64, copy=True)
        bt = self.apply_A(xt) if Ax is None else np.array(Ax, dtype=np.float64, copy=True)
        s0 = self._norm2(xt, bt)
        nu0 = float(np.sqrt(s0)) if s0 >= 0 else float("nan")
        self.last_nu0 = nu0
        if self.variant == "classic":
            if self.d == 0 or self.d >= self.M:
                self.reset()
                return self._restart(x, xt, bt, nu0)
            Xc, Bc, keep = self.X, self.B, None
        else:
            keep = None
            if self.d == self.M:
                Xc, Bc, rots = self._drop_oldest()
                keep = (Xc, Bc, self._rotated_scales(rots))
                self.S, self.T, self.sig, self.mu = [], [], [], []
            else:
                Xc, Bc = self.X, self.B
            if len(Xc) == 0:
                return self._restart(x, xt, bt, nu0)
        d = len(Xc)
        ctot = np.zeros(d)
        e = 0
        for p in range(2):
            c = [self._ip(xj, bj, bt) for xj, bj in zip(Xc, Bc)]
            for cj, xj, bj in zip(c, Xc, Bc):
                bt = bt - cj * bj
                xt = xt - cj * xj
            ctot += np.array(c)
            if p == 0:
                e = self._exp_for(xt, bt)
        s = self._norm2(xt, bt)
        nu = float(np.sqrt(s)) if s >= 0 else float("nan")
        self.last_nu = nu
        self.last_exp = e
        fin = bool(np.isfinite(nu))
        ok = fin and (nu > self.eps_rel * nu0 if decide is None else bool(decide))
        if keep is not None:
            # the rotated columns are stored (rounded) at the end of the update
            for xj, bj, sg in zip(*keep):
                self._put(xj / sg, bj / sg, sg)
        if ok:
            self._put_new(xt, bt, nu, e)
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
