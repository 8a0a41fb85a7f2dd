"""Projection through the Gram matrix of the stored raw solutions (oracle).

TEST INFRASTRUCTURE ONLY.

The guess of §2 is the A-norm-optimal combination of the stored solutions:
x0 minimises ||x* - x||_A over their span.  Algorithms 1 and 2 compute it from
an orthonormal basis built by Gram-Schmidt.  In exact arithmetic the same
guess follows from the stored solutions W themselves and their Gram matrix
G = W^T A W: x0 = W G^{-1} W^T b (the normal equations of the minimisation),
and the norm that the rejection test compares is that of the part of a new
solution w outside the span, nu^2 = w^T A w - g^T G^{-1} g with g = W^T A w
(the Schur complement of the Gram matrix extended by w); nu0^2 = w^T A w.

Reading for reduced-precision histories (the paper fixes no precision): the
stored solutions are rounded to the storage format -- FP16 as round(2^e x)
with e from max |x| (lowprec.f16_scale_exp), like the extrapolation ring --
and G is the exact FP64 Gram matrix of the vectors actually stored, A
applied to each stored vector.  The guess is then the A-norm-optimal
combination of what is stored: rounding moves the stored span a little but
leaves no inconsistency between a basis and its Gram matrix for
near-dependence to amplify (the Gram-Schmidt form's stored columns carry
rounding relative to their own small norms, which their normalisation
magnifies by nu0 / nu).

The history is bounded as in Algorithms 1 and 2: classic restarts (the
update that finds d = M starts again from the new solution) or the rolling
window (the update that finds d = M first drops the oldest solution).  The
rejection test is the relative reading of the Gram-Schmidt forms: keep w iff
nu > eps_rel * nu0.  Linear solves with G use the library routine (a step,
not a fusion of the method).
"""
from __future__ import annotations

import numpy as np

from .lowprec import f16_scale_exp, round_store


class RawProjection:
    def __init__(self, M: int, apply_A, eps_rel: float = 1e-6, dtype: str = "f64", variant: str = "classic"):
        if M < 1:
            raise ValueError("M must be >= 1")
        if variant not in ("classic", "qr"):
            raise ValueError("variant must be classic or qr")
        self.M, self.apply_A, self.eps_rel, self.dtype, self.variant = M, apply_A, eps_rel, dtype, variant
        self.reset()
        self.drops = 0
        self.last_accepted = None
        self.last_nu = None
        self.last_nu0 = None

    def reset(self) -> None:
        self.W = []            # stored solutions, oldest first (values they stand for, descaled)
        self.exps = []         # FP16: exponent of each stored solution; else 0
        self.G = np.zeros((0, 0))

    @property
    def d(self) -> int:
        return len(self.W)

    @property
    def R(self) -> np.ndarray:
        """Upper triangular factor with R^T R = G (raw solutions = X R, X = W R^-1
        A-orthonormal), by the library Cholesky routine."""
        return np.linalg.cholesky(self.G).T if self.d else np.zeros((0, 0))

    @property
    def amplification(self) -> float:
        """Condition number of G (1 for an empty history): the factor by which rounding in
        the Gram row and the right-hand side grows in the solve with G, so two correct FP64
        implementations agree on the guess only to about u times this."""
        return float(np.linalg.cond(self.G)) if self.d else 1.0

    # ------------------------------------------------------------ guess
    def form(self, b) -> np.ndarray:
        """x0 = W y with G y = W^T b, or 0 for an empty history."""
        b = np.asarray(b, dtype=np.float64)
        if self.d == 0:
            return np.zeros_like(b)
        c = np.array([float(w @ b) for w in self.W])
        y = np.linalg.solve(self.G, c)
        x0 = y[0] * self.W[0]
        for yj, w in zip(y[1:], self.W[1:]):
            x0 = x0 + yj * w
        return x0

    # ------------------------------------------------------------ update
    def _outside_norm2(self, s0: float, g) -> float:
        """nu^2 = s0 - g^T G^{-1} g: the squared A-norm of the new vector's part outside the
        stored span (Schur complement of the extended Gram matrix)."""
        return s0 - float(g @ np.linalg.solve(self.G, g))

    def update(self, x, Ax=None, decide=None) -> bool:
        """Store the rounded solution and extend G, or reject it.  A is applied to the stored
        vector (a given A x would belong to the unrounded one and is not used).  ``decide``
        replaces the rejection test by a given decision (a replay forces the other side's
        decision where nu / nu0 sits within rounding of eps_rel)."""
        x = np.asarray(x, dtype=np.float64)
        if self.variant == "classic" and self.d >= self.M:
            self.reset()
        elif self.variant == "qr" and self.d == self.M:
            self.W, self.exps = self.W[1:], self.exps[1:]
            self.G = self.G[1:, 1:].copy()
            self.drops += 1
        e = f16_scale_exp(float(np.max(np.abs(x)))) if self.dtype == "f16" and x.size else 0
        w = round_store(x, self.dtype, e)
        Aw = self.apply_A(w)
        s0 = float(w @ Aw)
        nu0 = float(np.sqrt(s0)) if s0 >= 0 else float("nan")
        if self.d == 0:
            g = np.zeros(0)
            nu = nu0
            ok = bool(np.isfinite(nu0) and nu0 > 0.0)
        else:
            g = np.array([float(wi @ Aw) for wi in self.W])
            s = self._outside_norm2(s0, g)
            nu = float(np.sqrt(s)) if s >= 0 else float("nan")
            fin = bool(np.isfinite(nu))
            ok = fin and (nu > self.eps_rel * nu0 if decide is None else bool(decide))
        self.last_nu0, self.last_nu, self.last_accepted = nu0, nu, ok
        if ok:
            d = self.d
            G = np.zeros((d + 1, d + 1))
            G[:d, :d] = self.G
            G[:d, d] = g
            G[d, :d] = g
            G[d, d] = s0
            self.G = G
            self.W.append(w)
            self.exps.append(e)
        return ok
