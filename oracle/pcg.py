"""Jacobi-preconditioned conjugate gradients (oracle; test infrastructure only).

The paper solves every system with PCG, point-Jacobi preconditioned for the
velocity systems (§5.3).  This is the textbook preconditioned CG recurrence.

Stopping rule (reading): the recurrence residual r_k satisfies
||r_k||_2 <= rtol ||b||_2 (the right-hand-side criterion of §6.4 without the
max(., 1) floor); it is tested before the first iteration, so an exact guess
costs zero iterations.  ``rule="initresid"`` selects the paper's default
||r_k||_2 < rtol max(||r_0||_2, 1) instead (§6.4).  The iteration count is
the number of operator applications inside the loop.

The preconditioner multiplies by the reciprocal diagonal, dinv = 1 / diag(A).
"""
from __future__ import annotations

import numpy as np

OK, NOTCONV, BREAKDOWN = 0, -4, -5


def pcg(apply_A, b, x0, dinv, rtol=1e-8, maxit=10000, rule="rhs"):
    """Solve A x = b from x0.  Returns (x, iterations, status, relres_recurrence)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_A(x)
    bnorm = float(np.sqrt(b @ b))
    rnorm = float(np.sqrt(r @ r))
    if rule == "rhs":
        thresh = rtol * bnorm
        stop = lambda rn: rn <= thresh          # noqa: E731
    elif rule == "initresid":
        thresh = rtol * max(rnorm, 1.0)
        stop = lambda rn: rn < thresh           # noqa: E731
    else:
        raise ValueError(rule)
    scale = bnorm if bnorm > 0 else 1.0
    if stop(rnorm):
        return x, 0, OK, rnorm / scale
    z = dinv * r
    p = z.copy()
    rho = float(r @ z)
    for it in range(1, maxit + 1):
        q = apply_A(p)
        pq = float(p @ q)
        if not (pq > 0.0) or not np.isfinite(pq):
            return x, it, BREAKDOWN, rnorm / scale
        alpha = rho / pq
        x = x + alpha * p
        r = r - alpha * q
        rnorm = float(np.sqrt(r @ r))
        if stop(rnorm):
            return x, it, OK, rnorm / scale
        z = dinv * r
        rho_new = float(r @ z)
        beta = rho_new / rho
        rho = rho_new
        p = z + beta * p
    return x, maxit, NOTCONV, rnorm / scale
