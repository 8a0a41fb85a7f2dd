"""Time-step driver: guess -> PCG -> history update (oracle; test infrastructure only).

For each right-hand side b_n of a sequence the initial guess is formed from
the history, the system is solved by PCG from that guess, and the solution is
added to the history (the loop of §2, Algorithm 1, and §3, used at every time
step as in §6.2-§6.3).
"""
from __future__ import annotations

import numpy as np

from .extrap import ExtrapHistory
from .operator import Operator
from .pcg import pcg
from .projection import AOrthoProjection, Projection


class ZeroGuess:
    def form(self, b, N=None):
        return np.zeros(len(b), dtype=np.float64)

    def update(self, x, Ax=None):
        return None


class LastGuess:
    """Previous solution as the guess (EXTRAP with M = 1)."""

    def __init__(self, dtype="f64"):
        self.h = ExtrapHistory(1, 0, dtype)

    def form(self, b, N=None):
        return self.h.form(b, N=len(b))

    def update(self, x, Ax=None):
        self.h.update(x)


class ExtrapGuess:
    def __init__(self, M, m, dtype="f64", sparse=False):
        self.h = ExtrapHistory(M, m, dtype, sparse)

    def form(self, b, N=None):
        return self.h.form(b, N=len(b))

    def update(self, x, Ax=None):
        self.h.update(x)


def make_guess(method: str, M: int, degree: int, op, eps_rel=1e-6, dtype="f64"):
    if method == "zero":
        return ZeroGuess()
    if method == "last":
        return LastGuess(dtype)
    if method == "extrap":
        return ExtrapGuess(M, degree, dtype)
    if method == "spextrap":
        return ExtrapGuess(M, degree, dtype, sparse=True)
    if method == "proj":
        return AOrthoProjection(M, op, eps_rel, dtype)
    if method in ("projqr", "proj_l2", "projqr_l2"):
        variant = "qr" if method.startswith("projqr") else "classic"
        return Projection(M, op, eps_rel, dtype, variant, "l2" if method.endswith("_l2") else "A")
    raise ValueError(method)


def run_sequence(op: Operator, rhs_seq, method: str, M: int = 8, degree: int = 2,
                 rtol: float = 1e-8, maxit: int = 10000, eps_rel: float = 1e-6,
                 dtype: str = "f64", keep=False):
    """Solve A x_n = b_n for every b_n in order.  Returns a dict of per-step data."""
    g = make_guess(method, M, degree, op, eps_rel, dtype)
    dinv = 1.0 / op.diag()
    iters, relres, guesses, sols, r0 = [], [], [], [], []
    for b in rhs_seq:
        x0 = g.form(b)
        bn = float(np.linalg.norm(b))
        r0.append(float(np.linalg.norm(b - op(x0))) / (bn if bn > 0 else 1.0))
        x, it, st, rr = pcg(op, b, x0, dinv, rtol, maxit)
        if st != 0:
            raise RuntimeError(f"oracle PCG failed with status {st}")
        g.update(x)
        iters.append(it)
        relres.append(rr)
        if keep:
            guesses.append(x0)
            sols.append(x)
    return {"iters": iters, "relres": relres, "r0": r0, "guesses": guesses, "solutions": sols}


def replay_guesses(method: str, M: int, degree: int, op, rhs_seq, sol_seq,
                   eps_rel=1e-6, dtype="f64"):
    """Guesses x0_n for given (b_n, x_n) pairs, without solving.

    Used to compare implementations on identical inputs: the history is fed
    the given solutions rather than each implementation's own PCG output.
    """
    g = make_guess(method, M, degree, op, eps_rel, dtype)
    out, accepted = [], []
    for b, x in zip(rhs_seq, sol_seq):
        out.append(g.form(b))
        r = g.update(x)
        accepted.append(r)
    return out, accepted
