"""Differentiable sequence of solves with initial guesses in both time directions.

Workload: right-hand sides b_n(c) = sum_k c_k s_{k,n} f_k (modes f_k, amplitudes
s_{k,n}), solutions x_n = A^{-1} b_n for n = 1..T, each solve started from the
library's initial guess.  ``GuessSolveFn.apply(c, seq)`` returns the stacked
solutions X (T x N).  Because A is symmetric, the adjoint of the sequence is a
second sequence of solves run backwards in time: lambda_n = A^{-1} g_n with
g_n = dL/dx_n, and dL/dc_k = sum_n s_{k,n} <f_k, lambda_n>.  The backward pass
uses its own guess history (extrapolation with uniform weights also works in
reverse time, the nodes being equispaced either way).

All vector work runs in libguess kernels: b_n is a vec_combine of the device
mode matrix, the gradient terms are vec_multidot calls, solves are pcg_solve,
guesses are guess_form / guess_update.  Torch holds the device memory.
"""
from __future__ import annotations

import torch

from . import libguess as L
from .sequence import GuessSequence, Operator


class SolveSequence:
    """Fixed data of a differentiable sequence: operator, modes, amplitudes, guess settings."""

    def __init__(self, op: Operator, modes: torch.Tensor, amps, method: str = "extrap", M: int = 8,
                 degree: int = 2, dtype: str = "f64", rtol: float = 1e-8, maxit: int = 20000):
        if modes.dim() != 2 or modes.shape[1] != op.N or not modes.is_cuda:
            raise ValueError("modes must be a device tensor of shape (K, N)")
        self.op = op
        self.F = modes.contiguous()
        self.K = modes.shape[0]
        self.S = torch.as_tensor(amps, dtype=torch.float64, device="cpu")   # (T, K)
        if self.S.dim() != 2 or self.S.shape[1] != self.K:
            raise ValueError("amps must have shape (T, K)")
        self.T = self.S.shape[0]
        self.method, self.M, self.degree, self.dtype = method, M, degree, dtype
        self.rtol, self.maxit = rtol, maxit
        self.stats = {"forward_iters": [], "adjoint_iters": []}

    def _solve_all(self, rhs_of, order, store):
        """Solve A y_n = rhs_of(n) for n in `order` with a fresh guess history."""
        N = self.op.N
        g = GuessSequence(N, self.M, self.method, self.degree, self.dtype, op=self.op)
        b = torch.empty(N, dtype=torch.float64, device="cuda")
        iters = []
        try:
            for n in order:
                rhs_of(n, b)
                y = store(n)
                g.form(b, y)
                st, it, _ = self.op.solve(b, y, self.rtol, self.maxit)
                if st != L.OK:
                    raise RuntimeError(f"PCG failed at step {n} (status {st})")
                g.update(y)
                iters.append(it)
        finally:
            g.close()
        return iters


class GuessSolveFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c: torch.Tensor, seq: SolveSequence):
        c64 = c.detach().to("cpu", torch.float64)
        N, T = seq.op.N, seq.T
        # rows padded to an even length so that every row is 16-byte aligned
        Npad = N + (N & 1)
        X = torch.empty((T, Npad), dtype=torch.float64, device="cuda")[:, :N]

        def rhs(n, b):
            L.vec_combine(N, seq.K, seq.F, (seq.S[n] * c64).tolist(), b, L.stream_handle())

        seq.stats["forward_iters"] = seq._solve_all(rhs, range(T), lambda n: X[n])
        ctx.seq = seq
        ctx.c_device, ctx.c_dtype = c.device, c.dtype
        return X

    @staticmethod
    def backward(ctx, gX: torch.Tensor):
        seq = ctx.seq
        N, T = seq.op.N, seq.T
        lam = torch.empty(N, dtype=torch.float64, device="cuda")
        grad = torch.zeros(seq.K, dtype=torch.float64)

        def rhs(n, b):
            b.copy_(gX[n])

        # reverse-time adjoint solves; the gradient term of each step is taken
        # right after its solve, before lam is reused
        g = GuessSequence(N, seq.M, seq.method, seq.degree, seq.dtype, op=seq.op)
        b = torch.empty(N, dtype=torch.float64, device="cuda")
        iters = []
        try:
            for n in range(T - 1, -1, -1):
                rhs(n, b)
                g.form(b, lam)
                st, it, _ = seq.op.solve(b, lam, seq.rtol, seq.maxit)
                if st != L.OK:
                    raise RuntimeError(f"adjoint PCG failed at step {n} (status {st})")
                g.update(lam)
                iters.append(it)
                d = L.vec_multidot(N, seq.K, seq.F, lam, L.stream_handle())
                grad += seq.S[n] * torch.tensor(d, dtype=torch.float64)
        finally:
            g.close()
        seq.stats["adjoint_iters"] = iters[::-1]
        return grad.to(ctx.c_device, ctx.c_dtype), None


def plane_wave_modes(params: dict, n: int) -> torch.Tensor:
    """Device mode matrix (K x n^3) evaluated by the library's RHS kernel (one mode at a time)."""
    K = params["K"]
    F = torch.empty((K, n ** 3), dtype=torch.float64, device="cuda")
    kvec = [int(v) for v in params["k"].reshape(-1)]
    theta = [float(v) for v in params["theta"]]
    for q in range(K):
        amp = [1.0 if j == q else 0.0 for j in range(K)]
        L.workload_plane_wave_rhs(n, kvec, theta, amp, F[q], L.stream_handle())
    return F
