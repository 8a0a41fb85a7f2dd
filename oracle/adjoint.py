"""Reference gradient of the differentiation workload (oracle; test infrastructure only).

Workload: x_n solves A x_n = b_n(c) with b_n(c) = sum_k c_k s_{k,n} f_k,
s_{k,n} = sin(w_k t_n + phi_k), and L(c) = sum_n ||x_n - y_n||^2.  A is
symmetric, so with lambda_n = A^{-1} 2 (x_n - y_n) the gradient is
dL/dc_k = sum_n s_{k,n} <f_k, lambda_n>.  Solves here are exact (DST-I), so
the result is the FP64 reference.  L is exactly quadratic in c, which makes a
central finite difference exact up to rounding (used as the pin).

The paper does not differentiate through its solver; this workload and its
reading are this library's extension.  The pin is the central finite
difference, exact for this quadratic loss up to rounding.
"""
from __future__ import annotations

import numpy as np

from .operator import dst_solve


def loss_and_grad(F, S, Y, n, c, shift=10.0):
    """F: K x N modes; S: T x K amplitudes s_{k,n}; Y: T x N targets; c: K."""
    c = np.asarray(c, dtype=np.float64)
    L = 0.0
    g = np.zeros_like(c)
    for t in range(S.shape[0]):
        b = (S[t] * c) @ F
        x = dst_solve(b, n, shift)
        e = x - Y[t]
        L += float(e @ e)
        lam = dst_solve(2.0 * e, n, shift)
        g += S[t] * (F @ lam)
    return L, g


def loss(F, S, Y, n, c, shift=10.0):
    return loss_and_grad(F, S, Y, n, c, shift)[0]
