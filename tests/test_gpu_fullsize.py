"""Parity at the benchmark's full size (256^3 = 16,777,216 unknowns, M = 8).

Same library launch configuration as bench.py.  The extrapolated guess is
checked at sampled unknowns (the oracle evaluates sum_j beta_j h_j one
unknown at a time); the projection guess is checked against the full FP64
oracle on random (well-conditioned) histories.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, assert_within, dev, host, rel_inf
from oracle import extrap, lowprec
from oracle import operator as op
from oracle.projection import AOrthoProjection

pytestmark = pytest.mark.gpu

n = 256
N = n ** 3


def sample_idx():
    idx = np.random.default_rng(11).integers(0, N, 8192)
    return np.unique(np.concatenate([idx, [0, 1, 2, 3, N - 4, N - 3, N - 2, N - 1, n * n, n * n - 1]]))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_extrap_256_sampled(lib, dtype):
    import torch

    announce(f"extrap 256^3 M=8 m=2 {dtype}")
    L = lib
    M, m = 8, 2
    idx = sample_idx()
    g = L.guess_create_ex(N, M, L.EXTRAP, m, L.DTYPES[dtype])
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    hist = []
    try:
        rng = np.random.default_rng(5)
        for s in range(M + 1):
            v = rng.standard_normal(N) * (1.0 + 0.1 * s)
            L.guess_update(g, dev(v))
            hist.append(lowprec.round_store(v[idx], dtype))
            hist = hist[-M:]
        L.guess_form(g, None, x0)
        got = host(x0)[idx]
    finally:
        L.guess_destroy(g)
    beta = extrap.to_f64(extrap.beta_ls_exact(m, M))
    want = extrap.form(hist, beta)
    if dtype == "f64":
        assert rel_inf(got, want) <= 1e-12
    else:
        mag = sum(abs(b) * np.abs(h) for b, h in zip(beta, hist))
        assert_within(got, want, (M + 1) * 2.0 ** -24 * mag + 2.0 ** -24 * np.abs(want), hist, dtype)


def test_proj_256_full(lib):
    import torch

    announce("proj 256^3 M=4 random replay")
    L = lib
    M, T = 4, 6
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, L.PROJ, 0, L.F64, 1e-6, A)
    Aop = op.Operator(n)
    ref = AOrthoProjection(M, Aop, 1e-6)
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    idx = sample_idx()
    rng = np.random.default_rng(8)
    try:
        for s in range(T):
            b = rng.standard_normal(N)
            x = rng.standard_normal(N)
            L.guess_form(g, dev(b), x0)
            want = ref.form(b)
            got = host(x0)
            if s == 0:
                assert not got.any()
            else:
                assert rel_inf(got, want) <= 1e-12, s
                assert rel_inf(got[idx], want[idx]) <= 1e-12
            L.guess_update(g, dev(x))
            ref.update(x)
            info = L.guess_get_info(g)
            assert info["count"] == ref.d and info["last_accepted"] == 1
            assert abs(info["nu0"] - ref.last_nu0) <= 1e-12 * ref.last_nu0
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
