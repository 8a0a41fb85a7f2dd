"""The non-separable workload: a Gaussian source moving through the unit cube, whose
solutions do not lie in a fixed low-dimensional space (unlike the plane-wave sequence).

The library's RHS kernel is compared with the input generator (exp evaluated on both
sides, so within a few ulps), and guess sequences on exact (DST) solutions are replayed
through the GPU and the oracle with the projection parity tolerance.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host
from oracle import extrap
from oracle import operator as op
from test_gpu_proj import check_rows
from test_gpu_proj_variants import replay

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 7, 33, 64])
def test_gaussian_rhs_kernel(lib, n):
    import torch

    announce(f"gaussian rhs n={n}")
    params = synth.gaussian_source_params(3)
    b = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    for t in (0.0, 0.37, 1.9):
        lib.workload_gaussian_rhs(n, synth.gaussian_center(params, t), params["sigma"], params["amp"], b,
                                  lib.stream_handle())
        want = synth.gaussian_source_rhs(params, n, t)
        got = host(b)
        assert np.max(np.abs(got - want)) <= 1e-14 * max(np.max(np.abs(want)), 1e-300)
    with pytest.raises(lib.GuessError):
        lib.workload_gaussian_rhs(n, [0.5, 0.5, 0.5], 0.0, 1.0, b, lib.stream_handle())


def _sequence(n, T, dt, seed=1):
    params = synth.gaussian_source_params(seed)
    B = [synth.gaussian_source_rhs(params, n, t) for t in synth.step_times(T, dt)]
    X = [op.dst_solve(b, n) for b in B]
    return B, X


@pytest.mark.parametrize("method", ["proj", "projqr", "proj_l2", "projqr_l2"])
def test_projection_replay_moving_source(lib, method):
    announce(f"{method} moving source 24^3")
    n, M, T = 24, 8, 30
    B, X = _sequence(n, T, 0.02)
    rows, _, ref, _ = replay(lib, n, M, B, X, method)
    assert check_rows(rows, 1e-6) >= 20
    if method.startswith("projqr"):
        assert ref.drops > 0           # the window really slides on this workload


@pytest.mark.parametrize("sparse", [False, True])
def test_extrapolation_replay_moving_source(lib, sparse):
    import torch

    announce(f"{'spextrap' if sparse else 'extrap'} moving source 24^3")
    L = lib
    n, M, m, T = 24, 8, 3, 14
    N = n ** 3
    B, X = _sequence(n, T, 0.02, seed=2)
    g = L.guess_create_ex(N, M, L.SPEXTRAP if sparse else L.EXTRAP, m, L.F64)
    ref = extrap.ExtrapHistory(M, m, sparse=sparse)
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    try:
        for q, x in enumerate(X):
            L.guess_form(g, None, x0)
            want = ref.form(N=N)
            got = host(x0)
            if q > 0:
                assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want)), q
            L.guess_update(g, dev(x))
            ref.update(x)
    finally:
        L.guess_destroy(g)
