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
from proj_replay import check_rows
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


def test_workload_generators_across_streams(lib):
    """One host thread alternating streams (and, for the plane waves, mode sets): every right-hand
    side equals the one made alone on a single stream (the per-thread tables are rewritten only
    after the previous call's kernels are done)."""
    import torch

    announce("workload generators across streams")
    L = lib
    n = 96
    N = n ** 3
    gp = synth.gaussian_source_params(4)
    pw = [synth.plane_wave_params(s, 16) for s in (1, 2)]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]

    def gauss(t, out, st):
        L.workload_gaussian_rhs(n, synth.gaussian_center(gp, t), gp["sigma"], gp["amp"], out, L.stream_handle(st))

    def plane(q, t, out, st):
        p = pw[q]
        L.workload_plane_wave_rhs(n, [int(v) for v in p["k"].reshape(-1)], p["theta"],
                                  np.sin(p["w"] * t + p["phi"]), out, L.stream_handle(st))

    ts = [0.1 * (i + 1) for i in range(6)]
    ref_g, ref_p = [], []
    for i, t in enumerate(ts):
        out = torch.empty(N, dtype=torch.float64, device="cuda")
        gauss(t, out, None)
        torch.cuda.synchronize()
        ref_g.append(host(out))
        out = torch.empty(N, dtype=torch.float64, device="cuda")
        plane(i % 2, t, out, None)
        torch.cuda.synchronize()
        ref_p.append(host(out))
    outs_g = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in ts]
    outs_p = [torch.empty(N, dtype=torch.float64, device="cuda") for _ in ts]
    torch.cuda.synchronize()
    for i, t in enumerate(ts):
        gauss(t, outs_g[i], streams[i % 2])
        plane(i % 2, t, outs_p[i], streams[(i + 1) % 2])
    torch.cuda.synchronize()
    for i in range(len(ts)):
        assert np.array_equal(host(outs_g[i]), ref_g[i]), i
        assert np.array_equal(host(outs_p[i]), ref_p[i]), i


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
    assert check_rows(rows, label=f"{method} gaussian") == len(rows)
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
