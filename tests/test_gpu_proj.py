"""GPU parity of the A-orthonormal projection path against the oracle.

Replay protocol (tests/proj_replay.py): both sides receive the same (b_n, x_n)
pairs, so the guesses can be compared at every step.  Tolerance: relative
1e-12, widened to 1e-14 * a where a = max nu0/nu over the stored columns (the
factor by which the Gram-Schmidt normalisation of a nearly dependent column
amplifies rounding; two correct FP64 implementations that sum in different
orders agree only to about u * a).  Random histories have a ~ 1 and are held
to 1e-12 exactly.  Accept / reject decisions must agree at every step; where
the oracle's ratio nu/nu0 lies within a relative 1e-6 of eps_rel (a decision
rounding can flip) the oracle takes the library's decision, and every step of
every sequence is compared.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rel_inf
from oracle import operator as op
from oracle.projection import AOrthoProjection
from proj_replay import check_rows
from proj_replay import replay as replay_rows

pytestmark = pytest.mark.gpu


def replay(L, n, M, B, X, eps=1e-6, use_ax=False, dtype="f64"):
    import torch

    N = n ** 3
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, L.PROJ, 0, L.DTYPES[dtype], eps, A)
    Aop = op.Operator(n)
    ref = AOrthoProjection(M, Aop, eps, dtype)
    try:
        rows, ref = replay_rows(L, g, ref, B, X, eps, Aop, use_ax)
        hist = []
        for j in range(L.guess_get_info(g)["count"]):
            xj = torch.empty(N, dtype=torch.float64, device="cuda")
            bj = torch.empty(N, dtype=torch.float64, device="cuda")
            L.guess_history_get(g, 0, j, xj)
            L.guess_history_get(g, 1, j, bj)
            hist.append((host(xj), host(bj)))
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
    return rows, hist, ref


@pytest.mark.parametrize("n,M", [(1, 2), (3, 4), (5, 1), (8, 8), (11, 16)])
def test_random_sequence_parity(lib, n, M):
    """Random solutions (well-conditioned history): strict parity incl. restarts."""
    announce(f"proj random n={n} M={M}")
    N = n ** 3
    T = 2 * M + 3
    X = synth.random_vectors(50 + n, T, N)
    B = synth.random_vectors(60 + n, T, N)
    rows, hist, ref = replay(lib, n, M, B, X)
    assert check_rows(rows, strict=(N > 2 * M), label=f"proj random n={n} M={M}") == T
    ds = [r["d"] for r in rows]
    expected, d = [], 0
    for _ in range(T):
        d = 1 if (d == 0 or d >= M) else d + 1
        expected.append(d)
    if N >= M:   # random vectors in dimension >= M are independent
        assert ds == expected


def test_history_invariants(lib):
    """X^T A X = I and B = A X for the GPU's stored history."""
    announce("proj invariants")
    n, M = 8, 8
    N = n ** 3
    X = synth.random_vectors(5, 7, N)
    rows, hist, _ = replay(lib, n, M, synth.random_vectors(6, 7, N), X)
    Aop = op.Operator(n)
    Xs = np.stack([h[0] for h in hist])
    Bs = np.stack([h[1] for h in hist])
    assert Xs.shape[0] == 7
    np.testing.assert_allclose(Xs @ Bs.T, np.eye(7), rtol=0, atol=1e-12)
    for x, b in zip(Xs, Bs):
        assert rel_inf(Aop(x), b) <= 1e-12


@pytest.mark.parametrize("use_ax", [False, True])
def test_plane_wave_replay_32(lib, use_ax):
    """C1 workload: 32^3, K = 4 plane waves, dt = 0.01, 50 steps, M = 8, exact solutions."""
    announce(f"proj replay 32^3 use_ax={use_ax}")
    n, M, T = 32, 8, 50
    params = synth.plane_wave_params(0, 4)
    B = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(T, 0.01)]
    X = [op.dst_solve(b, n) for b in B]
    rows, _, _ = replay(lib, n, M, B, X, use_ax=use_ax)
    assert check_rows(rows, label=f"proj 32^3 use_ax={use_ax}") == T


def test_plane_wave_replay_16_modes(lib):
    """K = 16 modes (more modes than M): restarts happen and guesses match."""
    announce("proj replay K=16")
    n, M, T = 24, 8, 40
    params = synth.plane_wave_params(1, 16)
    B = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(T, 0.05)]
    X = [op.dst_solve(b, n) for b in B]
    rows, _, _ = replay(lib, n, M, B, X)
    assert check_rows(rows, label="proj K=16") == T


def test_rejection_and_nonfinite(lib):
    import torch

    announce("proj rejection / non-finite")
    L = lib
    n = 4
    N = n ** 3
    A = L.guess_op_create(n, n, n, 25.0, 10.0, None)
    g = L.guess_create_ex(N, 4, L.PROJ, 0, L.F64, 1e-6, A)
    try:
        v = synth.random_vectors(1, 2, N)
        L.guess_update(g, dev(v[0]))
        L.guess_update(g, dev(2.0 * v[0]))          # dependent: rejected
        i = L.guess_get_info(g)
        assert i["count"] == 1 and i["last_accepted"] == 0 and i["rejects"] == 1
        bad = v[1].copy()
        bad[3] = np.nan
        L.guess_update(g, dev(bad))
        i = L.guess_get_info(g)
        assert i["count"] == 1 and i["nonfinite"] == 1 and i["last_accepted"] == 0
        L.guess_update(g, dev(v[1]))
        assert L.guess_get_info(g)["count"] == 2
        L.guess_reset(g)
        assert L.guess_get_info(g)["count"] == 0
        x0 = torch.full((N,), 5.0, dtype=torch.float64, device="cuda")
        L.guess_form(g, dev(v[1]), x0)
        assert not host(x0).any()
        L.guess_update(g, dev(np.zeros(N)))          # zero solution: nothing stored
        assert L.guess_get_info(g)["count"] == 0
        with pytest.raises(L.GuessError):
            L.guess_form(g, None, x0)                # projection needs b
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)


def test_update_without_operator_needs_ax(lib):
    announce("proj without operator")
    L = lib
    N = 100
    g = L.guess_create_ex(N, 4, L.PROJ, 0, L.F64, 1e-6, None)
    try:
        x = dev(np.ones(N))
        with pytest.raises(L.GuessError):
            L.guess_update(g, x)
        L.guess_update(g, x, dev(2.0 * np.ones(N)))     # B = A X given by the caller
        assert L.guess_get_info(g)["count"] == 1
    finally:
        L.guess_destroy(g)


def test_default_threshold_follows_storage_format(lib):
    """eps_rel <= 0 selects the format's default (1e-6 F64, 1e-4 F32, 1e-2 F16 / BF16); a given
    value is kept."""
    L = lib
    A = L.guess_op_create(8, 8, 8, 81.0, 10.0, None)
    try:
        for dt, want in (("f64", 1e-6), ("f32", 1e-4), ("f16", 1e-2), ("bf16", 1e-2)):
            for meth in (L.PROJ, L.PROJ_QR):
                g = L.guess_create_ex(512, 4, meth, 0, L.DTYPES[dt], 0.0, A)
                try:
                    assert L.guess_get_info(g)["eps_rel"] == want
                finally:
                    L.guess_destroy(g)
            g = L.guess_create_ex(512, 4, L.PROJ, 0, L.DTYPES[dt], 3e-5, A)
            try:
                assert L.guess_get_info(g)["eps_rel"] == 3e-5
            finally:
                L.guess_destroy(g)
    finally:
        L.guess_op_destroy(A)
