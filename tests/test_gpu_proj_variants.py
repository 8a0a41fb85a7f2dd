"""GPU parity of the rolling-QR projection (§2, Algorithm 2) and of the
paper's l2 inner product, against the oracle.

Same replay protocol and tolerances as the classic A-orthonormal path
(tests/proj_replay.py): both sides receive the same (b_n, x_n) pairs; guesses
agree to relative 1e-12 (random histories, amplification ~ 1) or 1e-14 times
the amplification max nu0/nu of the accepted columns (smooth histories), at
every step.  The triangular factor R (raw solutions = X R) is compared entry
by entry relative to its largest entry, and the GPU's own history is checked
against the invariants (orthonormality in the variant's inner product,
B = A X, raw window = X R).
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rel_inf
from oracle import operator as op
from oracle.projection import Projection
from proj_replay import check_rows
from proj_replay import replay as replay_rows

pytestmark = pytest.mark.gpu

VARIANTS = ["projqr", "proj_l2", "projqr_l2"]


def replay(L, n, M, B, X, method, eps=1e-6, use_ax=False, dtype="f64", factors=False):
    import torch

    N = n ** 3
    meth, inner = L.parse_method(method)
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, meth, 0, L.DTYPES[dtype], eps, A, None, inner)
    Aop = op.Operator(n)
    ref = Projection(M, Aop, eps, dtype, "qr" if method.startswith("projqr") else "classic",
                     "l2" if inner == L.INNER_L2 else "A")
    try:
        rows, ref = replay_rows(L, g, ref, B, X, eps, Aop, use_ax, factors=factors)
        hist = []
        for j in range(L.guess_get_info(g)["count"]):
            xj = torch.empty(N, dtype=torch.float64, device="cuda")
            bj = torch.empty(N, dtype=torch.float64, device="cuda")
            L.guess_history_get(g, 0, j, xj)
            L.guess_history_get(g, 1, j, bj)
            hist.append((host(xj), host(bj)))
        R = L.guess_proj_factor(g)
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
    return rows, hist, ref, R


@pytest.mark.parametrize("method", VARIANTS)
@pytest.mark.parametrize("n,M", [(1, 2), (3, 4), (5, 1), (5, 2), (8, 8), (11, 16)])
def test_random_sequence_parity(lib, method, n, M):
    """Random solutions: strict parity through restarts / drops, factor parity."""
    announce(f"{method} random n={n} M={M}")
    N = n ** 3
    T = 2 * M + 3
    X = synth.random_vectors(70 + n, T, N)
    B = synth.random_vectors(80 + n, T, N)
    rows, hist, ref, R = replay(lib, n, M, B, X, method, factors=True)
    assert check_rows(rows, strict=(N > 2 * M), label=f"{method} random n={n} M={M}") == T
    if N > M:                       # random vectors in dimension > M are independent
        ds = [r["d"] for r in rows]
        if method.startswith("projqr"):
            assert ds == [min(q + 1, M) for q in range(T)]
            assert rows[-1]["info"]["drops"] == T - M
            assert rows[-1]["info"]["restarts"] == 1
        for r in rows:
            Rg, Rr = r["R"], r["R_ref"]
            assert Rg.shape == Rr.shape
            assert np.max(np.abs(Rg - Rr)) <= 1e-12 * np.max(np.abs(Rr))


@pytest.mark.parametrize("method", VARIANTS)
def test_history_invariants_after_drops(lib, method):
    """Orthonormality, B = A X and raw window = X R for the GPU's stored history."""
    announce(f"{method} invariants")
    n, M, T = 8, 6, 15
    N = n ** 3
    X = synth.random_vectors(15, T, N)
    rows, hist, ref, R = replay(lib, n, M, synth.random_vectors(16, T, N), X, method)
    Aop = op.Operator(n)
    Xs = np.stack([h[0] for h in hist])
    Bs = np.stack([h[1] for h in hist])
    d = Xs.shape[0]
    assert d == (M if method.startswith("projqr") else (T - 1) % M + 1)
    G = Xs @ Bs.T if not method.endswith("_l2") else Bs @ Bs.T
    np.testing.assert_allclose(G, np.eye(d), rtol=0, atol=1e-12)
    for x, b in zip(Xs, Bs):
        assert rel_inf(Aop(x), b) <= 1e-12
    raw = np.stack(ref.raw)
    assert np.max(np.abs(R.T @ Xs - raw)) <= 1e-12 * np.max(np.abs(raw))


@pytest.mark.parametrize("method", ["projqr", "projqr_l2"])
@pytest.mark.parametrize("use_ax", [False, True])
def test_plane_wave_replay_32(lib, method, use_ax):
    """32^3, K = 4 plane waves, dt = 0.01, 50 steps, M = 8, exact solutions: the rolling window
    slides through 42 drops with rejections of nearly dependent solutions."""
    announce(f"{method} replay 32^3 use_ax={use_ax}")
    n, M, T = 32, 8, 50
    params = synth.plane_wave_params(0, 4)
    B = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(T, 0.01)]
    X = [op.dst_solve(b, n) for b in B]
    rows, _, _, _ = replay(lib, n, M, B, X, method, use_ax=use_ax)
    assert check_rows(rows, label=f"{method} 32^3 use_ax={use_ax}") == T


def test_plane_wave_replay_16_modes_qr(lib):
    """K = 16 modes (more modes than M): the window drops every step once full."""
    announce("projqr replay K=16")
    n, M, T = 24, 8, 40
    params = synth.plane_wave_params(1, 16)
    B = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(T, 0.05)]
    X = [op.dst_solve(b, n) for b in B]
    rows, _, ref, _ = replay(lib, n, M, B, X, "projqr")
    assert check_rows(rows, label="projqr K=16") == T
    assert ref.drops > 0


def test_rejection_drop_and_reset_qr(lib):
    import torch

    announce("projqr rejection / reset")
    L = lib
    n = 4
    N = n ** 3
    A = L.guess_op_create(n, n, n, 25.0, 10.0, None)
    g = L.guess_create_ex(N, 3, L.PROJ_QR, 0, L.F64, 1e-6, A)
    try:
        v = synth.random_vectors(2, 5, N)
        for q in range(3):
            L.guess_update(g, dev(v[q]))
        assert L.guess_get_info(g)["count"] == 3
        L.guess_update(g, dev(v[1] + v[2]))             # full: drop, then in the window's span
        i = L.guess_get_info(g)
        assert i["count"] == 2 and i["last_accepted"] == 0 and i["rejects"] == 1 and i["drops"] == 1
        L.guess_update(g, dev(v[3]))
        i = L.guess_get_info(g)
        assert i["count"] == 3 and i["drops"] == 1
        R = L.guess_proj_factor(g)
        assert R.shape == (3, 3) and np.all(np.tril(R, -1) == 0)
        L.guess_reset(g)
        assert L.guess_get_info(g)["count"] == 0
        x0 = torch.full((N,), 5.0, dtype=torch.float64, device="cuda")
        L.guess_form(g, dev(v[4]), x0)
        assert not host(x0).any()
        L.guess_update(g, dev(v[4]))
        assert L.guess_get_info(g)["count"] == 1
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
