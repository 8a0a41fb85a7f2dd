"""GPU parity of the raw-solution projection (GUESS_PROJ_RAW, GUESS_PROJ_RAW_QR) against the oracle.

Both sides store the rounded raw solutions -- numbers of the input, rounded
once (FP16 after an exact power-of-two scaling) -- so the stored values must
agree bit for bit, with the same exponents.  Everything else is FP64: the
Gram matrix of the stored vectors, the Cholesky solve (library) or LU solve
(oracle), the Schur complement of the rejection test.  Guesses agree to
relative max(1e-12, 1e-14 cond(G)); decisions must agree except within a
relative 1e-6 of eps_rel, where the oracle takes the library's decision
(tests/proj_replay.py).  The library's factor R = L^T must satisfy
R^T R = G of the oracle's stored vectors.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host
from oracle import lowprec
from oracle import operator as op
from oracle.rawproj import RawProjection
from proj_replay import check_rows, replay

pytestmark = pytest.mark.gpu

METHODS = ["proj_raw", "projqr_raw"]


def run(L, n, M, B, X, method, dtype, eps=1e-6):
    import torch

    N = n ** 3
    meth, inner = L.parse_method(method)
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, meth, 0, L.DTYPES[dtype], eps, A)
    Aop = op.Operator(n)
    ref = RawProjection(M, Aop, eps, dtype, "qr" if method == "projqr_raw" else "classic")
    stored = []
    try:
        rows, ref = replay(L, g, ref, B, X, eps, Aop, factors=True)
        buf = torch.empty(N, dtype=torch.float64, device="cuda")
        for j in range(L.guess_get_info(g)["count"]):
            sc = L.guess_history_raw(g, 0, j, buf)
            stored.append((host(buf).copy(), sc))
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
    return rows, ref, stored


def check_stored(ref, stored, dtype, label):
    assert len(stored) == ref.d, label
    for j, ((got, sc), w, e) in enumerate(zip(stored, ref.W, ref.exps)):
        assert sc == 2.0 ** -e, (label, j, sc, e)
        want = np.ldexp(w, e)                    # the stored values themselves
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (label, j)
        if dtype == "f16":
            assert np.max(np.abs(got)) <= 2 ** 15


def check_factors(rows, label):
    """R^T R of the library's factor equals the oracle's Gram matrix (both of the same
    stored vectors) to FP64 rounding."""
    for q, r in enumerate(rows):
        Rg, Rr = r["R"], r["R_ref"]
        if Rg.size == 0:
            continue
        G = Rr.T @ Rr
        assert Rg.shape == G.shape, (label, q)
        assert np.all(np.tril(Rg, -1) == 0)
        assert np.max(np.abs(Rg.T @ Rg - G)) <= 1e-12 * np.max(np.abs(G)), (label, q)


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("n", [7, 32])
def test_random_history(lib, method, dtype, n):
    """Random solutions of magnitudes 1e-2 .. 1e2 through restarts / drops (7^3: ragged tail
    and the chunk-form apply; 32^3: the z-marching apply)."""
    announce(f"{method} {dtype} random n={n}")
    M = 5
    N = n ** 3
    T = 2 * M + 2
    X = [v * 10.0 ** ((q % 5) - 2) for q, v in enumerate(synth.random_vectors(61, T, N))]
    B = synth.random_vectors(62, T, N)
    rows, ref, stored = run(lib, n, M, B, X, method, dtype)
    check_stored(ref, stored, dtype, f"{method} {dtype} n={n}")
    assert check_rows(rows, label=f"{method} {dtype} n={n}") == T
    check_factors(rows, f"{method} {dtype} n={n}")
    ds = [r["d"] for r in rows]
    if method == "projqr_raw":
        assert ds == [min(q + 1, M) for q in range(T)] and rows[-1]["info"]["drops"] == T - M
    else:
        assert ds == [(q % M) + 1 for q in range(T)]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("mag", [1e-6, 1e6])
def test_f16_far_outside_range(lib, method, mag):
    """FP16 solutions ~1e6 and ~1e-6: every stored solution carries its own exponent."""
    announce(f"{method} f16 magnitude {mag}")
    n, M = 9, 4
    T = 3 * M
    X = [v * mag * (1 + 0.3 * q) for q, v in enumerate(synth.random_vectors(63, T, n ** 3))]
    B = synth.random_vectors(64, T, n ** 3)
    rows, ref, stored = run(lib, n, M, B, X, method, "f16")
    check_stored(ref, stored, "f16", f"{method} f16 mag={mag}")
    assert check_rows(rows, label=f"{method} f16 mag={mag}") == T


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_plane_wave_history(lib, method, dtype):
    """Smooth plane-wave solutions (32^3, K = 16 modes, dt = 0.005, 30 steps): nearly dependent
    stored vectors, decisions near the threshold; stored values still bit for bit."""
    announce(f"{method} {dtype} plane waves")
    n, M, T = 32, 8, 30
    params = synth.plane_wave_params(1, 16)
    B = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(T, 0.005)]
    X = [op.dst_solve(b, n) for b in B]
    rows, ref, stored = run(lib, n, M, B, X, method, dtype)
    check_stored(ref, stored, dtype, f"{method} {dtype} plane waves")
    assert check_rows(rows, label=f"{method} {dtype} plane waves") == T


@pytest.mark.parametrize("method,dtype", [("projqr_raw", "f32"), ("proj_raw", "f16")])
def test_full_size_replay(lib, method, dtype):
    """The benchmark's size, 256^3, M = 8: ten random solutions (the rolling window drops its
    oldest twice, the classic one restarts once), every stored solution bit for bit, guesses to
    1e-12 and the factor against the oracle -- the z-marching apply (FP32) and the chunk-form
    apply (FP16) at the size the benchmark runs them."""
    announce(f"{method} {dtype} random 256^3")
    n, M, T = 256, 8, 10
    N = n ** 3
    X = [v * (1.0 + 0.5 * q) for q, v in enumerate(synth.random_vectors(65, T, N))]
    B = synth.random_vectors(66, T, N)
    rows, ref, stored = run(lib, n, M, B, X, method, dtype)
    check_stored(ref, stored, dtype, f"{method} {dtype} 256^3")
    assert check_rows(rows, strict=True, label=f"{method} {dtype} 256^3") == T
    check_factors(rows, f"{method} {dtype} 256^3")
    ds = [r["d"] for r in rows]
    if method == "projqr_raw":
        assert ds == [min(q + 1, M) for q in range(T)] and rows[-1]["info"]["drops"] == T - M
    else:
        assert ds == [(q % M) + 1 for q in range(T)]


def test_factor_is_the_cholesky_factor_of_the_gram_matrix(lib):
    announce("proj_raw factor")
    n, M, T = 8, 6, 9
    X = synth.random_vectors(65, T, n ** 3)
    rows, ref, stored = run(lib, n, M, synth.random_vectors(66, T, n ** 3), X, "projqr_raw", "f32")
    for q, r in enumerate(rows):
        Rg = r["R"]
        d = r["d"]
        assert Rg.shape == (d, d) and np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0)
    check_factors(rows, "projqr_raw f32")
    G = ref.G
    Rg = rows[-1]["R"]
    assert np.max(np.abs(Rg.T @ Rg - G)) <= 1e-12 * np.max(np.abs(G))


def test_argument_checks(lib):
    L = lib
    announce("proj_raw argument checks")
    n = 4
    N = n ** 3
    A = L.guess_op_create(n, n, n, 25.0, 10.0, None)
    try:
        with pytest.raises(L.GuessError) as e:       # FP64 histories use the Gram-Schmidt forms
            L.guess_create_ex(N, 4, L.PROJ_RAW, 0, L.F64, 0.0, A)
        assert e.value.code == L.EINVAL
        g = L.guess_create_ex(N, 4, L.PROJ_RAW, 0, L.F32, 0.0, None)
        try:
            assert L.guess_get_info(g)["eps_rel"] == 1e-6
            x = dev(np.ones(N))
            with pytest.raises(L.GuessError):        # no operator bound
                L.guess_update(g, x)
            L.guess_set_op(g, A)
            with pytest.raises(L.GuessError):        # A x of the unrounded solution is not used
                L.guess_update(g, x, dev(np.ones(N)))
            L.guess_update(g, x)
            assert L.guess_get_info(g)["count"] == 1
            L.guess_update(g, dev(np.zeros(N)))        # dependent (zero): rejected
            i = L.guess_get_info(g)
            assert i["count"] == 1 and i["last_accepted"] == 0
            L.guess_reset(g)
            assert L.guess_get_info(g)["count"] == 0
        finally:
            L.guess_destroy(g)
    finally:
        L.guess_op_destroy(A)
