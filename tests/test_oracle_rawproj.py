"""Pins of the oracle's raw-solution projection (oracle/rawproj.py).

References independent of its formula: exact rational arithmetic (the
A-norm minimiser over the stored vectors, solved by Fraction elimination),
the Gram-Schmidt projection of oracle/projection.py (another algorithm for
the same guess, pinned on its own), x^T A x of the remainder computed by
explicit orthogonal projection, IEEE rounding through numpy's float32 /
float16, and the FP16 range.  Planted mistakes must fail a pin.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import lowprec
from oracle import operator as op
from oracle.projection import Projection
from oracle.rawproj import RawProjection


def A_of(n):
    return lambda v: op.apply_const(v, n)


def _exact_minimiser(W, n, b):
    """x = W y with (W^T A W) y = W^T b, all in exact rationals (A applied exactly)."""
    N = n ** 3
    h2 = (n + 1) ** 2

    def A_exact(v):
        out = []
        for q in range(N):
            i, j, k = q % n, (q // n) % n, q // (n * n)
            s = 6 * v[q]
            for di, dj, dk in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                a, bb, c = i + di, j + dj, k + dk
                if 0 <= a < n and 0 <= bb < n and 0 <= c < n:
                    s -= v[a + n * (bb + n * c)]
            out.append(h2 * s + 10 * v[q])
        return out

    Wf = [[Fraction(float(t)) for t in w] for w in W]
    bf = [Fraction(float(t)) for t in b]
    AW = [A_exact(w) for w in Wf]
    d = len(Wf)
    G = [[sum(a * c for a, c in zip(Wf[i], AW[j])) for j in range(d)] for i in range(d)]
    r = [sum(a * c for a, c in zip(Wf[i], bf)) for i in range(d)]
    # Gauss-Jordan elimination (G is symmetric positive definite: no pivoting needed)
    M = [G[i][:] + [r[i]] for i in range(d)]
    for c in range(d):
        p = M[c][c]
        M[c] = [v / p for v in M[c]]
        for i in range(d):
            if i != c and M[i][c] != 0:
                f = M[i][c]
                M[i] = [a - f * bb for a, bb in zip(M[i], M[c])]
    y = [M[i][d] for i in range(d)]
    return np.array([float(sum(y[i] * Wf[i][q] for i in range(d))) for q in range(len(bf))])


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16", "bf16"])
def test_guess_is_the_exact_minimiser_over_the_stored_vectors(dtype):
    """3^3 grid, random solutions: the guess equals the exact-rational A-norm minimiser over
    the vectors the history holds (rounded to the format)."""
    n, M = 3, 4
    A = A_of(n)
    V = synth.random_vectors(11, M, n ** 3)
    P = RawProjection(M, A, 1e-8, dtype)
    for v in V:
        assert P.update(v)
    b = synth.random_vectors(12, 1, n ** 3)[0]
    want = _exact_minimiser(P.W, n, b)
    got = P.form(b)
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))


@pytest.mark.parametrize("variant", ["classic", "qr"])
def test_fp64_equals_the_gram_schmidt_projection(variant):
    """FP64 storage, random (well-conditioned) solutions: the same guesses, decisions and
    ratios nu / nu0 as Algorithm 1 / 2 in Gram-Schmidt form, through restarts and drops."""
    n, M = 6, 4
    A = A_of(n)
    V = synth.random_vectors(21, 3 * M + 1, n ** 3)
    Bs = synth.random_vectors(22, 3 * M + 1, n ** 3)
    R = RawProjection(M, A, 1e-6, "f64", variant)
    G = Projection(M, A, 1e-6, "f64", variant, "A")
    for v, b in zip(V, Bs):
        gr, gg = R.form(b), G.form(b)
        if np.max(np.abs(gg)) > 0:
            assert np.max(np.abs(gr - gg)) <= 1e-10 * np.max(np.abs(gg))
        else:
            assert not gr.any()
        assert R.update(v) == G.update(v)
        assert R.d == G.d
        assert abs(R.last_nu / R.last_nu0 - G.last_nu / G.last_nu0) <= 1e-10
    if variant == "qr":
        assert R.drops == G.drops > 0


def test_rejection_norm_is_the_remainder_norm():
    """nu^2 equals r^T A r for the remainder r = w - X X^T A w of w after A-orthogonal
    projection onto the stored span, X the A-orthonormal basis of the Gram-Schmidt oracle."""
    n, M = 5, 6
    A = A_of(n)
    V = synth.random_vectors(31, 4, n ** 3)
    R = RawProjection(M, A, 1e-12, "f64")
    G = Projection(M, A, 1e-12, "f64")
    for v in V[:3]:
        R.update(v)
        G.update(v)
    w = V[3] + 0.9 * V[0] - 0.5 * V[2]
    R.update(w)
    X = np.stack(G.X)
    r = w - X.T @ (X @ A(w))
    assert abs(R.last_nu - np.sqrt(r @ A(r))) <= 1e-10 * R.last_nu


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_stored_values_and_gram(dtype):
    """Stored vectors are the format's rounding of the solutions (FP16: of 2^e x, max in
    [2^14, 2^15)), and G is the Gram matrix of exactly those vectors."""
    n, M = 5, 4
    A = A_of(n)
    V = [v * 10.0 ** (q - 3) for q, v in enumerate(synth.random_vectors(41, 2 * M, n ** 3))]
    P = RawProjection(M, A, 1e-6, dtype, "qr")
    for v in V:
        P.update(v)
    for q, w in enumerate(P.W):
        x = V[len(V) - P.d + q]
        e = lowprec.f16_scale_exp(float(np.max(np.abs(x)))) if dtype == "f16" else 0
        np.testing.assert_array_equal(w, lowprec.round_store(x, dtype, e))
        if dtype == "f16":
            assert 2 ** 14 <= np.max(np.abs(np.ldexp(w, e))) <= 2 ** 15
    Wm = np.stack(P.W)
    G = Wm @ np.stack([A(w) for w in P.W]).T
    np.testing.assert_allclose(P.G, G, rtol=1e-13, atol=0)


def test_classic_restart_and_rolling_window():
    n, M = 4, 3
    A = A_of(n)
    V = synth.random_vectors(51, 8, n ** 3)
    C = RawProjection(M, A, 1e-6, "f64", "classic")
    Q = RawProjection(M, A, 1e-6, "f64", "qr")
    dc, dq = [], []
    for v in V:
        C.update(v)
        Q.update(v)
        dc.append(C.d)
        dq.append(Q.d)
    assert dc == [1, 2, 3, 1, 2, 3, 1, 2]
    assert dq == [1, 2, 3, 3, 3, 3, 3, 3] and Q.drops == 5
    for w, v in zip(Q.W, V[-3:]):          # the window holds the last M solutions
        np.testing.assert_array_equal(w, v)
    # a dependent solution is rejected; a zero one too
    assert not C.update(2.0 * C.W[-1] - C.W[0])
    assert not RawProjection(M, A).update(np.zeros(n ** 3))


def test_pins_catch_planted_mistakes(monkeypatch):
    def run(fn, *a):
        try:
            fn(*a)
            return True
        except AssertionError:
            return False

    assert run(test_guess_is_the_exact_minimiser_over_the_stored_vectors, "f16")
    assert run(test_fp64_equals_the_gram_schmidt_projection, "qr")
    assert run(test_stored_values_and_gram, "bf16")
    good_update = RawProjection.update

    # Gram matrix of the unrounded solutions instead of the stored ones
    def unrounded_gram(self, x, Ax=None, decide=None):
        ok = good_update(self, x, Ax, decide)
        if ok and self.dtype != "f64":
            W = [np.asarray(x, dtype=np.float64) if q == self.d - 1 else w for q, w in enumerate(self.W)]
            G = self.G.copy()
            G[-1, -1] = float(W[-1] @ self.apply_A(W[-1]))
            self.G = G
        return ok

    monkeypatch.setattr(RawProjection, "update", unrounded_gram)
    assert not run(test_stored_values_and_gram, "bf16")
    monkeypatch.setattr(RawProjection, "update", good_update)

    # wrong sign in the Schur complement: nu^2 = s0 + g^T G^{-1} g
    monkeypatch.setattr(RawProjection, "_outside_norm2",
                        lambda self, s0, g: s0 + float(g @ np.linalg.solve(self.G, g)))
    assert not run(test_fp64_equals_the_gram_schmidt_projection, "classic")
    assert not run(test_rejection_norm_is_the_remainder_norm)
    monkeypatch.undo()

    # dropping the newest instead of the oldest solution
    def drop_newest(self, x, Ax=None, decide=None):
        if self.variant == "qr" and self.d == self.M:
            self.W, self.exps, self.G = self.W[:-1], self.exps[:-1], self.G[:-1, :-1].copy()
            self.drops += 1
            self.variant = "classic_tmp"
            try:
                return good_update(self, x, Ax, decide)
            finally:
                self.variant = "qr"
        return good_update(self, x, Ax, decide)

    monkeypatch.setattr(RawProjection, "update", drop_newest)
    assert not run(test_fp64_equals_the_gram_schmidt_projection, "qr")
