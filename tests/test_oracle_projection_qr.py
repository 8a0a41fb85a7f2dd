"""Pins of the oracle's rolling-QR projection (§2, Algorithm 2) and of the
paper's ell-2 inner product, for both the classic and the rolling variant.

Independent references: the normal-equation minimisers over the retained raw
solutions (A-norm and residual-2-norm, FP64 and exact rationals), the
factorisation identity [raw solutions] = X R with R upper triangular, the orthonormality and A X = B invariants, and the
classic variant, which the rolling one must equal until the history is
first full.
"""
import numpy as np
import pytest

import synth
from oracle import operator as op
from oracle.projection import Projection, brute_force_guess, l2_residual_guess
from test_oracle_projection import A_of, _rational_minimiser


def _smooth_history(seed, T, N, K=5):
    """Columns drawn from a K-dimensional random subspace with smooth time
    coefficients plus a small independent part, so that every column is
    accepted and the window matters."""
    rng = np.random.default_rng(seed)
    basis = rng.standard_normal((K, N))
    out = []
    for t in range(T):
        coef = np.sin(0.3 * (t + 1) * (np.arange(K) + 1) + rng.uniform(0, 0.1, K))
        out.append(coef @ basis + 1e-2 * rng.standard_normal(N))
    return out


def _check_invariants(P, A, tol=1e-11):
    d = P.d
    if d == 0:
        return
    X, B = np.stack(P.X), np.stack(P.B)
    AX = np.stack([A(x) for x in P.X])
    assert np.max(np.abs(AX - B)) <= tol * np.max(np.abs(B))
    G = X @ B.T if P.inner == "A" else B @ B.T
    assert np.max(np.abs(G - np.eye(d))) <= tol
    R = P.R
    assert R.shape == (d, d)
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) != 0)
    raw = np.stack(P.raw)
    assert np.max(np.abs(R.T @ X - raw)) <= tol * np.max(np.abs(raw))


@pytest.mark.parametrize("inner", ["A", "l2"])
@pytest.mark.parametrize("M", [1, 2, 3, 5, 8])
def test_rolling_window_invariants_and_minimiser(inner, M):
    n = 4
    A = A_of(n)
    V = _smooth_history(3 + M, 3 * M + 4, n ** 3)
    b = synth.random_vectors(9, 1, n ** 3)[0]
    P = Projection(M, A, eps_rel=1e-10, variant="qr", inner=inner)
    for q, v in enumerate(V):
        assert P.update(v)
        assert P.d == min(q + 1, M)
        # the window is the last d raw solutions
        assert all(np.array_equal(r, w) for r, w in zip(P.raw, V[q + 1 - P.d: q + 1]))
        _check_invariants(P, A)
        ref = (brute_force_guess if inner == "A" else l2_residual_guess)(P.raw, A, b)
        got = P.form(b)
        assert np.max(np.abs(got - ref)) <= 1e-8 * np.max(np.abs(ref))
    assert P.drops == max(0, len(V) - M)


def test_rolling_guess_equals_exact_rational_minimiser():
    n = 3
    A = A_of(n)
    V = synth.random_vectors(21, 8, n ** 3)
    P = Projection(3, A, eps_rel=1e-10, variant="qr")
    for v in V[:6]:
        P.update(v)
    assert P.d == 3 and P.drops == 3
    ref = np.array([float(v) for v in _rational_minimiser(V[3:6], V[7], n)])
    got = P.form(V[7])
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("inner", ["A", "l2"])
def test_rolling_equals_classic_until_full(inner):
    n = 4
    A = A_of(n)
    V = _smooth_history(5, 6, n ** 3)
    Pc = Projection(6, A, eps_rel=1e-10, variant="classic", inner=inner)
    Pq = Projection(6, A, eps_rel=1e-10, variant="qr", inner=inner)
    b = V[-1] + 0.5
    for v in V:
        assert Pc.update(v) == Pq.update(v)
        assert np.array_equal(Pc.form(b), Pq.form(b))
    for xc, xq in zip(Pc.X, Pq.X):
        assert np.array_equal(xc, xq)


def test_classic_keeps_factor_too():
    n = 4
    A = A_of(n)
    V = _smooth_history(8, 11, n ** 3)
    P = Projection(4, A, eps_rel=1e-10)
    for v in V:
        P.update(v)
        _check_invariants(P, A)
    assert P.d == 11 - 8 and P.drops == 0       # restarts at steps 5 and 9


def test_rejection_keeps_window_consistent():
    """A rejected vector leaves the factor of the (possibly dropped) window intact."""
    n = 4
    A = A_of(n)
    V = _smooth_history(2, 4, n ** 3)
    P = Projection(4, A, eps_rel=1e-6, variant="qr")
    for v in V:
        assert P.update(v)
    dup = V[1] + V[2]                       # in the span of the window
    assert not P.update(dup)                # full: oldest dropped, then rejected
    assert P.d == 3 and len(P.raw) == 3
    _check_invariants(P, A)
    assert P.update(_smooth_history(7, 1, n ** 3)[0] * 3.0 + 1.0)
    assert P.d == 4
    _check_invariants(P, A)


def test_l2_guess_minimises_residual():
    n = 4
    A = A_of(n)
    V = synth.random_vectors(4, 5, n ** 3)
    P = Projection(8, A, eps_rel=1e-10, inner="l2")
    for v in V[:4]:
        P.update(v)
    b = V[4]
    x0 = P.form(b)
    r0 = np.linalg.norm(b - A(x0))
    rng = np.random.default_rng(0)
    for _ in range(20):
        y = x0 + 1e-3 * (rng.standard_normal(4) @ np.stack(P.raw))
        assert np.linalg.norm(b - A(y)) >= r0 * (1 - 1e-12)


def test_pins_catch_planted_mistakes(monkeypatch):
    n = 4
    A = A_of(n)
    V = _smooth_history(12, 9, n ** 3)
    b = synth.random_vectors(3, 1, n ** 3)[0]

    def pins_hold():
        try:
            P = Projection(4, A, eps_rel=1e-10, variant="qr")
            for v in V:
                P.update(v)
                _check_invariants(P, A)
                ref = brute_force_guess(P.raw, A, b)
                if np.max(np.abs(P.form(b) - ref)) > 1e-8 * np.max(np.abs(ref)):
                    return False
            return True
        except AssertionError:
            return False

    assert pins_hold()
    good = Projection._drop_oldest

    def drop_newest(self):           # drops the newest instead of the oldest
        self.raw = self.raw[1:]
        self.R = self.R[:-1, :-1]
        return self.X[:-1], self.B[:-1], [(1.0, 0.0)] * (self.d - 1)
    monkeypatch.setattr(Projection, "_drop_oldest", drop_newest)
    assert not pins_hold()

    def no_sign(self):               # c = a / r, s = -b / r: does not zero the subdiagonal
        d = self.d
        R = self.R[:, 1:].copy()
        X, B = list(self.X), list(self.B)
        for i in range(d - 1):
            a, bb = R[i, i], R[i + 1, i]
            r = float(np.hypot(a, bb))
            c, s = a / r, -bb / r
            G = np.array([[c, s], [-s, c]])
            R[i:i + 2, :] = G @ R[i:i + 2, :]
            R[i + 1, i] = 0.0
            X[i], X[i + 1] = c * X[i] + s * X[i + 1], -s * X[i] + c * X[i + 1]
            B[i], B[i + 1] = c * B[i] + s * B[i + 1], -s * B[i] + c * B[i + 1]
        self.R, self.raw = R[: d - 1], self.raw[1:]
        return X[: d - 1], B[: d - 1], [(1.0, 0.0)] * (d - 1)
    monkeypatch.setattr(Projection, "_drop_oldest", no_sign)
    assert not pins_hold()

    def transposed_rotation(self):   # columns rotated with G instead of G^T
        d = self.d
        R = self.R[:, 1:].copy()
        X, B = list(self.X), list(self.B)
        for i in range(d - 1):
            a, bb = R[i, i], R[i + 1, i]
            r = float(np.hypot(a, bb))
            c, s = abs(a) / r, (1.0 if a >= 0 else -1.0) * bb / r
            R[i:i + 2, :] = np.array([[c, s], [-s, c]]) @ R[i:i + 2, :]
            R[i + 1, i] = 0.0
            X[i], X[i + 1] = c * X[i] - s * X[i + 1], s * X[i] + c * X[i + 1]
            B[i], B[i + 1] = c * B[i] - s * B[i + 1], s * B[i] + c * B[i + 1]
        self.R, self.raw = R[: d - 1], self.raw[1:]
        return X[: d - 1], B[: d - 1], [(1.0, 0.0)] * (d - 1)
    monkeypatch.setattr(Projection, "_drop_oldest", transposed_rotation)
    assert not pins_hold()

    def columns_not_rotated(self):   # R rotated but X, B left alone
        d = self.d
        R = self.R[:, 1:].copy()
        for i in range(d - 1):
            a, bb = R[i, i], R[i + 1, i]
            r = float(np.hypot(a, bb))
            c, s = abs(a) / r, np.sign(a) * bb / r
            R[i:i + 2, :] = np.array([[c, s], [-s, c]]) @ R[i:i + 2, :]
            R[i + 1, i] = 0.0
        self.R, self.raw = R[: d - 1], self.raw[1:]
        return self.X[1:], self.B[1:], [(1.0, 0.0)] * (d - 1)
    monkeypatch.setattr(Projection, "_drop_oldest", columns_not_rotated)
    assert not pins_hold()
    monkeypatch.setattr(Projection, "_drop_oldest", good)
    assert pins_hold()
