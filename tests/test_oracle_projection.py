"""Pins of the oracle's A-orthonormal projection (§2, Algorithm 1, A inner product).

Independent references: the invariants the paper states for the history
(A X = B, orthonormality, span of the retained solutions), the normal-equation
minimiser written in exact rational arithmetic on a 3^3 grid, the same
minimiser in FP64 on 4^3 grids, and §4's theorem (i) in its A-norm form.
"""
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import extrap
from oracle import operator as op
from oracle.projection import AOrthoProjection, brute_force_guess


def A_of(n):
    return lambda v: op.apply_const(v, n)


def _rational_apply(u, n):
    """Exact 7-point operator on Fractions (c = (n+1)^2, shift 10)."""
    c = (n + 1) ** 2
    out = []
    for l in range(n):
        for j in range(n):
            for i in range(n):
                k = (l * n + j) * n + i
                s = 6 * u[k]
                for di, dj, dl in ((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)):
                    ii, jj, ll = i + di, j + dj, l + dl
                    if 0 <= ii < n and 0 <= jj < n and 0 <= ll < n:
                        s -= u[(ll * n + jj) * n + ii]
                out.append(c * s + 10 * u[k])
    return out


def _rational_minimiser(S, b, n):
    """x = S (S^T A S)^{-1} S^T b in exact arithmetic (rows of S are vectors)."""
    S = [[Fraction(float(v)) for v in s] for s in S]
    b = [Fraction(float(v)) for v in b]
    AS = [_rational_apply(s, n) for s in S]
    k = len(S)
    G = [[sum(a * c for a, c in zip(S[i], AS[j])) for j in range(k)] for i in range(k)]
    rhs = [sum(a * c for a, c in zip(S[i], b)) for i in range(k)]
    y = extrap._solve_exact(G, rhs)
    return [sum(y[i] * S[i][q] for i in range(k)) for q in range(len(b))]


def test_guess_equals_exact_rational_minimiser():
    n = 3
    A = A_of(n)
    V = synth.random_vectors(11, 6, n ** 3)
    P = AOrthoProjection(8, A, eps_rel=1e-10)
    for q in range(4):
        P.update(V[q])
    assert P.d == 4
    b = V[5]
    x0 = P.form(b)
    ref = np.array([float(v) for v in _rational_minimiser(P.raw, b, n)])
    assert np.max(np.abs(x0 - ref)) <= 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_guess_equals_normal_equation_minimiser(seed):
    n = 4
    A = A_of(n)
    V = synth.random_vectors(100 + seed, 5, n ** 3)
    P = AOrthoProjection(8, A, eps_rel=1e-10)
    for q in range(4):
        P.update(V[q])
        b = V[4]
        ref = brute_force_guess(P.raw, A, b)
        np.testing.assert_allclose(P.form(b), ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_history_invariants():
    n = 6
    A = A_of(n)
    V = synth.random_vectors(7, 7, n ** 3)
    P = AOrthoProjection(8, A, eps_rel=1e-10)
    for v in V:
        P.update(v)
    X, B = np.stack(P.X), np.stack(P.B)
    d = P.d
    assert d == 7
    np.testing.assert_allclose(X @ B.T, np.eye(d), rtol=0, atol=1e-12)       # X^T A X = I
    for x, bb in zip(X, B):
        np.testing.assert_allclose(A(x), bb, rtol=0, atol=1e-12 * np.abs(bb).max())
    # span X = span of accepted raw solutions: projecting each raw solution is exact
    for r in P.raw:
        proj = X.T @ (B @ r)
        np.testing.assert_allclose(proj, r, rtol=0, atol=1e-11 * np.abs(r).max())


def test_restart_when_full():
    n = 4
    A = A_of(n)
    V = synth.random_vectors(3, 6, n ** 3)
    P = AOrthoProjection(3, A)
    ds = []
    for v in V:
        P.update(v)
        ds.append(P.d)
    assert ds == [1, 2, 3, 1, 2, 3]
    assert len(P.raw) == 3


def test_rejects_dependent_vector():
    n = 4
    A = A_of(n)
    V = synth.random_vectors(4, 3, n ** 3)
    P = AOrthoProjection(8, A, eps_rel=1e-6)
    P.update(V[0])
    P.update(V[1])
    assert not P.update(0.3 * V[0] - 2.0 * V[1])      # in the span: rejected
    assert P.d == 2
    assert P.last_nu <= 1e-6 * P.last_nu0
    assert P.update(V[2])
    assert P.d == 3


def test_empty_history_and_zero_solution():
    n = 3
    P = AOrthoProjection(4, A_of(n))
    b = synth.random_vectors(0, 1, n ** 3)[0]
    assert not P.form(b).any()
    assert not P.update(np.zeros(n ** 3))              # nu0 = 0: nothing stored
    assert P.d == 0


def test_projection_beats_extrapolation_in_A_norm():
    """§4 theorem (i), A-norm form: on a shared span projection is optimal."""
    # time step large enough that the history is well conditioned in FP64
    # (with tiny steps the retained solutions are nearly dependent and the
    # computed basis, not the theorem, limits the projection)
    n = 8
    A = A_of(n)
    params = synth.plane_wave_params(0, 16)
    ts = synth.step_times(7, 0.1)
    B = [synth.plane_wave_rhs(params, n, t) for t in ts]
    X = [op.dst_solve(b, n) for b in B]
    P = AOrthoProjection(6, A, eps_rel=1e-10)
    for x in X[:6]:
        P.update(x)
    assert P.d == 6
    xs = X[6]
    xp = P.form(B[6])
    for m in (1, 2, 3):
        xe = extrap.form(X[:6], extrap.to_f64(extrap.beta_ls_exact(m, 6)))
        eP, eE = xs - xp, xs - xe
        assert eP @ A(eP) <= eE @ A(eE) * (1 + 1e-9)


def test_pins_catch_planted_mistakes(monkeypatch):
    """A wrong sign in the Gram-Schmidt step, or a single GS pass with a
    transposed operand, breaks the invariants or the minimiser pin."""
    n = 4
    A = A_of(n)
    V = synth.random_vectors(21, 5, n ** 3)

    def pins_hold():
        P = AOrthoProjection(8, A, eps_rel=1e-10)
        for v in V[:4]:
            P.update(v)
        X, B = np.stack(P.X), np.stack(P.B)
        ok = np.allclose(X @ B.T, np.eye(P.d), atol=1e-10)
        ref = brute_force_guess(P.raw, A, V[4])
        ok &= np.allclose(P.form(V[4]), ref, atol=1e-10 * np.abs(ref).max())
        return ok

    assert pins_hold()
    real_update = AOrthoProjection.update

    def update_wrong_sign(self, x, Ax=None):
        xt = np.array(x, dtype=float)
        bt = self.apply_A(xt)
        if self.d == 0 or self.d >= self.M:
            return real_update(self, x, Ax)
        for _ in range(2):
            c = [float(xj @ bt) for xj in self.X]
            for cj, xj, bj in zip(c, self.X, self.B):
                bt = bt - cj * bj
                xt = xt + cj * xj          # planted: wrong sign
        nu = np.sqrt(abs(xt @ bt))
        self._put_new(xt, bt, nu, 0)
        self.raw.append(np.array(x, dtype=float))
        return True

    monkeypatch.setattr(AOrthoProjection, "update", update_wrong_sign)
    assert not pins_hold()
