"""Pins of the oracle's sparse extrapolation (§3.3, eq. CPQRCoeffs).

Independent checks: polynomial exactness in monomials and in index time
(eq. PolyExactness), the count of nonzero weights, the Lagrange closed form
through the selected nodes, the minimum-norm property of the least-squares
weights it must not beat, the naive binomial weights when every node is
selected, the Legendre basis against numpy's Legendre evaluation, and the
pivot order re-derived by brute force from Gram determinants.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

from oracle import extrap
from test_oracle_extrap import _read_rows, pin_exactness

SHAPES = [(m, M) for M in range(1, 17) for m in range(0, M)]


def _det(A):
    """Exact determinant by fraction-valued elimination (independent of the oracle's solver)."""
    A = [list(r) for r in A]
    n, det = len(A), Fraction(1)
    for c in range(n):
        p = next((r for r in range(c, n) if A[r][c] != 0), None)
        if p is None:
            return Fraction(0)
        if p != c:
            A[c], A[p] = A[p], A[c]
            det = -det
        det *= A[c][c]
        for r in range(c + 1, n):
            f = A[r][c] / A[c][c]
            A[r] = [a - f * b for a, b in zip(A[r], A[c])]
    return det


def _brute_pivots(m, M):
    """Greedy volume maximisation: the next pivot maximises the Gram determinant of
    the chosen columns of V^T (equal to the product of squared residual norms);
    first index on exact ties."""
    V, _ = extrap.legendre_vandermonde(M, m)
    chosen = []
    for _ in range(m + 1):
        best, bi = None, None
        for i in range(M):
            if i in chosen:
                continue
            rows = [V[j] for j in chosen + [i]]
            gram = [[sum(a * b for a, b in zip(r, s)) for s in rows] for r in rows]
            d = _det(gram)
            if best is None or d > best:
                best, bi = d, i
        chosen.append(bi)
    return chosen


def _lagrange(S, M):
    t, tn = extrap.time_nodes(M)
    beta = [Fraction(0)] * M
    for a in S:
        w = Fraction(1)
        for b in S:
            if b != a:
                w *= (tn - t[b]) / (t[a] - t[b])
        beta[a] = w
    return beta


@pytest.mark.parametrize("m,M", SHAPES)
def test_sparse_weights_pins(m, M):
    beta = extrap.beta_sparse_exact(m, M)
    S = extrap.cpqr_pivots(m, M)
    assert len(beta) == M
    assert sum(1 for b in beta if b != 0) == m + 1
    assert sorted(S) == [i for i, b in enumerate(beta) if b != 0]
    assert pin_exactness(beta, m, M)
    assert beta == _lagrange(S, M)
    # the least-squares weights are the minimum 2-norm solution of the same system
    ls = extrap.beta_ls_exact(m, M)
    n2 = sum(b * b for b in beta)
    n2ls = sum(b * b for b in ls)
    assert n2 >= n2ls
    if m == M - 1:
        assert beta == ls


@pytest.mark.parametrize("m,M", [(m, M) for M in range(1, 11) for m in range(0, M)])
def test_pivots_are_greedy_volume_maximisers(m, M):
    assert extrap.cpqr_pivots(m, M) == _brute_pivots(m, M)


def test_full_degree_is_naive():
    for row in _read_rows("naive_rows_pascal.txt"):
        M = int(row[0])
        want = [(-1) ** (M - i) * mag for i, mag in enumerate(row[1:], start=1)]
        assert extrap.beta_sparse_exact(M - 1, M) == want


@pytest.mark.parametrize("M", [2, 3, 5, 8, 12, 16])
def test_endpoints_are_always_selected(M):
    """Column pivoting clusters the selected nodes at the ends, like Chebyshev points (§3.3):
    for m >= 1 both the oldest and the newest solution are used."""
    for m in range(1, M):
        S = extrap.cpqr_pivots(m, M)
        assert 0 in S and M - 1 in S


def test_legendre_basis_matches_numpy():
    for M, m in [(8, 3), (16, 7), (5, 4)]:
        V, v = extrap.legendre_vandermonde(M, m)
        t, tn = extrap.time_nodes(M)
        for j in range(m + 1):
            c = np.zeros(j + 1)
            c[j] = 1.0
            ref = np.polynomial.legendre.legval(np.array([float(x) for x in t] + [float(tn)]), c)
            got = np.array([float(V[i][j]) for i in range(M)] + [float(v[j])])
            np.testing.assert_allclose(got, ref, rtol=1e-14, atol=1e-14)


def test_sparse_form_exact_on_time_polynomials():
    import synth

    for m, M in [(1, 8), (2, 8), (3, 16), (2, 4)]:
        times = np.arange(1, M + 2) * 0.01
        X, _ = synth.polynomial_in_time_history(11, m, 129, times)
        beta = extrap.to_f64(extrap.beta_sparse_exact(m, M))
        x0 = extrap.form(list(X[:M]), beta)
        assert np.max(np.abs(x0 - X[M])) <= 1e-11 * np.max(np.abs(X)) * float(extrap.lebesgue(beta))


def test_history_object_sparse():
    h = extrap.ExtrapHistory(8, 2, sparse=True)
    for i in range(1, 12):
        g = h.form(N=3)
        if i >= 4:
            np.testing.assert_allclose(g, float(i) ** 2, rtol=1e-12)
        h.update(np.full(3, float(i) ** 2))
    assert np.array_equal(h.weights(8), extrap.to_f64(extrap.beta_sparse_exact(2, 8)))
    assert np.array_equal(h.weights(3), extrap.to_f64(extrap.beta_sparse_exact(2, 3)))


def test_pins_catch_planted_mistakes(monkeypatch):
    """Plausible bugs in the sparse oracle each fail at least one pin."""
    shapes = [(1, 4), (2, 8), (3, 8), (4, 8), (2, 5)]

    def check():
        try:
            for m, M in shapes:
                beta = extrap.beta_sparse_exact(m, M)
                S = extrap.cpqr_pivots(m, M)
                if not (pin_exactness(beta, m, M) and beta == _lagrange(S, M)
                        and sum(1 for b in beta if b != 0) == m + 1):
                    return False
                if S != _brute_pivots(m, M):
                    return False
        except Exception:
            return False
        return True

    assert check()
    good_piv, good_vdm = extrap.cpqr_pivots, extrap.legendre_vandermonde

    # 1. last-maximum tie-break
    def piv_last(m, M):
        V, _ = good_vdm(M, m)
        chosen = []
        for _ in range(m + 1):
            best = max((i for i in range(M) if i not in chosen),
                       key=lambda i: (_det([[sum(a * b for a, b in zip(V[r], V[s])) for s in chosen + [i]]
                                            for r in chosen + [i]]), i))
            chosen.append(best)
        return chosen
    monkeypatch.setattr(extrap, "cpqr_pivots", piv_last)
    assert not check()
    monkeypatch.setattr(extrap, "cpqr_pivots", good_piv)

    # 2. the last m+1 nodes (plain Lagrange extrapolation) instead of the pivots
    monkeypatch.setattr(extrap, "cpqr_pivots", lambda m, M: list(range(M - m - 1, M)))
    assert not check()
    monkeypatch.setattr(extrap, "cpqr_pivots", good_piv)

    # 3. a wrong Legendre recurrence coefficient
    def vdm_bad(M, m):
        V, v = good_vdm(M, m)
        if m >= 2:
            t, tn = extrap.time_nodes(M)
            V = [row[:2] + [Fraction(3) * ti * ti - 1 for _ in row[2:3]] + row[3:] for row, ti in zip(V, t)]
        return V, v
    monkeypatch.setattr(extrap, "legendre_vandermonde", vdm_bad)
    assert not check()
    monkeypatch.setattr(extrap, "legendre_vandermonde", good_vdm)

    # 4. weights assigned to the pivots in sorted instead of pivot order
    good_sparse = extrap.beta_sparse_exact

    def sparse_misassigned(m, M):
        beta = good_sparse(m, M)
        nz = [i for i, b in enumerate(beta) if b != 0]
        vals = [beta[i] for i in nz][::-1]
        out = [Fraction(0)] * M
        for i, b in zip(nz, vals):
            out[i] = b
        return out
    monkeypatch.setattr(extrap, "beta_sparse_exact", sparse_misassigned)
    assert not check()
    monkeypatch.setattr(extrap, "beta_sparse_exact", good_sparse)
    assert check()
