"""Pins of the oracle's extrapolation weights and guess against the paper.

Each pin is independent of the code under test: closed forms printed in the
paper (§3.1 theorem, worked example, Pascal rows, §6.5 Lebesgue theorem),
textbook closed forms (mean, simple linear regression), the defining
properties of the least-squares weights (polynomial exactness, eq.
PolyExactness, and minimum norm, §3.3) and a library pseudoinverse.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import extrap

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([Fraction(t) for t in line.split()])
    return rows


# ---------------------------------------------------------------- pin helpers
def pin_exactness(beta, m, M):
    """Scheme is exact on polynomials of degree <= m (eq. PolyExactness)."""
    t, tn = extrap.time_nodes(M)
    rng = np.random.default_rng(1234 + 31 * M + m)
    for _ in range(3):
        coef = [Fraction(int(c)) for c in rng.integers(-9, 10, size=m + 1)]
        p = lambda s: sum(c * s ** q for q, c in enumerate(coef))  # noqa: E731
        if sum(b * p(ti) for b, ti in zip(beta, t)) != p(tn):
            return False
    # also in index time (affine invariance): nodes 1..M, new node M+1
    for q in range(m + 1):
        if sum(b * Fraction(i) ** q for i, b in enumerate(beta, start=1)) != Fraction(M + 1) ** q:
            return False
    return True


def pin_min_norm(beta, m, M):
    """beta is the minimum-norm solution of V^T beta = v (pseudoinverse, §3.3)."""
    t, tn = extrap.time_nodes(M)
    # Legendre-free float check with numpy's SVD-based pseudoinverse of V^T
    tt = np.array([float(x) for x in t])
    Vt = np.stack([tt ** q for q in range(m + 1)])
    v = np.array([float(tn) ** q for q in range(m + 1)])
    ref = np.linalg.pinv(Vt) @ v
    return np.allclose(np.array([float(b) for b in beta]), ref, rtol=0, atol=1e-10)


# ---------------------------------------------------------------- paper pins
def test_worked_example_linear_M2():
    (row,) = _read_rows("extrap_linear_M2.txt")
    m, M, beta = int(row[0]), int(row[1]), row[2:]
    assert extrap.beta_ls_exact(m, M) == beta
    assert extrap.beta_naive_exact(M) == beta


def test_naive_weights_are_pascal_rows():
    for row in _read_rows("naive_rows_pascal.txt"):
        M = int(row[0])
        mags = row[1:]
        beta = extrap.beta_naive_exact(M)
        assert [abs(b) for b in beta] == mags
        assert [1 if b > 0 else -1 for b in beta] == [(-1) ** (M - i) for i in range(1, M + 1)]


@pytest.mark.parametrize("M", range(1, 13))
def test_ls_with_full_degree_is_lagrange(M):
    """Least squares with m = M-1 interpolates: weights of the §3.1 theorem."""
    assert extrap.beta_ls_exact(M - 1, M) == extrap.beta_naive_exact(M)


@pytest.mark.parametrize("M", range(1, 16))
def test_naive_lebesgue_constant(M):
    """§6.5 theorem: Lambda(naive EXTRAP(M-1, M)) = 2^M - 1."""
    assert extrap.lebesgue(extrap.beta_ls_exact(M - 1, M)) == 2 ** M - 1


@pytest.mark.parametrize("M", range(1, 17))
def test_degree_zero_is_mean(M):
    """Constant least-squares fit = mean of the history (textbook)."""
    assert extrap.beta_ls_exact(0, M) == [Fraction(1, M)] * M


@pytest.mark.parametrize("M", range(2, 17))
def test_degree_one_is_linear_regression(M):
    """Simple linear regression on index time i = 1..M evaluated at M+1.

    Textbook closed form: beta_i = 1/M + (M+1-ibar)(i-ibar)/S_ii with
    ibar = (M+1)/2 and S_ii = M(M^2-1)/12, i.e. 2(3i-M-2)/(M(M-1)).
    """
    ibar = Fraction(M + 1, 2)
    Sii = Fraction(M * (M * M - 1), 12)
    ref = [Fraction(1, M) + (M + 1 - ibar) * (i - ibar) / Sii for i in range(1, M + 1)]
    assert extrap.beta_ls_exact(1, M) == ref
    assert ref == [Fraction(2 * (3 * i - M - 2), M * (M - 1)) for i in range(1, M + 1)]


@pytest.mark.parametrize("m,M", [(m, M) for M in range(1, 17) for m in range(0, 6) if m <= M - 1])
def test_ls_exactness_and_min_norm(m, M):
    beta = extrap.beta_ls_exact(m, M)
    assert sum(beta) == 1
    assert pin_exactness(beta, m, M)
    assert pin_min_norm(beta, m, M)
    if m < M - 1:
        # not exact one degree higher (else the degree would be overstated)
        t, tn = extrap.time_nodes(M)
        assert sum(b * ti ** (m + 1) for b, ti in zip(beta, t)) != tn ** (m + 1)


def test_stabilized_lebesgue_stays_small():
    """§6.5 figure: EXTRAP(floor(sqrt M), M) has a slowly growing Lebesgue constant."""
    for M in range(2, 33):
        m = int(np.floor(np.sqrt(M)))
        lam = extrap.lebesgue(extrap.beta_ls_exact(m, M))
        assert 1 <= lam < 10
        assert lam <= extrap.lebesgue(extrap.beta_naive_exact(M))


def test_warm_up_rule():
    assert extrap.effective_params(2, 8, 0) is None
    assert extrap.effective_params(2, 8, 1) == (0, 1)
    assert extrap.effective_params(2, 8, 2) == (1, 2)
    assert extrap.effective_params(2, 8, 3) == (2, 3)
    assert extrap.effective_params(2, 8, 7) == (2, 7)
    assert extrap.effective_params(2, 8, 12) == (2, 8)


# ---------------------------------------------------------------- the guess
@pytest.mark.parametrize("m,M", [(0, 1), (1, 2), (2, 8), (3, 8), (1, 8), (3, 16), (2, 4)])
def test_form_exact_on_time_polynomials(m, M):
    """Vector histories x_i = sum_q t_i^q v_q of degree m are extrapolated exactly."""
    dt = 0.01
    times = np.arange(1, M + 2) * dt
    X, V = synth.polynomial_in_time_history(7, m, 257, times)
    beta = extrap.to_f64(extrap.beta_ls_exact(m, M))
    x0 = extrap.form(list(X[:M]), beta)
    ref = X[M]
    assert np.max(np.abs(x0 - ref)) <= 1e-12 * np.max(np.abs(X)) * extrap.lebesgue(beta) * 10


@pytest.mark.parametrize("m,M", [(1, 8), (2, 8), (3, 8), (2, 4), (1, 2)])
def test_error_order_under_step_halving(m, M):
    """§4 theorem (iii): the extrapolation error is O(dt^(m+1)).

    Smooth history x(t) = exp(t) v (no derivative vanishes); halving dt
    divides the error by about 2^(m+1).
    """
    v = np.linspace(0.5, 1.5, 16)
    beta = extrap.to_f64(extrap.beta_ls_exact(m, M))
    errs = []
    for dt in (0.01, 0.005, 0.0025):
        ts = 0.3 + np.arange(1, M + 2) * dt
        X = np.stack([np.exp(t) * v for t in ts])
        errs.append(np.max(np.abs(extrap.form(list(X[:M]), beta) - X[M])))
    for e1, e2 in zip(errs, errs[1:]):
        ratio = e1 / e2
        assert 2 ** (m + 1) * 0.8 < ratio < 2 ** (m + 1) * 1.25


def test_history_object_uses_warmup_and_ring_order():
    h = extrap.ExtrapHistory(4, 2)
    xs = [np.full(5, float(i)) for i in range(1, 8)]    # linear in time
    assert np.all(h.form(N=5) == 0)
    for i, x in enumerate(xs):
        g = h.form(N=5)
        if i >= 2:
            # linear data is reproduced exactly once two points are known
            np.testing.assert_allclose(g, float(i + 1), rtol=0, atol=1e-12)
        h.update(x)
    assert len(h.hist) == 4
    assert h.hist[0][0] == 4.0


# ---------------------------------------------------------------- planted mistakes
def test_pins_catch_planted_mistakes(monkeypatch):
    """Plausible bugs in the oracle's weights each fail at least one pin."""
    good_nodes = extrap.time_nodes

    def check_all():
        ok = True
        for (m, M) in [(1, 2), (2, 8), (3, 8), (2, 4), (1, 16)]:
            beta = extrap.beta_ls_exact(m, M)
            ok &= len(beta) == M
            ok &= pin_exactness(beta, m, M) and pin_min_norm(beta, m, M)
            ok &= beta == [Fraction(2 * (3 * i - M - 2), M * (M - 1)) for i in range(1, M + 1)] \
                if m == 1 else True
        return ok

    assert check_all()

    # 1. new node at the last history node (extrapolation distance dropped)
    def nodes_no_step(M):
        t, tn = good_nodes(M)
        return t, t[-1]
    monkeypatch.setattr(extrap, "time_nodes", nodes_no_step)
    assert not check_all()
    monkeypatch.setattr(extrap, "time_nodes", good_nodes)

    # 2. weights in reversed order (newest first)
    good_ls = extrap.beta_ls_exact
    monkeypatch.setattr(extrap, "beta_ls_exact", lambda m, M: list(reversed(good_ls(m, M))))
    assert not check_all()
    monkeypatch.setattr(extrap, "beta_ls_exact", good_ls)

    # 3. the highest basis function replaced by the next lower one times t
    #    evaluated at the wrong node (a transposed index in V)
    good_vdm = extrap.vandermonde

    def vdm_transposed_index(M, m):
        V, v = good_vdm(M, m)
        V = [row[:] for row in V]
        V[0], V[-1] = V[-1], V[0]          # rows of the first and last node swapped
        return V, v
    monkeypatch.setattr(extrap, "vandermonde", vdm_transposed_index)
    assert not check_all()

    # 4. new node one step too far
    monkeypatch.setattr(extrap, "vandermonde", good_vdm)

    def nodes_far(M):
        t, tn = good_nodes(M)
        return t, tn + (t[1] - t[0] if M > 1 else 1)
    monkeypatch.setattr(extrap, "time_nodes", nodes_far)
    assert not check_all()
    monkeypatch.setattr(extrap, "time_nodes", good_nodes)
    assert check_all()
