"""Pins of the oracle's reduced-precision projection storage and FP16 ring scaling.

The reading (oracle/projection.py, oracle/extrap.py): column j is a stored
pair S_j, T_j in the storage format with one FP64 scale sigma_j; a new pair
(x, b) of norm nu is stored as round(2^e x), round(2^e b) with
sigma = 1 / (nu 2^e), e = 0 except for FP16 (largest magnitude times 2^e in
[2^14, 2^15)); rotated columns of a rolling drop keep their slot's scale, or
in FP16 take a bound-based one.

Independent references used here: the raw solution itself (a restart stores
it, rounded), the A-orthogonal remainder of a new solution computed by normal
equations against the stored columns (not by Gram-Schmidt), ||x||_A from
x^T A x, IEEE rounding through numpy's float32 / float16 (lowprec's own pins
cover the BF16 bit manipulation), the FP16 range, and orthonormality.
"""
import numpy as np
import pytest

import synth
from oracle import lowprec
from oracle import operator as op
from oracle.extrap import ExtrapHistory, beta_ls_exact, to_f64
from oracle.projection import Projection

DT = ("f32", "f16", "bf16")
VARIANTS = [("classic", "A"), ("qr", "A"), ("classic", "l2"), ("qr", "l2")]


def A_of(n):
    return lambda v: op.apply_const(v, n)


def _is_format_value(v, dtype):
    return np.array_equal(lowprec.round_store(v, dtype), v)


def _round_bound(v, dtype):
    """Elementwise bound on |round(v) - v| for the storage format (FP16: plus half the
    subnormal spacing)."""
    u = lowprec.UNIT_ROUNDOFF[dtype]
    return u * np.abs(v) * (1 + 1e-12) + (2.0 ** -25 if dtype == "f16" else 0.0)


def _remainder_bf(Xs, Bs, A, x, inner):
    """The pair (x, A x) minus its projection on the stored pairs (Xs, Bs), by normal
    equations: y solves <C_i, A x - sum_j y_j B_j> = 0 for all i (C = X for the A inner
    product, B for l2), the condition that twice-iterated Gram-Schmidt meets to second
    order in the columns' departure from orthonormality.  Returns r = x - Xs^T y,
    w = A x - Bs^T y and the norm of the pair."""
    Xs, Bs = np.asarray(Xs), np.asarray(Bs)
    Ax = A(x)
    C = Xs if inner == "A" else Bs
    y = np.linalg.solve(C @ Bs.T, C @ Ax)
    r, w = x - y @ Xs, Ax - y @ Bs
    nu = np.sqrt(r @ w) if inner == "A" else np.linalg.norm(w)
    return r, w, nu, y


def _rough_smooth_history(seed, T, n):
    """Solutions alternating between rough (random) and smooth (low-frequency) vectors of
    magnitudes 1e-3 .. 1e3: the true columns' largest magnitudes differ a lot, which is
    what a rolling drop has to scale for in FP16."""
    rng = np.random.default_rng(seed)
    g = np.arange(1, n + 1) / (n + 1)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    out = []
    for t in range(T):
        mag = 10.0 ** rng.uniform(-3, 3)
        if t % 2 == 0:
            out.append(rng.standard_normal(n ** 3) * mag)
        else:
            k = rng.integers(1, 3, 3)
            s = np.sin(np.pi * (k[0] * x + k[1] * y + k[2] * z)).reshape(-1)
            out.append(mag * (s + 1e-3 * rng.standard_normal(n ** 3)))
    return out


# ---------------------------------------------------------------- restart column
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("inner", ["A", "l2"])
def test_restart_stores_the_rounded_solution(dtype, inner):
    """A restart stores the raw solution itself (times 2^e), rounded, with scale
    1 / (2^e ||x||)."""
    n = 5
    A = A_of(n)
    for mag in (1e-6, 1.0, 1e6):
        x = synth.random_vectors(3, 1, n ** 3)[0] * mag
        P = Projection(3, A, 1e-6, dtype, "classic", inner)
        assert P.update(x)
        Ax = A(x)
        e = P.last_exp
        if dtype == "f16":
            m = max(np.max(np.abs(x)), np.max(np.abs(Ax)))
            assert 2 ** 14 <= m * 2.0 ** e < 2 ** 15
        else:
            assert e == 0
        np.testing.assert_array_equal(P.S[0], lowprec.round_store(np.ldexp(x, e), dtype))
        np.testing.assert_array_equal(P.T[0], lowprec.round_store(np.ldexp(Ax, e), dtype))
        nrm = np.sqrt(x @ Ax) if inner == "A" else np.linalg.norm(Ax)
        assert abs(P.sig[0] * 2.0 ** e * nrm - 1.0) <= 1e-14
        assert np.all(np.isfinite(P.S[0])) and np.all(np.isfinite(P.T[0]))


# ---------------------------------------------------------------- Gram-Schmidt columns
@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("variant,inner", VARIANTS)
def test_new_column_is_the_rounded_remainder(dtype, variant, inner):
    """Every accepted Gram-Schmidt column is the rounded (2^e-scaled) remainder of the raw
    solution after projection on the stored columns, and its scale is 1 / (2^e nu)."""
    n, M = 5, 4
    A = A_of(n)
    V = synth.random_vectors(40, 2 * M + 3, n ** 3)
    for q, v in enumerate(V):
        V[q] = v * 10.0 ** (q % 5 - 2)
    P = Projection(M, A, 1e-6, dtype, variant, inner)
    checked = 0
    for v in V:
        restart = P.d == 0 or (variant == "classic" and P.d >= M)
        drop = variant == "qr" and P.d == M
        prev = None if (restart or drop) else (np.stack(P.X), np.stack(P.B))
        assert P.update(v)
        if prev is None:
            continue
        r, w, nu, y = _remainder_bf(*prev, A, v, inner)
        e = P.last_exp
        S, T, sg = P.S[-1], P.T[-1], P.sig[-1]
        assert _is_format_value(S, dtype) and _is_format_value(T, dtype)
        # stored = round(2^e r): the format's rounding, plus the second-order difference
        # between Gram-Schmidt and the normal equations (u_s^2 |y| in units of the columns)
        u = lowprec.UNIT_ROUNDOFF[dtype]
        for got, ref, cols in ((S, r, prev[0]), (T, w, prev[1])):
            ref = np.ldexp(ref, e)
            slack = (64 * u * u * np.abs(y).sum() * np.max(np.abs(cols)) * 2.0 ** e
                     + 1e-12 * np.max(np.abs(ref)))
            assert np.all(np.abs(got - ref) <= _round_bound(ref, dtype) + slack)
        assert abs(sg * 2.0 ** e * nu - 1.0) <= 64 * u * u * P.amplification + 1e-12
        if dtype == "f16":
            m = max(np.max(np.abs(S)), np.max(np.abs(T)))
            assert 2 ** 14 * (1 - 1e-6) <= m <= 2 ** 15
        else:
            assert e == 0
        checked += 1
    assert checked >= M - 1


@pytest.mark.parametrize("dtype", DT)
@pytest.mark.parametrize("variant,inner", VARIANTS)
def test_stored_values_and_orthonormality(dtype, variant, inner):
    """Stored values are values of the format; the true columns are orthonormal in the
    variant's inner product to a few units of the format's roundoff (random history, so
    the amplification max nu0/nu stays near 1), and B = A X to the same order."""
    n, M = 6, 5
    A = A_of(n)
    V = synth.random_vectors(50, 3 * M, n ** 3)
    P = Projection(M, A, 1e-6, dtype, variant, inner)
    u = lowprec.UNIT_ROUNDOFF[dtype]
    for v in V:
        P.update(v)
        X, B = np.stack(P.X), np.stack(P.B)
        for S, T in zip(P.S, P.T):
            assert _is_format_value(S, dtype) and _is_format_value(T, dtype)
        G = X @ B.T if inner == "A" else B @ B.T
        a = P.amplification
        assert np.max(np.abs(G - np.eye(P.d))) <= 16 * u * a
        AX = np.stack([A(x) for x in X])
        assert np.max(np.abs(AX - B)) <= 16 * u * a * np.max(np.abs(B))


def test_fp64_storage_unchanged_by_the_reading():
    """With FP64 storage the pair is the unrounded remainder and sigma = 1/nu: the true
    columns equal x''/nu to rounding, so the FP64 guesses are those of the textbook form."""
    n, M = 5, 4
    A = A_of(n)
    V = synth.random_vectors(60, 9, n ** 3)
    P = Projection(M, A, 1e-10, "f64")
    for v in V[:4]:
        prev = None if P.d == 0 else (np.stack(P.X), np.stack(P.B))
        P.update(v)
        if prev is not None:
            r, _, nu, _ = _remainder_bf(*prev, A, v, "A")
            assert np.max(np.abs(P.X[-1] - r / nu)) <= 1e-12 * np.max(np.abs(r / nu))


# ---------------------------------------------------------------- FP16 rolling drop
@pytest.mark.parametrize("inner", ["A", "l2"])
def test_f16_rolling_drop_stays_in_range(inner):
    """Rolling drops over rough / smooth solutions of very different magnitudes: every
    stored value stays within 2^15 (finite), the rotated columns are the rounded exact
    rotations at their slot's new scale, and the guesses stay close to FP64 storage."""
    n, M = 7, 4
    A = A_of(n)
    V = _rough_smooth_history(3, 14, n)
    P = Projection(M, A, 1e-6, "f16", "qr", inner)
    R64 = Projection(M, A, 1e-6, "f64", "qr", inner)
    b = synth.random_vectors(9, 1, n ** 3)[0]
    for v in V:
        if P.d == M:
            # the exact rotation of the current true columns, from a copy of the state
            import copy

            Q = copy.deepcopy(P)
            Xr, Br, rots = Q._drop_oldest()
            sc = Q._rotated_scales(rots)
        else:
            Xr = None
        P.update(v)
        R64.update(v)
        for S, T in zip(P.S, P.T):
            assert np.max(np.abs(S)) <= 2 ** 15 and np.max(np.abs(T)) <= 2 ** 15
        if Xr is not None:
            for i, (x, bb, s) in enumerate(zip(Xr, Br, sc)):
                assert P.sig[i] == s
                assert np.all(np.abs(P.S[i] - x / s) <= _round_bound(x / s, "f16") + 1e-12 * 2 ** 15)
                assert np.all(np.abs(P.T[i] - bb / s) <= _round_bound(bb / s, "f16") + 1e-12 * 2 ** 15)
        # FP16 rounding of the columns, amplified by max nu0/nu (measured: <= 2.7 u a here)
        g16, g64 = P.form(b), R64.form(b)
        assert np.max(np.abs(g16 - g64)) <= 16 * 2.0 ** -11 * P.amplification * np.max(np.abs(g64))
    assert P.drops >= 8


# ---------------------------------------------------------------- planted mistakes
def test_pins_catch_planted_storage_mistakes(monkeypatch):
    """Normalise-then-round, an FP16 exponent off by one, an exponent taken from x alone,
    and FP16 rotated columns kept at their old scale each break a pin above."""
    def run(fn, *args):
        try:
            fn(*args)
            return True
        except AssertionError:
            return False

    assert run(test_restart_stores_the_rounded_solution, "f32", "A")
    assert run(test_new_column_is_the_rounded_remainder, "bf16", "classic", "A")
    assert run(test_new_column_is_the_rounded_remainder, "f16", "classic", "A")
    assert run(test_f16_rolling_drop_stays_in_range, "A")

    good_put_new = Projection._put_new
    good_exp = Projection._exp_for
    good_scales = Projection._rotated_scales

    def normalise_then_round(self, x, b, nu, e):
        self._put(np.ldexp(x / nu, e), np.ldexp(b / nu, e), float(np.ldexp(1.0, -e)))

    monkeypatch.setattr(Projection, "_put_new", normalise_then_round)
    assert not run(test_restart_stores_the_rounded_solution, "f32", "A")
    assert not run(test_new_column_is_the_rounded_remainder, "bf16", "classic", "A")
    monkeypatch.setattr(Projection, "_put_new", good_put_new)

    monkeypatch.setattr(Projection, "_exp_for", lambda self, x, b: good_exp(self, x, b) + 1
                        if self.dtype == "f16" else 0)
    assert not run(test_new_column_is_the_rounded_remainder, "f16", "classic", "A")
    monkeypatch.setattr(Projection, "_exp_for", lambda self, x, b: lowprec.f16_scale_exp(
        float(np.max(np.abs(x)))) if self.dtype == "f16" else 0)
    assert not run(test_restart_stores_the_rounded_solution, "f16", "A")
    monkeypatch.setattr(Projection, "_exp_for", good_exp)

    monkeypatch.setattr(Projection, "_rotated_scales", lambda self, rots: list(self.sig[: len(rots)]))
    assert not run(test_f16_rolling_drop_stays_in_range, "A")
    monkeypatch.setattr(Projection, "_rotated_scales", good_scales)
    assert run(test_f16_rolling_drop_stays_in_range, "A")


# ---------------------------------------------------------------- FP16 extrapolation ring
@pytest.mark.parametrize("mag", [1e-6, 1e-2, 1.0, 1e6])
def test_f16_ring_scaled_store_and_exactness(mag):
    """FP16 ring slots hold round(2^e x) with max |x| 2^e in [2^14, 2^15): in range for
    solutions of any size, within FP16's relative roundoff of x, and the extrapolated guess
    of a degree-2 sequence is exact to the rounding bound Lambda u max |x|."""
    rng = np.random.default_rng(7)
    N, M, m = 4000, 8, 2
    v = [rng.standard_normal(N) * mag for _ in range(3)]
    H = ExtrapHistory(M, m, "f16")
    xs = []
    for i in range(M + 1):
        t = i * 0.25
        xs.append(v[0] + t * v[1] + t * t * v[2])
    for x in xs[:M]:
        H.update(x)
        e = H.exps[-1]
        stored = np.ldexp(H.hist[-1], e)
        assert 2 ** 14 <= np.max(np.abs(stored)) <= 2 ** 15
        assert _is_format_value(stored, "f16")
        assert np.all(np.abs(H.hist[-1] - x) <= np.ldexp(_round_bound(np.ldexp(x, e), "f16"), -e))
    beta = to_f64(beta_ls_exact(m, M))
    lam = float(np.sum(np.abs(beta)))
    got = H.form(N=N)
    scale = max(np.max(np.abs(x)) for x in xs)
    assert np.max(np.abs(got - xs[M])) <= lam * 2.0 ** -11 * scale * 1.01 + 1e-12 * scale


def test_f16_ring_pins_catch_an_unscaled_store(monkeypatch):
    from oracle import extrap

    monkeypatch.setattr(lowprec, "f16_scale_exp", lambda m: 0)
    for mag in (1e-6, 1e6):
        with pytest.raises(AssertionError):
            test_f16_ring_scaled_store_and_exactness(mag)
    assert extrap is not None
