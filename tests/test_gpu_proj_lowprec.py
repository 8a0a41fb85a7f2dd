"""GPU parity of reduced-precision projection histories (FP32, FP16, BF16) against the oracle.

The reading both sides follow (the paper fixes no precision): column j is the
stored pair round(2^e x''), round(2^e b'') with the FP64 scale 1 / (nu 2^e),
e = 0 except for FP16 (largest stored magnitude in [2^14, 2^15), from the
raw pair at a restart and from the pair after the first Gram-Schmidt pass
otherwise); a rolling drop keeps each rotated slot's scale, except in FP16,
where slot i takes a bound-based scale.  All arithmetic besides the stored
values is FP64 on both sides, so the values a storage format holds are the
same numbers: after every update the library's raw stored columns (fetched
without the scale) must equal the oracle's bit for bit, and the scales must
agree to FP64 rounding.  Rounding differences in the FP64 remainders could
put a value on the other side of a rounding boundary of the format; with
random histories the remainders agree to about 1e-16 relative, so that has
probability ~1e-13 per value and any such flip is counted and reported.
With identical stored values the guesses are FP64 evaluations of the same
numbers and must agree to relative max(1e-12, 1e-14 a) (a = max nu0 / nu).
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce
from oracle import lowprec
from oracle import operator as op
from oracle.projection import Projection
from proj_replay import check_rows, replay

pytestmark = pytest.mark.gpu

METHODS = ["proj", "projqr", "proj_l2", "projqr_l2"]


def run(L, n, M, B, X, method, dtype, eps, sync=False):
    N = n ** 3
    meth, inner = L.parse_method(method)
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, meth, 0, L.DTYPES[dtype], eps, A, None, inner)
    Aop = op.Operator(n)
    ref = Projection(M, Aop, eps, dtype, "qr" if method.startswith("projqr") else "classic",
                     "l2" if inner == L.INNER_L2 else "A")
    try:
        rows, ref = replay(L, g, ref, B, X, eps, Aop, raw=True, sync=sync)
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
    return rows, ref


def check_storage(rows, dtype, label):
    """Stored values bit for bit, except where the two FP64 computations of a value round to
    different neighbours of the format.  A differing value may differ by one unit of the
    format at that value, or by the FP64 difference of the two computations: 64 u times the
    magnitudes the value was formed from -- the raw pair (x, A x) scaled to stored units for a
    new Gram-Schmidt column (its remainder is formed by cancellation), the column itself
    otherwise (u = 2^-53).  Differing values are counted.  Scales agree to FP64 rounding
    (1e-13 a, a = max nu0 / nu); FP16 values lie within 2^15."""
    flips, worst = 0, 0.0
    u = lowprec.UNIT_ROUNDOFF[dtype]
    for q, r in enumerate(rows):
        assert len(r["raw"]) == len(r["ref_cols"]), (label, q)
        a = max(1.0, r["amp"], r["amp_after"])
        nu = r["info"]["nu"]
        for j, ((xs, bs, sc), (S, T, sg)) in enumerate(zip(r["raw"], r["ref_cols"])):
            assert abs(sc - sg) <= 1e-13 * a * abs(sg), (label, q, j, sc, sg)
            for got, want in ((xs, S), (bs, T)):
                diff = got.view(np.uint64) != want.view(np.uint64)
                if diff.any():
                    mag = a * float(np.max(np.abs(want)))
                    if r["acc"] and j == len(r["raw"]) - 1 and nu > 0:
                        mag = max(mag, r["xmax"] / (sc * nu))      # raw pair in stored units (2^e = 1 / (sc nu))
                    dv = np.abs(got[diff] - want[diff])
                    ok = dv <= 2 * u * np.abs(want[diff]) + 64 * 2.0 ** -53 * mag
                    assert np.all(ok), (label, q, j, float(np.max(dv)), mag, int(diff.sum()))
                    flips += int(diff.sum())
                    worst = max(worst, float(np.max(dv / (2 * u * np.abs(want[diff]) + 2.0 ** -53 * mag))))
            if dtype == "f16":
                assert np.max(np.abs(xs)) <= 2 ** 15 and np.max(np.abs(bs)) <= 2 ** 15
                assert np.all(np.isfinite(xs)) and np.all(np.isfinite(bs))
    values = sum(2 * xs.size for r in rows for xs, _, _ in r["raw"])
    print(f"[storage] {label}: {values} stored values compared, {flips} differ "
          f"(largest difference {worst:.2f} of one unit of the format + u a max|column|)", flush=True)
    return flips


def check_guesses(rows, dtype, flips, label):
    """With identical stored values: the FP64 tolerance max(1e-12, 1e-14 a).
    Once a stored value differs, the histories differ by one unit of the format there and in
    what later Gram-Schmidt steps derive from it: guesses within 4 d u_s a."""
    if flips == 0:
        return check_rows(rows, label=label)
    u = lowprec.UNIT_ROUNDOFF[dtype]
    for q, r in enumerate(rows):
        assert r["acc"] == r["acc_ref"] and r["d"] == r["d_ref"], (label, q)
        if np.max(np.abs(r["want"])) > 0:
            err = np.max(np.abs(r["got"] - r["want"])) / np.max(np.abs(r["want"]))
            assert err <= 4 * max(1, r["d"]) * u * r["amp"], (label, q, err)
    print(f"[replay] {label}: {len(rows)} steps within 4 d u_s a ({flips} stored values differ)", flush=True)
    return len(rows)


def magnitudes(V, lo, hi):
    """Scale the q-th vector by 10^(lo + (hi - lo) * (q mod 5) / 4)."""
    return [v * 10.0 ** (lo + (hi - lo) * (q % 5) / 4.0) for q, v in enumerate(V)]


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("n", [7, 32])
def test_random_history_bit_exact(lib, method, dtype, n):
    """Random solutions of magnitudes 1e-2 .. 1e2 through restarts / drops: stored columns
    equal the oracle's, guesses to 1e-12 (7^3: a ragged tail only; 32^3: the z-marching fused
    apply, also for the FP16 restart pass)."""
    announce(f"{method} {dtype} random n={n}")
    M = 5
    N = n ** 3
    T = 2 * M + 2
    X = magnitudes(synth.random_vectors(32, T, N), -2, 2)
    B = synth.random_vectors(31, T, N)
    rows, ref = run(lib, n, M, B, X, method, dtype, 1e-6)
    flips = check_storage(rows, dtype, f"{method} {dtype} n={n}")
    values = sum(2 * xs.size for r in rows for xs, _, _ in r["raw"])
    assert flips <= 1e-4 * values
    assert check_guesses(rows, dtype, flips, f"{method} {dtype} n={n}") == T


@pytest.mark.parametrize("method", METHODS)
@pytest.mark.parametrize("mag", [1e-6, 1e6])
def test_f16_far_outside_range(lib, method, mag):
    """FP16 histories of solutions ~1e6 (beyond FP16's 65504) and ~1e-6 (below its smallest
    normal): the exponent of every pair puts it in range, stored bits equal the oracle's."""
    announce(f"{method} f16 magnitude {mag}")
    n, M = 9, 4
    T = 3 * M
    X = [v * mag for v in synth.random_vectors(41, T, n ** 3)]
    B = synth.random_vectors(42, T, n ** 3)
    rows, ref = run(lib, n, M, B, X, method, "f16", 1e-6)
    flips = check_storage(rows, "f16", f"{method} f16 mag={mag}")
    assert flips <= 2
    assert check_guesses(rows, "f16", flips, f"{method} f16 mag={mag}") == T


@pytest.mark.parametrize("method", METHODS)
def test_f16_nearly_dependent(lib, method):
    """Each solution is the previous one plus 1e-2 of a new direction, so every Gram-Schmidt
    remainder is ~1e-2 of the raw solution (nu / nu0 ~ 1e-2) and its exponent lies ~7 above
    the raw solution's: the scaled path the stored pairs take away from a restart."""
    announce(f"{method} f16 nearly dependent")
    n, M = 8, 6
    N = n ** 3
    T = 2 * M + 1
    R = synth.random_vectors(43, T, N)
    X = [R[0]]
    for q in range(1, T):
        X.append(X[-1] + 1e-2 * R[q])
    B = synth.random_vectors(44, T, N)
    rows, ref = run(lib, n, M, B, X, method, "f16", 1e-4)
    # exponent of each newly accepted Gram-Schmidt pair (scale = 1 / (nu 2^e)) against the one
    # its raw solution would take
    Aop = op.Operator(n)
    ups = []
    for r, x in zip(rows, X):
        if r["acc"] and r["d"] >= 2:
            e_col = int(round(-np.log2(r["raw"][-1][2] * r["info"]["nu"])))
            e_raw = lowprec.f16_scale_exp(max(np.max(np.abs(x)), np.max(np.abs(Aop(x)))))
            ups.append(e_col - e_raw)
    assert len(ups) >= M - 1 and min(ups) >= 4, ups
    flips = check_storage(rows, "f16", f"{method} f16 nearly dependent")
    assert flips <= 2
    assert check_guesses(rows, "f16", flips, f"{method} f16 nearly dependent") == T


@pytest.mark.parametrize("inner", ["A", "l2"])
def test_f16_rolling_rough_smooth(lib, inner):
    """Rolling drops over solutions alternating between rough and smooth vectors of magnitudes
    1e-3 .. 1e3: the rotated FP16 slots take the bound-based scales and stay in range; stored
    bits and scales equal the oracle's."""
    announce(f"projqr f16 rough/smooth inner={inner}")
    n, M, T = 7, 4, 14
    rng = np.random.default_rng(3)
    g = np.arange(1, n + 1) / (n + 1)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    X = []
    for t in range(T):
        mag = 10.0 ** rng.uniform(-3, 3)
        if t % 2 == 0:
            X.append(rng.standard_normal(n ** 3) * mag)
        else:
            k = rng.integers(1, 3, 3)
            s = np.sin(np.pi * (k[0] * x + k[1] * y + k[2] * z)).reshape(-1)
            X.append(mag * (s + 1e-3 * rng.standard_normal(n ** 3)))
    B = synth.random_vectors(45, T, n ** 3)
    method = "projqr" if inner == "A" else "projqr_l2"
    rows, ref = run(lib, n, M, B, X, method, "f16", 1e-6)
    assert ref.drops >= 8
    flips = check_storage(rows, "f16", f"{method} f16 rough/smooth")
    assert flips <= 2
    assert check_guesses(rows, "f16", flips, f"{method} f16 rough/smooth") == T


@pytest.mark.parametrize("method", ["proj", "projqr"])
@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_plane_wave_history(lib, method, dtype):
    """Smooth plane-wave solutions (32^3, K = 4, 30 steps) with the format's default threshold.
    Nearly dependent columns are formed by cancellation, so the two FP64 computations of a
    stored value can round to neighbouring values of the format; once one has, the histories
    differ there and later columns inherit it.  Two replays: (1) after every step the oracle
    takes the library's stored history, so each step is compared from the same state: stored
    values equal up to counted rounding-boundary differences (check_storage), guesses to the
    FP64 tolerance; (2) free-running: guesses within 4 d u_s a of the oracle's."""
    announce(f"{method} {dtype} plane waves 32^3")
    n, M, T = 32, 8, 30
    params = synth.plane_wave_params(0, 4)
    B = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(T, 0.01)]
    X = [op.dst_solve(b, n) for b in B]
    eps = {"f32": 1e-4, "f16": 1e-2, "bf16": 1e-2}[dtype]
    label = f"{method} {dtype} plane waves"
    rows, ref = run(lib, n, M, B, X, method, dtype, eps, sync=True)
    flips = check_storage(rows, dtype, label + " (same state each step)")
    total = sum(2 * xs.size for r in rows for xs, _, _ in r["raw"])
    assert flips <= 1e-3 * total
    assert check_rows(rows, label=label + " (same state each step)") == T
    rows, ref = run(lib, n, M, B, X, method, dtype, eps)
    u = lowprec.UNIT_ROUNDOFF[dtype]
    worst = 0.0
    for q, r in enumerate(rows):
        assert r["acc"] == r["acc_ref"] and r["d"] == r["d_ref"], q
        if q > 0 and np.max(np.abs(r["want"])) > 0:
            err = np.max(np.abs(r["got"] - r["want"])) / np.max(np.abs(r["want"]))
            bound = max(1e-12, 4 * max(1, r["d"]) * u * r["amp"])
            worst = max(worst, err / bound)
            assert err <= bound, (q, err, r["amp"])
    print(f"[replay] {label} (free-running): {T} steps, largest error {worst:.3f} of 4 d u_s a", flush=True)
