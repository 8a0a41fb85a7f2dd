"""GPU parity of the extrapolation path (ring store + extrap_form) against the oracle.

Tolerances: FP64 history -- guesses within relative 1e-12 of the oracle
(inf-norm, relative to the oracle guess); stored FP64/FP32/FP16/BF16 values
bit-exact (a deterministic rounding); FP32-accumulated guesses from
reduced-precision history within the rigorous FP32 summation bound around
the oracle's exact evaluation of the stored values.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, assert_within, dev, host, rel_inf
from oracle import extrap, lowprec

pytestmark = pytest.mark.gpu

RAGGED_N = [1, 2, 3, 4, 5, 7, 1023, 1027, 32 ** 3, 33 ** 3 + 2]


def _seq(lib, N, M, m, dtype, steps, seed, sparse=False):
    import torch

    L = lib
    method = L.SPEXTRAP if sparse else (L.EXTRAP if M > 1 or m > 0 else L.LAST)
    g = L.guess_create_ex(N, M, method, m, L.DTYPES[dtype])
    ref = extrap.ExtrapHistory(M, m, dtype, sparse=sparse)
    X = synth.random_vectors(seed, steps, N) * np.linspace(0.5, 2.0, steps)[:, None]
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    out = []
    try:
        for s in range(steps):
            L.guess_form(g, None, x0)
            out.append((host(x0), ref.form(N=N), list(ref.hist)))
            xd = dev(X[s])
            L.guess_update(g, xd)
            ref.update(X[s])
        info = L.guess_get_info(g)
    finally:
        L.guess_destroy(g)
    return out, info


@pytest.mark.parametrize("N", RAGGED_N)
def test_f64_guesses_match_oracle(lib, N):
    announce(f"extrap f64 N={N}")
    M, m = 8, 2
    res, info = _seq(lib, N, M, m, "f64", 12, seed=N)
    assert info["count"] == M and info["head"] == 12 % (M + 1)   # FP64 rings keep a spare slot
    for q, (got, want, _) in enumerate(res):
        if q == 0:
            assert not got.any()
        else:
            assert rel_inf(got, want) <= 1e-12, (N, q)


@pytest.mark.parametrize("M,m", [(1, 0), (2, 1), (4, 2), (8, 1), (8, 3), (16, 3), (16, 4), (5, 4)])
def test_f64_all_shapes(lib, M, m):
    announce(f"extrap f64 M={M} m={m}")
    res, _ = _seq(lib, 4099, M, m, "f64", M + 3, seed=100 + M + m)
    for q, (got, want, _) in enumerate(res[1:], start=1):
        assert rel_inf(got, want) <= 1e-12, (M, m, q)


@pytest.mark.parametrize("M,m", [(8, 2), (8, 1), (8, 3), (16, 2), (16, 4), (4, 3), (3, 0), (1, 0)])
@pytest.mark.parametrize("N", [5, 1027, 33 ** 3 + 2])
def test_sparse_f64_matches_oracle(lib, M, m, N):
    """Sparse extrapolation (§3.3): the m+1 selected solutions, oldest first."""
    announce(f"spextrap f64 M={M} m={m} N={N}")
    res, info = _seq(lib, N, M, m, "f64", M + 3, seed=500 + M + m, sparse=True)
    for q, (got, want, _) in enumerate(res[1:], start=1):
        assert rel_inf(got, want) <= 1e-12, (M, m, q)
    # only the selected slots are read: (m+1) stored vectors + the FP64 guess
    assert info["form_bytes"] == N * (8.0 * (min(m, M - 1) + 1) + 8.0)


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_sparse_lowprec_within_fp32_bound(lib, dtype):
    announce(f"spextrap {dtype}")
    M, m = 8, 2
    res, _ = _seq(lib, 5003, M, m, dtype, M + 2, seed=9, sparse=True)
    u = 2.0 ** -24
    for q, (got, want, hist) in enumerate(res[1:], start=1):
        k = len(hist)
        beta = extrap.to_f64(extrap.beta_sparse_exact(min(m, k - 1), k))
        mag = sum(abs(b) * np.abs(h) for b, h in zip(beta, hist))
        bound = (m + 2) * u * mag + u * np.abs(want) + 1e-300
        assert_within(got, want, bound, hist, f"spextrap {dtype} step {q}")


@pytest.mark.parametrize("dtype", ["f64", "f32", "f16", "bf16"])
def test_ring_store_bit_exact(lib, dtype):
    """Stored values equal the oracle's two-step round-to-nearest-even (FP16: of 2^e x, e from
    max |x|; here one element of 20000 fixes e = 0 so the crafted ties stay ties)."""
    import torch

    announce(f"ring store {dtype}")
    L = lib
    # ties, subnormals, overflow, signed zero, and double-rounding cases
    # (FP64 -> FP32 lands exactly on an FP16 / BF16 midpoint)
    special = [1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -11, 1 + 3 * 2 ** -11, 1 + 2 ** -24,
               1 + 3 * 2 ** -24, 2.0 ** -24, 3e-8, -0.0, 0.0, 1e-40, -2.5,
               1 + 2 ** -11 + 2 ** -30, -(1 + 2 ** -11 + 2 ** -30), 1 + 2 ** -8 + 2 ** -30,
               3 * (1 + 2 ** -11) + 2 ** -28]
    if dtype == "f16":
        special = [20000.0] + special + [2 ** 14 + 2 ** 3 + 2 ** -20]
    else:
        special += [65504.0, 65519.0, 3.0e38, 1e300 if dtype == "f64" else 1.0]
    special = np.array(special)
    for N in (1, 3, 5, 1030, 70001):
        v = synth.random_vectors(N, 1, N)[0] * 10.0 ** np.random.default_rng(N).integers(-6, 4, N)
        if dtype == "f16":
            v = np.clip(v, -19000.0, 19000.0)
        v[: min(N, len(special))] = special[: min(N, len(special))]
        g = L.guess_create_ex(N, 2, L.EXTRAP, 0, L.DTYPES[dtype])
        try:
            L.guess_update(g, dev(v))
            out = torch.empty(N, dtype=torch.float64, device="cuda")
            L.guess_history_get(g, 0, 0, out)
            got = host(out)
            raw = torch.empty(N, dtype=torch.float64, device="cuda")
            scale = L.guess_history_raw(g, 0, 0, raw)
            got_raw = host(raw)
        finally:
            L.guess_destroy(g)
        e = lowprec.f16_scale_exp(float(np.max(np.abs(v)))) if dtype == "f16" else 0
        want = lowprec.round_store(v, dtype, e)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (dtype, N)
        assert np.array_equal(got_raw.view(np.uint64), lowprec.decode(lowprec.stored_bits(v, dtype, e), dtype).view(
            np.uint64)), (dtype, N)
        assert scale == 2.0 ** -e, (dtype, N, scale, e)


@pytest.mark.parametrize("mags", [(1e6, 1e6), (1e-6, 1e-6), (1e-6, 1e6), (1.0, 3e4)])
@pytest.mark.parametrize("N", [1027, 70001])
def test_f16_ring_scaled_slots(lib, mags, N):
    """FP16 slots hold round(2^e x), e from max |x| (max |x| 2^e in [2^14, 2^15)), so solutions
    far outside FP16's range (|x| ~ 1e6, 1e-6) are stored with FP16's relative precision: the
    raw stored bits and each slot's scale 2^-e equal the oracle's, and the guesses (weights
    beta_j 2^-e_j, FP32 accumulation) meet the FP32 summation bound around the oracle's exact
    evaluation of the stored values.  Magnitudes sweep geometrically from the first to the
    second value, so the exponent of the next solution differs from the previous one's (the
    slot is stored again) or not (one pass), and the update's byte count says which."""
    import torch

    announce(f"extrap f16 scaled slots mags={mags} N={N}")
    L = lib
    M, m, T = 8, 2, 12
    g = L.guess_create_ex(N, M, L.EXTRAP, m, L.F16)
    ref = extrap.ExtrapHistory(M, m, "f16")
    rng = np.random.default_rng([N, int(np.log10(mags[0]) + 10), int(np.log10(mags[1]) + 10)])
    base = rng.standard_normal(N)
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    raw = torch.empty(N, dtype=torch.float64, device="cuda")
    u = 2.0 ** -24
    fixes = 0
    try:
        for s in range(T):
            mag = mags[0] * (mags[1] / mags[0]) ** (s / (T - 1))
            x = mag * (base + 0.1 * s * rng.standard_normal(N))
            if s > 0:
                L.guess_form(g, None, x0)
                got, want = host(x0), ref.form(N=N)
                k = len(ref.hist)
                beta = extrap.to_f64(extrap.beta_ls_exact(min(m, k - 1), k))
                magsum = sum(abs(b) * np.abs(h) for b, h in zip(beta, ref.hist))
                assert_within(got, want, (k + 1) * u * magsum + u * np.abs(want) + 1e-300, ref.hist,
                              f"f16 scaled step {s}")
            prev_e = ref.exps[-1] if ref.exps else 0
            L.guess_update(g, dev(x))
            ref.update(x)
            e = ref.exps[-1]
            info = L.guess_get_info(g)
            fixed = e != prev_e
            fixes += fixed
            assert info["update_bytes"] == N * 10.0 * (2 if fixed else 1), (s, e, prev_e)
            scale = L.guess_history_raw(g, 0, info["count"] - 1, raw)
            assert scale == 2.0 ** -e, (s, scale, e)
            want_raw = lowprec.decode(lowprec.stored_bits(x, "f16", e), "f16")
            assert np.array_equal(host(raw).view(np.uint64), want_raw.view(np.uint64)), s
            assert np.all(np.isfinite(want_raw)) and np.max(np.abs(want_raw)) <= 2 ** 15
    finally:
        L.guess_destroy(g)
    if mags[0] == mags[1]:
        assert fixes < T // 2      # the first store, and the steps whose max |x| crosses a power of two
    else:
        assert fixes >= 3


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
@pytest.mark.parametrize("M,m", [(8, 2), (4, 1), (16, 3)])
def test_lowprec_guess_within_fp32_bound(lib, dtype, M, m):
    """|x0_gpu - sum beta_j h_j| <= (k+1) 2^-24 sum |beta_j h_j| + 2^-24 |x0| (h stored values)."""
    announce(f"extrap {dtype} M={M} m={m}")
    res, _ = _seq(lib, 5003, M, m, dtype, M + 2, seed=7)
    u = 2.0 ** -24
    for q, (got, want, hist) in enumerate(res[1:], start=1):
        k = len(hist)
        beta = extrap.to_f64(extrap.beta_ls_exact(min(m, k - 1), k))
        mag = sum(abs(b) * np.abs(h) for b, h in zip(beta, hist))
        bound = (k + 1) * u * mag + u * np.abs(want) + 1e-300
        assert_within(got, want, bound, hist, f"{dtype} M={M} m={m} step {q}")


def test_lowprec_error_vs_fp64_history(lib):
    """Guess error against the unrounded FP64 history stays within Lambda u_s max|x|."""
    announce("extrap low precision vs f64")
    N, M, m = 2048, 8, 2
    lam = float(extrap.lebesgue(extrap.beta_ls_exact(m, M)))
    res64, _ = _seq(lib, N, M, m, "f64", M + 1, seed=3)
    for dtype in ("f32", "f16", "bf16"):
        res, _ = _seq(lib, N, M, m, dtype, M + 1, seed=3)
        got, ref = res[-1][0], res64[-1][0]
        X = synth.random_vectors(3, M + 1, N) * np.linspace(0.5, 2.0, M + 1)[:, None]
        xmax = np.abs(X).max()
        u = lowprec.UNIT_ROUNDOFF[dtype]
        assert np.max(np.abs(got - ref)) <= (lam * u + (M + 1) * 2.0 ** -24 * lam) * xmax * 1.01, dtype


def test_reset_and_zero_guess(lib):
    import torch

    announce("extrap reset / zero method")
    L = lib
    N = 100
    g = L.guess_create(N, 4, L.EXTRAP, 1)
    z = L.guess_create(N, 1, L.ZERO, 0)
    x0 = torch.full((N,), 7.0, dtype=torch.float64, device="cuda")
    try:
        L.guess_update(g, dev(np.ones(N)))
        L.guess_form(g, None, x0)
        assert np.all(host(x0) == 1.0)
        L.guess_reset(g)
        assert L.guess_get_info(g)["count"] == 0
        L.guess_form(g, None, x0)
        assert not host(x0).any()
        x0.fill_(3.0)
        L.guess_form(z, None, x0)
        L.guess_update(z, x0)
        assert not host(x0).any()
    finally:
        L.guess_destroy(g)
        L.guess_destroy(z)


@pytest.mark.parametrize("method", ["extrap", "spextrap", "last"])
def test_in_place_sequence_matches_copy(lib, method):
    """Solving in the ring's spare slot (guess_next_slot): the same guesses, solutions and PCG
    counts as the copying update, bit for bit, and the update moves nothing."""
    import torch

    from paper_2009_10863_amd.sequence import GuessSequence, Operator, PlaneWaveRHS

    announce(f"in-place {method}")
    L = lib
    n, M, T = 16, 6, 12
    op = Operator(n)
    rhs = PlaneWaveRHS(synth.plane_wave_params(2, 4), n)
    gc = GuessSequence(op.N, M, method, 2, "f64", 0.0, op)
    gi = GuessSequence(op.N, M, method, 2, "f64", 0.0, op, in_place=True)
    b = torch.empty(op.N, dtype=torch.float64, device="cuda")
    xc = torch.empty_like(b)
    try:
        for k in range(1, T + 1):
            rhs(0.01 * k, b)
            gc.form(b, xc)
            xi = gi.slot()
            gi.form(b, xi)
            assert torch.equal(xc, xi), k
            s1 = op.solve(b, xc, 1e-10)
            s2 = op.solve(b, xi, 1e-10)
            assert s1[0] == s2[0] == L.OK and s1[1] == s2[1], k
            assert torch.equal(xc, xi), k
            gc.update(xc)
            gi.update(xi)
            assert gi.info()["update_bytes"] == 0.0 and gc.info()["update_bytes"] > 0.0
        for j in range(gc.info()["count"]):
            assert torch.equal(gc.history(j), gi.history(j)), j
    finally:
        gc.close()
        gi.close()
        op.close()
