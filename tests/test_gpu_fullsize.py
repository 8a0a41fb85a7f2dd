"""Parity at the benchmark's full size (256^3 = 16,777,216 unknowns, M = 8).

Same library launch configuration as bench.py.  The extrapolated guess is
checked at sampled unknowns (the oracle evaluates sum_j beta_j h_j one
unknown at a time); the projection guess of the benchmark's PROJ(8) is
replayed against the full FP64 oracle on random (well-conditioned)
histories.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, assert_within, dev, host, rel_inf
from oracle import extrap, lowprec
from oracle import operator as op
from oracle.projection import Projection

pytestmark = pytest.mark.gpu

n = 256
N = n ** 3


def sample_idx():
    idx = np.random.default_rng(11).integers(0, N, 8192)
    return np.unique(np.concatenate([idx, [0, 1, 2, 3, N - 4, N - 3, N - 2, N - 1, n * n, n * n - 1]]))


@pytest.mark.parametrize("dtype", ["f64", "f32", "bf16", "f16"])
def test_extrap_256_sampled(lib, dtype):
    import torch

    announce(f"extrap 256^3 M=8 m=2 {dtype}")
    L = lib
    M, m = 8, 2
    idx = sample_idx()
    g = L.guess_create_ex(N, M, L.EXTRAP, m, L.DTYPES[dtype])
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    hist = []
    try:
        rng = np.random.default_rng(5)
        for s in range(M + 1):
            v = rng.standard_normal(N) * (1.0 + 0.1 * s)
            L.guess_update(g, dev(v))
            hist.append(lowprec.round_store(v[idx], dtype))
            hist = hist[-M:]
        L.guess_form(g, None, x0)
        got = host(x0)[idx]
    finally:
        L.guess_destroy(g)
    beta = extrap.to_f64(extrap.beta_ls_exact(m, M))
    want = extrap.form(hist, beta)
    if dtype == "f64":
        assert rel_inf(got, want) <= 1e-12
    else:
        mag = sum(abs(b) * np.abs(h) for b, h in zip(beta, hist))
        assert_within(got, want, (M + 1) * 2.0 ** -24 * mag + 2.0 ** -24 * np.abs(want), hist, dtype)


@pytest.mark.parametrize("method", ["proj", "projqr"])
def test_proj_256_m8_replay(lib, method):
    """The benchmark's projection configuration, PROJ(8) at 256^3, replayed against the FP64
    oracle on ten random solutions and right-hand sides: the history grows to d = 8 (the
    Gram-Schmidt kernels at every d up to 7), then the classic variant restarts and the rolling
    one drops its oldest solution twice (the fused drop at d = 8).  Random histories keep the
    amplification max nu0 / nu near 1, so every guess is held to relative 1e-12, and the
    library's nu0 and nu to 1e-12 of the oracle's."""
    import torch

    announce(f"{method} 256^3 M=8 random replay")
    L = lib
    M, T = 8, 10
    meth, _ = L.parse_method(method)
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, meth, 0, L.F64, 1e-6, A)
    Aop = op.Operator(n)
    ref = Projection(M, Aop, 1e-6, "f64", "qr" if method == "projqr" else "classic", "A")
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(8)
    ds = []
    try:
        for s in range(T):
            b = rng.standard_normal(N)
            x = rng.standard_normal(N)
            L.guess_form(g, dev(b), x0)
            want = ref.form(b)
            got = host(x0)
            if s == 0:
                assert not got.any()
            else:
                err = rel_inf(got, want)
                print(f"[replay] {method} 256^3 step {s}: d = {ref.d}, relative error {err:.2e}", flush=True)
                assert err <= 1e-12, (s, err)
            L.guess_update(g, dev(x))
            ref.update(x)
            info = L.guess_get_info(g)
            assert info["count"] == ref.d and info["last_accepted"] == 1
            assert abs(info["nu0"] - ref.last_nu0) <= 1e-12 * ref.last_nu0
            assert abs(info["nu"] - ref.last_nu) <= 1e-12 * ref.last_nu
            ds.append(ref.d)
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
    if method == "proj":
        assert ds == [1, 2, 3, 4, 5, 6, 7, 8, 1, 2] and info["restarts"] == 2
    else:
        assert ds == [1, 2, 3, 4, 5, 6, 7, 8, 8, 8] and info["drops"] == 2


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_spextrap_256_sampled(lib, dtype):
    """Sparse extrapolation SPEXTRAP(2,8) at full size: only the pivot slots enter the guess."""
    import torch

    announce(f"spextrap 256^3 M=8 m=2 {dtype}")
    L = lib
    M, m = 8, 2
    idx = sample_idx()
    g = L.guess_create_ex(N, M, L.SPEXTRAP, m, L.DTYPES[dtype])
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    hist = []
    try:
        rng = np.random.default_rng(6)
        for s in range(M + 2):
            v = rng.standard_normal(N) * (1.0 + 0.1 * s)
            L.guess_update(g, dev(v))
            hist.append(lowprec.round_store(v[idx], dtype))
            hist = hist[-M:]
        L.guess_form(g, None, x0)
        got = host(x0)[idx]
    finally:
        L.guess_destroy(g)
    beta = extrap.to_f64(extrap.beta_sparse_exact(m, M))
    assert np.count_nonzero(beta) == m + 1
    want = extrap.form(hist, beta)
    if dtype == "f64":
        assert rel_inf(got, want) <= 1e-12
    else:
        mag = sum(abs(b) * np.abs(h) for b, h in zip(beta, hist))
        assert_within(got, want, (M + 1) * 2.0 ** -24 * mag + 2.0 ** -24 * np.abs(want), hist, dtype)


@pytest.mark.parametrize("method", ["projqr", "proj_l2", "projqr_l2"])
def test_projection_variants_256_m8_properties(lib, method):
    """The bench's configuration (256^3, M = 8) for the rolling window (two drops) and the l2
    forms, ten random solutions: the stored history is orthonormal in the variant's inner product
    with B = A X, and the guess meets the variant's Galerkin condition against the retained raw
    solutions (A form: raw^T r = 0; l2 form: (A raw)^T r = 0, r = b - A x0).  The FP64 oracle
    replays the same variants at 32^3 (test_gpu_proj_variants); at this size it would take
    minutes per case, so properties that hold at any size are checked instead."""
    import torch

    announce(f"{method} 256^3 M=8 properties")
    L = lib
    M, T = 8, 10
    meth, inner = L.parse_method(method)
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, meth, 0, L.F64, 1e-6, A, None, inner)
    S = L.stream_handle()
    raw = torch.empty((T, N), dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(12)
    try:
        for s in range(T):
            raw[s].normal_(generator=gen)
            L.guess_update(g, raw[s])
        info = L.guess_get_info(g)
        d = info["count"]
        rolling = method.startswith("projqr")
        assert d == (M if rolling else T - M)
        assert info["drops"] == (T - M if rolling else 0)
        window = raw[T - d:].contiguous()
        X = torch.empty((d, N), dtype=torch.float64, device="cuda")
        B = torch.empty((d, N), dtype=torch.float64, device="cuda")
        for j in range(d):
            L.guess_history_get(g, 0, j, X[j])
            L.guess_history_get(g, 1, j, B[j])
        l2 = inner == L.INNER_L2
        G = np.stack([L.vec_multidot(N, d, B if l2 else X, B[j].contiguous(), S) for j in range(d)])
        assert np.max(np.abs(G - np.eye(d))) <= 1e-12
        AX = torch.empty(N, dtype=torch.float64, device="cuda")
        for j in range(d):
            L.op_apply(A, X[j], AX)
            assert float(torch.max(torch.abs(AX - B[j]))) <= 1e-12 * float(torch.max(torch.abs(B[j])))
        b = torch.empty(N, dtype=torch.float64, device="cuda").normal_(generator=gen)
        x0 = torch.empty_like(b)
        L.guess_form(g, b, x0)
        L.op_apply(A, x0, AX)
        r = (b - AX).contiguous()
        if l2:
            W = torch.empty_like(window)
            for j in range(d):
                L.op_apply(A, window[j], W[j])
        else:
            W = window
        gal = np.array(L.vec_multidot(N, d, W, r, S))
        scale = np.array([float(torch.linalg.vector_norm(W[j])) for j in range(d)]) * float(
            torch.linalg.vector_norm(b))
        assert np.max(np.abs(gal) / scale) <= 1e-10
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)



@pytest.mark.parametrize("method,dtype", [("proj", "f32"), ("proj", "f16"), ("proj", "bf16"), ("projqr", "f16")])
def test_proj_256_lowprec_replay(lib, method, dtype):
    """Reduced-precision PROJ(8) at the benchmark's size against the oracle: seven random
    solutions of growing magnitude and random right-hand sides.  After every update the newest
    stored column equals the oracle's bit for bit, except where the two FP64 remainders round
    to different neighbours of the format (a difference within one unit of the format plus
    64 u times the raw pair in stored units; at most 1e-6 of the values); the oracle then takes
    the library's stored history, so every guess is compared from identical states and held
    to 1e-12 relative -- the per-format guess error against the oracle at 256^3.  The FP16
    rolling window runs ten steps, so that its last two updates drop the oldest column (the
    write pass then reduces M + 1 values per workgroup)."""
    import torch

    from proj_replay import resync

    announce(f"{method} 256^3 M=8 {dtype} random replay")
    L = lib
    M, T = 8, (10 if method == "projqr" else 7)
    meth, _ = L.parse_method(method)
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, M, meth, 0, L.DTYPES[dtype], 1e-6, A)
    Aop = op.Operator(n)
    ref = Projection(M, Aop, 1e-6, dtype, "qr" if method == "projqr" else "classic", "A")
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    buf = torch.empty(N, dtype=torch.float64, device="cuda")
    u = lowprec.UNIT_ROUNDOFF[dtype]
    rng = np.random.default_rng(18)
    flips, worst, compared, drops = 0, 0.0, 0, 0
    try:
        for s in range(T):
            b = rng.standard_normal(N)
            x = rng.standard_normal(N) * (1.0 + 0.5 * s)
            L.guess_form(g, dev(b), x0)
            want = ref.form(b)
            if s > 0:
                err = rel_inf(host(x0), want)
                worst = max(worst, err)
                assert err <= 1e-12, (s, err)
            L.guess_update(g, dev(x))
            ref.update(x)
            info = L.guess_get_info(g)
            assert info["count"] == ref.d and info["last_accepted"] == 1
            raw = []
            for j in range(ref.d):
                sx = L.guess_history_raw(g, 0, j, buf)
                xs = host(buf).copy()
                L.guess_history_raw(g, 1, j, buf)
                raw.append((xs, host(buf).copy(), sx))
            xmax = max(float(np.max(np.abs(x))), float(np.max(np.abs(Aop(x)))))
            # the newest column; after a rolling drop every column (all were rotated and stored again)
            cols = range(ref.d) if info["drops"] > drops else [ref.d - 1]
            drops = info["drops"]
            cmax = max(max(float(np.max(np.abs(S))), float(np.max(np.abs(T)))) for S, T in zip(ref.S, ref.T))
            for j in cols:
                xs, bs, sc = raw[j]
                assert abs(sc - ref.sig[j]) <= 1e-13 * ref.sig[j], (s, j)
                for got, wcol in ((xs, ref.S[j]), (bs, ref.T[j])):
                    diff = got.view(np.uint64) != wcol.view(np.uint64)
                    if diff.any():
                        mag = 2 * cmax if j < ref.d - 1 else max(cmax, xmax / (sc * info["nu"]))
                        dv = np.abs(got[diff] - wcol[diff])
                        assert np.all(dv <= 2 * u * np.abs(wcol[diff]) + 64 * 2.0 ** -53 * mag), (s, j, int(diff.sum()))
                        flips += int(diff.sum())
                if dtype == "f16":
                    assert np.max(np.abs(xs)) <= 2 ** 15 and np.max(np.abs(bs)) <= 2 ** 15
                compared += 2 * N
            resync(L, g, ref, raw)
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
    print(f"[replay] {method} {dtype} 256^3: {T} steps, {drops} drops, {flips} of {compared} stored values "
          f"differ, largest guess error {worst:.2e}", flush=True)
    assert flips <= 1e-6 * compared
    if method == "projqr":
        assert drops == T - M
