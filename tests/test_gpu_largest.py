"""The largest workload at full size: variable-coefficient -div(kappa grad u) + 10 u on 384^3
(56,623,104 unknowns), kappa = exp(g), g a unit-variance Gaussian field with correlation length
0.1; history M = 16.

At this size the oracle checks what it can compute: the operator bit for bit at sampled
unknowns (the oracle applies it to the whole vector) and the extrapolated guess at sampled
unknowns.  Projection and PCG are checked through properties that hold at any size, evaluated
with the library's own verified primitives (op_apply is bit-exact against the oracle, the
multi-dot is an FP64 reduction): orthonormality of the stored history in the A inner product,
B = A X, the Galerkin condition of the guess (residual b - A x0 orthogonal to the retained
solutions) and the true residual of the PCG solution.
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rel_inf
from oracle import extrap, lowprec
from oracle import operator as op

pytestmark = pytest.mark.gpu

n = 384
N = n ** 3
M = 16


@pytest.fixture(scope="module")
def field():
    announce("kappa 386^3 (oracle side)")
    return np.exp(synth.gaussian_field(5, n))


@pytest.fixture(scope="module")
def gpu_op(lib, field):
    A = lib.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, dev(field))
    yield A
    lib.guess_op_destroy(A)


def sample_idx():
    idx = np.random.default_rng(12).integers(0, N, 16384)
    edges = [0, 1, n - 1, n, n * n - 1, n * n, N - n * n, N - n - 1, N - 2, N - 1]
    return np.unique(np.concatenate([idx, edges]))


def test_varcoef_operator_bit_exact_sampled(lib, field, gpu_op):
    import torch

    announce("varcoef op_apply 384^3")
    u = np.random.default_rng(3).standard_normal(N)
    y = torch.empty(N, dtype=torch.float64, device="cuda")
    lib.op_apply(gpu_op, dev(u), y)
    idx = sample_idx()
    got = host(y)[idx]
    want = op.apply_var(u, n, op.face_coeffs(field, n))[idx]
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_extrap_384_m16_sampled(lib, dtype):
    import torch

    announce(f"extrap 384^3 M=16 m=3 {dtype}")
    L = lib
    m = 3
    idx = sample_idx()
    g = L.guess_create_ex(N, M, L.EXTRAP, m, L.DTYPES[dtype])
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    hist = []
    try:
        rng = np.random.default_rng(6)
        for s in range(M + 2):
            v = rng.standard_normal(N) * (1.0 + 0.05 * s)
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
        err = np.abs(got - want)
        assert np.all(err <= (M + 1) * 2.0 ** -24 * mag + 2.0 ** -24 * np.abs(want))


@pytest.mark.parametrize("method", ["proj", "projqr"])
def test_proj_384_m16_properties(lib, gpu_op, method):
    """18 random solutions through PROJ(16) / rolling PROJ(16) with the variable-coefficient
    operator: stored history A-orthonormal with B = A X, and the guess satisfies the
    Galerkin condition against the retained raw solutions."""
    import torch

    announce(f"{method} 384^3 M=16 varcoef")
    L = lib
    meth, inner = L.parse_method(method)
    T = M + 2
    g = L.guess_create_ex(N, M, meth, 0, L.F64, 1e-6, gpu_op)
    S = L.stream_handle()
    raw = torch.empty((T, N), dtype=torch.float64, device="cuda")
    gen = torch.Generator(device="cuda").manual_seed(4)
    try:
        for s in range(T):
            raw[s].normal_(generator=gen)
            L.guess_update(g, raw[s])
        info = L.guess_get_info(g)
        d = info["count"]
        window = raw[T - d:] if method == "projqr" else raw[T - d:]
        assert d == (M if method == "projqr" else T - M)
        X = torch.empty((d, N), dtype=torch.float64, device="cuda")
        B = torch.empty((d, N), dtype=torch.float64, device="cuda")
        for j in range(d):
            L.guess_history_get(g, 0, j, X[j])
            L.guess_history_get(g, 1, j, B[j])
        G = np.stack([L.vec_multidot(N, d, X, B[j].contiguous(), S) for j in range(d)])
        assert np.max(np.abs(G - np.eye(d))) <= 1e-12
        AX = torch.empty(N, dtype=torch.float64, device="cuda")
        for j in range(d):
            L.op_apply(gpu_op, X[j], AX)
            assert float(torch.max(torch.abs(AX - B[j]))) <= 1e-12 * float(torch.max(torch.abs(B[j])))
        # Galerkin: raw_j^T (b - A x0) = 0 for the retained raw solutions
        b = torch.empty(N, dtype=torch.float64, device="cuda").normal_(generator=gen)
        x0 = torch.empty_like(b)
        L.guess_form(g, b, x0)
        L.op_apply(gpu_op, x0, AX)
        r = (b - AX).contiguous()
        W = window.contiguous()
        gal = np.array(L.vec_multidot(N, d, W, r, S))
        scale = np.array([float(torch.linalg.vector_norm(W[j])) for j in range(d)]) * float(
            torch.linalg.vector_norm(b))
        assert np.max(np.abs(gal) / scale) <= 1e-10
    finally:
        L.guess_destroy(g)


def test_pcg_384_true_residual(lib, gpu_op):
    import torch

    announce("pcg 384^3 varcoef")
    L = lib
    params = synth.plane_wave_params(0, 16)
    from paper_2009_10863_amd.sequence import PlaneWaveRHS

    b = torch.empty(N, dtype=torch.float64, device="cuda")
    PlaneWaveRHS(params, n)(0.1, b)
    x = torch.zeros_like(b)
    st, it, rr = L.pcg_solve(gpu_op, b, x, 1e-8, 20000)
    assert st == L.OK and rr <= 1e-8
    Ax = torch.empty_like(b)
    L.op_apply(gpu_op, x, Ax)
    true = float(torch.linalg.vector_norm(b - Ax) / torch.linalg.vector_norm(b))
    assert true <= 2e-8, (it, true)


def test_pcg_384_stop_path_applies_last_update_everywhere(lib, gpu_op):
    """The solve that stops inside its stencil kernel (the stop test of iteration K+1 passes) must
    give bit for bit the x of the same solve capped at K iterations, which ends with the separate
    check and finishing kernels.  At this size the stencil kernel's workgroups run in several
    rounds, so workgroups that start after the stop decision was written must still apply their
    part of the last x update."""
    import torch

    announce("pcg 384^3 varcoef stop path")
    L = lib
    b = torch.empty(N, dtype=torch.float64, device="cuda").normal_(generator=torch.Generator(device="cuda").manual_seed(21))
    x1 = torch.zeros(N, dtype=torch.float64, device="cuda")
    st, its, rr = L.pcg_solve(gpu_op, b, x1, 1e-6, 20000)
    assert st == L.OK and its > 1
    x2 = torch.zeros(N, dtype=torch.float64, device="cuda")
    st2, its2, rr2 = L.pcg_solve(gpu_op, b, x2, 1e-6, its)
    assert st2 == L.OK and its2 == its and rr2 == rr
    assert torch.equal(x1, x2)
