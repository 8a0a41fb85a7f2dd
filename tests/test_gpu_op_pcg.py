"""GPU parity of the operator (bit-exact) and Jacobi-PCG (iterations +-1) against the oracle."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host, rel_inf
from oracle import operator as op
from oracle.pcg import pcg as oracle_pcg

pytestmark = pytest.mark.gpu


def make_op(L, n, kappa=None):
    return L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None if kappa is None else dev(kappa))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 32, 33])
def test_const_operator_bit_exact(lib, n):
    import torch

    announce(f"op const n={n}")
    L = lib
    A = make_op(L, n)
    try:
        x = synth.random_vectors(n, 1, n ** 3)[0]
        y = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
        L.op_apply(A, dev(x), y)
        got = host(y)
    finally:
        L.guess_op_destroy(A)
    want = op.apply_const(x, n)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n", [1, 3, 17])
def test_var_operator_bit_exact(lib, n):
    import torch

    announce(f"op var n={n}")
    L = lib
    kappa = np.exp(synth.gaussian_field(5, n, ell=0.2))
    A = make_op(L, n, kappa)
    try:
        x = synth.random_vectors(n + 1, 1, n ** 3)[0]
        y = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
        L.op_apply(A, dev(x), y)
        got = host(y)
    finally:
        L.guess_op_destroy(A)
    want = op.apply_var(x, n, op.face_coeffs(kappa, n))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n,seed", [(16, 0), (32, 1), (31, 2)])
def test_pcg_iterations_and_solution(lib, n, seed):
    import torch

    announce(f"pcg n={n}")
    L = lib
    params = synth.plane_wave_params(seed, 4)
    b = synth.plane_wave_rhs(params, n, 0.25)
    A = make_op(L, n)
    try:
        x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, it, rr = L.pcg_solve(A, dev(b), x, 1e-8, 5000)
        xg = host(x)
    finally:
        L.guess_op_destroy(A)
    Aop = op.Operator(n)
    xo, ito, sto, rro = oracle_pcg(Aop, b, np.zeros_like(b), 1.0 / Aop.diag(), 1e-8, 5000)
    assert st == L.OK and sto == 0
    assert abs(it - ito) <= 1
    assert rr <= 1e-8
    true_res = np.linalg.norm(b - Aop(xg)) / np.linalg.norm(b)
    assert true_res <= 1.5e-8
    xe = op.dst_solve(b, n)
    assert rel_inf(xg, xe) <= 1e-6
    assert rel_inf(xg, xo) <= 1e-6


BOXES = [(384, 8, 6), (512, 2, 5), (64, 16, 9), (6, 10, 7), (256, 4, 3)]


@pytest.mark.parametrize("shape", BOXES)
def test_box_operator_bit_exact(lib, shape):
    """Non-cubic grids: rows longer than a 256-element tile, tiles spanning several rows."""
    import torch

    announce(f"op box {shape}")
    L = lib
    nx, ny, nz = shape
    N = nx * ny * nz
    A = L.guess_op_create(nx, ny, nz, 900.0, 10.0, None)
    try:
        x = synth.random_vectors(nx + ny, 1, N)[0]
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        L.op_apply(A, dev(x), y)
        got = host(y)
    finally:
        L.guess_op_destroy(A)
    assert np.array_equal(got, op.apply_const_box(x, shape, 900.0))


@pytest.mark.parametrize("shape", BOXES)
def test_pcg_box_grids(lib, shape):
    """PCG on boxes (the z-marching stencil kernel runs where every plane is a whole number of
    4-tile groups): the first iterates agree with the oracle's to rounding, the converged
    iteration count to +-1."""
    import torch

    announce(f"pcg box {shape}")
    L = lib
    nx, ny, nz = shape
    N = nx * ny * nz
    c = 900.0
    b = synth.random_vectors(3 * nz, 1, N)[0]
    apply = lambda v: op.apply_const_box(v, shape, c)  # noqa: E731
    dinv = np.full(N, 1.0 / (c * 6.0 + 10.0))
    A = L.guess_op_create(nx, ny, nz, c, 10.0, None)
    try:
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st, it, _ = L.pcg_solve(A, dev(b), x, 1e-30, 5)
        assert st == L.ENOTCONV and it == 5
        xo, _, _, _ = oracle_pcg(apply, b, np.zeros(N), dinv, 1e-30, 5)
        assert rel_inf(host(x), xo) <= 1e-11
        x.zero_()
        st, it, rr = L.pcg_solve(A, dev(b), x, 1e-8, 5000)
        xo, ito, sto, _ = oracle_pcg(apply, b, np.zeros(N), dinv, 1e-8, 5000)
        assert st == L.OK and sto == 0 and abs(it - ito) <= 1
        assert np.linalg.norm(b - apply(host(x))) <= 1.5e-8 * np.linalg.norm(b)
        # stopping inside the stencil kernel and stopping at the iteration cap give the same x
        x2 = torch.zeros(N, dtype=torch.float64, device="cuda")
        st2, it2, _ = L.pcg_solve(A, dev(b), x2, 1e-8, it)
        assert st2 == L.OK and it2 == it and torch.equal(x, x2)
    finally:
        L.guess_op_destroy(A)


@pytest.mark.parametrize("shape", BOXES)
def test_box_var_operator_bit_exact(lib, shape):
    import torch

    announce(f"op var box {shape}")
    L = lib
    nx, ny, nz = shape
    N = nx * ny * nz
    kappa = np.exp(0.5 * synth.random_vectors(7, 1, (nx + 2) * (ny + 2) * (nz + 2))[0])
    A = L.guess_op_create(nx, ny, nz, 900.0, 10.0, dev(kappa))
    try:
        x = synth.random_vectors(nx + 2 * ny, 1, N)[0]
        y = torch.empty(N, dtype=torch.float64, device="cuda")
        L.op_apply(A, dev(x), y)
        got = host(y)
    finally:
        L.guess_op_destroy(A)
    want = op.apply_var_box(x, shape, op.face_coeffs_box(kappa, shape), 900.0)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("shape", [(384, 8, 6), (64, 16, 9), (6, 10, 7)])
def test_pcg_box_var(lib, shape):
    import torch

    announce(f"pcg var box {shape}")
    L = lib
    nx, ny, nz = shape
    N = nx * ny * nz
    c = 900.0
    kappa = np.exp(0.5 * synth.random_vectors(8, 1, (nx + 2) * (ny + 2) * (nz + 2))[0])
    faces = op.face_coeffs_box(kappa, shape)
    apply = lambda v: op.apply_var_box(v, shape, faces, c)  # noqa: E731
    kxa, kya, kza = faces
    diag = c * (kxa[:, :, :-1] + kxa[:, :, 1:] + kya[:, :-1, :] + kya[:, 1:, :] + kza[:-1] + kza[1:]) + 10.0
    b = synth.random_vectors(9, 1, N)[0]
    A = L.guess_op_create(nx, ny, nz, c, 10.0, dev(kappa))
    try:
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st, it, _ = L.pcg_solve(A, dev(b), x, 1e-30, 5)
        xo, _, _, _ = oracle_pcg(apply, b, np.zeros(N), 1.0 / diag.reshape(-1), 1e-30, 5)
        assert st == L.ENOTCONV and rel_inf(host(x), xo) <= 1e-11
        x.zero_()
        st, it, rr = L.pcg_solve(A, dev(b), x, 1e-8, 5000)
        xo, ito, sto, _ = oracle_pcg(apply, b, np.zeros(N), 1.0 / diag.reshape(-1), 1e-8, 5000)
        assert st == L.OK and sto == 0 and abs(it - ito) <= 1
    finally:
        L.guess_op_destroy(A)


def test_pcg_varcoef(lib):
    import torch

    announce("pcg var n=12")
    L = lib
    n = 12
    kappa = np.exp(synth.gaussian_field(2, n, ell=0.1))
    b = synth.random_vectors(4, 1, n ** 3)[0]
    A = make_op(L, n, kappa)
    try:
        x = torch.zeros(n ** 3, dtype=torch.float64, device="cuda")
        st, it, rr = L.pcg_solve(A, dev(b), x, 1e-8, 5000)
        xg = host(x)
    finally:
        L.guess_op_destroy(A)
    Aop = op.Operator(n, kappa_nodal=kappa)
    xo, ito, sto, _ = oracle_pcg(Aop, b, np.zeros_like(b), 1.0 / Aop.diag(), 1e-8, 5000)
    assert st == L.OK and abs(it - ito) <= 1
    assert rel_inf(xg, xo) <= 1e-6


def test_pcg_edge_cases(lib):
    import torch

    announce("pcg edge cases")
    L = lib
    n = 8
    N = n ** 3
    A = make_op(L, n)
    try:
        z = torch.zeros(N, dtype=torch.float64, device="cuda")
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st, it, rr = L.pcg_solve(A, z, x, 1e-8, 100)           # zero right-hand side
        assert st == L.OK and it == 0 and not host(x).any()
        b = synth.random_vectors(1, 1, N)[0]
        xe = op.dst_solve(b, n)
        x = dev(xe)
        st, it, rr = L.pcg_solve(A, dev(b), x, 1e-8, 100)       # exact guess
        assert st == L.OK and it == 0
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st, it, rr = L.pcg_solve(A, dev(b), x, 1e-14, 3)        # maxit
        assert st == L.ENOTCONV and it == 3
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st, it, rr = L.pcg_solve(A, dev(b), x, 1e-8, 0)         # no iterations allowed
        assert st == L.ENOTCONV and it == 0
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st, it, rr = L.pcg_solve(A, dev(1e-12 * b), x, 1e-8, 100, L.STOP_INITRESID)
        assert st == L.OK and it == 0                           # paper's rule: absolute floor
        x = torch.zeros(N, dtype=torch.float64, device="cuda")
        st, it, _ = L.pcg_solve(A, dev(b), x, 1e-8, 1000, L.STOP_INITRESID)
        Aop = op.Operator(n)
        _, ito, _, _ = oracle_pcg(Aop, b, np.zeros_like(b), 1.0 / Aop.diag(), 1e-8, 1000, rule="initresid")
        assert st == L.OK and abs(it - ito) <= 1
    finally:
        L.guess_op_destroy(A)


@pytest.mark.parametrize("n", [12, 32])
def test_pcg_deferred_updates_every_count(lib, n):
    """x is updated every other iteration (odd iterations apply the two updates before them), so
    what a solve leaves pending depends on the parity of its last iteration.  For K = 1 .. 7
    iterations: the solve capped at K (ending with the check and finishing kernels) equals the
    oracle's K-th iterate to 1e-12, and the solve that stops inside iteration K + 1's stencil
    kernel (its stop test passes on r_K) equals the capped one bit for bit.  12^3: chunk form
    with a ragged tail; 32^3: the z-marching form."""
    import torch

    L = lib
    N = n ** 3
    A = make_op(L, n)
    Aop = op.Operator(n)
    b = synth.random_vectors(91, 1, N)[0]
    capped, rrs = {}, {}
    try:
        for K in range(1, 8):
            announce(f"pcg n={n} capped at {K} iterations")
            x1 = torch.zeros(N, dtype=torch.float64, device="cuda")
            st, it, rrs[K] = L.pcg_solve(A, dev(b), x1, 1e-30, K)
            assert st == L.ENOTCONV and it == K
            capped[K] = host(x1).copy()
            xo, ito, _, _ = oracle_pcg(Aop, b, np.zeros_like(b), 1.0 / Aop.diag(), 1e-30, K)
            assert ito == K
            assert rel_inf(capped[K], xo) <= 1e-12, (K, rel_inf(capped[K], xo))
        # a tolerance just above the relative residual after K iterations stops the solve in
        # iteration K + 1 when no earlier residual was as small
        stops = [K for K in rrs if all(rrs[K] * (1.0 + 1e-9) < rrs[j] for j in range(1, K))]
        assert {K % 2 for K in stops} == {0, 1}, rrs
        for K in stops:
            announce(f"pcg n={n} stopping after {K} iterations")
            x2 = torch.zeros(N, dtype=torch.float64, device="cuda")
            st2, it2, _ = L.pcg_solve(A, dev(b), x2, rrs[K] * (1.0 + 1e-9), 100)
            assert st2 == L.OK and it2 == K, (K, it2)
            assert np.array_equal(host(x2), capped[K]), K
    finally:
        L.guess_op_destroy(A)


def test_plane_wave_rhs_kernel(lib):
    import torch

    announce("workload rhs")
    L = lib
    params = synth.plane_wave_params(0, 16)
    for n in (7, 32):
        amp = synth.mode_amplitudes(params, 0.37)
        b = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
        L.workload_plane_wave_rhs(n, params["k"].reshape(-1), params["theta"], amp, b)
        want = synth.plane_wave_rhs(params, n, 0.37)
        assert np.max(np.abs(host(b) - want)) <= 1e-12 * 16
    n = 256
    b = torch.empty(n ** 3, dtype=torch.float64, device="cuda")
    amp = synth.mode_amplitudes(params, 1.0)
    L.workload_plane_wave_rhs(n, params["k"].reshape(-1), params["theta"], amp, b)
    idx = np.random.default_rng(0).integers(0, n ** 3, 4096)
    idx = np.concatenate([idx, [0, n ** 3 - 1, n - 1, n * n - 1]])
    want = synth.plane_wave_rhs_at(params, n, 1.0, idx)
    assert np.max(np.abs(host(b)[idx] - want)) <= 1e-11 * 16


def test_vector_kernels(lib):
    import torch

    announce("multidot / combine / copy")
    L = lib
    for N, K in [(1, 1), (1001, 3), (70000, 17)]:
        V = synth.random_vectors(9, K, N)
        y = synth.random_vectors(10, 1, N)[0]
        got = L.vec_multidot(N, K, dev(V.reshape(-1)), dev(y))
        want = V @ y
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(V).sum(1).max())
        c = np.linspace(-1, 1, K)
        out = torch.empty(N, dtype=torch.float64, device="cuda")
        L.vec_combine(N, K, dev(V.reshape(-1)), c, out)
        assert rel_inf(host(out), c @ V) <= 1e-13
    src = dev(np.arange(12345, dtype=np.float64))
    dst = torch.zeros_like(src)
    L.guess_copy_kernel(dst, src, 12345 * 8)
    assert np.array_equal(host(dst), np.arange(12345, dtype=np.float64))


def test_roof_kernels(lib):
    """The bandwidth references read and write what they claim: the read kernels' partial rows
    sum to the sum of the bytes they read (one stream; 16 segments side by side, of which
    bytes / 16 rounded down to a multiple of 16 elements count), the write kernel fills dst,
    the copy copies."""
    import torch

    announce("roof kernels")
    L = lib
    n = 1 << 16                       # doubles; 2^15 16-byte elements
    v = np.arange(n, dtype=np.float64) % 97.0
    src = dev(v)
    part = torch.zeros(2048, dtype=torch.float64, device="cuda")
    L.guess_roof_kernel(L.ROOF_READ, part, src, n * 8)
    torch.cuda.synchronize()
    assert float(part.sum()) == float(v.sum())
    part.zero_()
    nbytes = n * 8 - 48                # 2^15 - 3 elements: 16 segments of 2047
    L.guess_roof_kernel(L.ROOF_READ_STREAMS, part, src, nbytes)
    torch.cuda.synchronize()
    seg = (nbytes // 16) // 16
    assert float(part.sum()) == float(v[: 2 * 16 * seg].sum())
    dst = torch.zeros(n, dtype=torch.float64, device="cuda")
    L.guess_roof_kernel(L.ROOF_WRITE, dst, None, n * 8)
    assert np.all(host(dst) == 1.0)
    dst.zero_()
    L.guess_roof_kernel(L.ROOF_COPY, dst, src, n * 8)
    assert np.array_equal(host(dst), v)
