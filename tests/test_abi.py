"""Host-side checks of the libguess C ABI (no GPU needed).

The library must load and export every function that include/libguess.h
declares; host-only entry points (least-squares weights, argument
validation, workspace sizes, error strings) are exercised directly.
Compute entry points are only called by the GPU tests.
"""
import ctypes
import os
import re

import pytest

from oracle import extrap

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libguess.h")


@pytest.fixture(scope="module")
def L():
    from paper_2009_10863_amd import _build

    if not os.path.exists(_build.LIB):
        _build.build()
    from paper_2009_10863_amd import libguess

    return libguess


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b([a-z_][a-z0-9_]*)\s*\([^;{]*\)\s*;", text)
    return sorted(set(n for n in names if n not in ("if", "sizeof")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("guess_create", "guess_form", "guess_update", "op_apply", "pcg_solve"):
        assert n in names


def test_library_exports_every_declared_function(L):
    lib = ctypes.CDLL(L.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(L.EXPORTED)


@pytest.mark.parametrize("k", range(1, 17))
def test_host_weights_match_exact_rationals(L, k):
    for m in range(0, k):
        got = L.guess_extrap_weights(m, k)
        ref = extrap.to_f64(extrap.beta_ls_exact(m, k))
        assert max(abs(a - b) for a, b in zip(got, ref)) <= 1e-14 * max(1.0, float(extrap.lebesgue(extrap.beta_ls_exact(m, k))))


@pytest.mark.parametrize("k", range(1, 17))
def test_host_sparse_weights_match_exact_rationals(L, k):
    """Same nonzero pattern as the oracle's exact pivoting (index work: exact), and
    weights within two roundings of the exact rationals."""
    for m in range(0, k):
        got = L.guess_spextrap_weights(m, k)
        exact = extrap.beta_sparse_exact(m, k)
        assert [g != 0.0 for g in got] == [b != 0 for b in exact], (m, k)
        ref = extrap.to_f64(exact)
        for a, b in zip(got, ref):
            assert abs(a - b) <= 2.0 ** -52 * abs(b), (m, k)


def test_weight_argument_checks(L):
    for m, k in [(-1, 4), (4, 4), (0, 0), (0, 17)]:
        for f in (L.guess_extrap_weights, L.guess_spextrap_weights):
            with pytest.raises(L.GuessError) as e:
                f(m, k)
            assert e.value.code == L.EINVAL


def test_create_argument_checks(L):
    bad = [
        dict(N=0, M=4, method=L.EXTRAP, degree=1),
        dict(N=10, M=0, method=L.EXTRAP, degree=0),
        dict(N=10, M=17, method=L.PROJ),
        dict(N=10, M=4, method=L.EXTRAP, degree=4),
        dict(N=10, M=4, method=L.EXTRAP, degree=-1),
        dict(N=10, M=4, method=7),
        dict(N=10, M=4, method=L.EXTRAP, degree=1, dtype=9),
        dict(N=10, M=4, method=L.SPEXTRAP, degree=4),
        dict(N=10, M=17, method=L.PROJ_QR),
        dict(N=10, M=4, method=L.PROJ, inner=2),
    ]
    for kw in bad:
        with pytest.raises(L.GuessError) as e:
            L.guess_create_ex(**kw)
        assert e.value.code == L.EINVAL, kw
    with pytest.raises(L.GuessError):
        L.guess_create(10, 0, L.EXTRAP, 0)


def test_operator_and_solver_argument_checks(L):
    for args in [(0, 4, 4, 25.0, 10.0), (4, 4, 4, 0.0, 10.0), (4, 4, 4, 25.0, -1.0),
                 (2048, 2048, 1024, 1.0, 1.0)]:
        with pytest.raises(L.GuessError) as e:
            L.guess_op_create(*args)
        assert e.value.code == L.EINVAL
    lib = L.lib()
    it, rr = ctypes.c_int(), ctypes.c_double()
    assert lib.pcg_solve(None, None, None, 1e-8, 10, ctypes.byref(it), ctypes.byref(rr)) == L.EINVAL
    assert lib.op_apply(None, None, None) == L.EINVAL
    assert lib.guess_form(None, None, None) == L.EINVAL
    assert lib.guess_update(None, None, None) == L.EINVAL
    d = ctypes.c_int()
    assert lib.guess_proj_factor(None, None, ctypes.byref(d)) == L.EINVAL
    assert "invalid" in L.guess_strerror(L.EINVAL)
    assert L.guess_strerror(12345) == "unknown status"


def test_workspace_bytes(L):
    N, M = 256 ** 3, 8
    col = N * 8
    assert L.guess_workspace_bytes(N, M, L.EXTRAP, L.F64) == (M + 1) * col   # one spare slot
    # FP16 rings also keep a small state (per-slot exponents) in 256 bytes
    assert L.guess_workspace_bytes(N, M, L.EXTRAP, L.F16) == M * N * 2 + 256
    assert L.guess_workspace_bytes(N, M, L.LAST, L.F64) == 2 * col
    assert L.guess_workspace_bytes(N, M, L.PROJ, L.F64) >= 2 * M * col + N * 8
    assert L.guess_workspace_bytes(N, M, L.PROJ_QR, L.F64) == L.guess_workspace_bytes(N, M, L.PROJ, L.F64)
    assert L.guess_workspace_bytes(N, M, L.SPEXTRAP, L.F32) == M * N * 4
    assert L.guess_workspace_bytes(N, M, L.PROJ, 9) == 0


def test_workspace_route_argument_checks(L):
    """A caller workspace that is too small or misaligned is refused before any allocation."""
    lib = L.lib()
    need = L.guess_workspace_bytes(1000, 4, L.PROJ, L.F64)
    assert need % 256 == 0
    o = L.guess_opts(N=1000, M=4, method=L.PROJ, degree=0, dtype=L.F64, eps_rel=0.0, op=None, stream=None,
                     inner=0, workspace=4096, workspace_bytes=need - 1)
    out = ctypes.c_void_p()
    assert lib.guess_create_ex(ctypes.byref(o), ctypes.byref(out)) == L.EINVAL and not out.value
    o.workspace, o.workspace_bytes = 4096 + 8, need
    assert lib.guess_create_ex(ctypes.byref(o), ctypes.byref(out)) == L.EINVAL and not out.value


def test_binding_refuses_undersized_or_mistyped_tensors(L):
    """The C ABI cannot see the size of a device buffer, so the binding checks every tensor it
    forwards against what the call will touch, before the call (CPU tensors: the size and type
    checks come first, so no device is needed here)."""
    import torch

    f64 = torch.float64
    with pytest.raises(ValueError, match="kappa"):   # (n+2)^2 instead of (n+2)^3 values
        L.guess_op_create(8, 8, 8, 81.0, 10.0, torch.zeros(10 * 10, dtype=f64))
    with pytest.raises(TypeError, match="float64"):
        L.guess_op_create(8, 8, 8, 81.0, 10.0, torch.zeros(10 ** 3, dtype=torch.float32))
    with pytest.raises(ValueError, match="device"):  # right size: only the device check is left
        L.guess_op_create(8, 8, 8, 81.0, 10.0, torch.zeros(10 ** 3, dtype=f64))
    fake = 0x1234   # a handle the binding knows the size of; the library is never reached
    L._sizes[fake] = 100
    try:
        short, ok = torch.zeros(99, dtype=f64), torch.zeros(100, dtype=f64)
        # the first tensor that is checked is the short one (a good CPU tensor would stop at the
        # device check)
        for call in (lambda: L.op_apply(fake, short, ok), lambda: L.op_apply(fake, None, short),
                     lambda: L.pcg_solve(fake, short, ok), lambda: L.pcg_solve(fake, None, short),
                     lambda: L.guess_form(fake, short, ok), lambda: L.guess_form(fake, None, short),
                     lambda: L.guess_update(fake, short), lambda: L.guess_update(fake, None, short),
                     lambda: L.guess_history_get(fake, 0, 0, short)):
            with pytest.raises(ValueError, match="needs 100"):
                call()
    finally:
        L._sizes.pop(fake)
    with pytest.raises(ValueError, match="needs 512"):
        L.workload_gaussian_rhs(8, (0.5, 0.5, 0.5), 0.1, 1.0, torch.zeros(511, dtype=f64))
    with pytest.raises(ValueError, match="needs 30"):
        L.vec_multidot(10, 3, torch.zeros(29, dtype=f64), torch.zeros(10, dtype=f64))
    with pytest.raises(ValueError, match="bytes"):
        L.guess_copy_kernel(torch.zeros(8, dtype=torch.uint8), torch.zeros(16, dtype=torch.uint8), 16)
