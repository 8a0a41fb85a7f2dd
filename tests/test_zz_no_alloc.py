"""The allocation-free multi-dot (vec_multidot_noalloc) against vec_multidot.

Called through the C ABI on two calls in a row, the second with a smaller
input (fewer vectors, a shorter length, other values): the static scratch
keeps the first call's contents, and the second call's results must not
depend on them.  Both entry points run the same kernels with the same grid,
so the results agree bit for bit; each is also within 1e-12 (relative to
sum |v_k||y|) of the plain NumPy dot products.
"""
import ctypes

import numpy as np
import pytest

from gpu_helpers import announce, dev

pytestmark = pytest.mark.gpu


def _call(L, name, N, K, V, y):
    out = (ctypes.c_double * K)()
    rc = getattr(L.lib(), name)(N, K, V.data_ptr(), y.data_ptr(), out, None)
    assert rc == L.OK, (name, rc, L.guess_last_error())
    return np.array(list(out))


def test_noalloc_multidot_matches_allocating_one(lib):
    import torch

    L = lib
    rng = np.random.default_rng(21)
    for N, K in ((70001, 13), (1027, 3)):
        announce(f"vec_multidot_noalloc N={N} K={K}")
        Vh = rng.standard_normal((K, N))
        yh = rng.standard_normal(N)
        V, y = dev(Vh.reshape(-1)), dev(yh)
        got = _call(L, "vec_multidot_noalloc", N, K, V, y)
        want = _call(L, "vec_multidot", N, K, V, y)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), (N, K)
        ref = Vh @ yh
        scale = np.abs(Vh) @ np.abs(yh)
        assert np.all(np.abs(got - ref) <= 1e-12 * scale), (N, K)
        torch.cuda.synchronize()


def test_noalloc_multidot_rejects_too_many_vectors(lib):
    import torch

    L = lib
    announce("vec_multidot_noalloc K=65")
    V = torch.zeros(65 * 8, dtype=torch.float64, device="cuda")
    y = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = (ctypes.c_double * 65)()
    assert L.lib().vec_multidot_noalloc(8, 65, V.data_ptr(), y.data_ptr(), out, None) == L.EINVAL
    assert "64" in L.guess_last_error()
