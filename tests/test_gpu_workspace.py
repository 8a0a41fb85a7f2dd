"""Contexts whose history lives in caller memory (guess_opts.workspace): same results as
library-allocated contexts, bit for bit, for every method."""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method,dtype", [("extrap", "f64"), ("spextrap", "f32"), ("last", "bf16"),
                                          ("proj", "f64"), ("projqr", "f32"), ("projqr_l2", "f64")])
def test_workspace_context_matches_allocated(lib, method, dtype):
    import torch

    announce(f"workspace {method} {dtype}")
    L = lib
    n, M, T = 9, 4, 11
    N = n ** 3
    meth, inner = L.parse_method(method)
    Mm = 1 if method == "last" else M
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    need = L.guess_workspace_bytes(N, Mm, meth, L.DTYPES[dtype])
    ws = torch.full((need + 256,), 0xAB, dtype=torch.uint8, device="cuda")[:need]   # 256-aligned start
    assert ws.data_ptr() % 256 == 0
    deg = 2 if method in ("extrap", "spextrap") else 0
    g1 = L.guess_create_ex(N, Mm, meth, deg, L.DTYPES[dtype], 1e-6, A, None, inner)
    g2 = L.guess_create_ex(N, Mm, meth, deg, L.DTYPES[dtype], 1e-6, A, None, inner, workspace=ws)
    X = synth.random_vectors(21, T, N)
    B = synth.random_vectors(22, T, N)
    y1 = torch.empty(N, dtype=torch.float64, device="cuda")
    y2 = torch.empty(N, dtype=torch.float64, device="cuda")
    try:
        for b, x in zip(B, X):
            L.guess_form(g1, dev(b), y1)
            L.guess_form(g2, dev(b), y2)
            assert np.array_equal(host(y1), host(y2))
            L.guess_update(g1, dev(x))
            L.guess_update(g2, dev(x))
        i1, i2 = L.guess_get_info(g1), L.guess_get_info(g2)
        assert i1["count"] == i2["count"] and i1["rejects"] == i2["rejects"]
    finally:
        L.guess_destroy(g2)
        L.guess_destroy(g1)
        L.guess_op_destroy(A)
    # the history was written into the workspace (its first buffer is the ring or X)
    first = N * L.ELEM_BYTES[L.DTYPES[dtype]]
    assert int((ws[:first] != 0xAB).sum()) > first // 2
