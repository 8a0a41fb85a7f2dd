"""The two byte models agree: bench.py's per-kernel algorithmic bytes (which set the reported
GB/s) sum, call by call, to the library's own guess_get_info form / update bytes, for every
method, through warm-up, restarts, drops and rejections."""
import numpy as np
import pytest

import bench
import synth
from gpu_helpers import announce, dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method", ["extrap", "spextrap", "last", "proj", "projqr", "proj_l2", "projqr_l2",
                                    "proj_raw", "projqr_raw"])
@pytest.mark.parametrize("dtype", ["f64", "bf16", "f16"])
def test_bench_bytes_match_library(lib, method, dtype):
    import torch

    if method in bench.RAW and dtype == "f64":
        pytest.skip("the raw-solution projection takes reduced-precision histories only")
    announce(f"bytes model {method} {dtype}")
    L = lib
    n, M, deg, T = 8, 4, 2, 11
    N = n ** 3
    meth, inner = L.parse_method(method)
    Mm = 1 if method == "last" else M
    A = L.guess_op_create(n, n, n, float((n + 1) ** 2), 10.0, None)
    g = L.guess_create_ex(N, Mm, meth, deg if method in ("extrap", "spextrap") else 0, L.DTYPES[dtype], 1e-6, A,
                          None, inner)
    s = L.ELEM_BYTES[L.DTYPES[dtype]]
    X = synth.random_vectors(5, T, N)
    X[6] = X[5]                          # one dependent solution: rejected by the projections
    x0 = torch.empty(N, dtype=torch.float64, device="cuda")
    b = dev(synth.random_vectors(6, 1, N)[0])
    try:
        for q in range(T):
            kd = L.guess_get_info(g)["count"]
            L.guess_form(g, b, x0)
            info = L.guess_get_info(g)
            if method == "spextrap":
                kf = min(deg, kd - 1) + 1 if kd > 0 else 0
            else:
                kf = kd if method.startswith("proj") else min(kd, Mm)
            want = sum(bench.kernel_bytes(method, "form", N, s, kf, Mm, False, dtype=dtype))
            if method in ("extrap", "spextrap", "last") and kd == 0:
                want = 8 * N                 # zero guess
            assert want == info["form_bytes"], (q, "form")
            L.guess_update(g, dev(X[q]))
            info = L.guess_get_info(g)
            d = kd
            restart = (d == 0 or Mm == 1) if method.startswith("projqr") else (d == 0 or d >= Mm)
            ring = method in bench.RING
            plain = sum(bench.kernel_bytes(method, "update", N, s, kd, Mm, False, dtype=dtype))
            fixed = dtype == "f16" and (ring or method in bench.RAW) and info["update_bytes"] > plain + 0.5 * N * (8 + s)
            if dtype == "f16" and ring:
                assert info["update_bytes"] in (N * (8 + s), 2 * N * (8 + s))
            want = sum(bench.kernel_bytes(method, "update", N, s, d, Mm, restart and method.startswith("proj"),
                                          dtype=dtype, fixed=fixed))
            assert want == info["update_bytes"], (q, "update", d)
    finally:
        L.guess_destroy(g)
        L.guess_op_destroy(A)
