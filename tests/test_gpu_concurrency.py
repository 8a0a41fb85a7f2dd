"""Independent sequences on their own streams from their own host threads.

Each field owns an operator, a guess context, a right-hand-side generator and a HIP stream; the
library keeps no state shared between them (per-operator PCG buffers, per-context histories,
per-thread workload tables and error strings).  Solving the fields side by side must reproduce,
bit for bit, the solutions and iteration counts of solving them one after another.
"""
import threading

import numpy as np
import pytest

import synth
from gpu_helpers import announce

pytestmark = pytest.mark.gpu


def _run(L, n, specs, steps, threaded):
    import torch

    from paper_2009_10863_amd.sequence import GuessSequence, Operator, PlaneWaveRHS

    N = n ** 3
    fields = []
    for shift, seed, method in specs:
        st = torch.cuda.Stream()
        op = Operator(n, shift, None, st)
        fields.append({"op": op, "st": st, "rhs": PlaneWaveRHS(synth.plane_wave_params(seed, 8), n, st),
                       "g": GuessSequence(N, 8, method, 2, "f64", 0.0, op, st),
                       "b": torch.empty(N, dtype=torch.float64, device="cuda"),
                       "x": torch.zeros(N, dtype=torch.float64, device="cuda"), "its": [], "xs": []})
    torch.cuda.synchronize()

    def work(f):
        for k in range(1, steps + 1):
            f["rhs"](0.01 * k, f["b"])
            f["g"].form(f["b"], f["x"])
            status, it, _ = f["op"].solve(f["b"], f["x"], 1e-9, 5000)
            assert status == L.OK
            f["g"].update(f["x"])
            f["its"].append(it)
        torch.cuda.synchronize(f["st"])
        f["xs"].append(f["x"].cpu().numpy())

    try:
        if threaded:
            errs = []

            def guarded(f):
                try:
                    work(f)
                except BaseException as e:  # noqa: BLE001
                    errs.append(e)
            th = [threading.Thread(target=guarded, args=(f,)) for f in fields]
            for t in th:
                t.start()
            for t in th:
                t.join()
            if errs:
                raise errs[0]
        else:
            for f in fields:
                work(f)
        return [(f["its"], f["xs"][-1]) for f in fields]
    finally:
        for f in fields:
            f["g"].close()
            f["op"].close()


def test_fields_side_by_side_match_one_after_another(lib):
    announce("concurrent fields 64^3 x4")
    specs = [(2.0e4, 1, "extrap"), (2.0e4, 2, "proj"), (2.0e4, 3, "projqr"), (0.0, 4, "extrap")]
    one = _run(lib, 64, specs, 12, threaded=False)
    par = _run(lib, 64, specs, 12, threaded=True)
    for (its1, x1), (its2, x2) in zip(one, par):
        assert its1 == its2
        assert np.array_equal(x1, x2)
