"""Python objects over the libguess C ABI and the time-step driver.

Torch supplies device memory and streams only; every operation below is one
or more calls into ``libguess.so``.
"""
from __future__ import annotations

import math

import torch

from . import libguess as L


def _dev_f64(n, device="cuda"):
    return torch.empty(n, dtype=torch.float64, device=device)


class Operator:
    """7-point Helmholtz operator on an n^3 unit-cube grid (kappa: nodal, (n+2)^3)."""

    def __init__(self, n: int, shift: float = 10.0, kappa: torch.Tensor = None, stream=None):
        self.n = n
        self.N = n ** 3
        self.shift = shift
        self.inv_h2 = float((n + 1) ** 2)
        if kappa is not None:
            if kappa.dtype != torch.float64 or kappa.numel() != (n + 2) ** 3:
                raise ValueError("kappa must be float64 with (n+2)^3 nodal values")
        self.handle = L.guess_op_create(n, n, n, self.inv_h2, shift, kappa)
        self.stream = L.stream_handle(stream)
        L.guess_op_set_stream(self.handle, self.stream)

    def apply(self, x: torch.Tensor, y: torch.Tensor = None) -> torch.Tensor:
        y = torch.empty_like(x) if y is None else y
        L.op_apply(self.handle, x, y)
        return y

    def solve(self, b, x, rtol=1e-8, maxit=20000, rule=L.STOP_RHS):
        """PCG from the guess held in x; returns (status, iterations, relres)."""
        return L.pcg_solve(self.handle, b, x, rtol, maxit, rule)

    def close(self):
        if getattr(self, "handle", None):
            L.guess_op_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GuessSequence:
    """Initial-guess history for one sequence of solves (one field).  eps_rel <= 0 selects the
    library's rejection threshold for the storage format (1e-6 for FP64).

    in_place (FP64 extrapolation only): the context lives in a torch-owned workspace and
    ``slot()`` is a view of the ring slot the next update writes; forming the guess into it,
    solving there and updating with it stores the solution without a copy."""

    def __init__(self, N: int, M: int = 8, method: str = "extrap", degree: int = 2,
                 dtype: str = "f64", eps_rel: float = 0.0, op: Operator = None, stream=None,
                 in_place: bool = False):
        self.N, self.M, self.method, self.degree, self.dtype = N, M, method, degree, dtype
        self.op = op
        self.stream = L.stream_handle(stream)
        meth, inner = L.parse_method(method)
        self.ws = None
        if in_place:
            if dtype != "f64" or method not in ("extrap", "spextrap", "last"):
                raise ValueError("in_place needs an FP64 extrapolation context")
            need = L.guess_workspace_bytes(N, M, meth, L.DTYPES[dtype])
            self.ws = torch.empty(need + 256, dtype=torch.uint8, device="cuda")
            off = (-self.ws.data_ptr()) % 256
            self.ws = self.ws[off:off + need]
        self.handle = L.guess_create_ex(N, M, meth, degree, L.DTYPES[dtype], eps_rel,
                                        op.handle if op is not None else None, self.stream, inner,
                                        workspace=self.ws)

    def slot(self) -> torch.Tensor:
        """View of the ring slot the next update writes (in_place contexts)."""
        if self.ws is None:
            raise ValueError("slot() needs a context made with in_place=True")
        off = L.guess_next_slot(self.handle) - self.ws.data_ptr()
        return self.ws[off:off + 8 * self.N].view(torch.float64)

    def form(self, b: torch.Tensor = None, out: torch.Tensor = None) -> torch.Tensor:
        out = _dev_f64(self.N, b.device if b is not None else "cuda") if out is None else out
        L.guess_form(self.handle, b, out)
        return out

    def update(self, x: torch.Tensor, Ax: torch.Tensor = None) -> None:
        L.guess_update(self.handle, x, Ax)

    def info(self) -> dict:
        return L.guess_get_info(self.handle)

    def reset(self) -> None:
        L.guess_reset(self.handle)

    def history(self, j: int, which: int = 0) -> torch.Tensor:
        out = _dev_f64(self.N)
        L.guess_history_get(self.handle, which, j, out)
        return out

    def close(self):
        if getattr(self, "handle", None):
            L.guess_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class PlaneWaveRHS:
    """b(t) = sum_k c_k sin(w_k t + phi_k) cos(2 pi k.x + theta_k) evaluated on the device.

    ``params`` is a dict with keys k (K x 3), theta, phi, w (as drawn by the
    seeded input generator); evaluation runs in the library's RHS kernel.
    """

    def __init__(self, params: dict, n: int, stream=None):
        self.n = n
        self.N = n ** 3
        self.kvec = [int(v) for v in params["k"].reshape(-1)]
        self.theta = [float(v) for v in params["theta"]]
        self.phi = [float(v) for v in params["phi"]]
        self.w = [float(v) for v in params["w"]]
        self.stream = L.stream_handle(stream)

    def amplitudes(self, t: float, c=None):
        a = [math.sin(w * t + p) for w, p in zip(self.w, self.phi)]
        if c is not None:
            a = [ai * float(ci) for ai, ci in zip(a, c)]
        return a

    def __call__(self, t: float, out: torch.Tensor = None, c=None) -> torch.Tensor:
        out = _dev_f64(self.N) if out is None else out
        L.workload_plane_wave_rhs(self.n, self.kvec, self.theta, self.amplitudes(t, c), out, self.stream)
        return out


def run_sequence(op: Operator, rhs_fn, T: int, method: str = "extrap", M: int = 8, degree: int = 2,
                 dtype: str = "f64", rtol: float = 1e-8, maxit: int = 20000, eps_rel: float = 0.0,
                 keep: bool = False, timing: bool = False):
    """Step loop: for n = 1..T, b = rhs_fn(n) -> guess -> PCG -> update.

    ``rhs_fn(n, out)`` fills the right-hand side of step n (1-based) into
    ``out``.  Returns per-step iteration counts, residuals and, with
    ``timing``, device times of guess form / update / solve in ms.
    """
    N = op.N
    g = GuessSequence(N, M, method, degree, dtype, eps_rel, op)
    b = _dev_f64(N)
    x = _dev_f64(N)
    out = {"iters": [], "relres": [], "status": [], "guesses": [], "solutions": [],
           "form_ms": [], "update_ms": [], "solve_ms": [], "form_bytes": [], "update_bytes": []}
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if timing else None
    for n in range(1, T + 1):
        rhs_fn(n, b)
        if timing:
            ev[0].record()
        g.form(b, x)
        if timing:
            ev[1].record()
        if keep:
            out["guesses"].append(x.clone())
        st, it, rr = op.solve(b, x, rtol, maxit)
        if timing:
            ev[2].record()
        g.update(x)
        if timing:
            ev[3].record()
            torch.cuda.synchronize()
            out["form_ms"].append(ev[0].elapsed_time(ev[1]))
            out["solve_ms"].append(ev[1].elapsed_time(ev[2]))
            out["update_ms"].append(ev[2].elapsed_time(ev[3]))
            inf = g.info()
            out["form_bytes"].append(inf["form_bytes"])
            out["update_bytes"].append(inf["update_bytes"])
        out["iters"].append(it)
        out["relres"].append(rr)
        out["status"].append(st)
        if keep:
            out["solutions"].append(x.clone())
    out["info"] = g.info()
    g.close()
    return out
