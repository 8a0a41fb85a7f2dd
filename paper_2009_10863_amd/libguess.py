"""ctypes binding of the libguess C ABI (``include/libguess.h``).

Argument marshalling only: every function below forwards to the entry point
of the same name in ``libguess.so``; all arithmetic runs in the library's HIP
kernels.  Vector arguments may be raw device addresses (int) or torch CUDA
tensors of dtype float64 (their ``data_ptr()`` is passed).  Errors raise
``GuessError`` with the library's message.  Importing this module fails
loudly when the shared library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("LIBGUESS_SO") or os.path.join(_HERE, "_lib", "libguess.so")

# ---------------------------------------------------------------- constants
ZERO, LAST, EXTRAP, PROJ, SPEXTRAP, PROJ_QR, PROJ_RAW, PROJ_RAW_QR = 0, 1, 2, 3, 4, 5, 6, 7
INNER_A, INNER_L2 = 0, 1
F64, F32, F16, BF16 = 0, 1, 2, 3
ROOF_COPY, ROOF_READ, ROOF_WRITE, ROOF_READ_STREAMS = 0, 1, 2, 3
OK, EINVAL, ENOMEM, EHIP, ENOTCONV, EBREAKDOWN, ENONFINITE = 0, -1, -2, -3, -4, -5, -6
STOP_RHS, STOP_INITRESID = 0, 1
MAX_M = 16
METHODS = {"zero": ZERO, "last": LAST, "extrap": EXTRAP, "proj": PROJ, "spextrap": SPEXTRAP,
           "projqr": PROJ_QR, "proj_raw": PROJ_RAW, "projqr_raw": PROJ_RAW_QR}
# method names with an inner-product suffix: "proj_l2", "projqr_l2"
PROJ_METHODS = ("proj", "projqr", "proj_l2", "projqr_l2", "proj_raw", "projqr_raw")


def parse_method(name: str):
    """(method, inner) of a method name; projection names take an optional "_l2" suffix."""
    if name.endswith("_l2") and name[:-3] in ("proj", "projqr"):
        return METHODS[name[:-3]], INNER_L2
    return METHODS[name], INNER_A
DTYPES = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
ELEM_BYTES = {F64: 8, F32: 4, F16: 2, BF16: 2}


class GuessError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libguess error {code}: {msg}")
        self.code = code


class guess_opts(C.Structure):
    _fields_ = [("N", C.c_int64), ("M", C.c_int), ("method", C.c_int), ("degree", C.c_int),
                ("dtype", C.c_int), ("eps_rel", C.c_double), ("op", C.c_void_p),
                ("stream", C.c_void_p), ("inner", C.c_int), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t)]


class guess_info(C.Structure):
    _fields_ = [("N", C.c_int64), ("method", C.c_int), ("dtype", C.c_int), ("M", C.c_int),
                ("degree", C.c_int), ("count", C.c_int), ("head", C.c_int),
                ("last_accepted", C.c_int), ("restarts", C.c_int), ("rejects", C.c_int),
                ("nonfinite", C.c_int), ("nu", C.c_double), ("nu0", C.c_double),
                ("form_bytes", C.c_double), ("update_bytes", C.c_double),
                ("drops", C.c_int), ("inner", C.c_int), ("eps_rel", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libguess.so not built at {LIB_PATH}; run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P, I, I64, D, S = C.c_void_p, C.c_int, C.c_int64, C.c_double, C.c_size_t
    sig = {
        "guess_op_create": (I, [I, I, I, D, D, P, C.POINTER(P)]),
        "guess_op_destroy": (None, [P]),
        "guess_op_set_stream": (I, [P, P]),
        "guess_op_size": (I64, [P]),
        "guess_next_slot": (I, [P, C.POINTER(C.c_void_p)]),
        "op_apply": (I, [P, P, P]),
        "pcg_solve": (I, [P, P, P, D, I, C.POINTER(I), C.POINTER(D)]),
        "pcg_solve_ex": (I, [P, P, P, D, I, I, C.POINTER(I), C.POINTER(D)]),
        "guess_create": (P, [I64, I, I, I]),
        "guess_create_ex": (I, [C.POINTER(guess_opts), C.POINTER(P)]),
        "guess_destroy": (None, [P]),
        "guess_set_stream": (I, [P, P]),
        "guess_set_op": (I, [P, P]),
        "guess_workspace_bytes": (S, [I64, I, I, I]),
        "guess_form": (I, [P, P, P]),
        "guess_update": (I, [P, P, P]),
        "guess_get_info": (I, [P, C.POINTER(guess_info)]),
        "guess_reset": (I, [P]),
        "guess_extrap_weights": (I, [I, I, C.POINTER(D)]),
        "guess_spextrap_weights": (I, [I, I, C.POINTER(D)]),
        "guess_history_get": (I, [P, I, I, P]),
        "guess_history_raw": (I, [P, I, I, P, C.POINTER(D)]),
        "guess_proj_factor": (I, [P, C.POINTER(D), C.POINTER(I)]),
        "workload_plane_wave_rhs": (I, [I, I, C.POINTER(I), C.POINTER(D), C.POINTER(D), P, P]),
        "workload_gaussian_rhs": (I, [I, C.POINTER(D), D, D, P, P]),
        "vec_multidot": (I, [I64, I, P, P, C.POINTER(D), P]),
        "vec_multidot_noalloc": (I, [I64, I, P, P, C.POINTER(D), P]),
        "vec_combine": (I, [I64, I, P, C.POINTER(D), P, P]),
        "guess_strerror": (C.c_char_p, [I]),
        "guess_last_error": (C.c_char_p, []),
        "guess_copy_kernel": (I, [P, P, S, P]),
        "guess_roof_kernel": (I, [I, P, P, S, P]),
        "guess_profile": (I, [P, I]),
        "guess_kernel_times": (I, [P, C.POINTER(D), I, C.POINTER(I)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load()
EXPORTED = (
    "guess_op_create", "guess_op_destroy", "guess_op_set_stream", "guess_op_size", "op_apply",
    "pcg_solve", "pcg_solve_ex", "guess_create", "guess_create_ex", "guess_destroy",
    "guess_set_stream", "guess_set_op", "guess_workspace_bytes", "guess_form", "guess_update",
    "guess_get_info", "guess_reset", "guess_extrap_weights", "guess_spextrap_weights", "guess_history_get",
    "guess_history_raw", "guess_proj_factor", "guess_next_slot",
    "workload_plane_wave_rhs", "workload_gaussian_rhs", "vec_multidot", "vec_multidot_noalloc", "vec_combine", "guess_strerror",
    "guess_last_error", "guess_copy_kernel", "guess_roof_kernel", "guess_profile", "guess_kernel_times",
)


def lib():
    return _lib


def _check(code):
    if code != OK:
        raise GuessError(code, _lib.guess_last_error().decode() or _lib.guess_strerror(code).decode())
    return code


def addr(v, need=None, what="vector", f64=True) -> int:
    """Device address of a vector argument (int, None, or torch tensor).  For a tensor,
    `need` is the number of elements (float64 unless f64 is False, then bytes) that the
    call reads or writes through it: a smaller tensor is refused here, since the library
    cannot see the size of a device buffer."""
    if v is None:
        return None
    if isinstance(v, int):
        return v
    import torch

    if not isinstance(v, torch.Tensor):
        raise TypeError("expected a device address or a torch tensor")
    if f64 and v.dtype != torch.float64:
        raise TypeError(f"{what}: libguess vectors are float64, got {v.dtype}")
    if need is not None:
        have = v.numel() if f64 else v.numel() * v.element_size()
        if have < need:
            raise ValueError(f"{what}: the call needs {need} {'elements' if f64 else 'bytes'}, "
                             f"the tensor has {have}")
    if not v.is_cuda:
        raise ValueError("libguess needs device (HIP) tensors")
    if not v.is_contiguous():
        raise ValueError("libguess needs contiguous tensors")
    return v.data_ptr()


# unknowns of the operators and contexts made through this module (tensor size checks)
_sizes: dict = {}


def stream_handle(stream=None):
    """hipStream_t of a torch stream (default: torch's current stream)."""
    import torch

    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


# ---------------------------------------------------------------- operator
def guess_op_create(nx, ny, nz, inv_h2, shift, kappa=None) -> int:
    out = C.c_void_p()
    kp = addr(kappa, (nx + 2) * (ny + 2) * (nz + 2) if min(nx, ny, nz) > 0 else None, "kappa")
    _check(_lib.guess_op_create(nx, ny, nz, inv_h2, shift, kp, C.byref(out)))
    _sizes[out.value] = nx * ny * nz
    return out.value


def guess_op_destroy(A) -> None:
    _sizes.pop(A, None)
    _lib.guess_op_destroy(A)


def guess_op_set_stream(A, stream) -> None:
    _check(_lib.guess_op_set_stream(A, stream))


def guess_op_size(A) -> int:
    return _lib.guess_op_size(A)


def op_apply(A, x, y) -> None:
    n = _sizes.get(A)
    _check(_lib.op_apply(A, addr(x, n, "x"), addr(y, n, "y")))


def pcg_solve(A, b, x, rtol=1e-8, maxit=10000, stop_rule=STOP_RHS, check=True):
    """Returns (status, iterations, relres)."""
    it, rr = C.c_int(0), C.c_double(0.0)
    n = _sizes.get(A)
    code = _lib.pcg_solve_ex(A, addr(b, n, "b"), addr(x, n, "x"), rtol, maxit, stop_rule, C.byref(it),
                             C.byref(rr))
    if check and code not in (OK, ENOTCONV, EBREAKDOWN):
        _check(code)
    return code, it.value, rr.value


# ---------------------------------------------------------------- contexts
def guess_create(N, M, method, degree) -> int:
    g = _lib.guess_create(N, M, method, degree)
    if not g:
        raise GuessError(EINVAL, _lib.guess_last_error().decode())
    _sizes[g] = N
    return g


def guess_create_ex(N, M, method, degree=0, dtype=F64, eps_rel=0.0, op=None, stream=None,
                    inner=INNER_A, workspace=None) -> int:
    """workspace: None, or a device tensor (or address) of at least guess_workspace_bytes
    bytes, 256-byte aligned, that holds the context's device buffers; it must outlive the context."""
    nbytes = 0
    if workspace is not None and not isinstance(workspace, int):
        nbytes = workspace.numel() * workspace.element_size()
    o = guess_opts(N=N, M=M, method=method, degree=degree, dtype=dtype, eps_rel=eps_rel,
                   op=op, stream=stream, inner=inner, workspace=addr(workspace, f64=False), workspace_bytes=nbytes)
    out = C.c_void_p()
    _check(_lib.guess_create_ex(C.byref(o), C.byref(out)))
    _sizes[out.value] = N
    return out.value


def guess_destroy(g) -> None:
    _sizes.pop(g, None)
    _lib.guess_destroy(g)


def guess_set_stream(g, stream) -> None:
    _check(_lib.guess_set_stream(g, stream))


def guess_set_op(g, A) -> None:
    _check(_lib.guess_set_op(g, A))


def guess_workspace_bytes(N, M, method, dtype) -> int:
    return _lib.guess_workspace_bytes(N, M, method, dtype)


def guess_form(g, b, x0) -> None:
    n = _sizes.get(g)
    _check(_lib.guess_form(g, addr(b, n, "b"), addr(x0, n, "x0")))


def guess_update(g, x, Ax=None) -> None:
    n = _sizes.get(g)
    _check(_lib.guess_update(g, addr(x, n, "x"), addr(Ax, n, "Ax")))


def guess_next_slot(g) -> int:
    """Device address of the ring slot the next update writes (FP64 extrapolation contexts)."""
    out = C.c_void_p()
    _check(_lib.guess_next_slot(g, C.byref(out)))
    return out.value


def guess_get_info(g) -> dict:
    info = guess_info()
    _check(_lib.guess_get_info(g, C.byref(info)))
    return info.as_dict()


def guess_reset(g) -> None:
    _check(_lib.guess_reset(g))


def guess_extrap_weights(m, k):
    buf = (C.c_double * k)()
    _check(_lib.guess_extrap_weights(m, k, buf))
    return list(buf)


def guess_spextrap_weights(m, k):
    buf = (C.c_double * k)()
    _check(_lib.guess_spextrap_weights(m, k, buf))
    return list(buf)


def guess_history_get(g, which, j, out) -> None:
    _check(_lib.guess_history_get(g, which, j, addr(out, _sizes.get(g), "out")))


def guess_history_raw(g, which, j, out) -> float:
    """Stored values of history vector j, widened without scale, into out; returns the FP64
    scale that turns them into the true values."""
    sc = C.c_double(0.0)
    _check(_lib.guess_history_raw(g, which, j, addr(out, _sizes.get(g), "out"), C.byref(sc)))
    return sc.value


def guess_proj_factor(g):
    """(d x d) triangular factor R of the projection history (raw solutions = X R)."""
    import numpy as np

    buf = (C.c_double * (MAX_M * MAX_M))()
    d = C.c_int(0)
    _check(_lib.guess_proj_factor(g, buf, C.byref(d)))
    n = d.value
    return np.array(buf[: n * n], dtype=np.float64).reshape(n, n)


def guess_profile(g, enable=True) -> None:
    _check(_lib.guess_profile(g, 1 if enable else 0))


def guess_kernel_times(g):
    """Device ms of each kernel launched by the last form / update call."""
    buf = (C.c_double * 8)()
    n = C.c_int(0)
    _check(_lib.guess_kernel_times(g, buf, 8, C.byref(n)))
    return list(buf[: n.value])


# ---------------------------------------------------------------- workload and vectors
def workload_plane_wave_rhs(n, kvec, theta, amp, b, stream=None) -> None:
    K = len(theta)
    kv = (C.c_int * (3 * K))(*[int(v) for v in kvec])
    th = (C.c_double * K)(*[float(v) for v in theta])
    am = (C.c_double * K)(*[float(v) for v in amp])
    _check(_lib.workload_plane_wave_rhs(n, K, kv, th, am, addr(b, n ** 3 if n > 0 else None, "b"), stream))


def workload_gaussian_rhs(n, center, sigma, amp, b, stream=None) -> None:
    c = (C.c_double * 3)(*[float(v) for v in center])
    _check(_lib.workload_gaussian_rhs(n, c, float(sigma), float(amp), addr(b, n ** 3 if n > 0 else None, "b"),
                                      stream))


def vec_multidot(N, K, V, y, stream=None):
    out = (C.c_double * K)()
    ok = N > 0 and K > 0
    _check(_lib.vec_multidot(N, K, addr(V, N * K if ok else None, "V"), addr(y, N if ok else None, "y"), out,
                             stream))
    return list(out)


def vec_multidot_noalloc(N, K, V, y, stream=None):
    """vec_multidot without any device allocation (the library's static scratch)."""
    out = (C.c_double * K)()
    ok = N > 0 and K > 0
    _check(_lib.vec_multidot_noalloc(N, K, addr(V, N * K if ok else None, "V"), addr(y, N if ok else None, "y"),
                                     out, stream))
    return list(out)


def vec_combine(N, K, V, c, y, stream=None) -> None:
    cc = (C.c_double * K)(*[float(v) for v in c])
    ok = N > 0 and K > 0
    _check(_lib.vec_combine(N, K, addr(V, N * K if ok else None, "V"), cc, addr(y, N if ok else None, "y"),
                            stream))


def guess_copy_kernel(dst, src, nbytes, stream=None) -> None:
    _check(_lib.guess_copy_kernel(addr(dst, nbytes, "dst", f64=False), addr(src, nbytes, "src", f64=False),
                                  nbytes, stream))


def guess_roof_kernel(mode, dst, src, nbytes, stream=None) -> None:
    """Copy / read-only / write-only bandwidth reference (the read mode writes 2048 partial
    sums into dst)."""
    need_dst = 2048 * 8 if mode in (ROOF_READ, ROOF_READ_STREAMS) else nbytes
    _check(_lib.guess_roof_kernel(mode, addr(dst, need_dst, "dst", f64=False),
                                  addr(src, nbytes if mode != ROOF_WRITE else None, "src", f64=False),
                                  nbytes, stream))


def guess_strerror(code) -> str:
    return _lib.guess_strerror(code).decode()


def guess_last_error() -> str:
    return _lib.guess_last_error().decode()
