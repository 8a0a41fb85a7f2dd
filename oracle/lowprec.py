"""Rounding of stored history to reduced precision (oracle; test infrastructure only).

The paper does not state a floating-point precision.  The low-precision
history forms store each history vector rounded to a narrower format while all
other arithmetic stays in FP64 (guess accumulation may be FP32).  Rounding is
round-to-nearest-even in two steps, FP64 -> FP32 -> target, which is what a
chain of hardware conversions does.

Each function returns float64 arrays holding exactly the representable stored
values, plus helpers that give the raw bit patterns so that stored bytes can
be compared bit for bit.
"""
from __future__ import annotations

import numpy as np

DTYPES = ("f64", "f32", "f16", "bf16")
BYTES = {"f64": 8, "f32": 4, "f16": 2, "bf16": 2}
# unit roundoff of each storage format
UNIT_ROUNDOFF = {"f64": 2.0 ** -53, "f32": 2.0 ** -24, "f16": 2.0 ** -11, "bf16": 2.0 ** -8}


def bf16_bits_from_f32(x32: np.ndarray) -> np.ndarray:
    """Upper 16 bits of FP32 values rounded to nearest even (NaN kept quiet)."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(x32)
    if nan.any():
        r = r.copy()
        r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


def bf16_bits_to_f32(bits: np.ndarray) -> np.ndarray:
    return (np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def stored_bits(x: np.ndarray, dtype: str, scale_exp: int = 0) -> np.ndarray:
    """Raw stored representation of x * 2^scale_exp in ``dtype``."""
    x = np.asarray(x, dtype=np.float64)
    if scale_exp:
        x = np.ldexp(x, scale_exp)
    if dtype == "f64":
        return x.copy()
    x32 = x.astype(np.float32)
    if dtype == "f32":
        return x32
    if dtype == "f16":
        with np.errstate(over="ignore"):   # beyond the FP16 range rounds to +-inf (IEEE)
            return x32.astype(np.float16)
    if dtype == "bf16":
        return bf16_bits_from_f32(x32)
    raise ValueError(dtype)


def decode(bits: np.ndarray, dtype: str, scale_exp: int = 0) -> np.ndarray:
    """Stored representation back to float64 values (exact)."""
    if dtype == "bf16":
        v = bf16_bits_to_f32(bits).astype(np.float64)
    else:
        v = np.asarray(bits).astype(np.float64)
    if scale_exp:
        v = np.ldexp(v, -scale_exp)
    return v


def round_store(x: np.ndarray, dtype: str, scale_exp: int = 0) -> np.ndarray:
    """Value actually held after storing x in ``dtype`` (float64 array)."""
    if dtype == "f64":
        return np.array(x, dtype=np.float64, copy=True)
    return decode(stored_bits(x, dtype, scale_exp), dtype, scale_exp)


def f16_scale_exp(maxabs: float) -> int:
    """Power-of-two exponent e with maxabs * 2^e in [2^14, 2^15).

    Used for FP16 storage so that the largest stored magnitude sits well
    inside the FP16 normal range (max 65504, min normal 2^-14) and no stored
    value of that vector can overflow.  Zero or non-finite maxabs gives e = 0;
    e is clamped to [-100, 100] (beyond that the data are far outside any
    range a solution of these systems takes), which keeps 2^-e times an
    extrapolation weight a normal FP32 number.
    """
    if not np.isfinite(maxabs) or maxabs <= 0.0:
        return 0
    _, E = np.frexp(maxabs)          # maxabs = f 2^E, f in [0.5, 1)
    return int(min(max(15 - E, -F16_EXP_CLAMP), F16_EXP_CLAMP))


F16_EXP_CLAMP = 100
