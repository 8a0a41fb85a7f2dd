"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and builds input fields (right-hand sides,
coefficient fields, regression targets, smooth histories).  It holds none of
the initial-guess arithmetic: no extrapolation weights, no inner products of
the method, no operator, no solver.  Both the CPU oracle and the HIP path take
their inputs from here, so that the two see identical data.

Grid convention used everywhere: an ``n x n x n`` grid of interior nodes of the
unit cube, spacing ``h = 1/(n+1)``, node ``(i, j, l)`` (1-based) at
``(i h, j h, l h)``, flattened lexicographically with ``i`` (x) fastest:
``flat = ((l-1) n + (j-1)) n + (i-1)``.  Boundary nodes carry the Dirichlet
value 0 and are not stored.

Workload recipe (plane waves): ``K`` distinct wave vectors ``k`` drawn from
``{1..kmax}^3``, phases ``theta_k`` and ``phi_k`` uniform on ``[0, 2 pi)``,
angular rates ``w_k`` uniform on ``[1, 5]`` -- drawn in that order from
``numpy.random.default_rng(seed)``.  Mode ``f_k(x) = cos(2 pi k.x + theta_k)``;
right-hand side at time ``t``: ``b(t) = sum_k c_k sin(w_k t + phi_k) f_k``.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


# --------------------------------------------------------------------------
# grid helpers
# --------------------------------------------------------------------------
def axis_coords(n: int) -> np.ndarray:
    """Coordinates ``i h`` (i = 1..n) of the interior nodes along one axis."""
    h = 1.0 / (n + 1)
    return np.arange(1, n + 1, dtype=np.float64) * h


def flat_index(i, j, l, n):
    """Flat index of 0-based interior node (i, j, l), x fastest."""
    return (np.asarray(l) * n + np.asarray(j)) * n + np.asarray(i)


# --------------------------------------------------------------------------
# plane-wave right-hand sides
# --------------------------------------------------------------------------
def plane_wave_params(seed: int, K: int, kmax: int = 4) -> dict:
    """Draw the parameters of a K-mode plane-wave workload (see module doc)."""
    if K > kmax ** 3:
        raise ValueError("K exceeds the number of distinct wave vectors")
    rng = np.random.default_rng(seed)
    code = rng.choice(kmax ** 3, size=K, replace=False)
    kx = code % kmax + 1
    ky = (code // kmax) % kmax + 1
    kz = code // (kmax * kmax) + 1
    theta = rng.uniform(0.0, TWO_PI, size=K)
    phi = rng.uniform(0.0, TWO_PI, size=K)
    w = rng.uniform(1.0, 5.0, size=K)
    return {
        "k": np.stack([kx, ky, kz], axis=1).astype(np.int64),
        "theta": theta,
        "phi": phi,
        "w": w,
        "K": K,
        "seed": seed,
    }


def mode_amplitudes(params: dict, t: float) -> np.ndarray:
    """``s_k(t) = sin(w_k t + phi_k)`` for every mode k."""
    return np.sin(params["w"] * t + params["phi"])


def plane_wave_modes(params: dict, n: int) -> np.ndarray:
    """Dense K x N matrix of mode values ``f_k`` at the interior nodes."""
    x = axis_coords(n)
    K = params["K"]
    out = np.empty((K, n * n * n), dtype=np.float64)
    for q in range(K):
        kx, ky, kz = params["k"][q]
        ph = (TWO_PI * kx * x)[None, None, :] + (TWO_PI * ky * x)[None, :, None] \
            + (TWO_PI * kz * x)[:, None, None] + params["theta"][q]
        out[q] = np.cos(ph).reshape(-1)
    return out


def plane_wave_rhs(params: dict, n: int, t: float, c=None, modes=None) -> np.ndarray:
    """``b(t) = sum_k c_k sin(w_k t + phi_k) f_k`` at the interior nodes."""
    a = mode_amplitudes(params, t)
    if c is not None:
        a = a * np.asarray(c, dtype=np.float64)
    F = plane_wave_modes(params, n) if modes is None else modes
    return a @ F


def plane_wave_rhs_at(params: dict, n: int, t: float, flat_idx, c=None) -> np.ndarray:
    """Values of ``b(t)`` at selected flat indices only (for huge grids)."""
    flat_idx = np.asarray(flat_idx, dtype=np.int64)
    i = flat_idx % n
    j = (flat_idx // n) % n
    l = flat_idx // (n * n)
    h = 1.0 / (n + 1)
    xs, ys, zs = (i + 1) * h, (j + 1) * h, (l + 1) * h
    a = mode_amplitudes(params, t)
    if c is not None:
        a = a * np.asarray(c, dtype=np.float64)
    out = np.zeros(flat_idx.shape, dtype=np.float64)
    for q in range(params["K"]):
        kx, ky, kz = params["k"][q]
        out += a[q] * np.cos(TWO_PI * kx * xs + TWO_PI * ky * ys + TWO_PI * kz * zs
                             + params["theta"][q])
    return out


# --------------------------------------------------------------------------
# moving Gaussian source (solutions not confined to a fixed low-rank space)
# --------------------------------------------------------------------------
def gaussian_source_params(seed: int, sigma: float = 0.08, radius: float = 0.25, amp: float = 1.0e3) -> dict:
    """Center path ``c(t) = 0.5 + radius * sin(om * t + ph)`` per axis, ``om ~ U[1, 5]``,
    ``ph ~ U[0, 2 pi)``, drawn in that order."""
    rng = np.random.default_rng(seed)
    om = rng.uniform(1.0, 5.0, 3)
    ph = rng.uniform(0.0, TWO_PI, 3)
    return {"omega": om, "phi": ph, "sigma": float(sigma), "radius": float(radius), "amp": float(amp)}


def gaussian_center(params: dict, t: float) -> np.ndarray:
    return 0.5 + params["radius"] * np.sin(params["omega"] * t + params["phi"])


def gaussian_source_rhs(params: dict, n: int, t: float) -> np.ndarray:
    """``b = amp * (g_x(i) * (g_y(j) * g_z(l)))``, ``g_a = exp(-(x - c_a)^2 / (2 sigma^2))``
    at the interior nodes ``x_i = (i + 1) / (n + 1)``, x fastest."""
    c = gaussian_center(params, t)
    x = (np.arange(n, dtype=np.float64) + 1.0) * (1.0 / (n + 1))
    inv2s2 = 1.0 / (2.0 * params["sigma"] * params["sigma"])
    g = [np.exp(-((x - c[a]) * (x - c[a])) * inv2s2) for a in range(3)]
    yz = g[1][None, :, None] * g[2][:, None, None]
    return (params["amp"] * (g[0][None, None, :] * yz)).reshape(-1)


def step_times(T: int, dt: float) -> np.ndarray:
    """``t_n = n dt`` for n = 1..T."""
    return np.arange(1, T + 1, dtype=np.float64) * dt


# --------------------------------------------------------------------------
# Dirichlet sine modes (exact eigenvectors of the constant-coefficient
# 7-point operator; used where closed forms are wanted)
# --------------------------------------------------------------------------
def sine_mode(p: int, q: int, r: int, n: int) -> np.ndarray:
    """``sin(p pi x) sin(q pi y) sin(r pi z)`` at the interior nodes."""
    x = axis_coords(n)
    sx, sy, sz = np.sin(p * math.pi * x), np.sin(q * math.pi * x), np.sin(r * math.pi * x)
    return (sz[:, None, None] * sy[None, :, None] * sx[None, None, :]).reshape(-1)


# --------------------------------------------------------------------------
# Gaussian random field for the variable coefficient kappa = exp(g)
# --------------------------------------------------------------------------
def gaussian_field(seed: int, n: int, ell: float = 0.1) -> np.ndarray:
    """Unit-variance Gaussian field with squared-exponential covariance.

    Sampled on all ``(n+2)^3`` nodes (boundary included), x fastest.  White
    noise is smoothed per axis by a 1-D Gaussian of standard deviation
    ``ell/sqrt(2)`` (so that the covariance is ``exp(-r^2 / (2 ell^2))``),
    then shifted to zero sample mean and scaled to unit sample variance.
    """
    from scipy.ndimage import gaussian_filter1d

    m = n + 2
    h = 1.0 / (n + 1)
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((m, m, m))
    sig = (ell / math.sqrt(2.0)) / h
    for ax in range(3):
        g = gaussian_filter1d(g, sig, axis=ax, mode="reflect", truncate=4.0)
    g = g - g.mean()
    g = g / g.std()
    return np.ascontiguousarray(g.reshape(-1))


# --------------------------------------------------------------------------
# regression targets for the differentiation workload
# --------------------------------------------------------------------------
def target_params(seed: int, J: int = 4, kmax: int = 4) -> dict:
    """Parameters of ``y(t) = 0.01 sum_j sin(om_j t + psi_j) cos(2 pi k'_j.x + th'_j)``."""
    rng = np.random.default_rng(seed)
    code = rng.choice(kmax ** 3, size=J, replace=False)
    k = np.stack([code % kmax + 1, (code // kmax) % kmax + 1, code // (kmax * kmax) + 1],
                 axis=1).astype(np.int64)
    theta = rng.uniform(0.0, TWO_PI, size=J)
    psi = rng.uniform(0.0, TWO_PI, size=J)
    om = rng.uniform(1.0, 5.0, size=J)
    return {"k": k, "theta": theta, "phi": psi, "w": om, "K": J, "seed": seed, "scale": 0.01}


def target_field(tparams: dict, n: int, t: float) -> np.ndarray:
    return tparams["scale"] * plane_wave_rhs(tparams, n, t)


# --------------------------------------------------------------------------
# generic seeded vectors
# --------------------------------------------------------------------------
def random_vectors(seed: int, count: int, N: int) -> np.ndarray:
    """``count`` standard-normal vectors of length N (count x N)."""
    return np.random.default_rng(seed).standard_normal((count, N))


def polynomial_in_time_history(seed: int, degree: int, N: int, times) -> np.ndarray:
    """Rows ``x(t) = sum_{q<=degree} t^q v_q`` for each t in ``times``.

    The ``v_q`` are seeded standard normals.  Returned as len(times) x N, plus
    the coefficient vectors (degree+1) x N so that a caller can evaluate x at
    any other time.
    """
    V = np.random.default_rng(seed).standard_normal((degree + 1, N))
    times = np.asarray(times, dtype=np.float64)
    X = np.stack([sum((t ** q) * V[q] for q in range(degree + 1)) for t in times])
    return X, V
