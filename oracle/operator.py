"""Matrix-free 7-point Helmholtz operators (oracle; test infrastructure only).

The paper's operator is a spectral-element discretisation inside an
incompressible-flow solver (§5); it is replaced here by the 7-point
finite-difference operators on an ``n^3`` grid of interior nodes of the unit
cube with zero Dirichlet values on the boundary (grid convention in
``synth``).  Two operators:

constant coefficient   (Au)_i = c (6 u_i - sum_nb u_nb) + s u_i
variable coefficient   (Au)_i = c sum_faces k_f (u_i - u_nb) + s u_i,
                       k_f = 2 k_i k_nb / (k_i + k_nb)  (harmonic mean)

with c = 1/h^2 = (n+1)^2 (exact in FP64) and shift s (10 in all workloads).
Nodal kappa lives on all (n+2)^3 nodes, boundary included.

The floating-point evaluation order is fixed so that any implementation that
follows it reproduces these results bit for bit: neighbour order
west(-x), east(+x), south(-y), north(+y), bottom(-z), top(+z), left to right,
no fused multiply-add, then ``c * s + shift * u``.
"""
from __future__ import annotations

import numpy as np


def inv_h2(n: int) -> float:
    return float((n + 1) * (n + 1))


def _pad(u: np.ndarray, n: int) -> np.ndarray:
    P = np.zeros((n + 2, n + 2, n + 2), dtype=np.float64)
    P[1:-1, 1:-1, 1:-1] = u.reshape(n, n, n)
    return P


def apply_const(u: np.ndarray, n: int, shift: float = 10.0, c: float = None) -> np.ndarray:
    """y = A u for the constant-coefficient operator (-Laplacian_h + shift I)."""
    c = inv_h2(n) if c is None else c
    return apply_const_box(u, (n, n, n), c, shift)


def apply_const_box(u: np.ndarray, shape, c: float, shift: float = 10.0) -> np.ndarray:
    """The same operator on an nx x ny x nz box of interior nodes, shape = (nx, ny, nz), x fastest."""
    nx, ny, nz = shape
    P = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.float64)
    P[1:-1, 1:-1, 1:-1] = np.asarray(u, dtype=np.float64).reshape(nz, ny, nx)
    U = P[1:-1, 1:-1, 1:-1]
    s = 6.0 * U
    s = s - P[1:-1, 1:-1, :-2]   # west
    s = s - P[1:-1, 1:-1, 2:]    # east
    s = s - P[1:-1, :-2, 1:-1]   # south
    s = s - P[1:-1, 2:, 1:-1]    # north
    s = s - P[:-2, 1:-1, 1:-1]   # bottom
    s = s - P[2:, 1:-1, 1:-1]    # top
    return (c * s + shift * U).reshape(-1)


def diag_const(n: int, shift: float = 10.0, c: float = None) -> float:
    c = inv_h2(n) if c is None else c
    return c * 6.0 + shift


def harmonic(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Face coefficient 2 a b / (a + b), evaluated as ((2a) b) / (a + b)."""
    return ((2.0 * a) * b) / (a + b)


def face_coeffs(kappa_nodal: np.ndarray, n: int):
    """Face coefficients of the variable-coefficient operator.

    Returns (kx, ky, kz) with shapes (n, n, n+1), (n, n+1, n), (n+1, n, n)
    in (z, y, x) order: ``kx[l, j, f]`` is the face between padded nodes
    f and f+1 along x at interior row (j, l); likewise for y and z.
    """
    return face_coeffs_box(kappa_nodal, (n, n, n))


def face_coeffs_box(kappa_nodal: np.ndarray, shape):
    """The same on an nx x ny x nz box: kappa on (nz+2, ny+2, nx+2) nodes, x fastest."""
    nx, ny, nz = shape
    K = np.asarray(kappa_nodal, dtype=np.float64).reshape(nz + 2, ny + 2, nx + 2)
    I = slice(1, -1)
    kx = harmonic(K[I, I, :-1], K[I, I, 1:])
    ky = harmonic(K[I, :-1, I], K[I, 1:, I])
    kz = harmonic(K[:-1, I, I], K[1:, I, I])
    return kx, ky, kz


def apply_var(u: np.ndarray, n: int, faces, shift: float = 10.0, c: float = None) -> np.ndarray:
    """y = A u for -div(kappa grad u) + shift u (harmonic-mean faces)."""
    c = inv_h2(n) if c is None else c
    return apply_var_box(u, (n, n, n), faces, c, shift)


def apply_var_box(u: np.ndarray, shape, faces, c: float, shift: float = 10.0) -> np.ndarray:
    """The same on an nx x ny x nz box (faces from face_coeffs_box)."""
    nx, ny, nz = shape
    kx, ky, kz = faces
    P = np.zeros((nz + 2, ny + 2, nx + 2), dtype=np.float64)
    P[1:-1, 1:-1, 1:-1] = np.asarray(u, dtype=np.float64).reshape(nz, ny, nx)
    U = P[1:-1, 1:-1, 1:-1]
    s = kx[:, :, :-1] * (U - P[1:-1, 1:-1, :-2])            # west
    s = s + kx[:, :, 1:] * (U - P[1:-1, 1:-1, 2:])          # east
    s = s + ky[:, :-1, :] * (U - P[1:-1, :-2, 1:-1])        # south
    s = s + ky[:, 1:, :] * (U - P[1:-1, 2:, 1:-1])          # north
    s = s + kz[:-1, :, :] * (U - P[:-2, 1:-1, 1:-1])        # bottom
    s = s + kz[1:, :, :] * (U - P[2:, 1:-1, 1:-1])          # top
    return (c * s + shift * U).reshape(-1)


def diag_var(n: int, faces, shift: float = 10.0, c: float = None) -> np.ndarray:
    c = inv_h2(n) if c is None else c
    kx, ky, kz = faces
    s = kx[:, :, :-1] + kx[:, :, 1:]
    s = s + ky[:, :-1, :]
    s = s + ky[:, 1:, :]
    s = s + kz[:-1, :, :]
    s = s + kz[1:, :, :]
    return (c * s + shift).reshape(-1)


class Operator:
    """Bundle of the operator, its Jacobi diagonal and (if constant) exact solver."""

    def __init__(self, n: int, shift: float = 10.0, kappa_nodal=None):
        self.n, self.shift = n, shift
        self.N = n ** 3
        self.c = inv_h2(n)
        self.faces = None if kappa_nodal is None else face_coeffs(kappa_nodal, n)

    def __call__(self, u: np.ndarray) -> np.ndarray:
        if self.faces is None:
            return apply_const(u, self.n, self.shift, self.c)
        return apply_var(u, self.n, self.faces, self.shift, self.c)

    def diag(self) -> np.ndarray:
        if self.faces is None:
            return np.full(self.N, diag_const(self.n, self.shift, self.c))
        return diag_var(self.n, self.faces, self.shift, self.c)

    def solve_exact(self, b: np.ndarray) -> np.ndarray:
        if self.faces is not None:
            raise NotImplementedError("closed-form solve only for constant coefficient")
        return dst_solve(b, self.n, self.shift, self.c)


def eigenvalues_const(n: int, shift: float = 10.0, c: float = None) -> np.ndarray:
    """Eigenvalues lambda_pqr on an (n, n, n) array indexed (r, q, p).

    The sine modes sin(p pi x) sin(q pi y) sin(r pi z) are eigenvectors of
    the constant-coefficient operator with eigenvalue
    shift + 4c [sin^2(p pi h/2) + sin^2(q pi h/2) + sin^2(r pi h/2)].
    """
    c = inv_h2(n) if c is None else c
    h = 1.0 / (n + 1)
    p = np.arange(1, n + 1)
    s2 = 4.0 * c * np.sin(p * np.pi * h / 2.0) ** 2
    return shift + s2[:, None, None] + s2[None, :, None] + s2[None, None, :]


def dst_solve(b: np.ndarray, n: int, shift: float = 10.0, c: float = None, workers: int = None) -> np.ndarray:
    """Exact solution of A x = b (constant coefficient) by DST-I diagonalisation.

    `workers` lets scipy spread the independent 1-D transforms over threads."""
    from scipy.fft import dstn, idstn

    B = np.asarray(b, dtype=np.float64).reshape(n, n, n)
    bh = dstn(B, type=1, norm="ortho", workers=workers)
    xh = bh / eigenvalues_const(n, shift, c)
    return idstn(xh, type=1, norm="ortho", workers=workers).reshape(-1)
