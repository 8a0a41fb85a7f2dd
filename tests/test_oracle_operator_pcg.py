"""Pins of the oracle's operators, exact solver and PCG.

Independent references: closed-form eigenpairs of the 7-point Dirichlet
Laplacian (sine modes), sparse matrices assembled a different way (Kronecker
sums; divergence form D^T diag(k) D), scipy's sparse direct solver and scipy's
conjugate-gradient routine, and CG's finite termination on a right-hand side
spanned by K eigenvectors.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import synth
from oracle import operator as op
from oracle.pcg import pcg, OK, NOTCONV


def kron_matrix(n, shift=10.0):
    c = float((n + 1) ** 2)
    T = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    I = sp.identity(n)
    L = sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)
    return (c * L + shift * sp.identity(n ** 3)).tocsr()


def divergence_form_matrix(n, kappa_nodal, shift=10.0):
    """A = c D^T diag(k_f) D + shift I with D the face-difference matrix.

    D maps the n^3 interior values (plus zero boundary values) to differences
    across every face touching an interior node; k_f is the harmonic mean of
    the nodal kappa on the two ends of the face.
    """
    m = n + 2
    K = kappa_nodal.reshape(m, m, m)
    rows, cols, vals, kf = [], [], [], []
    idx = lambda i, j, l: (l * n + j) * n + i          # noqa: E731
    r = 0
    # faces along each axis between padded nodes p and p+1 (p = 0..n)
    for axis in range(3):
        for l in range(n if axis != 2 else n + 1):
            for j in range(n if axis != 1 else n + 1):
                for i in range(n if axis != 0 else n + 1):
                    # ends a (lower) and b (upper) in padded coordinates (i, j, l) order x, y, z
                    a = [i + 1, j + 1, l + 1]
                    a[axis] -= 1
                    b = [i + 1, j + 1, l + 1]
                    ka, kb = K[a[2], a[1], a[0]], K[b[2], b[1], b[0]]
                    kf.append(2 * ka * kb / (ka + kb))
                    for sgn, pnt in ((-1.0, a), (1.0, b)):
                        if all(1 <= pnt[q] <= n for q in range(3)):
                            rows.append(r)
                            cols.append(idx(pnt[0] - 1, pnt[1] - 1, pnt[2] - 1))
                            vals.append(sgn)
                    r += 1
    D = sp.csr_matrix((vals, (rows, cols)), shape=(r, n ** 3))
    c = float((n + 1) ** 2)
    return (c * (D.T @ sp.diags(kf) @ D) + shift * sp.identity(n ** 3)).tocsr()


# ---------------------------------------------------------------- operator
@pytest.mark.parametrize("n", [4, 7])
def test_const_matches_kronecker_sum(n):
    A = kron_matrix(n)
    u = synth.random_vectors(1, 3, n ** 3)
    for v in u:
        np.testing.assert_allclose(op.apply_const(v, n), A @ v, rtol=1e-13, atol=1e-13 * np.abs(A @ v).max())
    Ad = A.toarray()
    assert np.array_equal(Ad, Ad.T)
    assert np.linalg.eigvalsh(Ad).min() > 0
    assert np.all(op.diag_const(n) == A.diagonal())


@pytest.mark.parametrize("pqr", [(1, 1, 1), (2, 3, 1), (5, 1, 4)])
def test_sine_modes_are_eigenvectors(pqr):
    n = 9
    u = synth.sine_mode(*pqr, n)
    lam = op.eigenvalues_const(n)[pqr[2] - 1, pqr[1] - 1, pqr[0] - 1]
    np.testing.assert_allclose(op.apply_const(u, n), lam * u, rtol=0, atol=1e-12 * lam)


@pytest.mark.parametrize("n", [3, 5])
def test_varcoef_matches_divergence_form(n):
    g = synth.gaussian_field(3, n, ell=0.3)
    kappa = np.exp(g)
    A = divergence_form_matrix(n, kappa)
    faces = op.face_coeffs(kappa, n)
    for v in synth.random_vectors(2, 3, n ** 3):
        ref = A @ v
        np.testing.assert_allclose(op.apply_var(v, n, faces), ref, rtol=1e-12,
                                   atol=1e-12 * np.abs(ref).max())
    np.testing.assert_allclose(op.diag_var(n, faces), A.diagonal(), rtol=1e-14)
    Ad = A.toarray()
    np.testing.assert_allclose(Ad, Ad.T, rtol=0, atol=1e-9)
    assert np.linalg.eigvalsh(Ad).min() > 0


def test_varcoef_with_unit_kappa_is_const():
    n = 6
    faces = op.face_coeffs(np.ones((n + 2) ** 3), n)
    v = synth.random_vectors(5, 1, n ** 3)[0]
    np.testing.assert_allclose(op.apply_var(v, n, faces), op.apply_const(v, n), rtol=1e-13, atol=1e-10)


def test_boundary_neighbours_are_zero():
    """A vector supported on one corner node sees only its in-grid neighbours."""
    n = 5
    e = np.zeros(n ** 3)
    e[0] = 1.0
    y = op.apply_const(e, n)
    c = (n + 1) ** 2
    assert y[0] == 6 * c + 10
    assert y[1] == -c and y[n] == -c and y[n * n] == -c
    assert np.count_nonzero(y) == 4


@pytest.mark.parametrize("n", [5, 8])
def test_dst_solver_is_exact(n):
    b = synth.random_vectors(9, 1, n ** 3)[0]
    x = op.dst_solve(b, n)
    np.testing.assert_allclose(op.apply_const(x, n), b, rtol=0, atol=1e-11 * np.abs(b).max())
    ref = spla.spsolve(kron_matrix(n).tocsc(), b)
    np.testing.assert_allclose(x, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------- PCG
def scipy_cg_iters(A, b, x0, rtol, dinv):
    count = [0]
    Mop = spla.LinearOperator(A.shape, matvec=lambda r: dinv * r)
    x, info = spla.cg(A, b, x0=x0, rtol=rtol, atol=0.0, M=Mop, maxiter=5000,
                      callback=lambda xk: count.__setitem__(0, count[0] + 1))
    return x, count[0], info


@pytest.mark.parametrize("n,seed", [(8, 0), (12, 1)])
def test_pcg_matches_scipy_cg(n, seed):
    A = kron_matrix(n)
    params = synth.plane_wave_params(seed, 4)
    b = synth.plane_wave_rhs(params, n, 0.37)
    x0 = np.zeros_like(b)
    dinv = 1.0 / op.diag_const(n) * np.ones(n ** 3)
    x, it, st, _ = pcg(lambda v: op.apply_const(v, n), b, x0, dinv, rtol=1e-8)
    xs, its, info = scipy_cg_iters(A, b, x0, 1e-8, dinv)
    assert st == OK and info == 0
    assert abs(it - its) <= 1
    xe = op.dst_solve(b, n)
    assert np.linalg.norm(x - xe) <= 1e-6 * np.linalg.norm(xe)
    assert np.linalg.norm(b - A @ x) <= 1.01e-8 * np.linalg.norm(b)


def test_pcg_varcoef_matches_scipy_cg():
    n = 6
    kappa = np.exp(synth.gaussian_field(4, n, ell=0.2))
    A = divergence_form_matrix(n, kappa)
    faces = op.face_coeffs(kappa, n)
    dinv = 1.0 / op.diag_var(n, faces)
    b = synth.random_vectors(3, 1, n ** 3)[0]
    x, it, st, _ = pcg(lambda v: op.apply_var(v, n, faces), b, np.zeros_like(b), dinv, 1e-8)
    xs, its, info = scipy_cg_iters(A, b, np.zeros_like(b), 1e-8, dinv)
    assert st == OK and abs(it - its) <= 1
    np.testing.assert_allclose(x, xs, rtol=0, atol=1e-6 * np.abs(xs).max())


def test_pcg_finite_termination_on_eigenvectors():
    """A right-hand side in a K-dimensional invariant subspace converges in <= K steps."""
    n = 10
    modes = [(1, 1, 1), (2, 1, 3), (4, 2, 2), (3, 5, 1)]
    b = sum((q + 1.0) * synth.sine_mode(*pqr, n) for q, pqr in enumerate(modes))
    dinv = np.full(n ** 3, 1.0 / op.diag_const(n))
    x, it, st, _ = pcg(lambda v: op.apply_const(v, n), b, np.zeros_like(b), dinv, 1e-10)
    assert st == OK and it <= len(modes) + 1


def test_pcg_edge_cases():
    n = 5
    A = lambda v: op.apply_const(v, n)                  # noqa: E731
    dinv = np.full(n ** 3, 1.0 / op.diag_const(n))
    z = np.zeros(n ** 3)
    x, it, st, _ = pcg(A, z, z, dinv)                   # zero right-hand side
    assert it == 0 and st == OK and not x.any()
    b = synth.random_vectors(1, 1, n ** 3)[0]
    xe = op.dst_solve(b, n)
    x, it, st, _ = pcg(A, b, xe, dinv)                  # exact guess
    assert it == 0 and st == OK
    x, it, st, _ = pcg(A, b, z, dinv, rtol=1e-14, maxit=3)
    assert st == NOTCONV and it == 3
    # the paper's default rule stops on rtol * max(||r0||, 1)
    x, it, st, _ = pcg(A, 1e-12 * b, z, dinv, rule="initresid")
    assert it == 0 and st == OK
