"""GPU checks of the differentiable solve sequence (reverse-time adjoint with its own guesses).

References: the oracle's FP64 gradient (exact DST solves) and central finite
differences of the GPU forward loss (L is exactly quadratic in c, so the
difference quotient is exact up to rounding and the solve tolerance).
"""
import numpy as np
import pytest

import synth
from gpu_helpers import announce, dev, host
from oracle import adjoint

pytestmark = pytest.mark.gpu


def setup_case(n=16, T=12, K=4, rtol=1e-12):
    from paper_2009_10863_amd.autograd import SolveSequence
    from paper_2009_10863_amd.sequence import Operator

    params = synth.plane_wave_params(3, K)
    tparams = synth.target_params(99)
    ts = synth.step_times(T, 0.005)
    S = np.stack([synth.mode_amplitudes(params, t) for t in ts])
    Fh = synth.plane_wave_modes(params, n)
    Y = np.stack([synth.target_field(tparams, n, t) for t in ts])
    op = Operator(n)
    seq = SolveSequence(op, dev(Fh.reshape(-1)).reshape(K, -1), S, method="extrap", M=8, degree=2,
                        rtol=rtol)
    return seq, Fh, S, Y, op


def test_gradient_matches_reference(lib):
    import torch

    from paper_2009_10863_amd.autograd import GuessSolveFn

    announce("adjoint gradient 16^3")
    seq, Fh, S, Y, op = setup_case()
    c = torch.ones(seq.K, dtype=torch.float64, requires_grad=True)
    X = GuessSolveFn.apply(c, seq)
    loss = ((X - dev(Y.reshape(-1)).reshape(Y.shape)) ** 2).sum()
    loss.backward()
    Lref, gref = adjoint.loss_and_grad(Fh, S, Y, 16, np.ones(seq.K))
    assert abs(float(loss) - Lref) <= 1e-9 * abs(Lref)
    g = c.grad.numpy()
    assert np.max(np.abs(g - gref)) <= 1e-8 * np.max(np.abs(gref))
    # the adjoint ran its own guess history: later solves need few iterations
    assert max(seq.stats["adjoint_iters"][:4]) < seq.stats["adjoint_iters"][-1]
    op.close()


def test_gradient_matches_finite_differences(lib):
    import torch

    from paper_2009_10863_amd.autograd import GuessSolveFn

    announce("adjoint FD 16^3")
    seq, Fh, S, Y, op = setup_case(T=8)
    Yd = dev(Y.reshape(-1)).reshape(Y.shape)

    def loss_of(cv):
        with torch.no_grad():
            return float(((GuessSolveFn.apply(cv, seq) - Yd) ** 2).sum())

    c = torch.ones(seq.K, dtype=torch.float64, requires_grad=True)
    X = GuessSolveFn.apply(c, seq)
    ((X - Yd) ** 2).sum().backward()
    g = c.grad.numpy()
    d = 1e-3
    for k in range(seq.K):
        e = torch.zeros(seq.K, dtype=torch.float64)
        e[k] = d
        fd = (loss_of(torch.ones(seq.K, dtype=torch.float64) + e)
              - loss_of(torch.ones(seq.K, dtype=torch.float64) - e)) / (2 * d)
        assert abs(fd - g[k]) <= 1e-6 * np.max(np.abs(g)), k
    op.close()


def test_mode_generator_matches_inputs(lib):
    from paper_2009_10863_amd.autograd import plane_wave_modes

    announce("mode generator")
    params = synth.plane_wave_params(2, 5)
    F = host(plane_wave_modes(params, 12))
    np.testing.assert_allclose(F, synth.plane_wave_modes(params, 12), rtol=0, atol=1e-13)


def test_gradient_128_matches_reference(lib):
    """The differentiation workload at its grid (128^3, 16 modes, EXTRAP(2,8) in both time
    directions), 30 steps: loss and gradient against the oracle's DST-exact FP64 reference."""
    import torch

    from paper_2009_10863_amd.autograd import GuessSolveFn, SolveSequence
    from paper_2009_10863_amd.sequence import Operator

    announce("adjoint gradient 128^3 K=16 T=30")
    n, T, K = 128, 30, 16
    params = synth.plane_wave_params(0, K)
    tparams = synth.target_params(99)
    ts = synth.step_times(T, 0.005)
    S = np.stack([synth.mode_amplitudes(params, t) for t in ts])
    Fh = synth.plane_wave_modes(params, n)
    Ft = synth.plane_wave_modes(tparams, n)
    Y = np.stack([tparams["scale"] * synth.plane_wave_rhs(tparams, n, t, modes=Ft) for t in ts])
    op = Operator(n)
    try:
        seq = SolveSequence(op, dev(Fh.reshape(-1)).reshape(K, -1), S, method="extrap", M=8, degree=2,
                            rtol=1e-10)
        c = torch.ones(K, dtype=torch.float64, requires_grad=True)
        X = GuessSolveFn.apply(c, seq)
        loss = ((X - dev(Y.reshape(-1)).reshape(Y.shape)) ** 2).sum()
        loss.backward()
        g = c.grad.numpy()
        fwd, adj = seq.stats["forward_iters"], seq.stats["adjoint_iters"]
    finally:
        op.close()
    Lref, gref = adjoint.loss_and_grad(Fh, S, Y, n, np.ones(K))
    assert abs(float(loss) - Lref) <= 1e-8 * abs(Lref)
    assert np.max(np.abs(g - gref)) <= 1e-7 * np.max(np.abs(gref))
    # both directions profit from their guess histories once they are warm
    assert np.mean(fwd[10:]) < 0.8 * fwd[0] and np.mean(adj[:-10]) < 0.8 * adj[-1]
