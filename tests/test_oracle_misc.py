"""Pins of the oracle's low-precision rounding, sequence driver and adjoint gradient."""
import numpy as np
import pytest

import synth
from oracle import adjoint, lowprec, sequence
from oracle import operator as op


# ---------------------------------------------------------------- rounding
def test_bf16_round_to_nearest_even_hand_cases():
    """Hand-worked IEEE cases: 1 + 2^-8 is a tie (rounds to 1), 1 + 3 2^-8 rounds
    up to 1 + 2^-6, just above a tie rounds up, inf and sign survive."""
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -2.5, np.inf,
                  3.0e38, 2.0 ** -130], dtype=np.float64)
    got = lowprec.round_store(x, "bf16")
    # 3.0e38 = 1.76324.. * 2^127; with 7 fraction bits .76324 * 128 = 97.69 -> 98,
    # so the nearest bf16 is (1 + 98/128) * 2^127
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -2.5, np.inf,
                     (1 + 98 / 128) * 2.0 ** 127, 2.0 ** -130])
    np.testing.assert_array_equal(got, want)


def test_f16_and_f32_rounding_and_two_step_chain():
    x = np.array([1 + 2 ** -11, 1 + 3 * 2 ** -11, 65504.0, 65520.0, 2.0 ** -24, 1e-9])
    got = lowprec.round_store(x, "f16")
    np.testing.assert_array_equal(got, [1.0, 1 + 2 ** -9, 65504.0, np.inf, 2.0 ** -24, 0.0])
    y = np.array([1 + 2 ** -24, 1 + 3 * 2 ** -24, 1 + 2 ** -24 + 2 ** -50])
    np.testing.assert_array_equal(lowprec.round_store(y, "f32"), [1.0, 1 + 2 ** -22, 1 + 2 ** -23])
    # two-step chain: 1 + 2^-11 + 2^-30 rounds to FP32 at 1 + 2^-11 (a tie in FP16 -> even = 1)
    z = np.array([1 + 2 ** -11 + 2 ** -30])
    assert lowprec.round_store(z, "f16")[0] == 1.0


@pytest.mark.parametrize("dtype", ["f32", "f16", "bf16"])
def test_rounding_error_within_unit_roundoff(dtype):
    x = synth.random_vectors(0, 1, 10000)[0]
    r = lowprec.round_store(x, dtype)
    u = lowprec.UNIT_ROUNDOFF[dtype]
    assert np.all(np.abs(r - x) <= u * np.abs(x) * (1 + 1e-12) + (2.0 ** -24 if dtype == "f16" else 0))
    # stored values are fixed points of the rounding
    np.testing.assert_array_equal(lowprec.round_store(r, dtype), r)


def test_f16_scale_exponent():
    for v in [1e-7, 3e-5, 0.02, 1.0, 1.5, 300.0]:
        e = lowprec.f16_scale_exp(v)
        assert 2 ** 14 <= v * 2.0 ** e < 2 ** 15
    assert lowprec.f16_scale_exp(0.0) == 0


# ---------------------------------------------------------------- driver
def test_sequence_guesses_reduce_iterations():
    """Qualitative ordering of §6.3 on a small synthetic sequence:
    zero > previous solution > extrapolation / projection."""
    n = 12
    A = op.Operator(n)
    params = synth.plane_wave_params(0, 4)
    rhs = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(24, 0.01)]
    res = {m: sequence.run_sequence(A, rhs, m, M=8, degree=2) for m in ("zero", "last", "extrap", "proj")}
    avg = {m: np.mean(r["iters"][10:]) for m, r in res.items()}
    assert avg["zero"] > avg["last"] > avg["extrap"]
    assert avg["last"] > avg["proj"]
    for r in res.values():
        assert max(r["relres"]) <= 1e-8


def test_projection_exact_on_finite_rank_sequence():
    """With K plane-wave modes every solution lies in a K-dimensional space, so
    projection with M > K is exact up to the solve tolerance of the stored
    solutions once K of them are stored; later solutions are rejected as
    dependent (relative A-norm below eps_rel) and the history stops growing."""
    n = 10
    A = op.Operator(n)
    params = synth.plane_wave_params(1, 3)
    rhs = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(14, 0.05)]
    r = sequence.run_sequence(A, rhs, "proj", M=8)
    assert max(r["r0"][3:]) <= 1e-6
    assert max(r["iters"][3:]) <= 8 < min(r["iters"][:3])


def test_replay_matches_run():
    n = 8
    A = op.Operator(n)
    params = synth.plane_wave_params(2, 4)
    rhs = [synth.plane_wave_rhs(params, n, t) for t in synth.step_times(12, 0.01)]
    run = sequence.run_sequence(A, rhs, "extrap", M=4, degree=2, keep=True)
    g, _ = sequence.replay_guesses("extrap", 4, 2, A, rhs, run["solutions"])
    for a, b in zip(g, run["guesses"]):
        np.testing.assert_array_equal(a, b)


# ---------------------------------------------------------------- adjoint
def test_adjoint_gradient_matches_central_difference():
    """L(c) is exactly quadratic in c, so a central difference is exact up to rounding."""
    n, T = 6, 8
    params = synth.plane_wave_params(3, 4)
    tparams = synth.target_params(99)
    F = synth.plane_wave_modes(params, n)
    ts = synth.step_times(T, 0.005)
    S = np.stack([synth.mode_amplitudes(params, t) for t in ts])
    Y = np.stack([synth.target_field(tparams, n, t) for t in ts])
    c = np.ones(4)
    L, g = adjoint.loss_and_grad(F, S, Y, n, c)
    d = 1e-3
    for k in range(4):
        e = np.zeros(4)
        e[k] = d
        fd = (adjoint.loss(F, S, Y, n, c + e) - adjoint.loss(F, S, Y, n, c - e)) / (2 * d)
        assert abs(fd - g[k]) <= 1e-7 * max(abs(g).max(), 1e-30)
