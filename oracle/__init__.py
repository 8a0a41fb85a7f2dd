"""CPU FP64 oracle for the initial-guess hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously-correct restatement of what the
method computes, written from the paper (Austin, Chalmers & Warburton,
"Initial Guesses for Sequences of Linear Systems in a GPU-Accelerated
Incompressible Flow Solver", 2020).  It exists so that the HIP path can be
checked against something independent of it.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (the ``libguess`` shared library
and its Python binding) never imports, links or executes anything here, and
nothing here imports the product package.  The two share no code; the only
common module is ``synth`` (seeded inputs, none of the method's arithmetic).

Modules
-------
extrap      least-squares / naive / sparse (column-pivoted QR) extrapolation
            weights in exact rationals, Lebesgue constant, the extrapolated
            guess, warm-up rule
lowprec     rounding of stored history to FP32 / FP16 / BF16
operator    7-point constant- and variable-coefficient Helmholtz operators,
            Jacobi diagonal, exact DST-I solver for the constant case
pcg         Jacobi-preconditioned conjugate gradients
projection  Fischer's projection: classic restarts (Algorithm 1) or the rolling
            window with its QR update (Algorithm 2), in the A inner product or
            the paper's l2 one, and the brute-force normal-equation minimiser
rawproj     the same A-norm projection through the Gram matrix of the stored
            (rounded) raw solutions, classic or rolling
sequence    the time-step driver: form guess -> solve -> update
adjoint     reference gradient of the differentiation workload

Functions whose result is pinned only by self-consistency say
"parity unpinned" in their docstring.
"""
from . import extrap, lowprec, operator, pcg, projection, rawproj, sequence, adjoint  # noqa: F401
