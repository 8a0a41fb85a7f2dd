"""MI355X-native initial guesses for sequences of SPD solves.

Implements the data-parallel hot path of Austin, Chalmers & Warburton (2020):
stabilized least-squares polynomial extrapolation and Fischer's projection
(A-orthonormal form) around a matrix-free 7-point operator and Jacobi-PCG.
All device work runs in the hand-written HIP kernels of ``libguess.so``
(C ABI in ``include/libguess.h``); Python only marshals arguments.

Submodules (imported on use, so that building does not need the library):
  libguess   ctypes binding of the C ABI (same function names)
  sequence   Operator / GuessSequence objects and the time-step driver
  autograd   GuessSolveFn: differentiable sequence of solves (adjoint PCG)
"""
import importlib

__all__ = ["libguess", "sequence", "autograd"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
