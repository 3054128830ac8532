"""MI355X (gfx950) 2SHOC-RK4 solver for the nonlinear Schroedinger equation.

The numerical work runs in hand-written HIP kernels behind the C ABI of
``include/nlse.h``; ``nlse.Solver`` is a thin ctypes binding of it.
"""
from .nlse import Batch, Corrector, NLSEError, Solver, inject, load, mass_noalloc  # noqa: F401

__all__ = ["Solver", "Batch", "Corrector", "inject", "NLSEError", "load", "mass_noalloc"]
