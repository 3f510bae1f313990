"""MI355X-native least-squares h-p spectral element hot path.

The library (``libsem.so``, HIP for gfx950) evaluates, matrix-free in every
PCG iteration, the normal-equation residual of the least-squares functional of
Husain's thesis (arXiv 1110.2316) and applies the block-diagonal separable
preconditioner.  ``semlib`` is the ctypes binding of its C ABI
(``include/sem.h``).
"""
from .semlib import Context, SemError, setup_problem, lib, pcg_solve_batch  # noqa: F401
from .adjoint import SourceSolve, solve_source  # noqa: F401,E402
