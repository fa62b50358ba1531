"""MI355X-native rAPDHG solver for convex quadratic programs.

Restarted accelerated PDHG (Lu & Yang, arXiv 2311.07710) with its whole
per-iteration hot path in hand-written HIP kernels for gfx950, behind the
C-ABI of include/qp.h.  This package is the thin Python binding; importing it
does not load the library, ``load()`` (or the first Solver) does, and raises
if the library has not been built: there is no CPU fallback.
"""
from ._binding import (  # noqa: F401
    QP_OK, QP_OPTIMAL, QP_ITERATION_LIMIT, QP_TIME_LIMIT, QP_NUMERICAL_ERROR,
    QP_PRIMAL_INFEASIBLE, QP_DUAL_INFEASIBLE,
    QP_RESTART_ADAPTIVE, QP_RESTART_FIXED_K, QP_RESTART_HALVING, QP_RESTART_NONE,
    QP_MEM_HOST, QP_MEM_DEVICE, QPError, LIB_PATH, SIGNATURES, load,
)
from .solver import Settings, Solver, BatchSolver  # noqa: F401
