"""CPU oracle for rAPDHG -- TEST INFRASTRUCTURE ONLY.

A plain, sequential, FP64 implementation of restarted accelerated PDHG for
convex QP (Lu & Yang, arXiv 2311.07710: Algorithm 1, Sec. 5 progress metric
and restart, Sec. 6 adaptive step size / primal weight / restart, the Sec. 5
diagonal preconditioning and the Sec. 5 PDHG baselines), written in
C (``rapdhg_oracle.c``) and wrapped with ctypes here.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the GPU library and never imports it.
"""
from .oracle import (  # noqa: F401
    OracleSettings,
    RESTART_ADAPTIVE,
    RESTART_FIXED_K,
    RESTART_HALVING,
    RESTART_NONE,
    OPTIMAL,
    ITERATION_LIMIT,
    TIME_LIMIT,
    NUMERICAL_ERROR,
    PRIMAL_INFEASIBLE,
    DUAL_INFEASIBLE,
    load,
    spmv,
    spmv_t,
    rel_kkt,
    norm_A,
    norm_Q,
    step_schedule,
    run_inner,
    solve,
    precondition,
    solve_scaled,
    infeas_check,
    set_threads,
    get_threads,
)
