"""Seeded synthetic convex-QP instances.

This module only builds problem data (CSR matrices, vectors, bounds, row
types).  It contains none of the solver's arithmetic, so both the CPU oracle
and the GPU path may consume the arrays it produces.

Problem form used throughout:
    min 1/2 x^T Q x + c^T x   s.t.  A_i x = b_i (EQ rows),  A_i x >= b_i (GE rows),
                                    l <= x <= u  (entries may be +-inf).
This generalises the paper's ``Ax <= b`` form (Sec. 1, eq. (qp) and its footnote).
"""
from .instances import (  # noqa: F401
    QPInstance,
    BatchInstances,
    tiny_random_qp,
    large_random_qp,
    portfolio_qp,
    mpc_qp,
    mpc_batch,
    portfolio_family,
    concat_batch,
    csr_from_dense,
    eq_qp,
    lasso_qp,
    huber_qp,
    svm_qp,
    ablation_set,
    ABLATION_CLASSES,
    primal_infeasible_qp,
    dual_infeasible_qp,
    with_contradictory_rows,
    with_unbounded_ray,
)
