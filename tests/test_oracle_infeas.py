"""Pins of the oracle's infeasibility certificates (the paper is silent on
infeasible inputs): hand-built Farkas rays and descent directions, the two
infeasible generators, and no false positives on feasible instances."""
import numpy as np
import pytest

import qpgen
from tests import qp_refs


def _budget_problem(budget):
    n = 4   # x >= 0, sum x = budget, min 1/2 |x|^2 + 1'x
    return qp_refs.make_qp(np.eye(n), np.ones((1, n)), np.ones(n), [budget], np.zeros(n),
                           np.full(n, np.inf), [0])


def test_farkas_ray_by_hand(orc):
    qp = _budget_problem(-1.0)
    # y = -1: A'y = -1 <= 0 needs only the finite lower bounds: support 0, b'y = 1
    r = orc.infeas_check(qp, np.zeros(4), np.array([-1.0]))
    assert r["primal_ratio"] == 0.0
    # the opposite ray needs the infinite upper bounds: no certificate
    r = orc.infeas_check(qp, np.zeros(4), np.array([1.0]))
    assert r["primal_ratio"] == np.inf
    # feasible budget: the same ray has b'y - support = -1 < 0
    r = orc.infeas_check(_budget_problem(1.0), np.zeros(4), np.array([-1.0]))
    assert r["primal_ratio"] == np.inf


def test_farkas_ratio_with_violation_by_hand(orc):
    # x1 free, 0 <= x2 <= 2;  rows x1 + x2 >= 3 (GE),  -x1 >= 0 (GE)
    qp = qp_refs.make_qp(np.eye(2), np.array([[1.0, 1.0], [-1.0, 0.0]]), [0.0, 0.0], [3.0, 0.0],
                         [-np.inf, 0.0], [np.inf, 2.0], [1, 1])
    # y = (1, 1): A'y = (0, 1) -> support of x2 in [0, 2] is 2;  b'y = 3;  margin 1
    r = orc.infeas_check(qp, np.zeros(2), np.array([1.0, 1.0]))
    assert r["primal_ratio"] == 0.0
    # y = (1, 0.9): A'y = (0.1, 1): 0.1 needs x1's infinite upper bound; margin 3 - 2 = 1
    r = orc.infeas_check(qp, np.zeros(2), np.array([1.0, 0.9]))
    assert r["primal_ratio"] == pytest.approx(0.1, rel=1e-15)
    # a negative component on a GE row is projected away: y = (1, -5) acts as (1, 0)
    r = orc.infeas_check(qp, np.zeros(2), np.array([1.0, -5.0]))
    assert r["primal_ratio"] == pytest.approx(1.0 / 1.0, rel=1e-15)


def test_descent_direction_by_hand(orc):
    # LP  min -x1  s.t.  x1 - x2 >= 0,  x >= 0: unbounded along (1, 1)
    qp = qp_refs.make_qp(np.zeros((2, 2)), np.array([[1.0, -1.0]]), [-1.0, 0.0], [0.0],
                         [0.0, 0.0], [np.inf, np.inf], [1])
    r = orc.infeas_check(qp, np.array([1.0, 1.0]), np.zeros(1))
    assert r["dual_ratio"] == 0.0
    # (1, 2) violates the row by 1 with c'd = -1
    r = orc.infeas_check(qp, np.array([1.0, 2.0]), np.zeros(1))
    assert r["dual_ratio"] == pytest.approx(1.0, rel=1e-15)
    # a component against a finite bound is projected away: (1, -3) acts as (1, 0)
    r = orc.infeas_check(qp, np.array([1.0, -3.0]), np.zeros(1))
    assert r["dual_ratio"] == 0.0
    # curvature along the direction: Q = diag(1, 0) makes (1, 1) no certificate
    qq = qp_refs.make_qp(np.diag([1.0, 0.0]), np.array([[1.0, -1.0]]), [-1.0, 0.0], [0.0],
                         [0.0, 0.0], [np.inf, np.inf], [1])
    r = orc.infeas_check(qq, np.array([1.0, 1.0]), np.zeros(1))
    assert r["dual_ratio"] == pytest.approx(1.0, rel=1e-15)
    # ascent is not a certificate
    assert orc.infeas_check(qp, np.array([-1.0, -1.0]), np.zeros(1))["dual_ratio"] == np.inf


@pytest.mark.parametrize("seed", range(1, 5))
@pytest.mark.parametrize("pre", [False, True])
def test_generators_detected(orc, seed, pre):
    for mk, want in ((qpgen.primal_infeasible_qp, orc.PRIMAL_INFEASIBLE),
                     (qpgen.dual_infeasible_qp, orc.DUAL_INFEASIBLE)):
        qp = mk(seed)
        s = orc.OracleSettings(eps=1e-6, detect_infeasibility=1, max_iter=100000)
        if pre:
            sc, dv, dr = orc.precondition(qp)
            _, _, r, _ = orc.solve_scaled(sc, qp, dv, dr, s)
        else:
            _, _, r, _ = orc.solve(qp, s)
        assert r["status"] == want, (qp.name, r)


def test_infeasible_generators_are_what_they_claim():
    # Farkas certificate of the planted pair, and the recession direction of the other
    qp = qpgen.primal_infeasible_qp(2)
    A = qp.A().toarray()
    y = np.zeros(qp.m)
    y[-2:] = 1.0
    np.testing.assert_allclose(A.T @ y, 0.0, atol=1e-12)
    assert qp.b @ y == 1.0
    qd = qpgen.dual_infeasible_qp(2)
    Q, A = qd.dense()
    d = np.zeros(qd.n)
    d[0] = -1.0
    assert np.all(Q @ d == 0.0) and qd.c @ d < 0 and np.isinf(qd.l[0])
    Ad = A @ d
    assert np.all(Ad[qd.row_type == 0] == 0.0) and np.all(Ad[qd.row_type == 1] >= 0.0)


@pytest.mark.parametrize("seed", range(1, 9))
def test_no_false_positives(orc, seed):
    qp = qpgen.tiny_random_qp(seed)
    a = orc.solve(qp, orc.OracleSettings(eps=1e-8, detect_infeasibility=1))
    b = orc.solve(qp, orc.OracleSettings(eps=1e-8))
    assert a[2]["status"] == b[2]["status"] == orc.OPTIMAL
    assert a[2]["iterations"] == b[2]["iterations"]
    np.testing.assert_array_equal(a[0], b[0])


def test_farkas_ratio_needs_the_right_bound(orc):
    # 0 <= x1 (no upper bound), 0 <= x2 <= 2;  0.1 x1 + x2 >= 3 (GE): y = 1 gives
    # A'y = (0.1, 1): x2's finite upper bound enters the support (margin 3 - 2 = 1),
    # x1's missing upper bound makes 0.1 a violation: ratio 0.1
    qp = qp_refs.make_qp(np.eye(2), np.array([[0.1, 1.0]]), [0.0, 0.0], [3.0],
                         [0.0, 0.0], [np.inf, 2.0], [1])
    r = orc.infeas_check(qp, np.zeros(2), np.array([1.0]))
    assert r["primal_ratio"] == pytest.approx(0.1, rel=1e-15)


def test_transforms_on_a_larger_instance(orc):
    base = qpgen.large_random_qp(seed=12, n=3000, m=1500)
    pi = qpgen.with_contradictory_rows(base, 1)
    A = pi.A()
    y = np.zeros(pi.m)
    y[-2:] = 1.0
    assert np.abs(A.T @ y).max() == 0.0 and pi.b @ y == 1.0
    ub = qpgen.with_unbounded_ray(base)
    Q, A = ub.Q(), ub.A()
    e0 = np.zeros(ub.n)
    e0[0] = 1.0
    assert np.abs(Q @ e0).max() == 0.0 and ub.c @ e0 < 0 and np.isinf(ub.u[0])
    Ae = A @ e0
    assert np.all(Ae[ub.row_type == 0] == 0.0) and np.all(Ae[ub.row_type == 1] >= 0.0)
    xf = ub.meta["x_feasible"]
    ax = A @ xf
    eq = ub.row_type == 0
    assert np.all(ax[eq] == ub.b[eq]) and np.all(ax[~eq] >= ub.b[~eq])
    assert np.all(xf >= ub.l) and np.all(xf <= ub.u)
    for qp, want in ((pi, orc.PRIMAL_INFEASIBLE), (ub, orc.DUAL_INFEASIBLE)):
        r = orc.solve(qp, orc.OracleSettings(eps=1e-6, detect_infeasibility=1, max_iter=50000))[2]
        assert r["status"] == want
