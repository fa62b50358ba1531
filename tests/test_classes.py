"""The further synthetic classes (random QP with equality constraints, Lasso,
Huber fitting, SVM): each generator must encode its textbook problem, checked on
the oracle's solution against that problem's own optimality conditions, which
never mention the QP reformulation."""
import numpy as np
import pytest

import qpgen
from tests import qp_refs


def _solve(orc, qp, eps=1e-9, precondition=True):
    if precondition:
        sc, dv, dr = orc.precondition(qp)
        x, y, r, _ = orc.solve_scaled(sc, qp, dv, dr, orc.OracleSettings(eps=eps, max_iter=400000))
    else:
        x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=eps, max_iter=400000))
    assert r["status"] == orc.OPTIMAL, r
    return x, y, r


def test_eq_qp_closed_form(orc):
    qp = qpgen.eq_qp(seed=3, n=120)
    assert np.all(qp.row_type == qpgen.instances.EQ) and np.all(np.isinf(qp.l))
    x, y, r = _solve(orc, qp)
    xs, ys = qp_refs.equality_kkt_solution(qp)
    np.testing.assert_allclose(x, xs, rtol=1e-5, atol=1e-6 * (1 + np.abs(xs).max()))
    np.testing.assert_allclose(y, ys, rtol=1e-4, atol=1e-5 * (1 + np.abs(ys).max()))


def test_lasso_subgradient_conditions(orc):
    qp = qpgen.lasso_qp(seed=4, n_features=40, m_samples=200, density=0.1)
    F, g, lam, n = qp.meta["F"], qp.meta["g"], qp.meta["lam"], qp.meta["n_features"]
    x, y, r = _solve(orc, qp)
    w = x[:n]
    grad = F.T @ (F @ w - g)
    scale = lam
    assert np.all(np.abs(grad) <= lam + 1e-5 * scale)
    on = np.abs(w) > 1e-6
    assert on.any() and (~on).any()
    np.testing.assert_allclose(grad[on], -lam * np.sign(w[on]), rtol=0, atol=1e-5 * scale)
    f_lasso = 0.5 * np.sum((F @ w - g) ** 2) + lam * np.abs(w).sum()
    assert r["primal_obj"] == pytest.approx(f_lasso, rel=1e-6)


def test_huber_stationarity(orc):
    qp = qpgen.huber_qp(seed=5, n_features=40, m_samples=200, density=0.1)
    F, g, n = qp.meta["F"], qp.meta["g"], qp.meta["n_features"]
    x, y, r = _solve(orc, qp)
    w = x[:n]
    s = F @ w - g
    dphi = np.where(np.abs(s) <= 1.0, 2.0 * s, 2.0 * np.sign(s))
    grad = F.T @ dphi
    assert np.abs(grad).max() <= 1e-5 * (1 + np.abs(F.T @ np.sign(s)).max())
    f_hub = np.sum(np.where(np.abs(s) <= 1.0, s * s, 2.0 * np.abs(s) - 1.0))
    assert r["primal_obj"] == pytest.approx(f_hub, rel=1e-6)
    assert (np.abs(s) > 1.0).any()   # the outliers are in the linear part


def test_svm_hinge_objective_and_margin(orc):
    qp = qpgen.svm_qp(seed=6, n_features=40, m_samples=200, density=0.1)
    F, lab, lam, n = qp.meta["F"], qp.meta["labels"], qp.meta["lam"], qp.meta["n_features"]
    x, y, r = _solve(orc, qp)
    w = x[:n]
    margin = lab * (F @ w)
    hinge = np.maximum(0.0, 1.0 - margin)
    f_svm = w @ w + lam * hinge.sum()
    assert r["primal_obj"] == pytest.approx(f_svm, rel=1e-6)
    # subgradient optimality: 2w = lam * sum_i a_i g_i f_i with a_i = 1 (margin < 1),
    # 0 (margin > 1), in [0, 1] (margin = 1); the QP duals of the margin rows are a_i*lam
    yv = y[:qp.m]
    assert np.all(yv >= -1e-9) and np.all(yv <= lam + 1e-6)
    np.testing.assert_allclose(2.0 * w, (F.T @ (lab * yv)), rtol=0, atol=1e-5)
    assert np.all(yv[margin > 1.0 + 1e-4] <= 1e-5)
    assert np.all(np.abs(yv[margin < 1.0 - 1e-4] - lam) <= 1e-5)


@pytest.mark.parametrize("maker", [lambda: qpgen.eq_qp(seed=3, n=120),
                                   lambda: qpgen.lasso_qp(seed=4, n_features=40, m_samples=200,
                                                          density=0.1),
                                   lambda: qpgen.huber_qp(seed=5, n_features=40, m_samples=200,
                                                          density=0.1),
                                   lambda: qpgen.svm_qp(seed=6, n_features=40, m_samples=200,
                                                        density=0.1)])
def test_class_generators_are_seeded_and_valid(maker):
    a, b = maker(), maker()
    for f in ("q_val", "a_val", "a_col", "c", "b", "l", "u"):
        np.testing.assert_array_equal(getattr(a, f), getattr(b, f))
    Q = a.Q()
    assert abs(Q - Q.T).max() == 0.0
    assert np.linalg.eigvalsh(Q.toarray()).min() >= -1e-9
    assert np.all(a.l <= a.u)
