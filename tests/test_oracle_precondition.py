"""Pins of the oracle's diagonal preconditioning (Sec. 5 "Preprocessing": Ruiz
steps, an l2 step and a Pock-Chambolle step on K = [[Q, A'], [A, 0]]) and of the
solve on the scaled problem, whose relKKT is measured on the original one."""
import numpy as np
import pytest

import qpgen
from tests import qp_refs


def _k_dense(qp):
    Q, A = qp.dense()
    n, m = qp.n, qp.m
    K = np.zeros((n + m, n + m))
    K[:n, :n] = Q
    K[n:, :n] = A
    K[:n, n:] = A.T
    return K


def test_scaled_data_are_the_stated_products(orc):
    qp = qpgen.tiny_random_qp(1)
    sc, dv, dr = orc.precondition(qp)
    Q, A = qp.dense()
    Qs, As = sc.dense()
    np.testing.assert_allclose(Qs, dv[:, None] * Q * dv[None, :], rtol=1e-13, atol=0)
    np.testing.assert_allclose(As, dr[:, None] * A * dv[None, :], rtol=1e-13, atol=0)
    np.testing.assert_allclose(sc.c, dv * qp.c, rtol=1e-15)
    np.testing.assert_allclose(sc.b, dr * qp.b, rtol=1e-15)
    fin = np.isfinite(qp.l)
    np.testing.assert_allclose(sc.l[fin], qp.l[fin] / dv[fin], rtol=1e-15)
    assert np.all(np.isinf(sc.l[~fin]))
    assert np.all(dv > 0) and np.all(dr > 0)


def test_diagonal_matrix_one_ruiz_step(orc):
    """K diagonal: one infinity-norm step gives |K~_jj| = 1 and d_j = 1/sqrt|K_jj|; the
    l2 and Pock-Chambolle steps then change nothing."""
    q = np.array([4.0, 0.25, 9.0, 1e-4, 2.5e3])
    n = q.size
    qp = qp_refs.make_qp(np.diag(q), np.zeros((0, n)), np.ones(n), [], np.full(n, -1.0),
                         np.full(n, 1.0), [])
    for ruiz, l2, pc in ((1, False, False), (10, True, True)):
        sc, dv, _ = orc.precondition(qp, ruiz, l2, pc)
        np.testing.assert_allclose(sc.q_val, 1.0, rtol=4e-16)
        np.testing.assert_allclose(dv, 1.0 / np.sqrt(q), rtol=4e-16)


def _circulant_q(n=8):
    # symmetric circulant: every row has the same entries, so every row statistic is equal
    row = np.zeros(n)
    row[0], row[1], row[-1], row[3], row[-3] = 3.0, -1.0, -1.0, 0.5, 0.5
    return np.array([np.roll(row, i) for i in range(n)])


@pytest.mark.parametrize("kind", ["l2", "pc"])
def test_equal_row_statistics_scale_uniformly(orc, kind):
    Q = _circulant_q()
    n = Q.shape[0]
    qp = qp_refs.make_qp(Q, np.zeros((0, n)), np.ones(n), [], np.full(n, -1.0),
                         np.full(n, 1.0), [])
    stat = np.sqrt(np.sum(Q[0] ** 2)) if kind == "l2" else np.sum(np.abs(Q[0]))
    sc, dv, _ = orc.precondition(qp, 0, kind == "l2", kind == "pc")
    np.testing.assert_allclose(dv, 1.0 / np.sqrt(stat), rtol=1e-15)
    Qs, _ = sc.dense()
    np.testing.assert_allclose(Qs, Q / stat, rtol=1e-14)


def test_ruiz_converges_to_unit_row_maxima(orc):
    """Ruiz's equilibration: repeated infinity-norm steps drive every row (and, K being
    symmetric, every column) maximum of K~ to 1."""
    qp = qpgen.tiny_random_qp(2)
    rng = np.random.default_rng(3)
    # badly scaled rows and columns
    qp.a_val = qp.a_val * np.repeat(10.0 ** rng.uniform(-3, 3, qp.m), np.diff(qp.a_rowptr))
    sc, dv, dr = orc.precondition(qp, 60, False, False)
    K = _k_dense(sc)
    np.testing.assert_allclose(np.abs(K).max(axis=1), 1.0, rtol=1e-9)
    K0 = _k_dense(qp)
    d = np.concatenate([dv, dr])
    np.testing.assert_allclose(K, d[:, None] * K0 * d[None, :], rtol=1e-12)


def test_identity_scaling_reproduces_plain_solve(orc):
    qp = qpgen.tiny_random_qp(3)
    sc, dv, dr = orc.precondition(qp, 0, False, False)
    assert np.all(dv == 1.0) and np.all(dr == 1.0)
    s = orc.OracleSettings(eps=1e-7)
    x1, y1, r1, _ = orc.solve(qp, s)
    x2, y2, r2, _ = orc.solve_scaled(sc, qp, dv, dr, s)
    np.testing.assert_array_equal(x1, x2)
    np.testing.assert_array_equal(y1, y2)
    assert r1["iterations"] == r2["iterations"] and r1["rel_kkt"] == r2["rel_kkt"]


@pytest.mark.parametrize("seed", range(6))
def test_preconditioned_solve_reaches_bruteforce_kkt(orc, seed):
    qp = qp_refs.random_tiny_qp(seed, n=5, m=3)
    best = qp_refs.brute_force_kkt(qp)
    assert best is not None
    f_star, x_star, _ = best
    sc, dv, dr = orc.precondition(qp)
    x, y, r, _ = orc.solve_scaled(sc, qp, dv, dr, orc.OracleSettings(eps=1e-10, max_iter=400000))
    assert r["status"] == orc.OPTIMAL, r
    # the reported relKKT is the original problem's at the returned point
    assert orc.rel_kkt(qp, x, y)["rel_kkt"] == pytest.approx(r["rel_kkt"], rel=1e-6, abs=1e-15)
    assert r["primal_obj"] == pytest.approx(f_star, rel=1e-7, abs=1e-7)
    np.testing.assert_allclose(x, x_star, rtol=1e-5, atol=1e-6)


def test_warm_start_is_taken_in_original_space(orc):
    qp = qpgen.tiny_random_qp(1)
    x, y, _, _ = orc.solve(qp, orc.OracleSettings(eps=1e-9))
    sc, dv, dr = orc.precondition(qp)
    _, _, r, _ = orc.solve_scaled(sc, qp, dv, dr, orc.OracleSettings(eps=1e-8), x0=x, y0=y)
    assert r["used_warm_start"] == 1 and r["iterations"] == 0


def test_preconditioning_helps_badly_scaled_rows(orc):
    """The purpose stated in Sec. 5: rows scaled over six decades slow the method down;
    the preconditioned solve needs fewer iterations."""
    qp = qpgen.tiny_random_qp(4)
    rng = np.random.default_rng(8)
    sc_rows = 10.0 ** rng.uniform(-3, 3, qp.m)
    qp.a_val = qp.a_val * np.repeat(sc_rows, np.diff(qp.a_rowptr))
    qp.b = qp.b * sc_rows
    s = orc.OracleSettings(eps=1e-6, max_iter=200000)
    _, _, r_plain, _ = orc.solve(qp, s)
    sc, dv, dr = orc.precondition(qp)
    _, _, r_pre, _ = orc.solve_scaled(sc, qp, dv, dr, s)
    assert r_pre["status"] == orc.OPTIMAL
    assert r_pre["iterations"] < r_plain["iterations"]


@pytest.mark.parametrize("kind", ["ruiz", "l2", "pc"])
def test_one_step_on_a_two_variable_k(orc, kind):
    """K = [[diag(q), a'], [a, 0]] with q = (1e-4, 4), a = (100, -2): one step of each kind
    worked by hand.  Variable row j of K holds q_j and a_j; the constraint row holds a."""
    q, a = np.array([1e-4, 4.0]), np.array([100.0, -2.0])
    qp = qp_refs.make_qp(np.diag(q), a[None, :], np.ones(2), [1.0], np.full(2, -1.0),
                         np.full(2, 1.0), [0])
    if kind == "ruiz":
        stat = np.array([100.0, 4.0, 100.0])
    elif kind == "l2":
        stat = np.array([np.hypot(1e-4, 100.0), np.hypot(4.0, 2.0), np.hypot(100.0, 2.0)])
    else:
        stat = np.array([100.0001, 6.0, 102.0])
    f = 1.0 / np.sqrt(stat)
    sc, dv, dr = orc.precondition(qp, 1 if kind == "ruiz" else 0, kind == "l2", kind == "pc")
    np.testing.assert_allclose(dv, f[:2], rtol=1e-15)
    np.testing.assert_allclose(dr, f[2:], rtol=1e-15)
    np.testing.assert_allclose(sc.q_val, q * f[:2] ** 2, rtol=1e-15)
    np.testing.assert_allclose(sc.a_val, a * f[:2] * f[2], rtol=1e-15)
