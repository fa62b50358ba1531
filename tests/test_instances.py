"""Structure and feasibility of the seeded synthetic instances (host only)."""
import numpy as np
import pytest

import qpgen


def _feasible(qp, x, tol=1e-9):
    ax = qp.A() @ x
    eq = qp.row_type == 0
    assert np.all(np.abs(ax[eq] - qp.b[eq]) <= tol * (1 + np.abs(qp.b[eq])))
    assert np.all(ax[~eq] >= qp.b[~eq] - tol)
    assert np.all(x >= qp.l - tol) and np.all(x <= qp.u + tol)


def _symmetric_psd_diag_dominant(qp):
    Q = qp.Q()
    assert abs(Q - Q.T).max() == 0
    d = Q.diagonal()
    off = np.asarray(abs(Q).sum(axis=1)).ravel() - np.abs(d)
    assert np.all(d >= off)


def test_tiny_random_qp():
    qp = qpgen.tiny_random_qp(1)
    assert (qp.n, qp.m) == (100, 50)
    assert list(qp.row_type[:30]) == [0] * 30 and list(qp.row_type[30:]) == [1] * 20
    assert np.isfinite(qp.l).sum() == 50 and np.all(qp.l[np.isfinite(qp.l)] == -10)
    _symmetric_psd_diag_dominant(qp)
    _feasible(qp, qp.meta["x_feasible"])
    q2 = qpgen.tiny_random_qp(1)
    assert np.array_equal(qp.a_val, q2.a_val) and np.array_equal(qp.c, q2.c)   # seeded


def test_large_random_scaled():
    qp = qpgen.large_random_qp(seed=2, n=5000, m=2500)
    assert np.all(np.diff(qp.a_rowptr) == 10)
    for i in range(0, qp.m, 97):
        cols = qp.a_col[qp.a_rowptr[i]:qp.a_rowptr[i + 1]]
        assert len(set(cols)) == 10 and np.all(np.diff(cols) > 0)
    _symmetric_psd_diag_dominant(qp)
    assert np.all(qp.l == 0) and np.all(np.isinf(qp.u))
    assert qp.row_type[:1250].sum() == 0 and qp.row_type[1250:].min() == 1
    _feasible(qp, qp.meta["x_feasible"], tol=1e-9)
    assert 9.0 < qp.q_nnz / qp.n < 12.0


def test_portfolio_scaled():
    qp = qpgen.portfolio_qp(seed=3, n_assets=20000, k=40)
    na, k = qp.meta["n_assets"], qp.meta["k"]
    assert qp.n == na + k and qp.m == k + 1
    assert np.all(qp.row_type == 0)
    assert qp.a_rowptr[-1] - qp.a_rowptr[-2] == na           # budget row is dense
    x = np.full(na, 1.0 / na)
    Ft = -qp.A()[:k, :na]                                     # rows y_i - (F'x)_i = 0
    _feasible(qp, np.concatenate([x, Ft @ x]), tol=1e-9)
    assert qp.q_nnz == qp.n


def test_mpc_batch_and_segments():
    batch = qpgen.mpc_batch(seed=4, count=12)
    assert batch.count == 12
    for i in range(batch.count):
        qp = batch.instance(i)
        assert qp.n == batch.var_off[i + 1] - batch.var_off[i]
        assert (10 + 1) * 4 + 10 * 2 <= qp.n <= (100 + 1) * 12 + 100 * 4
        assert qp.a_col.max() < qp.n
    one = qpgen.mpc_qp(np.random.default_rng([4, 0]), 10, 4, 2)
    _feasible(one, one.meta["x_feasible"], tol=1e-9)
    b2 = qpgen.concat_batch([batch.instance(i) for i in range(batch.count)])
    assert np.array_equal(b2.a_rowptr, batch.a_rowptr) and np.array_equal(b2.q_val, batch.q_val)


def test_mpc_instances_feasible():
    for i in range(20):
        rng = np.random.default_rng([4, i])
        T = int(rng.integers(10, 101)); nx = int(rng.integers(4, 13)); nu = int(rng.integers(2, 5))
        qp = qpgen.mpc_qp(rng, T, nx, nu)
        _feasible(qp, qp.meta["x_feasible"], tol=1e-6)


def test_portfolio_family():
    fam = qpgen.portfolio_family(seed=5, n_assets=500, k=10, count=30)
    assert fam.mu.shape == (30, 500) and fam.budget.min() >= 0.5 and fam.budget.max() <= 1.5
    q = fam.instance(3)
    assert q.b[-1] == fam.budget[3] and np.array_equal(q.c[:500], -fam.mu[3])
    bt = fam.batch([0, 1, 2])
    assert bt.count == 3 and bt.var_off[-1] == 3 * q.n
