"""Sec. 5 preprocessing on the device vs the oracle's: the scaling vectors, and the
preconditioned solves (iterating on the scaled problem, relKKT, warm starts and
outputs on the given one) element by element, single instance and batch, with
the tolerances of test_gpu_parity."""
import numpy as np
import pytest

import qpgen
from tests import qp_refs
from tests.test_gpu_parity import _assert_parity, _pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpa():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2311_07710_amd as m
    m.load()
    return m


def _badly_scaled(seed=4):
    qp = qpgen.tiny_random_qp(seed)
    rng = np.random.default_rng(8)
    rows = 10.0 ** rng.uniform(-3, 3, qp.m)
    qp.a_val = qp.a_val * np.repeat(rows, np.diff(qp.a_rowptr))
    qp.b = qp.b * rows
    return qp


def _ulp_diff(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return int(np.max(np.abs(a.view(np.int64) - b.view(np.int64)))) if a.size else 0


@pytest.mark.parametrize("maker", [lambda: qpgen.tiny_random_qp(1), _badly_scaled,
                                   lambda: qpgen.portfolio_qp(seed=3, n_assets=20000, k=40),
                                   lambda: qpgen.large_random_qp(seed=2, n=30000, m=15000)])
def test_device_scaling_matches_oracle(orc, qpa, maker):
    qp = maker()
    _, dv, dr = orc.precondition(qp)
    with qpa.Solver(qp, qpa.Settings(precondition=1, norm_A=1.0, norm_Q=1.0)) as s:
        gv, gr = s.scaling()
    print(f"  scaling ulp difference: D2 {_ulp_diff(gv, dv)}, D1 {_ulp_diff(gr, dr)}", flush=True)
    np.testing.assert_allclose(gv, dv, rtol=1e-14)
    np.testing.assert_allclose(gr, dr, rtol=1e-14)


@pytest.mark.parametrize("ruiz", [0, 1, 3])
def test_ruiz_pass_count_setting(orc, qpa, ruiz):
    """ruiz_iters (the Ruiz passes before the l2 and Pock-Chambolle steps) reaches the
    device: the scaling equals the oracle's for the same count, which differs from the
    default count's, and the preconditioned solve keeps parity."""
    qp = _badly_scaled()
    _, dv, dr = orc.precondition(qp, ruiz_iters=ruiz)
    _, dv10, dr10 = orc.precondition(qp)
    assert np.max(np.abs(dr - dr10)) > 1e-6 * np.max(np.abs(dr10))
    with qpa.Solver(qp, qpa.Settings(precondition=1, ruiz_iters=ruiz, norm_A=1.0,
                                     norm_Q=1.0)) as s:
        gv, gr = s.scaling()
    np.testing.assert_allclose(gv, dv, rtol=1e-14)
    np.testing.assert_allclose(gr, dr, rtol=1e-14)
    o, g = _pair(orc, qpa, qp, eps=1e-6, precondition=True, ruiz=ruiz)
    _assert_parity(orc, qp, o, g)


@pytest.mark.parametrize("maker,eps", [(lambda: qpgen.tiny_random_qp(1), 1e-6),
                                       (_badly_scaled, 1e-6),
                                       (lambda: qpgen.portfolio_family(seed=5, count=2).instance(0),
                                        1e-6),
                                       (lambda: qpgen.mpc_qp(np.random.default_rng([4, 2]), 36, 9, 4),
                                        1e-6)])
def test_preconditioned_solve_to_tolerance(orc, qpa, maker, eps):
    qp = maker()
    o, g = _pair(orc, qpa, qp, eps=eps, precondition=True)
    _assert_parity(orc, qp, o, g)
    assert g[2]["status"] == 0


@pytest.mark.parametrize("panels", [(1, 1), (4, 4)])
def test_preconditioned_large_fixed_iterations(orc, qpa, panels):
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=300, precondition=True, panels=panels)
    _assert_parity(orc, qp, o, g)


def test_preconditioned_long_rows(orc, qpa):
    qp = qpgen.portfolio_qp(seed=3, n_assets=20000, k=40)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=512, precondition=True)
    _assert_parity(orc, qp, o, g)


def test_preconditioned_warm_start(orc, qpa):
    qp = qpgen.tiny_random_qp(1)
    x, y, _, _ = orc.solve(qp, orc.OracleSettings(eps=1e-7))
    rng = np.random.default_rng(1)
    x0 = x + 1e-3 * rng.standard_normal(qp.n)
    y0 = y + 1e-3 * rng.standard_normal(qp.m)
    o, g = _pair(orc, qpa, qp, eps=1e-8, x0=x0, y0=y0, precondition=True)
    _assert_parity(orc, qp, o, g)
    assert g[2]["used_warm_start"] == 1


def test_preconditioned_update_vectors(orc, qpa):
    fam = qpgen.portfolio_family(seed=5, n_assets=400, k=20, count=3)
    base, other = fam.instance(0), fam.instance(2)
    sc, dv, dr = orc.precondition(other)
    nA, _ = orc.norm_A(sc, 1000, 1e-7)
    nQ, _ = orc.norm_Q(sc, 1000, 1e-7)
    s = orc.OracleSettings(eps=1e-6, norm_A=nA, norm_Q=nQ)
    xo, yo, ro, _ = orc.solve_scaled(sc, other, dv, dr, s)
    with qpa.Solver(base, qpa.Settings(eps=1e-6, norm_A=nA, norm_Q=nQ, precondition=1)) as gs:
        gs.update_vectors(c=other.c, b=other.b)
        xg, yg, rg = gs.solve()
    assert rg["iterations"] == ro["iterations"]
    assert abs(rg["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
    np.testing.assert_allclose(xg, xo, rtol=0, atol=1e-8 * (1 + np.abs(xo).max()))


def test_batch_preconditioned(orc, qpa):
    from tests.test_gpu_batch import _long_row_instance
    insts = [qpgen.mpc_qp(np.random.default_rng([4, i]), 20 + 7 * i, 6, 3) for i in range(4)]
    insts += [qpgen.tiny_random_qp(2), _badly_scaled(), _long_row_instance()]
    batch = qpgen.concat_batch(insts)
    refs = []
    for qp in insts:
        sc, dv, dr = orc.precondition(qp)
        nA, _ = orc.norm_A(sc, 1000, 1e-7)
        nQ, _ = orc.norm_Q(sc, 1000, 1e-7)
        x, y, r, _ = orc.solve_scaled(sc, qp, dv, dr,
                                      orc.OracleSettings(eps=1e-6, norm_A=nA, norm_Q=nQ))
        refs.append((x, y, r, nA, nQ, dv, dr))
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, precondition=1))
    bs.set_norms([r[3] for r in refs], [r[4] for r in refs])
    gv, gr = bs.scaling()
    xg, yg, rg = bs.solve()
    bs.close()
    for i, (xo, yo, ro, _, _, dv, dr) in enumerate(refs):
        v0, v1 = batch.var_off[i], batch.var_off[i + 1]
        r0, r1 = batch.row_off[i], batch.row_off[i + 1]
        g = rg[i]
        print(f"  [{i}] oracle it={ro['iterations']} rel={ro['rel_kkt']:.3e} | "
              f"gpu it={g['iterations']} rel={g['rel_kkt']:.3e}", flush=True)
        np.testing.assert_allclose(gv[v0:v1], dv, rtol=1e-14)
        np.testing.assert_allclose(gr[r0:r1], dr, rtol=1e-14)
        assert g["status"] == ro["status"] and g["iterations"] == ro["iterations"]
        assert abs(g["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
        zo = np.concatenate([xo, yo])
        zg = np.concatenate([xg[v0:v1], yg[r0:r1]])
        assert np.max(np.abs(zg - zo)) <= 1e-8 * (1 + np.max(np.abs(zo)))
