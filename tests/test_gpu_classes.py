"""GPU vs oracle on the further synthetic classes (random QP with equality
constraints, Lasso, Huber fitting, SVM), plain and with the Sec. 5 preprocessing,
single instance and batched, to the tolerances of test_gpu_parity."""
import numpy as np
import pytest

import qpgen
from tests.test_gpu_parity import _assert_parity, _pair

pytestmark = pytest.mark.gpu

CLASSES = {
    "eq_qp": lambda: qpgen.eq_qp(seed=3, n=600),
    "lasso": lambda: qpgen.lasso_qp(seed=4, n_features=80, m_samples=600, density=0.08),
    "huber": lambda: qpgen.huber_qp(seed=5, n_features=80, m_samples=600, density=0.08),
    "svm": lambda: qpgen.svm_qp(seed=6, n_features=80, m_samples=600, density=0.08),
}


@pytest.fixture(scope="module")
def qpa():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2311_07710_amd as m
    m.load()
    return m


@pytest.mark.parametrize("precondition", [False, True])
@pytest.mark.parametrize("name", sorted(CLASSES))
def test_class_to_tolerance(orc, qpa, name, precondition):
    qp = CLASSES[name]()
    o, g = _pair(orc, qpa, qp, eps=1e-6, precondition=precondition)
    _assert_parity(orc, qp, o, g)
    assert g[2]["status"] == 0


def test_classes_in_one_batch(orc, qpa):
    insts = [CLASSES[k]() for k in sorted(CLASSES)]
    batch = qpgen.concat_batch(insts)
    refs = []
    for qp in insts:
        sc, dv, dr = orc.precondition(qp)
        nA, _ = orc.norm_A(sc, 1000, 1e-7)
        nQ, _ = orc.norm_Q(sc, 1000, 1e-7)
        x, y, r, _ = orc.solve_scaled(sc, qp, dv, dr,
                                      orc.OracleSettings(eps=1e-6, norm_A=nA, norm_Q=nQ))
        refs.append((x, y, r, nA, nQ))
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, precondition=1))
    bs.set_norms([r[3] for r in refs], [r[4] for r in refs])
    xg, yg, rg = bs.solve()
    bs.close()
    for i, (xo, yo, ro, _, _) in enumerate(refs):
        v0, v1 = batch.var_off[i], batch.var_off[i + 1]
        r0, r1 = batch.row_off[i], batch.row_off[i + 1]
        g = rg[i]
        print(f"  [{i}] {insts[i].name}: oracle it={ro['iterations']} | gpu it={g['iterations']}",
              flush=True)
        assert g["status"] == ro["status"] == 0 and g["iterations"] == ro["iterations"]
        assert abs(g["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
        zo = np.concatenate([xo, yo])
        zg = np.concatenate([xg[v0:v1], yg[r0:r1]])
        assert np.max(np.abs(zg - zo)) <= 1e-8 * (1 + np.max(np.abs(zo)))
