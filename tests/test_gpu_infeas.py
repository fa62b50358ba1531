"""Infeasibility certificates on the GPU vs the oracle: the same status at the
same evaluation for primal-infeasible and unbounded instances (plain and
preconditioned, unpanelled and column-panelled, single and batched), and no
change to feasible solves when detection is on."""
import numpy as np
import pytest

import qpgen
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


@pytest.mark.parametrize("pre", [False, True])
@pytest.mark.parametrize("kind", ["primal", "dual"])
@pytest.mark.parametrize("seed", [1, 3])
def test_infeasible_status_matches_oracle(orc, qpa, kind, seed, pre):
    qp = (qpgen.primal_infeasible_qp if kind == "primal" else qpgen.dual_infeasible_qp)(seed)
    o, g = _pair(orc, qpa, qp, eps=1e-6, max_iter=100000, detect=True, precondition=pre)
    want = orc.PRIMAL_INFEASIBLE if kind == "primal" else orc.DUAL_INFEASIBLE
    print(f"  {qp.name}: oracle status {o[2]['status']} at {o[2]['iterations']}, "
          f"gpu status {g[2]['status']} at {g[2]['iterations']}", flush=True)
    assert o[2]["status"] == want
    assert g[2]["status"] == want
    assert g[2]["iterations"] == o[2]["iterations"]


@pytest.mark.parametrize("eps_inf", [1e-4, 1e-12])
@pytest.mark.parametrize("kind", ["primal", "dual"])
def test_certificate_tolerance_setting(orc, qpa, kind, eps_inf):
    """eps_infeasible reaches the device: at a tolerance that moves the oracle's
    detection to another evaluation than the default's, the GPU detects at that one."""
    qp = (qpgen.primal_infeasible_qp if kind == "primal" else qpgen.dual_infeasible_qp)(1)
    nA, _ = orc.norm_A(qp, 1000, 1e-7)
    nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
    base = orc.solve(qp, orc.OracleSettings(eps=1e-6, max_iter=100000, norm_A=nA, norm_Q=nQ,
                                            detect_infeasibility=1))[2]
    o, g = _pair(orc, qpa, qp, eps=1e-6, max_iter=100000, detect=True, norms=(nA, nQ),
                 extra={"eps_infeasible": eps_inf})
    want = orc.PRIMAL_INFEASIBLE if kind == "primal" else orc.DUAL_INFEASIBLE
    print(f"  {qp.name}: default detects at {base['iterations']}, oracle at "
          f"{o[2]['iterations']}, gpu at {g[2]['iterations']}", flush=True)
    assert o[2]["status"] == want and o[2]["iterations"] != base["iterations"]
    assert g[2]["status"] == want
    assert g[2]["iterations"] == o[2]["iterations"]


@pytest.mark.parametrize("panels", [(1, 1), (4, 4)])
@pytest.mark.parametrize("kind", ["primal", "dual"])
def test_larger_instances_with_panels(orc, qpa, kind, panels):
    base = qpgen.large_random_qp(seed=12, n=3000, m=1500)
    qp = qpgen.with_contradictory_rows(base, 1) if kind == "primal" else qpgen.with_unbounded_ray(base)
    o, g = _pair(orc, qpa, qp, eps=1e-6, max_iter=50000, detect=True, panels=panels)
    print(f"  {qp.name}: oracle {o[2]['status']}@{o[2]['iterations']}, "
          f"gpu {g[2]['status']}@{g[2]['iterations']}", flush=True)
    assert g[2]["status"] == o[2]["status"] == (4 if kind == "primal" else 5)
    assert g[2]["iterations"] == o[2]["iterations"]


@pytest.mark.parametrize("panels", [(1, 1), (4, 4)])
def test_detection_on_keeps_feasible_solves(orc, qpa, panels):
    qp = qpgen.large_random_qp(seed=22, n=4000, m=2000)
    o, g = _pair(orc, qpa, qp, eps=1e-6, detect=True, panels=panels)
    _assert_parity(orc, qp, o, g)
    assert g[2]["status"] == 0


def test_batch_detects_per_instance(orc, qpa):
    insts = [qpgen.primal_infeasible_qp(1), qpgen.tiny_random_qp(2), qpgen.dual_infeasible_qp(3),
             qpgen.mpc_qp(np.random.default_rng([4, 5]), 30, 6, 3)]
    batch = qpgen.concat_batch(insts)
    ref, nAs, nQs = [], [], []
    for qp in insts:
        nA, _ = orc.norm_A(qp, 1000, 1e-7)
        nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
        nAs.append(nA)
        nQs.append(nQ)
        ref.append(orc.solve(qp, orc.OracleSettings(eps=1e-6, max_iter=100000, norm_A=nA,
                                                    norm_Q=nQ, detect_infeasibility=1))[2])
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, max_iter=100000, detect_infeasibility=1))
    bs.set_norms(nAs, nQs)
    _, _, rg = bs.solve()
    bs.close()
    for i, (ro, g) in enumerate(zip(ref, rg)):
        print(f"  [{i}] {insts[i].name}: oracle {ro['status']}@{ro['iterations']} "
              f"gpu {g['status']}@{g['iterations']}", flush=True)
        assert g["status"] == ro["status"] and g["iterations"] == ro["iterations"]
    assert [r["status"] for r in ref] == [4, 0, 5, 0]
