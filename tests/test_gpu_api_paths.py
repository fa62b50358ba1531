"""API paths beyond a plain solve: new right-hand sides and costs on an existing
handle (single and batched), and the wall-clock limit."""
import numpy as np
import pytest

import qpgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpa():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2311_07710_amd as m
    m.load()
    return m


def _oracle(orc, qp, nA, nQ, eps=1e-6):
    s = orc.OracleSettings(eps=eps, norm_A=nA, norm_Q=nQ)
    return orc.solve(qp, s)[:3]


def _close(xg, yg, g, ref):
    xo, yo, ro = ref
    assert g["status"] == ro["status"] and g["iterations"] == ro["iterations"]
    assert abs(g["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
    zo, zg = np.concatenate([xo, yo]), np.concatenate([xg, yg])
    assert np.max(np.abs(zg - zo)) <= 1e-8 * (1 + np.max(np.abs(zo)))


def test_update_vectors_single_and_batch(orc, qpa):
    """Family members share Q and A: a handle created for members 0 (and 1) and given
    the c and b of members 2 (and 3) solves those members exactly as the oracle does,
    including a graph captured before the update."""
    fam = qpgen.portfolio_family(seed=5, n_assets=400, k=20, count=4)
    insts = [fam.instance(i) for i in range(4)]
    nA, _ = orc.norm_A(insts[0], 1000, 1e-7)
    nQ, _ = orc.norm_Q(insts[0], 1000, 1e-7)
    refs = [_oracle(orc, qp, nA, nQ) for qp in insts]
    with qpa.Solver(insts[0], qpa.Settings(eps=1e-6, norm_A=nA, norm_Q=nQ)) as s:
        _close(*s.solve(), refs[0])
        s.update_vectors(c=insts[2].c, b=insts[2].b)
        _close(*s.solve(), refs[2])
        s.update_vectors(b=insts[0].b)              # b of member 0, c of member 2 kept
        mixed = qpgen.instances._make("mixed", insts[0].Q(), insts[0].A(), insts[2].c,
                                      insts[0].b, insts[0].l, insts[0].u, insts[0].row_type)
        _close(*s.solve(), _oracle(orc, mixed, nA, nQ))
    batch = qpgen.concat_batch(insts[:2])
    with qpa.BatchSolver(batch, qpa.Settings(eps=1e-6)) as bs:
        bs.set_norms([nA, nA], [nQ, nQ])
        bs.update_vectors(c=np.concatenate([insts[2].c, insts[3].c]),
                          b=np.concatenate([insts[2].b, insts[3].b]))
        xb, yb, rb = bs.solve()
    for j, i in enumerate((2, 3)):
        v0, v1 = batch.var_off[j], batch.var_off[j + 1]
        r0, r1 = batch.row_off[j], batch.row_off[j + 1]
        _close(xb[v0:v1], yb[r0:r1], rb[j], refs[i])


def test_time_limit(qpa):
    """A wall-clock limit far below the solve time ends single and batched solves with
    the time-limit status and a valid point."""
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    with qpa.Solver(qp, qpa.Settings(eps=1e-12, time_limit_s=0.002)) as s:
        x, y, r = s.solve()
    assert r["status"] == qpa.QP_TIME_LIMIT and 0 < r["iterations"] < 200000
    assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
    batch = qpgen.mpc_batch(seed=4, count=64)
    with qpa.BatchSolver(batch, qpa.Settings(eps=1e-12, time_limit_s=0.002)) as bs:
        xb, yb, rb = bs.solve()
    st = np.array([q["status"] for q in rb])
    assert (st == qpa.QP_TIME_LIMIT).any() and np.isin(st, [qpa.QP_OPTIMAL, qpa.QP_TIME_LIMIT]).all()
    assert np.all(np.isfinite(xb)) and np.all(np.isfinite(yb))


def test_log_callback(orc, qpa):
    """settings.log_cb sees every relKKT evaluation of a single solve, in order, with the
    records qp_get_check_log keeps and the oracle's restart decisions; a batch handle
    never calls it."""
    qp = qpgen.tiny_random_qp(3)
    nA, _ = orc.norm_A(qp, 1000, 1e-7)
    nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
    _, _, ro, lo = orc.solve(qp, orc.OracleSettings(eps=1e-6, norm_A=nA, norm_Q=nQ),
                             log_cap=100000)
    seen = []
    with qpa.Solver(qp, qpa.Settings(eps=1e-6, norm_A=nA, norm_Q=nQ, log_checks=1,
                                     log_cb=seen.append)) as s:
        _, _, r = s.solve()
        kept = s.check_log()
        assert r["iterations"] == ro["iterations"] and r["restarts"] == ro["restarts"]
        assert seen == kept and len(seen) == len(lo) > 1
        for a, b in zip(seen, lo):
            assert (a["total"], a["k"], a["candidate"], a["restarted"]) == \
                (b["total"], b["k"], b["candidate"], b["restarted"])
        assert sum(c["restarted"] for c in seen) == r["restarts"]
        # a second solve calls it again from the start; without log_checks as well
        seen.clear()
        s.solve()
        assert seen == kept
    seen2 = []
    with qpa.Solver(qp, qpa.Settings(eps=1e-6, norm_A=nA, norm_Q=nQ,
                                     log_cb=seen2.append)) as s:
        s.solve()
        assert s.check_log() == [] and seen2 == kept
    calls = []
    batch = qpgen.concat_batch([qpgen.tiny_random_qp(k) for k in (1, 2)])
    with qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, log_cb=calls.append)) as bs:
        _, _, rb = bs.solve()
    assert all(q["status"] == qpa.QP_OPTIMAL for q in rb) and calls == []
