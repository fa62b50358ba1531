"""Seeded sweep of small mixed-feature QPs: the single-instance GPU path and one
batched launch against the CPU oracle, instance by instance.

Each instance draws its own size (n up to 80, m up to 60, m = 0 included), row
types (EQ / GE), empty rows, variable bounds (boxed, one-sided, free; a free
variable only where Q is positive definite, so the problem stays bounded), Q
(diagonal + low rank, low rank only, or zero with every variable boxed) and a
feasible right-hand side.  Runs are compared at equal iteration counts with the
tolerances of the other parity tests.
"""
import numpy as np
import pytest

import qpgen
from tests import qp_refs

pytestmark = pytest.mark.gpu

SEEDS = range(24)


@pytest.fixture(scope="module")
def qpa():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2311_07710_amd as m
    m.load()
    return m


def _instance(seed):
    rng = np.random.default_rng([77, seed])
    n = int(rng.integers(1, 81))
    m = int(rng.integers(0, 61)) if seed % 6 else 0
    kind = seed % 3                      # 0: diag + low rank, 1: low rank only, 2: Q = 0
    r = int(rng.integers(1, max(2, n // 3) + 1))
    G = rng.standard_normal((n, r))
    if kind == 0:
        Q = np.diag(rng.uniform(0.1, 2.0, n)) + G @ G.T / r
    elif kind == 1:
        Q = G @ G.T / r
    else:
        Q = np.zeros((n, n))
    density = rng.uniform(0.05, 0.5)
    A = np.where(rng.random((m, n)) < density, rng.standard_normal((m, n)), 0.0)
    if m:
        A[rng.random(m) < 0.1] = 0.0     # some empty rows
    # bounds: boxed, lower only, upper only, free (free only with positive definite Q)
    pick = rng.integers(0, 4 if kind == 0 else 1, n)
    l = np.where((pick == 0) | (pick == 1), -rng.uniform(0.5, 5.0, n), -np.inf)
    u = np.where((pick == 0) | (pick == 2), rng.uniform(0.5, 5.0, n), np.inf)
    if kind != 0:                         # a singular Q: keep every variable boxed
        l, u = -rng.uniform(0.5, 5.0, n), rng.uniform(0.5, 5.0, n)
    lo, hi = np.where(np.isfinite(l), l, -1.0), np.where(np.isfinite(u), u, 1.0)
    xf = lo + (hi - lo) * rng.uniform(0.1, 0.9, n)
    row_type = (rng.random(m) < 0.5).astype(np.uint8)
    ax = A @ xf
    b = np.where(row_type == 1, ax - rng.uniform(0.0, 1.0, m), ax)
    b[~A.any(axis=1) & (row_type == 0)] = 0.0
    return qp_refs.make_qp(Q, A, rng.standard_normal(n), b, l, u, row_type,
                           name=f"sweep{seed}_n{n}_m{m}_k{kind}")


def _oracle(orc, qp, eps, max_iter):
    nA, _ = orc.norm_A(qp, 1000, 1e-7)
    nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
    s = orc.OracleSettings(eps=eps, max_iter=max_iter, norm_A=nA, norm_Q=nQ)
    x, y, r, _ = orc.solve(qp, s)
    return x, y, r, nA, nQ


def _close(g, xg, yg, ref):
    xo, yo, ro = ref[:3]
    assert g["status"] == ro["status"]
    assert g["iterations"] == ro["iterations"]
    assert abs(g["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
    assert abs(g["primal_obj"] - ro["primal_obj"]) <= 1e-8 * (1 + abs(ro["primal_obj"]))
    zo = np.concatenate([xo, yo])
    zg = np.concatenate([xg, yg])
    assert np.max(np.abs(zg - zo)) <= 1e-8 * (1 + np.max(np.abs(zo)))


def test_random_sweep_single_and_batch(orc, qpa):
    eps, max_iter = 1e-6, 6000
    insts = [_instance(s) for s in SEEDS]
    refs = [_oracle(orc, qp, eps, max_iter) for qp in insts]
    for qp, ref in zip(insts, refs):
        if ref[3] == 0.0 and ref[4] == 0.0:
            continue                      # nothing to solve (rejected by qp_create)
        with qpa.Solver(qp, qpa.Settings(eps=eps, max_iter=max_iter, norm_A=ref[3],
                                         norm_Q=ref[4])) as s:
            xg, yg, g = s.solve()
        print(f"  {qp.name}: oracle it={ref[2]['iterations']} st={ref[2]['status']} | "
              f"gpu it={g['iterations']} st={g['status']}", flush=True)
        _close(g, xg, yg, ref)
    keep = [i for i, r in enumerate(refs) if r[3] > 0.0 or r[4] > 0.0]
    batch = qpgen.concat_batch([insts[i] for i in keep])
    with qpa.BatchSolver(batch, qpa.Settings(eps=eps, max_iter=max_iter)) as bs:
        bs.set_norms([refs[i][3] for i in keep], [refs[i][4] for i in keep])
        xb, yb, rb = bs.solve()
    for j, i in enumerate(keep):
        v0, v1 = batch.var_off[j], batch.var_off[j + 1]
        r0, r1 = batch.row_off[j], batch.row_off[j + 1]
        _close(rb[j], xb[v0:v1], yb[r0:r1], refs[i])


def _oracle_pre(orc, qp, eps, max_iter):
    sc, dv, dr = orc.precondition(qp)
    nA, _ = orc.norm_A(sc, 1000, 1e-7)
    nQ, _ = orc.norm_Q(sc, 1000, 1e-7)
    s = orc.OracleSettings(eps=eps, max_iter=max_iter, norm_A=nA, norm_Q=nQ)
    x, y, r, _ = orc.solve_scaled(sc, qp, dv, dr, s)
    return x, y, r, nA, nQ


def test_random_sweep_preconditioned(orc, qpa):
    """The same sweep with the Sec. 5 preprocessing on (device scaling, single and
    batched, against the oracle's own scaling)."""
    eps, max_iter = 1e-6, 6000
    insts = [_instance(s) for s in SEEDS]
    refs = [_oracle_pre(orc, qp, eps, max_iter) for qp in insts]
    keep = [i for i, r in enumerate(refs) if r[3] > 0.0 or r[4] > 0.0]
    for i in keep:
        qp, ref = insts[i], refs[i]
        with qpa.Solver(qp, qpa.Settings(eps=eps, max_iter=max_iter, norm_A=ref[3],
                                         norm_Q=ref[4], precondition=1)) as s:
            xg, yg, g = s.solve()
        _close(g, xg, yg, ref)
    batch = qpgen.concat_batch([insts[i] for i in keep])
    with qpa.BatchSolver(batch, qpa.Settings(eps=eps, max_iter=max_iter,
                                             precondition=1)) as bs:
        bs.set_norms([refs[i][3] for i in keep], [refs[i][4] for i in keep])
        xb, yb, rb = bs.solve()
    for j, i in enumerate(keep):
        v0, v1 = batch.var_off[j], batch.var_off[j + 1]
        r0, r1 = batch.row_off[j], batch.row_off[j + 1]
        _close(rb[j], xb[v0:v1], yb[r0:r1], refs[i])


def test_random_sweep_plain_pdhg(orc, qpa):
    """The sweep in the Sec. 5 PDHG baseline (no momentum, restarts off)."""
    eps, max_iter = 1e-6, 3000
    insts = [_instance(s) for s in SEEDS]
    refs = []
    for qp in insts:
        nA, _ = orc.norm_A(qp, 1000, 1e-7)
        nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
        s = orc.OracleSettings(eps=eps, max_iter=max_iter, norm_A=nA, norm_Q=nQ, momentum=0,
                               restart_mode=orc.RESTART_NONE)
        x, y, r, _ = orc.solve(qp, s)
        refs.append((x, y, r, nA, nQ))
    keep = [i for i, r in enumerate(refs) if r[3] > 0.0 or r[4] > 0.0]
    batch = qpgen.concat_batch([insts[i] for i in keep])
    with qpa.BatchSolver(batch, qpa.Settings(eps=eps, max_iter=max_iter, momentum=0,
                                             restart_mode=3)) as bs:
        bs.set_norms([refs[i][3] for i in keep], [refs[i][4] for i in keep])
        xb, yb, rb = bs.solve()
    for j, i in enumerate(keep):
        v0, v1 = batch.var_off[j], batch.var_off[j + 1]
        r0, r1 = batch.row_off[j], batch.row_off[j + 1]
        _close(rb[j], xb[v0:v1], yb[r0:r1], refs[i])
