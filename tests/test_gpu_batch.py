"""Batched persistent-kernel solver vs the CPU oracle, instance by instance.

Each instance of the batch must reproduce a single-instance oracle run with the
same norms and settings: equal status, iteration and restart counts, relKKT
within 1e-8, objective within 1e-8 relative, iterates within 1e-8 relative.
"""
import numpy as np
import pytest

import qpgen
from tests import qp_refs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qpa():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible MI355X")
    import paper_2311_07710_amd as m
    m.load()
    return m


def _mixed_batch():
    insts = []
    for i in range(10):                      # MPC instances of every size class
        rng = np.random.default_rng([4, i])
        T = int(rng.integers(10, 101)); nx = int(rng.integers(4, 13)); nu = int(rng.integers(2, 5))
        insts.append(qpgen.mpc_qp(rng, T, nx, nu, name=f"mpc{i}"))
    insts += [qpgen.tiny_random_qp(s) for s in (1, 2, 3)]
    fam = qpgen.portfolio_family(seed=5, count=2)
    insts.append(fam.instance(1))            # n + m = 5201: the largest class
    rng = np.random.default_rng(9)          # an instance without constraint rows
    n = 30
    G = rng.standard_normal((n, n))
    insts.append(qp_refs.make_qp(G @ G.T / n + np.eye(n), np.zeros((0, n)), rng.standard_normal(n),
                                 [], np.full(n, -1.0), np.full(n, 1.0), []))
    insts.append(_long_row_instance())
    return insts


def _long_row_instance(seed=11, n=300, m=160):
    """Rows of A and of P = [Q | -A'] longer than one team pass: Q = diag + v v'
    is dense, A has one dense row and one dense column, the rest is sparse."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    Q = np.diag(rng.uniform(0.5, 2.0, n)) + np.outer(v, v) / n
    A = np.zeros((m, n))
    for i in range(m):
        A[i, rng.choice(n, 5, replace=False)] = rng.standard_normal(5)
    A[0, :] = rng.standard_normal(n)
    A[:, 0] = rng.standard_normal(m)
    l, u = np.full(n, -2.0), np.full(n, 2.0)
    xf = rng.uniform(-1.0, 1.0, n)
    row_type = np.where(np.arange(m) % 3 == 0, qpgen.instances.EQ, qpgen.instances.GE)
    ax = A @ xf                                      # xf is strictly feasible for GE rows
    b = np.where(row_type == qpgen.instances.EQ, ax, ax - rng.uniform(0.0, 1.0, m))
    return qp_refs.make_qp(Q, A, rng.standard_normal(n), b, l, u, row_type, name="long_rows")


def _oracle_all(orc, insts, eps, max_iter=200000, x0s=None, y0s=None, fb=1, momentum=1,
                restart_mode=0, extra=None):
    out = []
    for i, qp in enumerate(insts):
        nA, _ = orc.norm_A(qp, 1000, 1e-7)
        nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
        s = orc.OracleSettings(eps=eps, max_iter=max_iter, norm_A=nA, norm_Q=nQ, warm_fallback=fb,
                               momentum=momentum, restart_mode=restart_mode, **(extra or {}))
        x, y, r, _ = orc.solve(qp, s, x0=None if x0s is None else x0s[i],
                               y0=None if y0s is None else y0s[i])
        out.append((x, y, r, nA, nQ))
    return out


def _compare(batch, xg, yg, rg, ref):
    for i, (xo, yo, ro, _, _) in enumerate(ref):
        v0, v1 = batch.var_off[i], batch.var_off[i + 1]
        r0, r1 = batch.row_off[i], batch.row_off[i + 1]
        g = rg[i]
        print(f"  [{i}] {batch.names[i]}: oracle it={ro['iterations']} rel={ro['rel_kkt']:.3e} | "
              f"gpu it={g['iterations']} rel={g['rel_kkt']:.3e}", flush=True)
        assert g["status"] == ro["status"]
        assert g["iterations"] == ro["iterations"]
        assert g["restarts"] == ro["restarts"]
        assert g["used_warm_start"] == ro["used_warm_start"]
        assert abs(g["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
        assert abs(g["primal_obj"] - ro["primal_obj"]) <= 1e-8 * (1 + abs(ro["primal_obj"]))
        zo = np.concatenate([xo, yo])
        zg = np.concatenate([xg[v0:v1], yg[r0:r1]])
        assert np.max(np.abs(zg - zo)) <= 1e-8 * (1 + np.max(np.abs(zo)))


def test_batch_matches_oracle_per_instance(orc, qpa):
    insts = _mixed_batch()
    batch = qpgen.concat_batch(insts)
    ref = _oracle_all(orc, insts, eps=1e-6)
    with_norms = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6))
    with_norms.set_norms([r[3] for r in ref], [r[4] for r in ref])
    xg, yg, rg = with_norms.solve()
    with_norms.close()
    _compare(batch, xg, yg, rg, ref)


@pytest.mark.parametrize("extra,max_iter", [
    ({"beta_sufficient": 0.15, "beta_necessary": 0.85, "beta_artificial": 0.5,
      "pw_smoothing": 0.3, "step_safety": 0.95}, 200000),
    ({"eps_zero": 1e6}, 8192)], ids=["sec6_constants", "eps_zero"])
def test_batch_method_constants_as_settings(orc, qpa, extra, max_iter):
    """The Sec. 6 constants given as settings reach the persistent kernel (and the
    host's initial primal weight): at values that change the oracle's iteration counts,
    every instance matches the oracle run with the same values (with epsilon_zero above
    the norms the primal weight stays 1 and slow instances stop at the limit)."""
    insts = _mixed_batch()[:8] + [_long_row_instance()]
    batch = qpgen.concat_batch(insts)
    ref = _oracle_all(orc, insts, eps=1e-6, max_iter=max_iter, extra=extra)
    base = _oracle_all(orc, insts, eps=1e-6, max_iter=max_iter)
    assert any(r[2]["iterations"] != b[2]["iterations"] for r, b in zip(ref, base))
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, max_iter=max_iter, **extra))
    bs.set_norms([r[3] for r in ref], [r[4] for r in ref])
    xg, yg, rg = bs.solve()
    bs.close()
    _compare(batch, xg, yg, rg, ref)


@pytest.mark.parametrize("restart_mode", [0, 2])
def test_batch_plain_pdhg(orc, qpa, restart_mode):
    """Sec. 5 baseline (no momentum) in the persistent kernel, long rows included."""
    insts = _mixed_batch()[:5] + [_long_row_instance()]
    batch = qpgen.concat_batch(insts)
    ref = _oracle_all(orc, insts, eps=1e-6, momentum=0, restart_mode=restart_mode)
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, momentum=0, restart_mode=restart_mode))
    bs.set_norms([r[3] for r in ref], [r[4] for r in ref])
    xg, yg, rg = bs.solve()
    bs.close()
    _compare(batch, xg, yg, rg, ref)


def test_batch_power_iteration_norms(orc, qpa):
    insts = _mixed_batch()
    batch = qpgen.concat_batch(insts)
    bs = qpa.BatchSolver(batch, qpa.Settings())
    gA, gQ = bs.norms()
    bs.close()
    for i, qp in enumerate(insts):
        nA, _ = orc.norm_A(qp, 1000, 1e-7)
        nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
        assert gA[i] == pytest.approx(nA, rel=1e-5, abs=1e-12)
        assert gQ[i] == pytest.approx(nQ, rel=1e-5)


def test_batch_power_iteration_limits(orc, qpa):
    """power_iter_max reaches the batched power iteration: after three steps every
    instance's norms equal the oracle's three-step estimates, which for some instances
    differ from the converged ones."""
    insts = _mixed_batch()
    batch = qpgen.concat_batch(insts)
    bs = qpa.BatchSolver(batch, qpa.Settings(power_iter_max=3, power_iter_rtol=0.0))
    gA, gQ = bs.norms()
    bs.close()
    moved = 0
    for i, qp in enumerate(insts):
        nA, _ = orc.norm_A(qp, 3, 0.0)
        nQ, _ = orc.norm_Q(qp, 3, 0.0)
        fA, _ = orc.norm_A(qp, 1000, 1e-7)
        moved += abs(nA - fA) > 1e-6 * fA
        assert gA[i] == pytest.approx(nA, rel=1e-9, abs=1e-12)
        assert gQ[i] == pytest.approx(nQ, rel=1e-9, abs=1e-12)
    assert moved > 0


def test_batch_team_sizes_agree(orc, qpa):
    """Every team size gives the same iterates (row sums are per thread in CSR order);
    the autotuner returns valid team sizes."""
    insts = _mixed_batch()[:8]
    batch = qpgen.concat_batch(insts)
    ref = _oracle_all(orc, insts, eps=1e-6)
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6))
    bs.set_norms([r[3] for r in ref], [r[4] for r in ref])
    for t in (64, 128, 256, 512, 1024):
        bs.set_threads([t] * 4)
        xg, yg, rg = bs.solve()
        _compare(batch, xg, yg, rg, ref)
    chosen = bs.autotune(sample=8, iters=64)
    assert all(c in (64, 128, 256, 512, 1024) for c in chosen)
    xg, yg, rg = bs.solve()
    _compare(batch, xg, yg, rg, ref)
    bs.close()


def test_batch_warm_starts_and_limits(orc, qpa):
    insts = _mixed_batch()[:6]
    batch = qpgen.concat_batch(insts)
    sols = _oracle_all(orc, insts, eps=1e-9)
    rng = np.random.default_rng(1)
    x0s = [s[0] + 1e-6 * rng.standard_normal(s[0].size) for s in sols]
    y0s = [s[1] + 1e-6 * rng.standard_normal(s[1].size) for s in sols]
    x0s[2] = np.full_like(x0s[2], 1e6)       # rejected by the fallback test
    ref = _oracle_all(orc, insts, eps=1e-6, x0s=x0s, y0s=y0s)
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6))
    bs.set_norms([r[3] for r in ref], [r[4] for r in ref])
    xg, yg, rg = bs.solve(x0=np.concatenate(x0s), y0=np.concatenate(y0s))
    _compare(batch, xg, yg, rg, ref)
    assert rg[2]["used_warm_start"] == 0
    assert sum(r["used_warm_start"] for r in rg) >= 4
    bs.close()
    # iteration limit not a multiple of the evaluation interval
    ref2 = _oracle_all(orc, insts, eps=0.0, max_iter=150)
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=0.0, max_iter=150))
    bs.set_norms([r[3] for r in ref2], [r[4] for r in ref2])
    xg, yg, rg = bs.solve()
    _compare(batch, xg, yg, rg, ref2)
    assert all(r["iterations"] == 150 and r["status"] == 1 for r in rg)
    bs.close()


def test_batch_equals_single_solves(qpa):
    insts = _mixed_batch()[:5]
    batch = qpgen.concat_batch(insts)
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6))
    gA, gQ = bs.norms()
    xg, yg, rg = bs.solve()
    bs.close()
    for i, qp in enumerate(insts):
        with qpa.Solver(qp, qpa.Settings(eps=1e-6, norm_A=gA[i], norm_Q=gQ[i])) as s:
            x, y, r = s.solve()
        assert r["iterations"] == rg[i]["iterations"]
        np.testing.assert_allclose(x, xg[batch.var_off[i]:batch.var_off[i + 1]], rtol=1e-9,
                                   atol=1e-9)


def _full_batch_sampled(orc, qpa, precondition):
    """The 4096-instance MPC batch with autotuned team sizes, checked instance by instance
    against the oracle on a sample that includes the instance needing the most iterations.
    The sampled instances run with the oracle's own power-iteration norms (set on the
    batch before the solve; the other instances keep the library's); with preprocessing
    the oracle solves its own Sec. 5 scaling of each sampled instance."""
    batch = qpgen.mpc_batch(seed=4, count=4096)
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, precondition=1 if precondition else 0))
    bs.autotune(sample=128, iters=256)
    gA, gQ = (np.array(v, dtype=float) for v in bs.norms())
    _, _, r0 = bs.solve()
    its = np.array([r["iterations"] for r in r0])
    slow = int(np.argmax(its))
    sample = sorted({0, 1000, 2047, 3071, 4095, slow})
    print(f"  slowest instance {slow}: {its[slow]} iterations (mean {its.mean():.0f})", flush=True)
    ref = {}
    for i in sample:
        qp = batch.instance(i)
        if precondition:
            sc, dv, dr = orc.precondition(qp)
            nA, _ = orc.norm_A(sc, 1000, 1e-7)
            nQ, _ = orc.norm_Q(sc, 1000, 1e-7)
            s = orc.OracleSettings(eps=1e-6, norm_A=nA, norm_Q=nQ)
            ref[i] = orc.solve_scaled(sc, qp, dv, dr, s)[:3]
        else:
            nA, _ = orc.norm_A(qp, 1000, 1e-7)
            nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
            ref[i] = orc.solve(qp, orc.OracleSettings(eps=1e-6, norm_A=nA, norm_Q=nQ))[:3]
        gA[i], gQ[i] = nA, nQ
    bs.set_norms(gA, gQ)
    xg, yg, rg = bs.solve()
    bs.close()
    assert all(r["status"] == 0 for r in rg)
    for i in sample:
        xo, yo, ro = ref[i]
        v0, v1 = batch.var_off[i], batch.var_off[i + 1]
        r0_, r1_ = batch.row_off[i], batch.row_off[i + 1]
        g = rg[i]
        print(f"  [{i}] oracle it={ro['iterations']} | gpu it={g['iterations']}", flush=True)
        assert g["iterations"] == ro["iterations"] and g["status"] == ro["status"]
        assert g["restarts"] == ro["restarts"]
        assert abs(g["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
        assert abs(g["primal_obj"] - ro["primal_obj"]) <= 1e-8 * (1 + abs(ro["primal_obj"]))
        zo = np.concatenate([xo, yo])
        zg = np.concatenate([xg[v0:v1], yg[r0_:r1_]])
        assert np.max(np.abs(zg - zo)) <= 1e-8 * (1 + np.max(np.abs(zo)))


def test_batch_full_size_sampled(orc, qpa):
    """4096 MPC QPs without preprocessing (autotuned teams)."""
    _full_batch_sampled(orc, qpa, precondition=False)


def test_batch_full_size_preconditioned_sampled(orc, qpa):
    """4096 MPC QPs exactly as the benchmark times them: Sec. 5 preprocessing on the
    device, autotuned teams, relKKT 1e-6; the sample includes the slowest instance."""
    _full_batch_sampled(orc, qpa, precondition=True)


def _slice_edge_instance(seed=21, n=200, m=300):
    """Rows around the 128-entry long-row limit (127, 128, 129) in A and in P (a
    column of A with 231 entries, one with about 120), an all-empty 64-row slice
    (rows 64-127) and a partial last slice (rows 256-299)."""
    rng = np.random.default_rng(seed)
    A = np.zeros((m, n))
    for i, L in enumerate((127, 128, 129, 0, 1)):
        A[i, rng.choice(n, L, replace=False)] = rng.standard_normal(L)
    live = [i for i in range(5, m) if not 64 <= i < 128]
    for i in live:
        A[i, rng.choice(np.arange(2, n), 3, replace=False)] = rng.standard_normal(3)
    A[live, 0] = rng.standard_normal(len(live))              # P row 0: > 128 entries
    A[np.array(live[:118]), 1] = rng.standard_normal(118)      # P row 1: about 120
    Q = np.diag(rng.uniform(0.5, 2.0, n))
    l, u = np.full(n, -2.0), np.full(n, 2.0)
    xf = rng.uniform(-1.0, 1.0, n)
    row_type = np.where(np.arange(m) % 2 == 0, qpgen.instances.EQ, qpgen.instances.GE)
    ax = A @ xf
    b = np.where(row_type == qpgen.instances.EQ, ax, ax - rng.uniform(0.0, 1.0, m))
    return qp_refs.make_qp(Q, A, rng.standard_normal(n), b, l, u, row_type, name="slice_edges")


def test_batch_sliced_layout_edges(orc, qpa):
    """The sliced row layout at its edges, next to instances of other size classes."""
    edge = _slice_edge_instance()
    lens_a = np.diff(edge.a_rowptr)
    assert {127, 128, 129}.issubset(set(lens_a.tolist())) and (lens_a[64:128] == 0).all()
    P_lens = np.diff(edge.q_rowptr) + np.bincount(edge.a_col, minlength=edge.n)
    assert P_lens.max() > 128 and ((P_lens > 64) & (P_lens <= 128)).any()
    insts = [edge, qpgen.tiny_random_qp(4), _mixed_batch()[3]]
    batch = qpgen.concat_batch(insts)
    ref = _oracle_all(orc, insts, eps=1e-6, max_iter=4000)   # the edge instance stops at the cap
    for threads in (64, 1024):
        bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, max_iter=4000))
        bs.set_norms([r[3] for r in ref], [r[4] for r in ref])
        bs.set_threads([threads] * 4)
        xg, yg, rg = bs.solve()
        bs.close()
        _compare(batch, xg, yg, rg, ref)


def test_batch_instance_too_large_for_lds(orc, qpa):
    """An instance whose vectors cannot live in LDS (3 n + m = 24500 doubles) runs
    with all vectors in HBM next to instances that keep them in LDS."""
    big = qpgen.eq_qp(seed=8, n=7000)
    assert 3 * big.n + big.m > 160 * 1024 // 8
    insts = [big, qpgen.tiny_random_qp(5), _mixed_batch()[2]]
    batch = qpgen.concat_batch(insts)
    ref = _oracle_all(orc, insts, eps=1e-6)
    for threads in (256, 1024):
        bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6))
        bs.set_norms([r[3] for r in ref], [r[4] for r in ref])
        bs.set_threads([threads] * 4)
        xg, yg, rg = bs.solve()
        bs.close()
        _compare(batch, xg, yg, rg, ref)


@pytest.mark.parametrize("mom,mode,K", [(1, 2, 100), (0, 2, 100), (1, 3, 100), (0, 3, 100),
                                        (1, 1, 10)])
def test_batch_ablation_modes_preconditioned(orc, qpa, mom, mode, K):
    """The configuration of the Sec. 5 comparison in the benchmark: preprocessing on, each
    method as a batched launch over instances of the seven synthetic classes (two each),
    checked per instance against the oracle's solve of its own scaling of the instance
    (the no-restart methods stop at the iteration limit)."""
    per = 2
    insts = [q for k, q in enumerate(qpgen.ablation_set(24)) if k % 24 < per]
    batch = qpgen.concat_batch(insts)
    cap = 6000
    refs = []
    for qp in insts:
        sc, dv, dr = orc.precondition(qp)
        nA, _ = orc.norm_A(sc, 1000, 1e-7)
        nQ, _ = orc.norm_Q(sc, 1000, 1e-7)
        s = orc.OracleSettings(eps=1e-6, max_iter=cap, momentum=mom, restart_mode=mode,
                               fixed_K=K, norm_A=nA, norm_Q=nQ)
        refs.append((*orc.solve_scaled(sc, qp, dv, dr, s)[:3], nA, nQ))
    bs = qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, max_iter=cap, momentum=mom,
                                             restart_mode=mode, fixed_K=K, precondition=1))
    bs.set_norms([r[3] for r in refs], [r[4] for r in refs])
    xg, yg, rg = bs.solve()
    bs.close()
    for i, (xo, yo, ro, _, _) in enumerate(refs):
        v0, v1 = batch.var_off[i], batch.var_off[i + 1]
        r0, r1 = batch.row_off[i], batch.row_off[i + 1]
        g = rg[i]
        assert g["status"] == ro["status"] and g["iterations"] == ro["iterations"], (i, g, ro)
        assert g["restarts"] == ro["restarts"]
        assert abs(g["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
        zo = np.concatenate([xo, yo])
        zg = np.concatenate([xg[v0:v1], yg[r0:r1]])
        assert np.max(np.abs(zg - zo)) <= 1e-8 * (1 + np.max(np.abs(zo)))
