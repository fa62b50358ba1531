"""GPU path vs CPU oracle, element by element, through the C-ABI.

Both sides get the same seeded instance and the same operator norms (the
oracle's power-iteration values are passed to the library as overrides, so
step sizes agree).  Tolerances (FP64):
  * relKKT of the returned point: |gpu - oracle| <= 1e-8 (the metric is
    already relative);
  * primal objective: |gpu - oracle| <= 1e-8 (1 + |oracle|);
  * iterates (diagnostic): ||z_gpu - z_or||_inf <= 1e-8 (1 + ||z_or||_inf);
  * iteration counts, restart counts and the evaluation log (iteration,
    candidate, restart flag) identical.
The GPU's reported relKKT is also re-evaluated by the oracle's own KKT routine
at the GPU's returned point (1e-7 relative; the gap term's cancellation makes
reduction-order effects ~1e-9): this pins the KKT kernels independently of the
trajectory.
"""
import math

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


def _norms(orc, qp):
    nA, _ = orc.norm_A(qp, 1000, 1e-7)
    nQ, _ = orc.norm_Q(qp, 1000, 1e-7)
    return nA, nQ


def _pair(orc, qpa, qp, *, eps=1e-6, max_iter=200000, check_every=64, mode=0, fixed_K=100,
          x0=None, y0=None, omega0=0.0, warm_fallback=1, use_graph=1, norms=None, log=True,
          panels=(0, 0), momentum=1, precondition=False, scaling_out=None, detect=False,
          ruiz=10, extra=None):
    """Oracle and GPU runs of the same instance and settings.  With precondition the
    oracle solves its own Sec. 5 scaling of qp (relKKT on qp, `ruiz` Ruiz passes) and the
    GPU scales on the device; norms are then those of the scaled problem.  `extra`: more
    settings, given to both sides under the same names."""
    extra = extra or {}
    if precondition:
        sc, dv, dr = orc.precondition(qp, ruiz_iters=ruiz)
        nA, nQ = norms if norms is not None else _norms(orc, sc)
    else:
        nA, nQ = norms if norms is not None else _norms(orc, qp)
    os_ = orc.OracleSettings(eps=eps, max_iter=max_iter, check_every=check_every,
                             restart_mode=mode, fixed_K=fixed_K, norm_A=nA, norm_Q=nQ,
                             warm_fallback=warm_fallback, momentum=momentum,
                             detect_infeasibility=1 if detect else 0, **extra)
    if precondition:
        xo, yo, ro, lo = orc.solve_scaled(sc, qp, dv, dr, os_, x0=x0, y0=y0, omega0=omega0,
                                          log_cap=100000)
    else:
        xo, yo, ro, lo = orc.solve(qp, os_, x0=x0, y0=y0, omega0=omega0, log_cap=100000)
    gs = qpa.Settings(eps=eps, max_iter=max_iter, check_every=check_every, restart_mode=mode,
                      fixed_K=fixed_K, norm_A=nA, norm_Q=nQ, warm_fallback=warm_fallback,
                      use_graph=use_graph, log_checks=1 if log else 0,
                      panels_dual=panels[0], panels_primal=panels[1], momentum=momentum,
                      precondition=1 if precondition else 0, ruiz_iters=ruiz,
                      detect_infeasibility=1 if detect else 0, **extra)
    with qpa.Solver(qp, gs) as s:
        if scaling_out is not None:
            scaling_out.append((s.scaling(), (dv, dr) if precondition else None))
        xg, yg, rg = s.solve(x0=x0, y0=y0, omega0=omega0)
        lg = s.check_log()
    return (xo, yo, ro, lo), (xg, yg, rg, lg)


def _assert_parity(orc, qp, o, g, *, z_tol=1e-8, check_log=True):
    xo, yo, ro, lo = o
    xg, yg, rg, lg = g
    print(f"  oracle: status={ro['status']} it={ro['iterations']} restarts={ro['restarts']} "
          f"relKKT={ro['rel_kkt']:.3e} obj={ro['primal_obj']:.12g}", flush=True)
    print(f"  gpu:    status={rg['status']} it={rg['iterations']} restarts={rg['restarts']} "
          f"relKKT={rg['rel_kkt']:.3e} obj={rg['primal_obj']:.12g}", flush=True)
    assert rg["status"] == ro["status"]
    assert rg["iterations"] == ro["iterations"]
    assert rg["restarts"] == ro["restarts"]
    assert rg["kkt_evals"] == ro["kkt_evals"]
    assert rg["used_warm_start"] == ro["used_warm_start"]
    assert abs(rg["rel_kkt"] - ro["rel_kkt"]) <= 1e-8
    assert abs(rg["primal_obj"] - ro["primal_obj"]) <= 1e-8 * (1 + abs(ro["primal_obj"]))
    assert abs(rg["dual_obj"] - ro["dual_obj"]) <= 1e-8 * (1 + abs(ro["dual_obj"]))
    # omega is driven by restart distances, which near machine-precision convergence are
    # themselves rounding noise: agreement to 1e-6 relative
    assert rg["omega"] == pytest.approx(ro["omega"], rel=1e-6)
    zo = np.concatenate([xo, yo])
    zg = np.concatenate([xg, yg])
    assert np.max(np.abs(zg - zo)) <= z_tol * (1 + np.max(np.abs(zo)))
    # the GPU's KKT kernels, re-checked at the GPU's own point
    k = orc.rel_kkt(qp, xg, yg)
    # (block-ordered reductions vs sequential sums; the gap term cancels P - D, so the
    # relative agreement is ~1e-9 near convergence.  With large bounds the sums behind P
    # and D hold terms a million times larger than P - D (control instances: state
    # bounds of several hundred), and their summation order alone moves the gap term by
    # ~1e-12; hence 1e-11 absolute beside 1e-7 relative, far inside the 1e-8 bar above.)
    assert rg["rel_kkt"] == pytest.approx(k["rel_kkt"], rel=1e-7, abs=1e-11)
    assert rg["primal_obj"] == pytest.approx(k["primal_obj"], rel=1e-12, abs=1e-12)
    if check_log:
        assert len(lg) == len(lo)
        for a, b in zip(lg, lo):
            assert (a["total"], a["k"], a["candidate"], a["restarted"]) == \
                (b["total"], b["k"], b["candidate"], b["restarted"])
            assert a["r_cur"] == pytest.approx(b["r_cur"], rel=1e-6, abs=1e-12)
            assert a["r_avg"] == pytest.approx(b["r_avg"], rel=1e-6, abs=1e-12)


# ---------------------------------------------------------------------------
# tiny random config (n=100, m=50) to tolerance
# ---------------------------------------------------------------------------
def test_tiny_config_to_tolerance(orc, qpa):
    qp = qpgen.tiny_random_qp(1)
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    _assert_parity(orc, qp, o, g)
    assert g[2]["status"] == 0 and g[2]["rel_kkt"] <= 1e-6


@pytest.mark.parametrize("seed", list(range(1001, 1101)))
def test_tiny_config_seed_sweep(orc, qpa, seed):
    qp = qpgen.tiny_random_qp(seed)
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    _assert_parity(orc, qp, o, g)


# ---------------------------------------------------------------------------
# operator norms: GPU power iteration vs the oracle's
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("maker", ["tiny", "large", "portfolio"])
def test_power_iteration_norms(orc, qpa, maker):
    qp = {"tiny": lambda: qpgen.tiny_random_qp(1),
          "large": lambda: qpgen.large_random_qp(seed=2, n=30000, m=15000),
          "portfolio": lambda: qpgen.portfolio_qp(seed=3, n_assets=20000, k=40)}[maker]()
    nA, nQ = _norms(orc, qp)
    with qpa.Solver(qp, qpa.Settings()) as s:
        gA, gQ = s.norms()
    assert gA == pytest.approx(nA, rel=1e-5)
    assert gQ == pytest.approx(nQ, rel=1e-5)


@pytest.mark.parametrize("maxit,rtol", [(3, 0.0), (200, 1e-3)])
def test_power_iteration_limits(orc, qpa, maxit, rtol):
    """power_iter_max and power_iter_rtol reach the device: stopped after `maxit` steps,
    or once the estimate moves by at most rtol, the GPU's norms equal the oracle's under
    the same limits (the same iteration from the same start), which differ from the
    converged norms."""
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    nA, itA = orc.norm_A(qp, maxit, rtol)
    nQ, itQ = orc.norm_Q(qp, maxit, rtol)
    fA, fQ = _norms(orc, qp)
    print(f"  oracle: ||A|| {nA:.12g} after {itA} steps, ||Q|| {nQ:.12g} after {itQ}", flush=True)
    assert abs(nA - fA) > 1e-6 * fA and abs(nQ - fQ) > 1e-6 * fQ
    with qpa.Solver(qp, qpa.Settings(power_iter_max=maxit, power_iter_rtol=rtol)) as s:
        gA, gQ = s.norms()
    assert gA == pytest.approx(nA, rel=1e-9)
    assert gQ == pytest.approx(nQ, rel=1e-9)


# ---------------------------------------------------------------------------
# the method's constants as settings (Sec. 6 restart criteria, primal-weight
# smoothing, step-size factor, epsilon_zero).  Each value below changes the oracle's
# trajectory on these instances, so agreement with the oracle run at that value shows
# that the GPU applied it.
# ---------------------------------------------------------------------------
_CONSTANTS = {
    "restart_criteria": {"beta_sufficient": 0.1, "beta_necessary": 0.9, "beta_artificial": 1.0},
    "pw_smoothing": {"pw_smoothing": 0.6},
    "step_safety": {"step_safety": 0.9},
    "eps_zero": {"eps_zero": 1e6},
}


@pytest.mark.parametrize("name", sorted(_CONSTANTS))
@pytest.mark.parametrize("seed", [1, 7])
def test_method_constants_as_settings(orc, qpa, name, seed):
    qp = qpgen.tiny_random_qp(seed)
    norms = _norms(orc, qp)
    extra = _CONSTANTS[name]
    base = orc.solve(qp, orc.OracleSettings(eps=1e-6, norm_A=norms[0], norm_Q=norms[1]),
                     log_cap=100000)
    o, g = _pair(orc, qpa, qp, eps=1e-6, norms=norms, extra=extra)

    def trace(log):
        return [(e["total"], e["restarted"], e["r_cur"]) for e in log]

    assert trace(o[3]) != trace(base[3])
    _assert_parity(orc, qp, o, g)


# ---------------------------------------------------------------------------
# scaled large random QP and portfolio QP at a fixed iteration count
# ---------------------------------------------------------------------------
def test_large_random_scaled_fixed_iterations(orc, qpa):
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=640)
    _assert_parity(orc, qp, o, g)


@pytest.mark.parametrize("panels", [(2, 2), (4, 8), (8, 4), (8, 8)])
def test_column_panels_match_oracle(orc, qpa, panels):
    """XCD-pinned column panels (partial sums + combine) on both phases."""
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=320, panels=panels)
    _assert_parity(orc, qp, o, g)


@pytest.mark.parametrize("panels", [(8, 8), (2, 4)])
def test_column_panels_long_rows(orc, qpa, panels):
    """The 20000-nonzero budget row is split across panels and chunks."""
    qp = qpgen.portfolio_qp(seed=3, n_assets=20000, k=40)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=256, panels=panels)
    _assert_parity(orc, qp, o, g)


@pytest.mark.parametrize("panels", [(8, 8), (4, 2)])
def test_column_panels_tiny_to_tolerance(orc, qpa, panels):
    qp = qpgen.tiny_random_qp(1)
    o, g = _pair(orc, qpa, qp, eps=1e-6, panels=panels)
    _assert_parity(orc, qp, o, g)


def test_large_random_scaled_to_tolerance(orc, qpa):
    qp = qpgen.large_random_qp(seed=22, n=4000, m=2000)
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    _assert_parity(orc, qp, o, g)


def test_portfolio_scaled_long_rows(orc, qpa):
    """Budget row of 20000 nonzeros: chunked rows combined across workgroups."""
    qp = qpgen.portfolio_qp(seed=3, n_assets=20000, k=40)
    assert qp.a_rowptr[-1] - qp.a_rowptr[-2] > 2048
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=512)
    _assert_parity(orc, qp, o, g)


def test_portfolio_family_member_to_tolerance(orc, qpa):
    fam = qpgen.portfolio_family(seed=5, count=2)
    qp = fam.instance(0)
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    _assert_parity(orc, qp, o, g)


def test_mpc_instance_to_tolerance(orc, qpa):
    rng = np.random.default_rng([4, 2])
    qp = qpgen.mpc_qp(rng, 36, 9, 4)
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    _assert_parity(orc, qp, o, g)


# ---------------------------------------------------------------------------
# restart modes, evaluation cadences, graph vs direct launches, warm starts
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("mode,kw", [(1, {"fixed_K": 100}), (1, {"fixed_K": 37}),
                                     (2, {}), (3, {"eps": 1e-4, "max_iter": 3000})])
def test_restart_modes(orc, qpa, mode, kw):
    qp = qpgen.tiny_random_qp(1)
    args = dict(eps=1e-6)
    args.update(kw)
    o, g = _pair(orc, qpa, qp, mode=mode, **args)
    _assert_parity(orc, qp, o, g)


# Sec. 5 baselines: plain PDHG (no momentum) under every restart rule
@pytest.mark.parametrize("mode,kw", [(0, {}), (1, {"fixed_K": 100}), (2, {}),
                                     (3, {"eps": 1e-4, "max_iter": 6000})])
def test_pdhg_modes(orc, qpa, mode, kw):
    qp = qpgen.tiny_random_qp(2)
    args = dict(eps=1e-6)
    args.update(kw)
    o, g = _pair(orc, qpa, qp, mode=mode, momentum=0, **args)
    _assert_parity(orc, qp, o, g)


@pytest.mark.parametrize("panels", [(1, 1), (4, 4)])
def test_pdhg_scaled_fixed_iterations(orc, qpa, panels):
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=300, momentum=0, panels=panels)
    _assert_parity(orc, qp, o, g)


@pytest.mark.parametrize("check_every,max_iter", [(1, 50), (7, 300), (64, 300), (100, 277)])
def test_cadence_and_partial_interval(orc, qpa, check_every, max_iter):
    qp = qpgen.tiny_random_qp(3)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=max_iter, check_every=check_every)
    _assert_parity(orc, qp, o, g)
    assert g[2]["iterations"] == max_iter and g[2]["status"] == 1


def test_graph_and_direct_launch_identical(qpa, orc):
    qp = qpgen.tiny_random_qp(4)
    nA, nQ = _norms(orc, qp)
    out = []
    for ug in (0, 1):
        with qpa.Solver(qp, qpa.Settings(norm_A=nA, norm_Q=nQ, use_graph=ug)) as s:
            out.append(s.solve())
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][2]["iterations"] == out[1][2]["iterations"]


def test_repeat_solve_is_deterministic(qpa):
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    with qpa.Solver(qp, qpa.Settings(eps=0.0, max_iter=256)) as s:
        a = s.solve()
        b = s.solve()
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_array_equal(a[1], b[1])


def test_warm_start_paths(orc, qpa):
    qp = qpgen.tiny_random_qp(1)
    xs, ys, _, _ = orc.solve(qp, orc.OracleSettings(eps=1e-9))
    rng = np.random.default_rng(0)
    xw = xs + 1e-3 * rng.standard_normal(qp.n)
    yw = ys + 1e-3 * rng.standard_normal(qp.m)
    for fb in (1, 0):
        o, g = _pair(orc, qpa, qp, eps=1e-6, x0=xw, y0=yw, omega0=2.0, warm_fallback=fb)
        _assert_parity(orc, qp, o, g)
        assert g[2]["used_warm_start"] == 1
    # a bad warm start is rejected by the fallback test
    o, g = _pair(orc, qpa, qp, eps=1e-6, x0=np.full(qp.n, 1e6), y0=np.zeros(qp.m))
    _assert_parity(orc, qp, o, g)
    assert g[2]["used_warm_start"] == 0
    # warm start at the solution terminates before the first iteration
    o, g = _pair(orc, qpa, qp, eps=1e-8, x0=xs, y0=ys)
    _assert_parity(orc, qp, o, g)
    assert g[2]["iterations"] == 0


# ---------------------------------------------------------------------------
# edge cases: no rows, empty rows, rows at/above the LDS block size, free and
# one-sided bounds, equality-only, singular Q
# ---------------------------------------------------------------------------
def test_unconstrained_m0(orc, qpa):
    rng = np.random.default_rng(11)
    n = 300
    G = rng.standard_normal((n, n)) * (rng.random((n, n)) < 0.05)
    Q = G @ G.T / n + np.eye(n)
    qp = qp_refs.make_qp(Q, np.zeros((0, n)), rng.standard_normal(n), [], np.full(n, -np.inf),
                         np.full(n, np.inf), [])
    o, g = _pair(orc, qpa, qp, eps=1e-9)
    _assert_parity(orc, qp, o, g)
    np.testing.assert_allclose(g[0], np.linalg.solve(Q, -qp.c), rtol=1e-6, atol=1e-7)


def test_row_lengths_around_block_size(orc, qpa):
    """Rows of 0 and 1 nonzeros, either side of 1024 and of the 2048-entry block size,
    4097 and 6000, among short rows."""
    rng = np.random.default_rng(12)
    n = 7000
    lens = [0, 1, 1023, 1024, 1025, 2047, 2048, 2049, 5, 4097, 0, 6000, 3] + [7] * 300
    rows, cols, vals = [], [], []
    for i, L in enumerate(lens):
        c = rng.choice(n, size=L, replace=False)
        rows += [i] * L
        cols += list(c)
        vals += list(rng.standard_normal(L) / math.sqrt(max(L, 1)))
    import scipy.sparse as sp
    A = sp.csr_matrix((vals, (rows, cols)), shape=(len(lens), n))
    x0 = rng.uniform(0, 1, n)
    b = A @ x0
    rt = (rng.random(len(lens)) < 0.5).astype(np.uint8)
    b[rt == 1] -= 0.1
    q = rng.uniform(0.5, 2.0, n)
    qp = qpgen.instances._make("rowlens", sp.diags(q), A, rng.standard_normal(n), b,
                               np.where(rng.random(n) < 0.5, 0.0, -np.inf),
                               np.where(rng.random(n) < 0.3, 2.0, np.inf), rt)
    for panels in ((1, 1), (8, 8)):
        o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=300, panels=panels)
        _assert_parity(orc, qp, o, g)


def test_equality_only_and_singular_q(orc, qpa):
    # rank-5 Q with every variable boxed (bounded, so an optimum exists)
    for seed in range(3):
        qp = qp_refs.random_tiny_qp(200 + seed, n=40, m=15, bounded_frac=1.0, eq_frac=1.0,
                                    psd_rank=5)
        o, g = _pair(orc, qpa, qp, eps=1e-7)
        _assert_parity(orc, qp, o, g)


def test_numerical_error_status(orc, qpa):
    qp = qpgen.tiny_random_qp(1)
    qp.c = qp.c.copy()
    qp.c[3] = np.nan
    o, g = _pair(orc, qpa, qp, norms=(6.0, 24.0))
    assert o[2]["status"] == 3 and g[2]["status"] == 3


def test_device_arrays_path(orc, qpa):
    import torch
    qp = qpgen.tiny_random_qp(1)
    nA, nQ = _norms(orc, qp)
    with qpa.Solver(qp, qpa.Settings(norm_A=nA, norm_Q=nQ), device_arrays=True) as s:
        xg, yg, rg = s.solve()
    assert isinstance(xg, torch.Tensor) and xg.is_cuda
    with qpa.Solver(qp, qpa.Settings(norm_A=nA, norm_Q=nQ)) as s:
        xh, yh, rh = s.solve()
    np.testing.assert_array_equal(xg.cpu().numpy(), xh)
    np.testing.assert_array_equal(yg.cpu().numpy(), yh)


# ---------------------------------------------------------------------------
# the full-size large random QP (n=1e6, m=5e5), in the benchmark's launch
# configuration, at a fixed iteration count
# ---------------------------------------------------------------------------
def test_large_random_full_size(orc, qpa):
    qp = qpgen.large_random_qp()
    nA, _ = orc.norm_A(qp, 40, 1e-7)
    nQ, _ = orc.norm_Q(qp, 40, 1e-7)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=64, norms=(nA, nQ))
    _assert_parity(orc, qp, o, g)


@pytest.fixture
def oracle_threads(orc):
    """The oracle's threaded mode (bitwise the one-thread result) for full-size legs."""
    import os
    orc.set_threads(min(16, os.cpu_count() or 1))
    yield
    orc.set_threads(1)


def test_large_random_full_size_to_tolerance(orc, qpa, oracle_threads):
    """The full-size large random QP solved to relKKT 1e-6 (about 2000 iterations, with
    restarts and primal-weight updates), in the benchmark's launch configuration."""
    qp = qpgen.large_random_qp()
    nA, _ = orc.norm_A(qp, 40, 1e-7)
    nQ, _ = orc.norm_Q(qp, 40, 1e-7)
    o, g = _pair(orc, qpa, qp, eps=1e-6, norms=(nA, nQ))
    _assert_parity(orc, qp, o, g)
    assert o[2]["restarts"] > 3


def test_portfolio_full_size_preconditioned(orc, qpa, oracle_threads):
    """The full factor-model portfolio QP with Sec. 5 preprocessing (the configuration
    the benchmark solves to tolerance), 1024 iterations through several restarts."""
    qp = qpgen.portfolio_qp()
    sc, _, _ = orc.precondition(qp)
    nA, _ = orc.norm_A(sc, 40, 1e-7)
    nQ, _ = orc.norm_Q(sc, 40, 1e-7)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=1024, precondition=True, norms=(nA, nQ))
    _assert_parity(orc, qp, o, g)
    assert o[2]["restarts"] > 3


def test_portfolio_full_size(orc, qpa):
    """The full factor-model portfolio QP (n = 5e5 + 1000, a 5e5-nonzero budget row)."""
    qp = qpgen.portfolio_qp()
    nA, _ = orc.norm_A(qp, 40, 1e-7)
    nQ, _ = orc.norm_Q(qp, 40, 1e-7)
    o, g = _pair(orc, qpa, qp, eps=0.0, max_iter=64, norms=(nA, nQ))
    _assert_parity(orc, qp, o, g)


def test_symmetry_check_accepts_generated_instances(orc, qpa):
    qp = qpgen.tiny_random_qp(1)
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    with qpa.Solver(qp, qpa.Settings(eps=1e-6, norm_A=o[2]["norm_A"], norm_Q=o[2]["norm_Q"],
                                     check_symmetry=1)) as s:
        x, y, r = s.solve()
    assert r["iterations"] == g[2]["iterations"]
    np.testing.assert_array_equal(x, g[0])
    batch = qpgen.concat_batch([qpgen.tiny_random_qp(k) for k in (1, 2)])
    with qpa.BatchSolver(batch, qpa.Settings(eps=1e-6, check_symmetry=1)) as bs:
        _, _, rb = bs.solve()
    assert all(r["status"] == 0 for r in rb)


def _lp_instance(seed=31, n=60, m=30):
    """A bounded LP (Q = 0, no stored entries): min c'x, Ax >= b, 0 <= x <= 10."""
    rng = np.random.default_rng(seed)
    A = np.where(rng.random((m, n)) < 0.2, rng.standard_normal((m, n)), 0.0)
    xf = rng.uniform(0.5, 2.0, n)
    b = A @ xf - rng.uniform(0.0, 1.0, m)
    qp = qp_refs.make_qp(np.zeros((n, n)), A, rng.standard_normal(n), b, np.zeros(n),
                         np.full(n, 10.0), np.ones(m, dtype=int))
    assert qp.q_nnz == 0
    return qp


def test_linear_program_without_q(orc, qpa):
    qp = _lp_instance()
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    _assert_parity(orc, qp, o, g)
    assert g[2]["status"] == 0 and g[2]["norm_Q"] == 0.0


def test_single_variable(orc, qpa):
    # n = 1, m = 1: min 1/2 x^2 - 3x  s.t.  x >= 1, x <= 2  ->  x = 2
    qp = qp_refs.make_qp(np.eye(1), np.ones((1, 1)), [-3.0], [1.0], [-np.inf], [2.0], [1])
    o, g = _pair(orc, qpa, qp, eps=1e-9)
    _assert_parity(orc, qp, o, g)
    assert g[0][0] == pytest.approx(2.0, abs=1e-6)


def test_rows_without_entries(orc, qpa):
    """Constraint rows with no nonzeros (0 >= b_i with b_i <= 0, and 0 = 0): empty row
    blocks read the arrays' pad entry and contribute nothing."""
    qp0 = qpgen.tiny_random_qp(5)
    A = qp0.A().toarray()
    A[::3, :] = 0.0                       # every third row empty
    b = qp0.b.copy()
    empty = ~A.any(axis=1)
    b[empty & (qp0.row_type == 1)] = -1.0
    b[empty & (qp0.row_type == 0)] = 0.0
    Q, _ = qp0.dense()
    qp = qp_refs.make_qp(Q, A, qp0.c, b, qp0.l, qp0.u, qp0.row_type)
    assert (np.diff(qp.a_rowptr) == 0).sum() >= 10
    o, g = _pair(orc, qpa, qp, eps=1e-6)
    _assert_parity(orc, qp, o, g)


@pytest.mark.parametrize("every", [1, 4])
def test_profile_mode_matches_graph_mode(orc, qpa, every):
    """Profiling (direct launches, events around the phases of every k-th iteration,
    two event sets so one interval stays in flight) computes exactly what graph
    replay does, and times the phases of every k-th iteration that ran."""
    qp = qpgen.large_random_qp(seed=2, n=30000, m=15000)
    out = {}
    for prof in (0, every):
        with qpa.Solver(qp, qpa.Settings(eps=1e-6, max_iter=1000, profile=prof)) as s:
            out[prof] = s.solve()
            if prof:
                p = s.profile()
    (x0, y0, r0), (x1, y1, r1) = out[0], out[every]
    assert r1["iterations"] == r0["iterations"] and r1["status"] == r0["status"]
    np.testing.assert_array_equal(x1, x0)
    np.testing.assert_array_equal(y1, y0)
    # within each check interval of 64, iterations 0, k, 2k, ... are timed
    full, rest = divmod(r1["iterations"], 64)
    timed = full * len(range(0, 64, every)) + len(range(0, rest, every))
    assert p["dual_launches"] == timed and p["primal_launches"] == timed
    assert p["dual_ms"] > 0.0 and p["primal_ms"] > 0.0


@pytest.mark.parametrize("panels", [(1, 1), (8, 8)])
def test_long_row_chunks_repeatable(orc, qpa, panels):
    """Rows split into chunks that finish on different XCDs (a 20000-entry budget row,
    and with 8 panels every row of P spread over all XCDs): repeated solves give
    bitwise the same iterates, and match the oracle."""
    qp = qpgen.portfolio_qp(seed=3, n_assets=20000, k=40)
    o, g = _pair(orc, qpa, qp, eps=1e-6, max_iter=3000, panels=panels)
    _assert_parity(orc, qp, o, g)
    nA, nQ = g[2]["norm_A"], g[2]["norm_Q"]
    runs = []
    with qpa.Solver(qp, qpa.Settings(eps=1e-6, max_iter=3000, norm_A=nA, norm_Q=nQ,
                                     panels_dual=panels[0], panels_primal=panels[1])) as s:
        for _ in range(3):
            runs.append(s.solve())
    for x, y, r in runs[1:]:
        assert r["iterations"] == runs[0][2]["iterations"]
        np.testing.assert_array_equal(x, runs[0][0])
        np.testing.assert_array_equal(y, runs[0][1])


_SWEEP_MAKERS = {
    "random": lambda s: qpgen.large_random_qp(seed=s, n=6000, m=3000),
    "eq": lambda s: qpgen.eq_qp(seed=s, n=6000),
    "lasso": lambda s: qpgen.lasso_qp(seed=s, n_features=200, m_samples=2000, density=0.05),
    "huber": lambda s: qpgen.huber_qp(seed=s, n_features=200, m_samples=2000, density=0.05),
    "svm": lambda s: qpgen.svm_qp(seed=s, n_features=200, m_samples=2000, density=0.05),
    "portfolio": lambda s: qpgen.portfolio_qp(seed=s, n_assets=6000, k=30),
    "control": lambda s: qpgen.mpc_qp(np.random.default_rng(s), 150, 8, 3, name="control"),
}
_SWEEP_PANELS = [(4, 4), (2, 8), (8, 2), (4, 1)]


@pytest.mark.parametrize("seed", [3, 4])
@pytest.mark.parametrize("pre", [False, True])
@pytest.mark.parametrize("kind", sorted(_SWEEP_MAKERS))
def test_column_panels_class_sweep(orc, qpa, kind, pre, seed):
    """Every synthetic class on the column-panel kernels (panel partial sums, the KKT
    evaluation's interleaved pairs, the workgroup-built step table), to relKKT 1e-6
    with and without the Sec. 5 preprocessing, against the oracle."""
    panels = _SWEEP_PANELS[(sorted(_SWEEP_MAKERS).index(kind) + 2 * seed + int(pre)) % 4]
    qp = _SWEEP_MAKERS[kind](seed)
    print(f"  {kind} seed={seed} pre={pre} panels={panels} n={qp.n} m={qp.m}", flush=True)
    o, g = _pair(orc, qpa, qp, eps=1e-6, max_iter=40000, panels=panels, precondition=pre)
    _assert_parity(orc, qp, o, g)
