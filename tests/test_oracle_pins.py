"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test cites what it checks.  None of them compares the oracle with itself:
closed-form solutions, brute-force KKT enumeration, hand-computed values,
library routines and the paper's theorems are the references.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

import qpgen
from tests import qp_refs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _inf(v):
    return np.array([float(t) if not isinstance(t, str) else float(t.replace("inf", "inf"))
                     for t in v])


# ---------------------------------------------------------------------------
# SpMV: the definition of a sparse matrix-vector product (library routine)
# ---------------------------------------------------------------------------
def test_spmv_matches_scipy(orc):
    rng = np.random.default_rng(0)
    M = sp.random(300, 200, density=0.05, random_state=rng, format="csr")
    M.sort_indices()
    x = rng.standard_normal(200)
    y = orc.spmv(M.indptr, M.indices, M.data, x)
    np.testing.assert_allclose(y, M @ x, rtol=1e-13, atol=1e-13)
    z = orc.spmv_t(M.indptr, M.indices, M.data, rng.standard_normal(300), 200)
    assert z.shape == (200,)
    xr = rng.standard_normal(300)
    np.testing.assert_allclose(orc.spmv_t(M.indptr, M.indices, M.data, xr, 200), M.T @ xr,
                               rtol=1e-12, atol=1e-12)


# ---------------------------------------------------------------------------
# relKKT: hand-computed values (Sec. 5 definition, generalised)
# ---------------------------------------------------------------------------
def test_rel_kkt_hand_values(orc):
    g = json.load(open(os.path.join(GOLDEN, "relkkt_hand.json")))
    P = g["problem"]
    for case in g["cases"]:
        qp = qp_refs.make_qp(P["Q"], P["A"], case["c"], case.get("b", P["b"]), _inf(case["l"]),
                             _inf(case["u"]), P["row_type"])
        k = orc.rel_kkt(qp, np.array(case.get("x", P["x"])), np.array(case.get("y", P["y"])))
        for key in ("r_primal", "r_dual", "r_gap", "rel_kkt", "primal_obj", "dual_obj"):
            assert k[key] == pytest.approx(case[key], abs=1e-15, rel=1e-14), (case["name"], key)


def test_rel_kkt_reduces_to_paper_form(orc):
    """GE rows only, no bounds: the Sec. 5 formulas for A_p x <= b_p with
    A_p = -A, b_p = -b and the paper's sign of y (L = ... + y'A_p x - b_p'y)."""
    rng = np.random.default_rng(3)
    n, m = 7, 4
    G = rng.standard_normal((n, n))
    Q = G @ G.T
    A = rng.standard_normal((m, n))
    b = rng.standard_normal(m)
    c = rng.standard_normal(n)
    qp = qp_refs.make_qp(Q, A, c, b, np.full(n, -np.inf), np.full(n, np.inf), np.ones(m))
    x = rng.standard_normal(n)
    y = np.abs(rng.standard_normal(m))
    Ap, bp = -A, -b
    inf = lambda v: np.max(np.abs(v))  # noqa: E731
    rp = inf(np.maximum(Ap @ x - bp, 0)) / (1 + max(inf(Ap @ x), inf(bp)))
    rd = inf(Q @ x + Ap.T @ y + c) / (1 + max(inf(Q @ x), inf(Ap.T @ y), inf(c)))
    rg = abs(x @ Q @ x + c @ x + bp @ y) / (1 + max(abs(0.5 * x @ Q @ x + c @ x),
                                                    abs(0.5 * x @ Q @ x + bp @ y)))
    k = orc.rel_kkt(qp, x, y)
    assert k["r_primal"] == pytest.approx(rp, rel=1e-12)
    assert k["r_dual"] == pytest.approx(rd, rel=1e-12)
    assert k["r_gap"] == pytest.approx(rg, rel=1e-12)
    assert k["rel_kkt"] == pytest.approx(max(rp, rd, rg), rel=1e-12)


# ---------------------------------------------------------------------------
# operator norms: power iteration vs dense SVD / eigvalsh
# ---------------------------------------------------------------------------
def test_power_iteration_norms(orc):
    qp = qpgen.tiny_random_qp(1)
    Q, A = qp.dense()
    nA, itA = orc.norm_A(qp, 5000, 1e-12)
    nQ, itQ = orc.norm_Q(qp, 5000, 1e-12)
    assert nA == pytest.approx(np.linalg.norm(A, 2), rel=1e-5)
    assert nQ == pytest.approx(np.max(np.abs(np.linalg.eigvalsh(Q))), rel=1e-5)
    assert nA <= np.linalg.norm(A, 2) * (1 + 1e-12)  # Rayleigh quotient never overshoots
    assert itA > 1 and itQ > 1


# ---------------------------------------------------------------------------
# step sizes (Sec. 6 rule; eq. (param) of Lemma 1; Lemma 2 identity)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nA,nQ,omega", [(6.2, 24.4, 8.5), (1.0, 0.0, 1.0), (3.0, 100.0, 0.01),
                                         (0.5, 2.0, 50.0)])
def test_adaptive_step_conditions(orc, nA, nQ, omega):
    s = orc.OracleSettings()
    K = 400
    p, d, sc = orc.step_schedule(s, nA, nQ, omega, K)
    k = np.arange(K)
    beta = (k + 2) / 2.0
    # primal/dual split of Sec. 6: tau = eta/omega, sigma = eta*omega
    np.testing.assert_allclose(p, sc / omega, rtol=1e-15)
    np.testing.assert_allclose(d, sc * omega, rtol=1e-15)
    # start value 1.98 / (||Q||/w + sqrt(4||A||^2 + ||Q||^2/w^2))
    assert sc[0] == pytest.approx(1.98 / (nQ / omega + math.sqrt(4 * nA**2 + (nQ / omega) ** 2)),
                                  rel=1e-15)
    # growth never faster than (1 + 1/k): theta_k = k/(k+1) <= s_{k-1}/s_k (3rd condition of
    # eq. (param) with theta_k = k/(k+1))
    theta = k[1:] / (k[1:] + 1.0)
    assert np.all(theta <= sc[:-1] / sc[1:] * (1 + 1e-14))
    # step condition used in the proof of Lemma 2: 1/eta - ||Q||/beta - ||A||^2 tau >= 0
    slack = 1.0 / p - nQ / beta - nA**2 * d
    assert np.all(slack >= -1e-9 * (1.0 / p))
    # without the 0.99 safety factor the cap makes the condition tight
    s1 = orc.OracleSettings(step_safety=1.0)
    p1, d1, _ = orc.step_schedule(s1, nA, nQ, omega, 1)
    assert 1.0 / p1[0] - nQ / 1.0 - nA**2 * d1[0] == pytest.approx(0.0, abs=1e-9 / p1[0])


@pytest.mark.parametrize("K", [1, 10, 137])
def test_fixed_k_step_identity(orc, K):
    """Lemma 2 (i): with eq. (param-choice), eq. (param) holds and
    1/eta_k - ||Q||/beta_k - 4||A||^2 tau_k = 2||Q||/((k+1)(k+2)) + 2||A||(K/(k+1) - (k+1)/K)."""
    nA, nQ = 2.5, 7.0
    s = orc.OracleSettings(restart_mode=orc.RESTART_FIXED_K, fixed_K=K)
    p, d, _ = orc.step_schedule(s, nA, nQ, 1.0, K)
    k = np.arange(K)
    beta = (k + 2) / 2.0
    lhs = 1.0 / p - nQ / beta - 4 * nA**2 * d
    rhs = 2 * nQ / ((k + 1) * (k + 2)) + 2 * nA * (K / (k + 1) - (k + 1) / K)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    assert np.all(lhs >= -1e-12)
    if K > 1:
        theta_next = (k[1:]) / (k[1:] + 1.0)
        np.testing.assert_allclose(theta_next, p[:-1] / p[1:], rtol=1e-14)
        np.testing.assert_allclose(theta_next, d[:-1] / d[1:], rtol=1e-14)


# ---------------------------------------------------------------------------
# first iteration from zeros and the averaging identity (Algorithm 1)
# ---------------------------------------------------------------------------
def test_first_iteration_by_hand(orc):
    qp = qpgen.tiny_random_qp(1)
    Q, A = qp.dense()
    nA, nQ, omega = 6.0, 24.0, 2.0
    s = orc.OracleSettings()
    p, d, _ = orc.step_schedule(s, nA, nQ, omega, 1)
    x, y, xb, yb = orc.run_inner(qp, s, nA, nQ, omega, 1)
    # x~ = 0 at k = 0  =>  y1 = proj_Y(d0 * b);  x1 = proj_X(-p0 (c - A'y1))
    y1 = d[0] * qp.b
    y1[qp.row_type == 1] = np.maximum(y1[qp.row_type == 1], 0.0)
    x1 = np.clip(-p[0] * (qp.c - A.T @ y1), qp.l, qp.u)
    np.testing.assert_allclose(y, y1, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(x, x1, rtol=1e-13, atol=1e-15)
    np.testing.assert_array_equal(xb, x)   # 1/beta_0 = 1
    np.testing.assert_array_equal(yb, y)


def test_three_iterations_hand_worked(orc):
    """Exact-fraction hand computation of three accelerated PDHG steps (Algorithm 1 with the
    eq. (param-choice) parameters); pins theta_k, 1/beta_k, both step sizes and the averages."""
    g = json.load(open(os.path.join(GOLDEN, "apdhg_three_steps.json")))
    P = g["problem"]
    qp = qp_refs.make_qp(P["Q"], P["A"], P["c"], P["b"], _inf(P["l"]), _inf(P["u"]),
                         P["row_type"])
    s = orc.OracleSettings(restart_mode=orc.RESTART_FIXED_K, fixed_K=g["K"])
    for it in g["iterates"]:
        x, y, xb, yb = orc.run_inner(qp, s, g["norm_A"], g["norm_Q"], 1.0, it["k"])
        for got, key in ((x, "x"), (y, "y"), (xb, "xbar"), (yb, "ybar")):
            num, den = it[key]
            assert got[0] == pytest.approx(num / den, rel=1e-14), (it["k"], key)


def _golden_qp(P):
    return qp_refs.make_qp(P["Q"], P["A"], P["c"], P["b"], _inf(P["l"]), _inf(P["u"]),
                           P["row_type"])


def _frac(v):
    return v[0] / v[1]


def test_primal_weight_init_and_update_hand_worked(orc):
    """Sec. 6 InitializePrimalWeight and PrimalWeightUpdate pinned by an exact-fraction hand
    computation: omega0 = ||c||/||b||, the first iterate it yields through the step-size rule,
    the tie-broken candidate, restart (iii) at the first evaluation, and
    omega1 = (dy/dx)^theta * omega0^(1 - theta) with theta = 0.2."""
    g = json.load(open(os.path.join(GOLDEN, "primal_weight_first_restart.json")))
    qp = _golden_qp(g["problem"])
    base = dict(eps=0.0, check_every=g["check_every"], norm_A=g["norm_A"], norm_Q=g["norm_Q"])
    # one iteration, stopped at the limit before any restart: the weight is still omega0
    x, y, r, log = orc.solve(qp, orc.OracleSettings(max_iter=1, **base), log_cap=8)
    assert r["status"] == orc.ITERATION_LIMIT and r["restarts"] == 0
    assert r["omega"] == pytest.approx(_frac(g["omega0"]), rel=1e-15)
    assert x[0] == pytest.approx(_frac(g["x1"]), rel=1e-14)
    assert y[0] == pytest.approx(_frac(g["y1"]), rel=1e-14)
    assert r["rel_kkt"] == pytest.approx(_frac(g["rel_kkt_z1"]), rel=1e-13)
    # two iterations: the evaluation after the first restarts and updates the weight
    _, _, r2, log2 = orc.solve(qp, orc.OracleSettings(max_iter=2, **base), log_cap=8)
    e = log2[0]
    fc = g["first_check"]
    assert (e["total"], e["candidate"], e["restarted"]) == (fc["total"], fc["candidate"],
                                                            fc["restarted"])
    assert e["r_cur"] == e["r_avg"] == pytest.approx(_frac(g["rel_kkt_z1"]), rel=1e-13)
    w = g["omega1"]
    th = _frac(w["theta"])
    omega1 = _frac(w["ratio"]) ** th * _frac(w["omega0"]) ** (1.0 - th)
    assert e["omega"] == pytest.approx(omega1, rel=1e-14)
    assert r2["restarts"] >= 1


def test_halving_first_check_hand_worked(orc):
    """Sec. 5 halving rule at the first evaluation, from exact-fraction hand computations:
    one case where relKKT of the average falls below half of relKKT(z0) (restart, to the
    average) and one where it stays above it (no restart)."""
    g = json.load(open(os.path.join(GOLDEN, "halving_first_check.json")))
    for case in g["cases"]:
        qp = _golden_qp(case["problem"])
        s = orc.OracleSettings(eps=0.0, max_iter=2, check_every=1, norm_A=case["norm_A"],
                               norm_Q=case["norm_Q"], restart_mode=orc.RESTART_HALVING)
        _, _, r, log = orc.solve(qp, s, log_cap=8)
        e = log[0]
        assert e["total"] == 1
        assert e["r_avg"] == pytest.approx(_frac(case["rel_kkt_zbar1"]), rel=1e-13)
        assert e["restarted"] == case["restarted"], case["derivation"]
        if case["restarted"]:
            assert e["candidate"] == 1  # the restart point is the average
        if "x1" in case:
            x, y, r1, _ = orc.solve(qp, orc.OracleSettings(
                eps=0.0, max_iter=1, check_every=1, norm_A=case["norm_A"], norm_Q=case["norm_Q"],
                restart_mode=orc.RESTART_HALVING), log_cap=8)
            assert x[0] == pytest.approx(_frac(case["x1"]), rel=1e-14)
            assert y[0] == pytest.approx(_frac(case["y1"]), rel=1e-14)
        r0 = orc.rel_kkt(qp, np.zeros(1), np.zeros(1))["rel_kkt"]
        assert r0 == pytest.approx(_frac(case["rel_kkt_z0"]), rel=1e-15)


def test_halving_log_replay(orc):
    """Over a whole halving-restarted solve, every evaluation restarts exactly when
    relKKT(z-bar) <= relKKT(z^{n,0}) / 2, always to the average, and the next cycle's
    reference is the restart point's relKKT (Sec. 5)."""
    held = 0  # evaluations after a restart that do not restart: they see the new reference
    for seed in (2, 7):
        qp = qpgen.tiny_random_qp(seed)
        s = orc.OracleSettings(eps=1e-8, restart_mode=orc.RESTART_HALVING)
        _, _, r, log = orc.solve(qp, s, log_cap=100000)
        r0 = orc.rel_kkt(qp, np.clip(np.zeros(qp.n), qp.l, qp.u), np.zeros(qp.m))["rel_kkt"]
        nrs = 0
        for e in log[:-1]:
            want = e["r_avg"] <= 0.5 * r0
            assert bool(e["restarted"]) == want, (seed, e, r0)
            if want:
                assert e["candidate"] == 1
                r0 = e["r_avg"]
                nrs += 1
            elif nrs:
                held += 1
        assert nrs >= 3 and r["restarts"] == nrs
        assert r["status"] == orc.OPTIMAL
    assert held >= 2


@pytest.mark.parametrize("mode", ["halving", "none"])
def test_sec5_methods_are_measured_at_the_average(orc, mode):
    """Algorithm 1 outputs the average (its restart points are averages) and Sec. 5 tests
    progress on relKKT(z-bar): under the Sec. 5 restart rules every evaluation's candidate
    is the average, the solve stops at the first evaluation whose average meets eps (not
    earlier when the current iterate does), and the returned relKKT is the average's.  The
    choice of the better of the two belongs to the Sec. 6 rule only."""
    rm = orc.RESTART_HALVING if mode == "halving" else orc.RESTART_NONE
    # (the unrestarted average converges sublinearly: a looser tolerance there)
    eps = 1e-4 if mode == "halving" else 1e-2
    seen_cur_first = 0
    for seed in range(1, 9):
        qp = qpgen.tiny_random_qp(seed)
        s = orc.OracleSettings(eps=eps, restart_mode=rm, momentum=0, max_iter=100000)
        x, y, r, log = orc.solve(qp, s, log_cap=100000)
        assert r["status"] == orc.OPTIMAL
        assert all(e["candidate"] == 1 for e in log)
        assert all(e["r_avg"] > eps for e in log[:-1]) and log[-1]["r_avg"] <= eps
        assert r["rel_kkt"] == log[-1]["r_avg"]
        assert r["rel_kkt"] == pytest.approx(orc.rel_kkt(qp, x, y)["rel_kkt"], rel=1e-12)
        seen_cur_first += any(e["r_cur"] <= eps for e in log[:-1])
    # plain PDHG's current iterate often meets the tolerance long before its average:
    # the rule is exercised
    assert seen_cur_first >= 1


def test_averaging_identity(orc):
    """With 1/beta_k = 2/(k+2): x-bar^K = sum_{i=1..K} 2i/(K(K+1)) x^i."""
    qp = qpgen.tiny_random_qp(2)
    s = orc.OracleSettings()
    nA, nQ, omega = 6.5, 25.0, 1.3
    K = 12
    xs, ys = [], []
    for i in range(1, K + 1):
        x, y, _, _ = orc.run_inner(qp, s, nA, nQ, omega, i)
        xs.append(x); ys.append(y)
    _, _, xb, yb = orc.run_inner(qp, s, nA, nQ, omega, K)
    w = np.array([2.0 * i / (K * (K + 1)) for i in range(1, K + 1)])
    np.testing.assert_allclose(xb, w @ np.array(xs), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(yb, w @ np.array(ys), rtol=1e-12, atol=1e-13)


# ---------------------------------------------------------------------------
# closed-form fixed points (KKT system of Sec. 3, textbook special cases)
# ---------------------------------------------------------------------------
def test_unconstrained_closed_form(orc):
    rng = np.random.default_rng(11)
    n = 40
    G = rng.standard_normal((n, n))
    Q = G @ G.T / n + np.eye(n)
    c = rng.standard_normal(n)
    qp = qp_refs.make_qp(Q, np.zeros((0, n)), c, [], np.full(n, -np.inf), np.full(n, np.inf), [])
    x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-11))
    assert r["status"] == orc.OPTIMAL
    np.testing.assert_allclose(x, np.linalg.solve(Q, -c), rtol=1e-8, atol=1e-9)


def test_equality_only_closed_form(orc):
    rng = np.random.default_rng(12)
    n, m = 30, 12
    G = rng.standard_normal((n, n))
    Q = G @ G.T / n + 0.5 * np.eye(n)
    A = rng.standard_normal((m, n))
    qp = qp_refs.make_qp(Q, A, rng.standard_normal(n), rng.standard_normal(m),
                         np.full(n, -np.inf), np.full(n, np.inf), np.zeros(m))
    xs, ys = qp_refs.equality_kkt_solution(qp)
    x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-11))
    assert r["status"] == orc.OPTIMAL
    np.testing.assert_allclose(x, xs, rtol=1e-7, atol=1e-8)
    np.testing.assert_allclose(y, ys, rtol=1e-7, atol=1e-8)


def test_diagonal_box_closed_form(orc):
    rng = np.random.default_rng(13)
    n = 50
    q = rng.uniform(0.5, 4.0, n)
    c = 3 * rng.standard_normal(n)
    l = np.where(rng.random(n) < 0.7, -1.0, -np.inf)
    u = np.where(rng.random(n) < 0.7, 1.0, np.inf)
    # no constraint rows: m = 0
    qp = qp_refs.make_qp(np.diag(q), np.zeros((0, n)), c, [], l, u, [])
    x, _, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-12))
    assert r["status"] == orc.OPTIMAL
    np.testing.assert_allclose(x, qp_refs.diag_box_solution(q, c, l, u), rtol=1e-9, atol=1e-10)


def test_diagonal_budget_water_filling(orc):
    rng = np.random.default_rng(14)
    n = 60
    q = rng.uniform(0.2, 3.0, n)
    c = rng.standard_normal(n)
    budget = 1.7
    qp = qp_refs.make_qp(np.diag(q), np.ones((1, n)), c, [budget], np.zeros(n),
                         np.full(n, np.inf), [0])
    xs, nu = qp_refs.diag_budget_solution(q, c, budget)
    x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-11))
    assert r["status"] == orc.OPTIMAL
    np.testing.assert_allclose(x, xs, rtol=1e-7, atol=1e-8)
    # the budget row's multiplier is the water level nu (stationarity: q x + c - nu = 0 on
    # the support)
    assert y[0] == pytest.approx(nu, rel=1e-7)


# ---------------------------------------------------------------------------
# brute-force active-set enumeration on tiny general QPs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(12))
def test_bruteforce_tiny(orc, seed):
    qp = qp_refs.random_tiny_qp(seed, n=5, m=3)
    best = qp_refs.brute_force_kkt(qp)
    assert best is not None
    f_star, x_star, _ = best
    x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-10, max_iter=400000))
    assert r["status"] == orc.OPTIMAL, r
    assert r["primal_obj"] == pytest.approx(f_star, rel=1e-7, abs=1e-7)
    np.testing.assert_allclose(x, x_star, rtol=1e-5, atol=1e-6)  # Q positive definite


@pytest.mark.parametrize("seed", range(4))
def test_bruteforce_tiny_psd_singular(orc, seed):
    """Q rank-deficient (LP-like directions): the objective is still unique."""
    qp = qp_refs.random_tiny_qp(100 + seed, n=5, m=3, bounded_frac=1.0, psd_rank=2)
    best = qp_refs.brute_force_kkt(qp)
    assert best is not None
    x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-10, max_iter=400000))
    assert r["status"] == orc.OPTIMAL, r
    assert r["primal_obj"] == pytest.approx(best[0], rel=1e-7, abs=1e-7)


# ---------------------------------------------------------------------------
# the tiny random config: the identified active set solves the KKT system
# ---------------------------------------------------------------------------
def test_tiny_config_active_set_kkt(orc):
    qp = qpgen.tiny_random_qp(1)
    Q, A = qp.dense()
    x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-11, max_iter=400000))
    assert r["status"] == orc.OPTIMAL
    n, m = qp.n, qp.m
    tol = 1e-6
    active = [i for i in range(m) if qp.row_type[i] == 0 or y[i] > tol]
    at_lo = [j for j in range(n) if np.isfinite(qp.l[j]) and x[j] - qp.l[j] < tol]
    at_hi = [j for j in range(n) if np.isfinite(qp.u[j]) and qp.u[j] - x[j] < tol]
    fixed = set(at_lo) | set(at_hi)
    na = len(active)
    M = np.zeros((n + na, n + na))
    rhs = np.zeros(n + na)
    for j in range(n):
        if j in fixed:
            M[j, j] = 1.0
            rhs[j] = qp.l[j] if j in at_lo else qp.u[j]
        else:
            M[j, :n] = Q[j]
            M[j, n:] = -A[active, j]
            rhs[j] = -qp.c[j]
    for t, i in enumerate(active):
        M[n + t, :n] = A[i]
        rhs[n + t] = qp.b[i]
    sol = np.linalg.solve(M, rhs)
    xs = sol[:n]
    ys = np.zeros(m)
    ys[active] = sol[n:]
    lam = Q @ xs + qp.c - A.T @ ys
    # the polished point satisfies every KKT condition exactly (up to rounding)
    assert np.all(A[qp.row_type == 1] @ xs >= qp.b[qp.row_type == 1] - 1e-9)
    assert np.all(ys[qp.row_type == 1] >= -1e-9)
    assert np.all(xs >= qp.l - 1e-9) and np.all(xs <= qp.u + 1e-9)
    assert np.all(lam[at_lo] >= -1e-9) and np.all(lam[at_hi] <= 1e-9)
    np.testing.assert_allclose(x, xs, rtol=1e-7, atol=1e-8)
    assert r["primal_obj"] == pytest.approx(qp_refs.objective(qp, xs), rel=1e-9)


# ---------------------------------------------------------------------------
# zero duality gap (strong duality of eq. (minimax)) as the tolerance shrinks
# ---------------------------------------------------------------------------
def test_gap_closes_with_tolerance(orc):
    qp = qpgen.tiny_random_qp(1)
    gaps = []
    for eps in (1e-4, 1e-6, 1e-8, 1e-10):
        _, _, r, _ = orc.solve(qp, orc.OracleSettings(eps=eps, max_iter=400000))
        assert r["status"] == orc.OPTIMAL
        assert r["r_gap"] <= eps and r["rel_kkt"] <= eps
        gaps.append(abs(r["primal_obj"] - r["dual_obj"]))
    assert gaps[-1] < 1e-7 * (1 + abs(r["primal_obj"]))
    assert gaps[-1] <= gaps[0]


# ---------------------------------------------------------------------------
# Lemma 2 (fixed-K accelerated PDHG, no bounds, GE rows: the paper's setting)
# ---------------------------------------------------------------------------
def _lagrangian(Q, A, c, b, x, y):
    return 0.5 * x @ Q @ x + c @ x - y @ (A @ x - b)


@pytest.mark.parametrize("K", [5, 40, 300])
def test_lemma2_gap_bound(orc, K):
    rng = np.random.default_rng(21)
    n, m = 8, 5
    G = rng.standard_normal((n, n))
    Q = G @ G.T / n
    A = rng.standard_normal((m, n))
    b = A @ rng.standard_normal(n) - rng.uniform(0, 1, m)
    c = rng.standard_normal(n)
    qp = qp_refs.make_qp(Q, A, c, b, np.full(n, -np.inf), np.full(n, np.inf), np.ones(m))
    nA = np.linalg.norm(A, 2)
    nQ = np.max(np.linalg.eigvalsh(Q))
    s = orc.OracleSettings(restart_mode=orc.RESTART_FIXED_K, fixed_K=K)
    z0x = rng.standard_normal(n)
    z0y = np.abs(rng.standard_normal(m))
    _, _, xb, yb = orc.run_inner(qp, s, nA, nQ, 1.0, K, z0x, z0y)
    coef = 8 * (nQ / K**2 + nA / K)
    for t in range(20):
        xh = 3 * rng.standard_normal(n)
        yh = 3 * np.abs(rng.standard_normal(m))
        gap = _lagrangian(Q, A, c, b, xb, yh) - _lagrangian(Q, A, c, b, xh, yb)
        dist2 = np.sum((z0x - xh) ** 2) + np.sum((z0y - yh) ** 2)
        assert gap <= coef * dist2 + 1e-10, (t, gap, coef * dist2)


def test_lemma2_bounded_iterates(orc):
    """Lemma 2 (iii): 1/4 ||z^k - z*||^2 <= ||z^0 - z*||^2 for k < K when K >= ||Q||/||A||."""
    qp = qp_refs.random_tiny_qp(7, n=5, m=3, bounded_frac=0.0, eq_frac=0.0)
    best = qp_refs.brute_force_kkt(qp)
    _, xs, ys = best
    Q, A = qp.dense()
    nA = np.linalg.norm(A, 2)
    nQ = np.max(np.linalg.eigvalsh(Q))
    K = max(60, int(math.ceil(nQ / nA)))
    s = orc.OracleSettings(restart_mode=orc.RESTART_FIXED_K, fixed_K=K)
    d0 = np.sum(xs**2) + np.sum(ys**2)
    for k in range(1, K):
        x, y, _, _ = orc.run_inner(qp, s, nA, nQ, 1.0, k)
        assert 0.25 * (np.sum((x - xs) ** 2) + np.sum((y - ys) ** 2)) <= d0 * (1 + 1e-12)


# ---------------------------------------------------------------------------
# Theorem 1 on the Theorem 3 worst-case instances (alpha_xi in closed form)
# ---------------------------------------------------------------------------
def _restarted_fixed_k(orc, qp, nA, nQ, K, n_outer, dist_fn):
    s = orc.OracleSettings(restart_mode=orc.RESTART_FIXED_K, fixed_K=K)
    x = np.zeros(qp.n)
    y = np.zeros(qp.m)
    z0 = np.concatenate([x, y])
    out = [(dist_fn(x, y), 0.0)]
    for _ in range(n_outer):
        _, _, x, y = orc.run_inner(qp, s, nA, nQ, 1.0, K, x, y)   # restart at the average
        out.append((dist_fn(x, y), np.linalg.norm(np.concatenate([x, y]) - z0)))
    return out


def test_theorem1_strongly_convex_instance(orc):
    """Thm 3 (ii) instance: Q = diag(H, 0), c = (h, 0), A = diag(0, sqrt(||Q|| mu)) with free
    duals; alpha_xi = min(mu^2/(2 xi), mu/2).  Thm 1: dist(z^{n,0}) <= e^{-n} dist_0 and
    ||z^{n,0} - z^{0,0}|| <= 3/(1-1/e) dist_0 once K meets its lower bound."""
    H = np.array([1.0, 1.7, 2.6, 4.0])
    mu, L = H.min(), H.max()
    h = np.array([1.0, -2.0, 0.5, 3.0])
    n = H.size + 1
    Q = np.diag(np.concatenate([H, [0.0]]))
    A = np.zeros((n, n))
    A[-1, -1] = math.sqrt(L * mu)
    qp = qp_refs.make_qp(Q, A, np.concatenate([h, [0.0]]), np.zeros(n), np.full(n, -np.inf),
                         np.full(n, np.inf), np.zeros(n))
    nQ, nA = L, math.sqrt(L * mu)
    xi = 1.0
    alpha = min(mu**2 / (2 * xi), mu / 2)
    e2 = math.e ** 2
    K = int(math.ceil(max(math.sqrt(32 * e2 * nQ / alpha), 32 * e2 * nA / alpha,
                          math.sqrt(64 * nQ / xi), 64 * nA / xi, nQ / nA)))
    x_star = np.concatenate([-h / H, [0.0]])

    def dist(x, y):  # Y* = R^{n-1} x {0}
        return math.sqrt(np.sum((x - x_star) ** 2) + y[-1] ** 2)

    traj = _restarted_fixed_k(orc, qp, nA, nQ, K, 4, dist)
    d0 = traj[0][0]
    for t, (d, moved) in enumerate(traj):
        assert d <= math.exp(-t) * d0 * (1 + 1e-12), (t, d, d0)
        assert moved <= 3 / (1 - 1 / math.e) * d0


def test_theorem1_bilinear_instance(orc):
    """Thm 3 (i) instance: L = y'A x + b'y with A = H^{1/2}; alpha_xi = sigma_min(A)^2/(2 xi)."""
    rng = np.random.default_rng(5)
    n = 4
    U, _ = np.linalg.qr(rng.standard_normal((n, n)))
    sig = np.array([0.6, 0.8, 1.1, 1.5])
    Ah = U @ np.diag(sig) @ U.T            # symmetric square root of H = U diag(sig^2) U'
    bp = rng.standard_normal(n)
    # our form: -y'(A_o x - b_o) = y'(Ah x + bp)  =>  A_o = -Ah, b_o = bp
    qp = qp_refs.make_qp(np.zeros((n, n)), -Ah, np.zeros(n), bp, np.full(n, -np.inf),
                         np.full(n, np.inf), np.zeros(n))
    x_star = np.linalg.solve(-Ah, bp)
    nA = sig.max()
    xi = sig.min()
    alpha = sig.min() ** 2 / (2 * xi)
    e2 = math.e ** 2
    K = int(math.ceil(max(32 * e2 * nA / alpha, 64 * nA / xi)))

    def dist(x, y):
        return math.sqrt(np.sum((x - x_star) ** 2) + np.sum(y**2))

    traj = _restarted_fixed_k(orc, qp, nA, 0.0, K, 3, dist)
    d0 = traj[0][0]
    for t, (d, moved) in enumerate(traj):
        assert d <= math.exp(-t) * d0 * (1 + 1e-12), (t, d, d0)
        assert moved <= 3 / (1 - 1 / math.e) * d0


# ---------------------------------------------------------------------------
# restart / termination bookkeeping (Sec. 6 rules (i)-(iii), Sec. 5 halving)
# ---------------------------------------------------------------------------
def test_restart_log_follows_rules(orc):
    qp = qpgen.tiny_random_qp(1)
    s = orc.OracleSettings(eps=1e-8)
    _, _, r, log = orc.solve(qp, s, log_cap=100000)
    r0 = orc.rel_kkt(qp, np.clip(np.zeros(qp.n), qp.l, qp.u), np.zeros(qp.m))["rel_kkt"]
    prev = math.inf
    k = 0
    last_total = 0
    for e in log[:-1]:
        k += e["total"] - last_total
        last_total = e["total"]
        rc = e["r_cur"] if e["r_cur"] < e["r_avg"] else e["r_avg"]
        assert e["candidate"] == (0 if e["r_cur"] < e["r_avg"] else 1)
        want = (rc <= 0.2 * r0) or (rc <= 0.8 * r0 and rc > prev) or (k >= 0.36 * e["total"])
        assert bool(e["restarted"]) == want, e
        if want:
            r0, prev, k = rc, math.inf, 0
        else:
            prev = rc
    assert r["status"] == orc.OPTIMAL
    assert r["restarts"] == sum(e["restarted"] for e in log)
    assert r["iterations"] == log[-1]["total"]


@pytest.mark.parametrize("mode", ["halving", "fixed", "none"])
def test_other_restart_modes_make_progress(orc, mode):
    qp = qpgen.tiny_random_qp(1)
    if mode == "halving":
        s = orc.OracleSettings(restart_mode=orc.RESTART_HALVING, eps=1e-6)
    elif mode == "fixed":
        s = orc.OracleSettings(restart_mode=orc.RESTART_FIXED_K, fixed_K=100, eps=1e-6)
    else:
        s = orc.OracleSettings(restart_mode=orc.RESTART_NONE, eps=1e-4, max_iter=20000)
    x, y, r, log = orc.solve(qp, s, log_cap=10000)
    r_init = orc.rel_kkt(qp, np.clip(np.zeros(qp.n), qp.l, qp.u), np.zeros(qp.m))["rel_kkt"]
    assert r["rel_kkt"] < 1e-2 * r_init
    if mode == "fixed":
        assert all(e["restarted"] == 1 for e in log[:-1])
        assert all(e["total"] % 100 == 0 for e in log)
    if mode == "halving":
        assert r["status"] == orc.OPTIMAL


def test_warm_start_at_solution_and_fallback(orc):
    qp = qpgen.tiny_random_qp(1)
    x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-9))
    x2, y2, r2, _ = orc.solve(qp, orc.OracleSettings(eps=1e-8), x0=x, y0=y)
    assert r2["status"] == orc.OPTIMAL and r2["iterations"] == 0 and r2["used_warm_start"] == 1
    bad = np.full(qp.n, 1e6)
    _, _, r3, _ = orc.solve(qp, orc.OracleSettings(eps=1e-6), x0=bad, y0=np.zeros(qp.m))
    assert r3["used_warm_start"] == 0
    _, _, r4, _ = orc.solve(qp, orc.OracleSettings(eps=1e-6))
    assert r3["iterations"] == r4["iterations"]


def test_iteration_limit_and_numerical_error(orc):
    qp = qpgen.tiny_random_qp(1)
    _, _, r, log = orc.solve(qp, orc.OracleSettings(eps=1e-12, max_iter=100), log_cap=10)
    assert r["status"] == orc.ITERATION_LIMIT and r["iterations"] == 100
    assert [e["total"] for e in log] == [64, 100]
    bad = qpgen.tiny_random_qp(1)
    bad.c = bad.c.copy()
    bad.c[3] = np.nan
    _, _, r2, _ = orc.solve(bad, orc.OracleSettings(norm_A=6.0, norm_Q=24.0))
    assert r2["status"] == orc.NUMERICAL_ERROR


# ---------------------------------------------------------------------------
# Sec. 5 baselines: PDHG without momentum (beta = theta = 1), with and without restart
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("nA,nQ,omega", [(6.2, 24.4, 8.5), (1.0, 0.0, 1.0), (3.0, 100.0, 0.01)])
def test_pdhg_constant_step_condition(orc, nA, nQ, omega):
    """Plain PDHG: the step condition of Lemma 2 with beta = 1 (1/eta - ||Q|| - ||A||^2 tau >= 0)
    holds with equality without the 0.99 factor, and the step is the same at every k."""
    s = orc.OracleSettings(momentum=0)
    p, d, sc = orc.step_schedule(s, nA, nQ, omega, 50)
    assert np.all(p == p[0]) and np.all(d == d[0])
    np.testing.assert_allclose(p, sc / omega, rtol=1e-15)
    np.testing.assert_allclose(d, sc * omega, rtol=1e-15)
    assert 1.0 / p[0] - nQ - nA**2 * d[0] > 0.0
    p1, d1, _ = orc.step_schedule(orc.OracleSettings(momentum=0, step_safety=1.0), nA, nQ, omega, 1)
    assert 1.0 / p1[0] - nQ - nA**2 * d1[0] == pytest.approx(0.0, abs=1e-9 / p1[0])
    # the fixed-K restart mode does not switch plain PDHG to the Theorem 1 schedule
    pk, dk, _ = orc.step_schedule(orc.OracleSettings(momentum=0, restart_mode=orc.RESTART_FIXED_K,
                                                     fixed_K=10), nA, nQ, omega, 10)
    np.testing.assert_array_equal(pk, p[:10])
    np.testing.assert_array_equal(dk, d[:10])


def test_pdhg_uniform_average(orc):
    """Without momentum z-bar is the plain mean of the cycle's iterates z^1..z^K."""
    qp = qpgen.tiny_random_qp(2)
    s = orc.OracleSettings(momentum=0)
    nA, nQ, omega = 6.5, 25.0, 1.3
    K = 12
    xs, ys = [], []
    for i in range(1, K + 1):
        x, y, _, _ = orc.run_inner(qp, s, nA, nQ, omega, i)
        xs.append(x); ys.append(y)
    _, _, xb, yb = orc.run_inner(qp, s, nA, nQ, omega, K)
    np.testing.assert_allclose(xb, np.mean(xs, axis=0), rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(yb, np.mean(ys, axis=0), rtol=1e-12, atol=1e-13)


def test_pdhg_without_rows_is_projected_gradient(orc):
    """m = 0: PDHG without momentum is projected gradient descent x+ = clip(x - eta (Qx + c))
    with the constant step; the accelerated variant is not (it evaluates Q at x_md)."""
    rng = np.random.default_rng(21)
    n = 9
    G = rng.standard_normal((n, n))
    Q = G @ G.T / n + np.eye(n)
    c = rng.standard_normal(n)
    l, u = np.full(n, -0.3), np.full(n, 0.4)
    qp = qp_refs.make_qp(Q, np.zeros((0, n)), c, [], l, u, [])
    nQ = float(np.linalg.eigvalsh(Q).max())
    s = orc.OracleSettings(momentum=0)
    p, _, _ = orc.step_schedule(s, 0.0, nQ, 1.0, 1)
    x = np.zeros(n)
    for _ in range(25):
        x = np.clip(x - p[0] * (Q @ x + c), l, u)
    xg, _, _, _ = orc.run_inner(qp, s, 0.0, nQ, 1.0, 25)
    np.testing.assert_allclose(xg, x, rtol=1e-12, atol=1e-14)
    xa, _, _, _ = orc.run_inner(qp, orc.OracleSettings(), 0.0, nQ, 1.0, 25)
    assert np.max(np.abs(xa - x)) > 1e-6


def test_pdhg_second_iteration_by_hand(orc):
    """theta = 1 and beta = 1: the second dual step extrapolates to 2 x^1 - x^0 and the
    second primal step applies Q at x^1 itself."""
    qp = qpgen.tiny_random_qp(1)
    Q, A = qp.dense()
    nA, nQ, omega = 6.0, 24.0, 2.0
    s = orc.OracleSettings(momentum=0)
    p, d, _ = orc.step_schedule(s, nA, nQ, omega, 2)
    x1, y1, _, _ = orc.run_inner(qp, s, nA, nQ, omega, 1)
    ge = qp.row_type == 1
    y2 = y1 - d[1] * (A @ (2.0 * x1) - qp.b)
    y2[ge] = np.maximum(y2[ge], 0.0)
    x2 = np.clip(x1 - p[1] * (Q @ x1 + qp.c - A.T @ y2), qp.l, qp.u)
    x, y, xb, yb = orc.run_inner(qp, s, nA, nQ, omega, 2)
    np.testing.assert_allclose(y, y2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(x, x2, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(xb, 0.5 * (x1 + x2), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_restarted_pdhg_reaches_bruteforce_kkt(orc, seed):
    qp = qp_refs.random_tiny_qp(seed, n=5, m=3)
    best = qp_refs.brute_force_kkt(qp)
    assert best is not None
    f_star, x_star, _ = best
    for mode in (orc.RESTART_ADAPTIVE, orc.RESTART_HALVING):
        x, y, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-10, max_iter=400000, momentum=0,
                                                      restart_mode=mode))
        assert r["status"] == orc.OPTIMAL, r
        assert r["primal_obj"] == pytest.approx(f_star, rel=1e-7, abs=1e-7)
        np.testing.assert_allclose(x, x_star, rtol=1e-5, atol=1e-6)


def test_momentum_and_restart_cut_iterations(orc):
    """Sec. 5's ablation on the tiny random class: under the same restart rule the
    accelerated method needs fewer iterations than plain PDHG (shifted geometric mean,
    shift 10, as in the paper's tables), and restarts help plain PDHG too."""
    def sgm(v):
        return math.exp(np.mean(np.log(np.asarray(v, float) + 10.0))) - 10.0
    its = {}
    for name, mom, mode in (("rAPDHG", 1, orc.RESTART_ADAPTIVE),
                            ("rPDHG", 0, orc.RESTART_ADAPTIVE),
                            ("rAPDHG-halving", 1, orc.RESTART_HALVING),
                            ("rPDHG-halving", 0, orc.RESTART_HALVING),
                            ("PDHG", 0, orc.RESTART_NONE)):
        its[name] = sgm([orc.solve(qpgen.tiny_random_qp(seed),
                                   orc.OracleSettings(eps=1e-6, max_iter=50000, momentum=mom,
                                                      restart_mode=mode))[2]["iterations"]
                         for seed in range(1, 9)])
    assert its["rAPDHG"] < its["rPDHG"] < its["PDHG"]
    assert its["rAPDHG-halving"] < its["rPDHG-halving"] < its["PDHG"]


# ---------------------------------------------------------------------------
# Sec. 4 smoothed duality gap (Fercoq's definition as the paper states it) in the
# paper's form min 1/2 x'Qx + c'x s.t. A_p x <= b_p, Z = R^n x R^m_+.  The closed form
# eq. (gap-explicit) and the split of lem. (pd=p-d) are checked against a generic
# numerical maximisation of the definition; the gap is zero exactly at a saddle point,
# which the oracle's solution must be.
# ---------------------------------------------------------------------------
def _paper_form(qp):
    """GE rows A x >= b are the paper's rows with A_p = -A, b_p = -b (same y >= 0)."""
    Q, A = qp.dense()
    return Q, -A, qp.c, -qp.b


def _gap_by_maximisation(Q, Ap, c, bp, x, y, xs, ys, xi):
    """max over (xh, yh >= 0) of L(x,yh) - L(xh,y) - xi/2 ||(xh,yh) - (xs,ys)||^2 with
    L(x,y) = 1/2 x'Qx + c'x + y'(A_p x - b_p), by bounded quasi-Newton iterations."""
    from scipy.optimize import minimize
    n, m = x.size, y.size
    Lx = lambda xx, yy: 0.5 * xx @ Q @ xx + c @ xx + yy @ (Ap @ xx - bp)  # noqa: E731

    def f(z):
        xh, yh = z[:n], z[n:]
        val = Lx(x, yh) - Lx(xh, y) - 0.5 * xi * (np.sum((xh - xs) ** 2) + np.sum((yh - ys) ** 2))
        gx = -(Q @ xh + c + Ap.T @ y) - xi * (xh - xs)
        gy = (Ap @ x - bp) - xi * (yh - ys)
        return -val, -np.concatenate([gx, gy])

    z0 = np.concatenate([xs, np.maximum(ys, 0.0)])
    r = minimize(f, z0, jac=True, method="L-BFGS-B",
                 bounds=[(None, None)] * n + [(0.0, None)] * m,
                 options={"ftol": 1e-16, "gtol": 1e-13, "maxiter": 20000})
    return -r.fun


def _gap_closed_form(Q, Ap, c, bp, x, y, xs, ys, xi):
    """eq. (gap-explicit), y >= 0 (the indicator term is zero)."""
    Minv = np.linalg.inv(np.eye(Q.shape[0]) + Q / xi)
    v = xs - (c + Ap.T @ y) / xi
    w = np.maximum(ys + (Ap @ x - bp) / xi, 0.0)
    return (0.5 * x @ Q @ x + c @ x + bp @ y + 0.5 * xi * (w @ w) - 0.5 * xi * (ys @ ys)
            + 0.5 * xi * (v @ Minv @ v) - 0.5 * xi * (xs @ xs))


def _gap_primal_part(Q, Ap, c, bp, x, xs, ys, xi):
    """lem. (pd=p-d) (ii): the gap at (x, y*)."""
    r = Ap @ x - bp
    w = np.maximum(ys + r / xi, 0.0)
    d = x - xs
    return 0.5 * xi * (w @ w) - 0.5 * xi * (ys @ ys) - ys @ r + 0.5 * d @ Q @ d


def _gap_dual_part(Q, Ap, c, bp, y, xs, xi):
    """lem. (pd=p-d) (iii): the gap at (x*, y), y >= 0."""
    Minv = np.linalg.inv(np.eye(Q.shape[0]) + Q / xi)
    g = Q @ xs + c + Ap.T @ y
    return g @ Minv @ g / (2 * xi) + y @ (bp - Ap @ xs)


@pytest.mark.parametrize("seed", [3, 11])
def test_smoothed_gap_closed_form_split_and_oracle_saddle(orc, seed):
    qp = qp_refs.random_tiny_qp(seed, n=6, m=4, bounded_frac=0.0, eq_frac=0.0)
    Q, Ap, c, bp = _paper_form(qp)
    _, xs, ys = qp_refs.brute_force_kkt(qp)
    rng = np.random.default_rng(seed)
    for xi in (0.5, 2.0, 10.0):
        for _ in range(3):
            x = xs + rng.standard_normal(6)
            y = np.abs(ys + rng.standard_normal(4))
            g_max = _gap_by_maximisation(Q, Ap, c, bp, x, y, xs, ys, xi)
            g_cf = _gap_closed_form(Q, Ap, c, bp, x, y, xs, ys, xi)
            assert g_cf == pytest.approx(g_max, rel=1e-8, abs=1e-9)
            gp = _gap_primal_part(Q, Ap, c, bp, x, xs, ys, xi)
            gd = _gap_dual_part(Q, Ap, c, bp, y, xs, xi)
            assert gp == pytest.approx(_gap_by_maximisation(Q, Ap, c, bp, x, ys, xs, ys, xi),
                                       rel=1e-8, abs=1e-9)
            assert gd == pytest.approx(_gap_by_maximisation(Q, Ap, c, bp, xs, y, xs, ys, xi),
                                       rel=1e-8, abs=1e-9)
            assert gp + gd == pytest.approx(g_cf, rel=1e-10, abs=1e-10)
            assert g_cf > 1e-6  # a point off the saddle has a positive gap
    # the oracle's solution is a saddle point: its smoothed gap centred at itself vanishes
    xo, yo, r, _ = orc.solve(qp, orc.OracleSettings(eps=1e-12, max_iter=400000))
    assert r["status"] == orc.OPTIMAL
    yo = yo[:qp.m]
    for xi in (0.5, 2.0):
        assert abs(_gap_closed_form(Q, Ap, c, bp, xo, yo, xo, yo, xi)) < 1e-9
        assert _gap_by_maximisation(Q, Ap, c, bp, xo, yo, xo, yo, xi) < 1e-9
    # ... and a shifted dual (not a saddle point) does not
    assert _gap_closed_form(Q, Ap, c, bp, xo, yo + 0.1, xo, yo + 0.1, 2.0) > 1e-4
