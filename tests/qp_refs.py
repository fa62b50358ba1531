"""Independent test-side references used to pin the oracle.

Nothing here runs rAPDHG: these are closed forms, brute-force enumeration of
KKT systems and textbook solvers, built only on numpy linear algebra.  The KKT
conditions used are those of the paper's Sec. 3 (eq. (KKT)), generalised to
equality rows and bounds.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

import qpgen


def make_qp(Q, A, c, b, l, u, row_type, name="handmade"):
    Q = np.asarray(Q, dtype=float)
    A = np.asarray(A, dtype=float).reshape(-1, Q.shape[0])
    return qpgen.instances._make(name, sp.csr_matrix(Q), sp.csr_matrix(A), np.asarray(c, float),
                                 np.asarray(b, float), np.asarray(l, float),
                                 np.asarray(u, float), np.asarray(row_type, np.uint8))


def objective(qp, x):
    Q = qp.Q()
    return 0.5 * x @ (Q @ x) + qp.c @ x


def brute_force_kkt(qp, tol=1e-9):
    """Enumerate every active set of a tiny QP and return the objective value and
    a primal-dual pair satisfying all KKT conditions.

    Active set: EQ rows always active; each GE row active (A_i x = b_i) or
    inactive (y_i = 0); each variable at a finite lower bound, at a finite upper
    bound, or free (stationarity component zero).
    """
    Q, A = qp.dense()
    n, m = qp.n, qp.m
    c, b, l, u = qp.c, qp.b, qp.l, qp.u
    ge = [i for i in range(m) if qp.row_type[i] == 1]
    var_opts = []
    for j in range(n):
        o = ["free"]
        if np.isfinite(l[j]):
            o.append("lo")
        if np.isfinite(u[j]):
            o.append("hi")
        var_opts.append(o)
    best = None
    for row_act in itertools.product([True, False], repeat=len(ge)):
        active = [i for i in range(m) if qp.row_type[i] == 0]
        active += [ge[t] for t, a in enumerate(row_act) if a]
        active.sort()
        for vs in itertools.product(*var_opts):
            na = len(active)
            # unknowns: x (n), y_active (na)
            M = np.zeros((n + na, n + na))
            r = np.zeros(n + na)
            for j in range(n):
                if vs[j] == "free":
                    M[j, :n] = Q[j]
                    M[j, n:] = -A[active, j]
                    r[j] = -c[j]
                else:
                    M[j, j] = 1.0
                    r[j] = l[j] if vs[j] == "lo" else u[j]
            for t, i in enumerate(active):
                M[n + t, :n] = A[i]
                r[n + t] = b[i]
            try:
                sol, *_ = np.linalg.lstsq(M, r, rcond=None)
            except np.linalg.LinAlgError:
                continue
            if np.linalg.norm(M @ sol - r) > 1e-8 * (1 + np.linalg.norm(r)):
                continue
            x = sol[:n]
            y = np.zeros(m)
            y[active] = sol[n:]
            ax = A @ x
            lam = Q @ x + c - A.T @ y
            ok = True
            for i in range(m):
                if qp.row_type[i] == 0:
                    ok &= abs(ax[i] - b[i]) <= tol * (1 + abs(b[i]))
                else:
                    ok &= ax[i] >= b[i] - tol * (1 + abs(b[i]))
                    ok &= y[i] >= -tol
            for j in range(n):
                ok &= l[j] - tol <= x[j] <= u[j] + tol
                if vs[j] == "free":
                    ok &= abs(lam[j]) <= 1e-7 * (1 + np.abs(c).max())
                elif vs[j] == "lo":
                    ok &= lam[j] >= -tol * 10
                else:
                    ok &= lam[j] <= tol * 10
            if not ok:
                continue
            f = objective(qp, x)
            if best is None or f < best[0]:
                best = (f, x, y)
    return best


def unconstrained_solution(qp):
    Q, _ = qp.dense()
    return np.linalg.solve(Q, -qp.c)


def equality_kkt_solution(qp):
    """Q x + c - A'y = 0, A x = b (all rows EQ, no bounds)."""
    Q, A = qp.dense()
    n, m = qp.n, qp.m
    K = np.block([[Q, -A.T], [A, np.zeros((m, m))]])
    sol = np.linalg.solve(K, np.concatenate([-qp.c, qp.b]))
    return sol[:n], sol[n:]


def diag_box_solution(qdiag, c, l, u):
    return np.clip(-c / qdiag, l, u)


def diag_budget_solution(qdiag, c, budget, iters=200):
    """min 1/2 sum q_j x_j^2 + c'x s.t. sum x = budget, x >= 0 (q > 0).
    x_j(nu) = max(0, (nu - c_j)/q_j); bisection on nu for sum x = budget."""
    lo = np.min(c) - 1.0
    hi = np.max(c) + budget * np.max(qdiag) + 1.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        s = np.maximum(0.0, (mid - c) / qdiag).sum()
        if s > budget:
            hi = mid
        else:
            lo = mid
    nu = 0.5 * (lo + hi)
    return np.maximum(0.0, (nu - c) / qdiag), nu


def random_tiny_qp(seed, n=5, m=3, bounded_frac=0.5, eq_frac=0.34, psd_rank=None):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, psd_rank or n))
    Q = G @ G.T / n + (0.1 if psd_rank is None else 0.0) * np.eye(n)
    A = rng.standard_normal((m, n))
    x0 = rng.uniform(-1, 1, n)
    b = A @ x0
    row_type = (rng.random(m) > eq_frac).astype(np.uint8)
    b[row_type == 1] -= rng.uniform(0, 1, int((row_type == 1).sum()))
    l = np.full(n, -np.inf)
    u = np.full(n, np.inf)
    for j in range(n):
        if rng.random() < bounded_frac:
            l[j] = x0[j] - rng.uniform(0.1, 1.5)
            u[j] = x0[j] + rng.uniform(0.1, 1.5)
    c = rng.standard_normal(n) * 2
    return make_qp(Q, A, c, b, l, u, row_type, name=f"tiny_bf_{seed}")
