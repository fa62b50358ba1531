"""Seeded generators for the synthetic QP workloads.

Every generator is deterministic given its seed (numpy PCG64 through
``np.random.default_rng``).  The arrays are produced once on the host; the
oracle and the GPU library both consume exactly these arrays.

The paper evaluates on synthetic random-QP, control and portfolio classes
(Sec. 6.1, experimental set-up); the shapes below are our own stand-ins for
those classes, not reproductions of any third-party generator.

CSR convention: int32 ``rowptr``/``col``, float64 values, column indices sorted
within each row, Q stored as a full symmetric matrix (both triangles).
Row types: 0 = equality row (A_i x = b_i), 1 = ``>=`` row (A_i x >= b_i).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

EQ = 0
GE = 1


@dataclass
class QPInstance:
    name: str
    n: int
    m: int
    q_rowptr: np.ndarray
    q_col: np.ndarray
    q_val: np.ndarray
    a_rowptr: np.ndarray
    a_col: np.ndarray
    a_val: np.ndarray
    c: np.ndarray
    b: np.ndarray
    l: np.ndarray
    u: np.ndarray
    row_type: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def q_nnz(self) -> int:
        return int(self.q_rowptr[-1])

    @property
    def a_nnz(self) -> int:
        return int(self.a_rowptr[-1])

    def Q(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.q_val, self.q_col, self.q_rowptr), shape=(self.n, self.n))

    def A(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.a_val, self.a_col, self.a_rowptr), shape=(self.m, self.n))

    def dense(self):
        return self.Q().toarray(), self.A().toarray()


def _to_csr(mat) -> tuple:
    mat = sp.csr_matrix(mat)
    mat.sum_duplicates()
    mat.sort_indices()
    return (mat.indptr.astype(np.int32), mat.indices.astype(np.int32),
            mat.data.astype(np.float64))


def csr_from_dense(M: np.ndarray) -> tuple:
    """CSR (rowptr, col, val) of the nonzero pattern of a dense matrix."""
    return _to_csr(sp.csr_matrix(np.asarray(M, dtype=np.float64)))


def _make(name, Q, A, c, b, l, u, row_type, meta=None) -> QPInstance:
    qr, qc, qv = _to_csr(Q)
    ar, ac, av = _to_csr(A)
    n = Q.shape[0]
    m = A.shape[0]
    return QPInstance(name, n, m, qr, qc, qv, ar, ac, av,
                      np.ascontiguousarray(c, dtype=np.float64),
                      np.ascontiguousarray(b, dtype=np.float64),
                      np.ascontiguousarray(l, dtype=np.float64),
                      np.ascontiguousarray(u, dtype=np.float64),
                      np.ascontiguousarray(row_type, dtype=np.uint8),
                      meta or {})


def _distinct_cols(rng, nrows: int, ncols: int, k: int, exclude_self: bool = False):
    """(nrows, k) matrix of distinct uniform column indices per row, sorted."""
    k = min(k, ncols - (1 if exclude_self else 0))
    cols = rng.integers(0, ncols, size=(nrows, k), dtype=np.int64)
    rows = np.arange(nrows, dtype=np.int64)[:, None]
    while True:
        cols.sort(axis=1)
        bad = np.zeros(nrows, dtype=bool)
        if k > 1:
            bad |= (np.diff(cols, axis=1) == 0).any(axis=1)
        if exclude_self:
            bad |= (cols == rows).any(axis=1)
        nb = int(bad.sum())
        if nb == 0:
            return cols
        cols[bad] = rng.integers(0, ncols, size=(nb, k), dtype=np.int64)


def _diag_dominant_from_offdiag(off: sp.spmatrix) -> sp.csr_matrix:
    off = sp.csr_matrix(off)
    off.sum_duplicates()
    off.setdiag(0.0)
    off.eliminate_zeros()
    d = np.asarray(abs(off).sum(axis=1)).ravel() + 1.0
    return sp.csr_matrix(off + sp.diags(d))


# ---------------------------------------------------------------------------
# Tiny random QP: n=100, m=50 (30 EQ, 20 GE), A 10 % dense, Q = S+S^T + diag.
# ---------------------------------------------------------------------------
def tiny_random_qp(seed: int = 1, n: int = 100, m: int = 50, n_eq: int = 30,
                   a_density: float = 0.10, s_density: float = 0.05,
                   bound: float = 10.0) -> QPInstance:
    rng = np.random.default_rng(seed)
    A = np.where(rng.random((m, n)) < a_density, rng.standard_normal((m, n)), 0.0)
    S = np.where(rng.random((n, n)) < s_density, rng.standard_normal((n, n)), 0.0)
    np.fill_diagonal(S, 0.0)
    Q = _diag_dominant_from_offdiag(sp.csr_matrix(S + S.T))
    c = rng.standard_normal(n)
    l = np.full(n, -np.inf)
    u = np.full(n, np.inf)
    bounded = rng.permutation(n)[: n // 2]
    l[bounded] = -bound
    u[bounded] = bound
    x0 = rng.uniform(-1.0, 1.0, n)
    b = A @ x0
    row_type = np.array([EQ] * n_eq + [GE] * (m - n_eq), dtype=np.uint8)
    b[n_eq:] -= rng.uniform(0.0, 1.0, m - n_eq)
    return _make(f"tiny_random_n{n}_m{m}_s{seed}", Q, sp.csr_matrix(A), c, b, l, u,
                 row_type, {"x_feasible": x0})


# ---------------------------------------------------------------------------
# Large sparse random QP: n=1e6, m=5e5 (half EQ, half GE), A 10 nnz/row,
# Q = S + S^T (S 5 nnz/row) + diagonal making it diagonally dominant, x >= 0.
# ---------------------------------------------------------------------------
def large_random_qp(seed: int = 2, n: int = 1_000_000, m: int = 500_000,
                    a_per_row: int = 10, s_per_row: int = 5) -> QPInstance:
    rng = np.random.default_rng(seed)
    acols = _distinct_cols(rng, m, n, a_per_row)
    k = acols.shape[1]
    avals = rng.standard_normal((m, k))
    A = sp.csr_matrix((avals.ravel(), acols.ravel(), np.arange(0, m * k + 1, k)), shape=(m, n))
    scols = _distinct_cols(rng, n, n, s_per_row, exclude_self=True)
    ks = scols.shape[1]
    svals = rng.standard_normal((n, ks))
    srows = np.repeat(np.arange(n), ks)
    S = sp.csr_matrix((svals.ravel(), (srows, scols.ravel())), shape=(n, n))
    Q = _diag_dominant_from_offdiag(S + S.T)
    c = rng.standard_normal(n)
    l = np.zeros(n)
    u = np.full(n, np.inf)
    x0 = rng.uniform(0.0, 1.0, n)
    b = A @ x0
    n_eq = m // 2
    row_type = np.array([EQ] * n_eq + [GE] * (m - n_eq), dtype=np.uint8)
    b[n_eq:] -= rng.uniform(0.0, 1.0, m - n_eq)
    return _make(f"large_random_n{n}_m{m}_s{seed}", Q, A, c, b, l, u, row_type,
                 {"x_feasible": x0})


# ---------------------------------------------------------------------------
# Factor-model portfolio QP: variables (x, y), x in R^{n_assets} (x >= 0),
# y in R^k (free).  min x^T D x + y^T y - mu^T x,  y = F^T x,  1^T x = budget.
# In 1/2 form: Q = diag(2D, 2I), c = (-mu, 0).
# ---------------------------------------------------------------------------
def _sparse_factor(rng, n_assets: int, k: int, density: float) -> sp.csc_matrix:
    rows, cols = [], []
    for j in range(k):
        cnt = int(rng.binomial(n_assets, density))
        r = np.unique(rng.integers(0, n_assets, size=cnt))
        rows.append(r)
        cols.append(np.full(r.size, j))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = rng.standard_normal(rows.size)
    return sp.csc_matrix((vals, (rows, cols)), shape=(n_assets, k))


def _portfolio_from_parts(name, D, F, mu, budget, k) -> QPInstance:
    n_assets = D.size
    n = n_assets + k
    Q = sp.diags(np.concatenate([2.0 * D, np.full(k, 2.0)]))
    c = np.concatenate([-mu, np.zeros(k)])
    # rows 0..k-1: y_i - (F^T x)_i = 0 ; row k: 1^T x = budget
    Ft = sp.csr_matrix(F.T)
    top = sp.hstack([-Ft, sp.identity(k, format="csr")])
    bottom = sp.csr_matrix((np.ones(n_assets), (np.zeros(n_assets, dtype=np.int64),
                                                np.arange(n_assets))), shape=(1, n))
    A = sp.vstack([top, bottom]).tocsr()
    b = np.zeros(k + 1)
    b[k] = budget
    l = np.concatenate([np.zeros(n_assets), np.full(k, -np.inf)])
    u = np.full(n, np.inf)
    row_type = np.zeros(k + 1, dtype=np.uint8)
    return _make(name, Q, A, c, b, l, u, row_type, {"n_assets": n_assets, "k": k})


def portfolio_qp(seed: int = 3, n_assets: int = 500_000, k: int = 1000,
                 f_density: float = 0.01, budget: float = 1.0) -> QPInstance:
    rng = np.random.default_rng(seed)
    F = _sparse_factor(rng, n_assets, k, f_density)
    D = rng.uniform(0.0, np.sqrt(k) * 0.1, n_assets)
    mu = rng.standard_normal(n_assets)
    return _portfolio_from_parts(f"portfolio_n{n_assets}_k{k}_s{seed}", D, F, mu, budget, k)


@dataclass
class PortfolioFamily:
    """A parametrised family sharing D and F; instance i has its own mu and budget."""
    base: QPInstance
    mu: np.ndarray        # (count, n_assets)
    budget: np.ndarray    # (count,)
    mu_bar: np.ndarray
    mu_sigma: float

    @property
    def count(self) -> int:
        return self.budget.size

    def c_of(self, i: int) -> np.ndarray:
        k = self.base.meta["k"]
        return np.concatenate([-self.mu[i], np.zeros(k)])

    def b_of(self, i: int) -> np.ndarray:
        b = np.zeros(self.base.m)
        b[-1] = self.budget[i]
        return b

    def instance(self, i: int) -> QPInstance:
        bi = self.base
        return QPInstance(f"{bi.name}_i{i}", bi.n, bi.m, bi.q_rowptr, bi.q_col, bi.q_val,
                          bi.a_rowptr, bi.a_col, bi.a_val, self.c_of(i), self.b_of(i),
                          bi.l, bi.u, bi.row_type, dict(bi.meta))

    def batch(self, idx) -> "BatchInstances":
        return concat_batch([self.instance(int(i)) for i in idx])


def portfolio_family(seed: int = 5, n_assets: int = 5000, k: int = 100, count: int = 20000,
                     f_density: float = 0.01, mu_sigma: float = 0.1,
                     budget_lo: float = 0.5, budget_hi: float = 1.5) -> PortfolioFamily:
    rng = np.random.default_rng(seed)
    F = _sparse_factor(rng, n_assets, k, f_density)
    D = rng.uniform(0.0, np.sqrt(k) * 0.1, n_assets)
    mu_bar = rng.standard_normal(n_assets)
    base = _portfolio_from_parts(f"portfolio_family_n{n_assets}_k{k}_s{seed}", D, F, mu_bar,
                                 1.0, k)
    mu = mu_bar[None, :] + mu_sigma * rng.standard_normal((count, n_assets))
    budget = rng.uniform(budget_lo, budget_hi, count)
    return PortfolioFamily(base, mu, budget, mu_bar, mu_sigma)


# ---------------------------------------------------------------------------
# MPC-style QP: z = (x_0..x_T, u_0..u_{T-1}); x_0 = x_init,
# x_{t+1} - A_t x_t - B_t u_t = 0; diagonal state/input weights; box bounds.
# ---------------------------------------------------------------------------
def mpc_qp(rng, T: int, nx: int, nu: int, name: str = "mpc",
           state_bound_cap: float = 1e3) -> QPInstance:
    n = (T + 1) * nx + T * nu
    m = (T + 1) * nx
    At = np.eye(nx)[None] + 0.1 * rng.standard_normal((T, nx, nx))
    Bt = 0.1 * rng.standard_normal((T, nx, nu))
    qd = rng.uniform(0.1, 10.0, (T + 1) * nx)
    rd = rng.uniform(0.1, 10.0, T * nu)
    x_init = rng.uniform(-1.0, 1.0, nx)
    u_sim = rng.uniform(-0.5, 0.5, (T, nu))
    xs = [x_init]
    for t in range(T):
        xs.append(At[t] @ xs[-1] + Bt[t] @ u_sim[t])
    xmax = float(np.max(np.abs(np.array(xs))))
    xb = max(10.0, 2.0 * xmax)
    if xb > state_bound_cap:
        xb = np.inf
    # rows 0..nx-1: x_0 = x_init ; row (t+1)*nx + j: x_{t+1,j} - A_t[j,:] x_t - B_t[j,:] u_t = 0
    t_idx = np.arange(T)[:, None, None]
    j_idx = np.arange(nx)[None, :, None]
    r_dyn = (t_idx + 1) * nx + j_idx                                   # (T, nx, 1)
    qx = np.arange(nx)[None, None, :]
    qu = np.arange(nu)[None, None, :]
    rows = np.concatenate([
        np.arange(nx),
        np.broadcast_to(r_dyn, (T, nx, nx)).ravel(),
        r_dyn.ravel(),
        np.broadcast_to(r_dyn, (T, nx, nu)).ravel()])
    cols = np.concatenate([
        np.arange(nx),
        (t_idx * nx + qx + 0 * j_idx).ravel(),
        ((t_idx + 1) * nx + j_idx).ravel(),
        ((T + 1) * nx + t_idx * nu + qu + 0 * j_idx).ravel()])
    vals = np.concatenate([
        np.ones(nx),
        (-At).ravel(),
        np.ones(T * nx),
        (-Bt).ravel()])
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    Q = sp.diags(np.concatenate([qd, rd]))
    c = np.zeros(n)
    b = np.zeros(m)
    b[:nx] = x_init
    l = np.concatenate([np.full((T + 1) * nx, -xb), np.full(T * nu, -1.0)])
    u = -l
    row_type = np.zeros(m, dtype=np.uint8)
    z_sim = np.concatenate([np.array(xs).ravel(), u_sim.ravel()])
    return _make(name, Q, A, c, b, l, u, row_type,
                 {"T": T, "nx": nx, "nu": nu, "x_feasible": z_sim, "state_bound": xb})


def mpc_batch(seed: int = 4, count: int = 4096, T_range=(10, 100), nx_range=(4, 12),
              nu_range=(2, 4)) -> "BatchInstances":
    insts = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        T = int(rng.integers(T_range[0], T_range[1] + 1))
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        nu = int(rng.integers(nu_range[0], nu_range[1] + 1))
        insts.append(mpc_qp(rng, T, nx, nu, name=f"mpc_s{seed}_i{i}"))
    return concat_batch(insts)


# ---------------------------------------------------------------------------
# Segment-CSR batch: instances concatenated; row pointers are global offsets
# into the concatenated nnz arrays, column indices stay local to the instance.
# ---------------------------------------------------------------------------
@dataclass
class BatchInstances:
    count: int
    var_off: np.ndarray   # int64 [B+1]
    row_off: np.ndarray   # int64 [B+1]
    q_rowptr: np.ndarray  # int32 [sum n + 1]  (global nnz offsets)
    q_col: np.ndarray     # int32 local column ids
    q_val: np.ndarray
    a_rowptr: np.ndarray  # int32 [sum m + 1]
    a_col: np.ndarray
    a_val: np.ndarray
    c: np.ndarray
    b: np.ndarray
    l: np.ndarray
    u: np.ndarray
    row_type: np.ndarray
    names: list

    def instance(self, i: int) -> QPInstance:
        v0, v1 = int(self.var_off[i]), int(self.var_off[i + 1])
        r0, r1 = int(self.row_off[i]), int(self.row_off[i + 1])
        qp = self.q_rowptr[v0:v1 + 1].astype(np.int64)
        ap = self.a_rowptr[r0:r1 + 1].astype(np.int64)
        return QPInstance(self.names[i], v1 - v0, r1 - r0,
                          (qp - qp[0]).astype(np.int32), self.q_col[qp[0]:qp[-1]].copy(),
                          self.q_val[qp[0]:qp[-1]].copy(),
                          (ap - ap[0]).astype(np.int32), self.a_col[ap[0]:ap[-1]].copy(),
                          self.a_val[ap[0]:ap[-1]].copy(),
                          self.c[v0:v1].copy(), self.b[r0:r1].copy(),
                          self.l[v0:v1].copy(), self.u[v0:v1].copy(),
                          self.row_type[r0:r1].copy())


def concat_batch(insts) -> BatchInstances:
    B = len(insts)
    var_off = np.zeros(B + 1, dtype=np.int64)
    row_off = np.zeros(B + 1, dtype=np.int64)
    for i, q in enumerate(insts):
        var_off[i + 1] = var_off[i] + q.n
        row_off[i + 1] = row_off[i] + q.m
    qnnz = np.cumsum([0] + [q.q_nnz for q in insts])
    annz = np.cumsum([0] + [q.a_nnz for q in insts])
    if qnnz[-1] >= 2**31 or annz[-1] >= 2**31:
        raise ValueError("batch too large for int32 row pointers")
    q_rowptr = np.concatenate([insts[i].q_rowptr[:-1].astype(np.int64) + qnnz[i] for i in range(B)]
                              + [np.array([qnnz[-1]])]).astype(np.int32)
    a_rowptr = np.concatenate([insts[i].a_rowptr[:-1].astype(np.int64) + annz[i] for i in range(B)]
                              + [np.array([annz[-1]])]).astype(np.int32)
    cat = lambda attr: np.concatenate([getattr(q, attr) for q in insts])  # noqa: E731
    return BatchInstances(B, var_off, row_off, q_rowptr, cat("q_col"), cat("q_val"),
                          a_rowptr, cat("a_col"), cat("a_val"), cat("c"), cat("b"),
                          cat("l"), cat("u"), cat("row_type"), [q.name for q in insts])


# ---------------------------------------------------------------------------
# Further synthetic classes of the paper's large-scale set (Sec. 6.1 lists random
# QP, random QP with equality constraints, control, portfolio, Huber regression,
# Lasso and SVM).  Each is the textbook problem written in the QP form above;
# the data distributions are our own choices.
# ---------------------------------------------------------------------------
def _sprandn(rng, m: int, n: int, density: float) -> sp.csr_matrix:
    return sp.random(m, n, density=density, format="csr", random_state=rng,
                     data_rvs=rng.standard_normal)


def eq_qp(seed: int = 7, n: int = 2000, nnz_per_row: int = 4) -> QPInstance:
    """min 1/2 x'Qx + c'x  s.t.  Ax = b:  Q = MM' + 0.01 I, A with m = n/2 rows; M and A
    have nnz_per_row N(0,1) entries in distinct uniform columns of every row; b = A x0 for
    a random x0; no bounds."""
    rng = np.random.default_rng(seed)
    m = n // 2
    k = min(nnz_per_row, n)

    def rows_k(nrows):   # exactly k distinct columns per row: no empty row
        cols = _distinct_cols(rng, nrows, n, k)
        return sp.csr_matrix((rng.standard_normal(nrows * k), cols.ravel(),
                              np.arange(0, nrows * k + 1, k)), shape=(nrows, n))
    M = rows_k(n)
    Q = sp.csr_matrix(M @ M.T + 0.01 * sp.identity(n))
    A = rows_k(m)
    x0 = rng.standard_normal(n)
    b = A @ x0
    c = rng.standard_normal(n)
    return _make(f"eq_qp_n{n}_s{seed}", Q, A, c, b, np.full(n, -np.inf), np.full(n, np.inf),
                 np.full(m, EQ, np.uint8), {"class": "eq_qp"})


def lasso_qp(seed: int = 8, n_features: int = 500, m_samples: int = 5000,
             density: float = 0.05) -> QPInstance:
    """Lasso  min 1/2 ||Fx - g||^2 + lam ||x||_1  as a QP in z = (x, y, t):
    min 1/2 y'y + lam 1't  s.t.  Fx - y = g (EQ),  t - x >= 0,  t + x >= 0 (GE).
    F sparse N(0,1); g = F v + noise with v half zeros; lam = ||F'g||_inf / 5."""
    rng = np.random.default_rng(seed)
    n, m = n_features, m_samples
    F = _sprandn(rng, m, n, density)
    v = np.where(rng.random(n) < 0.5, rng.standard_normal(n) / np.sqrt(n), 0.0)
    g = F @ v + rng.standard_normal(m)
    lam = float(np.abs(F.T @ g).max()) / 5.0
    N = n + m + n
    Q = sp.diags(np.concatenate([np.zeros(n), np.ones(m), np.zeros(n)])).tocsr()
    I_n = sp.identity(n, format="csr")
    A = sp.vstack([sp.hstack([F, -sp.identity(m), sp.csr_matrix((m, n))]),
                   sp.hstack([-I_n, sp.csr_matrix((n, m)), I_n]),
                   sp.hstack([I_n, sp.csr_matrix((n, m)), I_n])]).tocsr()
    b = np.concatenate([g, np.zeros(2 * n)])
    c = np.concatenate([np.zeros(n + m), np.full(n, lam)])
    rt = np.concatenate([np.full(m, EQ), np.full(2 * n, GE)]).astype(np.uint8)
    return _make(f"lasso_n{n}_m{m}_s{seed}", Q, A, c, b, np.full(N, -np.inf),
                 np.full(N, np.inf), rt,
                 {"class": "lasso", "F": F, "g": g, "lam": lam, "n_features": n})


def huber_qp(seed: int = 9, n_features: int = 500, m_samples: int = 5000,
             density: float = 0.05, outlier_frac: float = 0.05) -> QPInstance:
    """Huber fitting  min sum_i phi(f_i'x - g_i),  phi(s) = s^2 (|s| <= 1), 2|s| - 1
    (otherwise), as a QP in z = (x, u, r, s):  min u'u + 2 1'(r + s)  s.t.
    Fx - u - r + s = g (EQ),  r, s >= 0.  g = F v + noise with a few large outliers."""
    rng = np.random.default_rng(seed)
    n, m = n_features, m_samples
    F = _sprandn(rng, m, n, density)
    v = rng.standard_normal(n) / np.sqrt(n)
    noise = np.where(rng.random(m) < outlier_frac, 10.0 * rng.standard_normal(m),
                     0.5 * rng.standard_normal(m))
    g = F @ v + noise
    N = n + 3 * m
    Q = sp.diags(np.concatenate([np.zeros(n), np.full(m, 2.0), np.zeros(2 * m)])).tocsr()
    I_m = sp.identity(m, format="csr")
    A = sp.hstack([F, -I_m, -I_m, I_m]).tocsr()
    c = np.concatenate([np.zeros(n + m), np.full(2 * m, 2.0)])
    l = np.concatenate([np.full(n + m, -np.inf), np.zeros(2 * m)])
    return _make(f"huber_n{n}_m{m}_s{seed}", Q, A, c, g, l, np.full(N, np.inf),
                 np.full(m, EQ, np.uint8),
                 {"class": "huber", "F": F, "g": g, "n_features": n})


def svm_qp(seed: int = 10, n_features: int = 500, m_samples: int = 5000,
           density: float = 0.05, lam: float = 1.0) -> QPInstance:
    """Soft-margin SVM  min x'x + lam sum_i max(0, 1 - g_i f_i'x)  as a QP in
    z = (x, t):  min x'x + lam 1't  s.t.  t_i + g_i f_i'x >= 1 (GE),  t >= 0.
    Labels g = +1 for the first half of the samples, -1 for the rest; a sample's
    nonzero features are N(+-1/n, 1/n) by class."""
    rng = np.random.default_rng(seed)
    n, m = n_features, m_samples
    F = _sprandn(rng, m, n, density).tocoo()
    lab = np.where(np.arange(m) < m // 2, 1.0, -1.0)
    F.data = (lab[F.row] + rng.standard_normal(F.data.size)) / n
    F = F.tocsr()
    N = n + m
    Q = sp.diags(np.concatenate([np.full(n, 2.0), np.zeros(m)])).tocsr()
    A = sp.hstack([sp.diags(lab) @ F, sp.identity(m)]).tocsr()
    c = np.concatenate([np.zeros(n), np.full(m, lam)])
    l = np.concatenate([np.full(n, -np.inf), np.zeros(m)])
    return _make(f"svm_n{n}_m{m}_s{seed}", Q, A, c, np.ones(m), l, np.full(N, np.inf),
                 np.full(m, GE, np.uint8),
                 {"class": "svm", "F": F, "labels": lab, "lam": lam, "n_features": n})


# ---------------------------------------------------------------------------
# Infeasible and unbounded variants (inputs for infeasibility detection).
# ---------------------------------------------------------------------------
ABLATION_CLASSES = ("random", "eq", "control", "portfolio", "huber", "lasso", "svm")


def ablation_set(per_class: int = 24) -> list:
    """Small instances of the seven synthetic classes of the paper's QP test set (random,
    equality-constrained, control, portfolio, Huber, Lasso, SVM), `per_class` of each in
    that class order, with sizes in the tens to hundreds of variables: a synthetic stand-in
    for a mixed benchmark set, solved by every method of the momentum / restart
    comparison."""
    out = []
    for cls in ABLATION_CLASSES:
        for k in range(per_class):
            if cls == "random":
                out.append(tiny_random_qp(k + 1))
            elif cls == "eq":
                out.append(eq_qp(seed=100 + k, n=300))
            elif cls == "control":
                out.append(mpc_qp(np.random.default_rng([6, k]), 20 + 5 * (k % 16), 6, 3))
            elif cls == "portfolio":
                out.append(portfolio_qp(seed=200 + k, n_assets=400, k=20))
            elif cls == "huber":
                out.append(huber_qp(seed=300 + k, n_features=40, m_samples=300))
            elif cls == "lasso":
                out.append(lasso_qp(seed=400 + k, n_features=40, m_samples=300))
            else:
                out.append(svm_qp(seed=500 + k, n_features=40, m_samples=300))
    return out


def primal_infeasible_qp(seed: int = 1, n: int = 100, m: int = 50) -> QPInstance:
    """The tiny random QP plus two contradictory rows a'x >= 1 and -a'x >= 0 for a dense
    random a: y = (1, 1) on them is a Farkas certificate (A'y = 0, b'y = 1)."""
    base = tiny_random_qp(seed, n=n, m=m)
    rng = np.random.default_rng([seed, 77])
    a = rng.standard_normal(n)
    A = sp.vstack([base.A(), sp.csr_matrix(a[None, :]), sp.csr_matrix(-a[None, :])]).tocsr()
    b = np.concatenate([base.b, [1.0, 0.0]])
    rt = np.concatenate([base.row_type, [GE, GE]]).astype(np.uint8)
    return _make(f"primal_infeasible_s{seed}", base.Q(), A, base.c, b, base.l, base.u, rt,
                 {"class": "primal_infeasible"})


def dual_infeasible_qp(seed: int = 1, n: int = 100, m: int = 50) -> QPInstance:
    """A feasible QP that is unbounded below along d = -e_0: Q has no curvature along
    variable 0 (its row and column are zero), x_0 has no lower bound, c_0 = 1, and
    column 0 of A is 0 on equality rows and <= 0 on >= rows (so A d >= 0)."""
    base = tiny_random_qp(seed, n=n, m=m)
    Q = base.Q().tolil()
    Q[0, :] = 0.0
    Q[:, 0] = 0.0
    A = base.A().tolil()
    col0 = A[:, 0].toarray().ravel()
    eq = base.row_type == EQ
    col0[eq] = 0.0
    col0[~eq] = -np.abs(col0[~eq])
    A[:, 0] = col0[:, None]
    c = base.c.copy()
    c[0] = 1.0
    l, u = base.l.copy(), base.u.copy()
    l[0], u[0] = -np.inf, np.inf
    x0 = base.meta["x_feasible"].copy()
    A = sp.csr_matrix(A)
    A.eliminate_zeros()
    b = A @ x0
    b[~eq] -= np.random.default_rng([seed, 78]).uniform(0.0, 1.0, int((~eq).sum()))
    Qc = sp.csr_matrix(Q)
    Qc.eliminate_zeros()
    return _make(f"dual_infeasible_s{seed}", Qc, A, c, b, l, u, base.row_type,
                 {"class": "dual_infeasible"})


def with_contradictory_rows(qp: QPInstance, seed: int = 0) -> QPInstance:
    """qp plus the pair a'x >= 1, -a'x >= 0 (a: 64 N(0,1) entries in distinct uniform
    columns): primal infeasible with the Farkas certificate y = 1 on the pair."""
    rng = np.random.default_rng([seed, 79])
    k = min(64, qp.n)
    cols = np.sort(rng.choice(qp.n, k, replace=False))
    a = np.zeros(qp.n)
    a[cols] = rng.standard_normal(k)
    A = sp.vstack([qp.A(), sp.csr_matrix(a[None, :]), sp.csr_matrix(-a[None, :])]).tocsr()
    return _make(qp.name + "_contradictory", qp.Q(), A, qp.c, np.concatenate([qp.b, [1.0, 0.0]]),
                 qp.l, qp.u, np.concatenate([qp.row_type, [GE, GE]]).astype(np.uint8),
                 {"class": "primal_infeasible"})


def with_unbounded_ray(qp: QPInstance) -> QPInstance:
    """qp made unbounded below along +e_0: Q's row and column 0 zeroed, x_0 without an
    upper bound, c_0 = -1, column 0 of A zeroed on EQ rows and made >= 0 on GE rows (so
    A e_0 >= 0).  qp's feasible point (meta "x_feasible") with x_0 moved to its lower
    bound stays feasible: b is re-derived on EQ rows and lowered where needed on GE rows."""
    Q = qp.Q().tolil()
    Q[0, :] = 0.0
    Q[:, 0] = 0.0
    A = qp.A().tocsc()
    col = A[:, 0].toarray().ravel()
    eq = qp.row_type == EQ
    col[eq] = 0.0
    col[~eq] = np.abs(col[~eq])
    A = A.tolil()
    A[:, 0] = col[:, None]
    c = qp.c.copy()
    c[0] = -1.0
    u = qp.u.copy()
    u[0] = np.inf
    Ac = sp.csr_matrix(A)
    Ac.eliminate_zeros()
    Qc = sp.csr_matrix(Q)
    Qc.eliminate_zeros()
    xf = np.array(qp.meta["x_feasible"], dtype=np.float64)
    xf[0] = qp.l[0] if np.isfinite(qp.l[0]) else 0.0
    ax = Ac @ xf
    b = np.where(eq, ax, np.minimum(qp.b, ax))
    return _make(qp.name + "_unbounded", Qc, Ac, c, b, qp.l, u, qp.row_type,
                 {"class": "dual_infeasible", "x_feasible": xf})
