"""ctypes wrapper of the C oracle (test infrastructure only).

Problems are passed as any object with the attributes of ``qpgen.QPInstance``
(n, m, q_rowptr, q_col, q_val, a_rowptr, a_col, a_val, c, b, l, u, row_type).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of the same source (the sanitizer test builds one with
# AddressSanitizer and UndefinedBehaviorSanitizer and runs the oracle's tests against it)
LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

RESTART_ADAPTIVE, RESTART_FIXED_K, RESTART_HALVING, RESTART_NONE = 0, 1, 2, 3
OPTIMAL, ITERATION_LIMIT, TIME_LIMIT, NUMERICAL_ERROR = 0, 1, 2, 3
PRIMAL_INFEASIBLE, DUAL_INFEASIBLE = 4, 5

_pd = C.POINTER(C.c_double)
_pi = C.POINTER(C.c_int32)
_pu8 = C.POINTER(C.c_uint8)


class _Problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64),
                ("q_rowptr", _pi), ("q_col", _pi), ("q_val", _pd),
                ("a_rowptr", _pi), ("a_col", _pi), ("a_val", _pd),
                ("c", _pd), ("b", _pd), ("l", _pd), ("u", _pd), ("row_type", _pu8)]


class _Settings(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
                ("check_every", C.c_int32), ("restart_mode", C.c_int32), ("fixed_K", C.c_int32),
                ("beta_sufficient", C.c_double), ("beta_necessary", C.c_double),
                ("beta_artificial", C.c_double), ("pw_smoothing", C.c_double),
                ("eps_zero", C.c_double), ("step_safety", C.c_double),
                ("norm_A", C.c_double), ("norm_Q", C.c_double),
                ("power_iter_max", C.c_int32), ("power_iter_rtol", C.c_double),
                ("warm_fallback", C.c_int32), ("detect_infeasibility", C.c_int32),
                ("eps_infeasible", C.c_double), ("momentum", C.c_int32)]


class _Infeas(C.Structure):
    _fields_ = [("primal_ratio", C.c_double), ("dual_ratio", C.c_double)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("iterations", C.c_int64), ("restarts", C.c_int64),
                ("kkt_evals", C.c_int64), ("rel_kkt", C.c_double), ("r_primal", C.c_double),
                ("r_dual", C.c_double), ("r_gap", C.c_double), ("primal_obj", C.c_double),
                ("dual_obj", C.c_double), ("omega", C.c_double), ("norm_A", C.c_double),
                ("norm_Q", C.c_double), ("used_warm_start", C.c_int32)]


class _CheckLog(C.Structure):
    _fields_ = [("total", C.c_int64), ("k", C.c_int64), ("r_cur", C.c_double),
                ("r_avg", C.c_double), ("candidate", C.c_int32), ("restarted", C.c_int32),
                ("omega", C.c_double)]


class _Kkt(C.Structure):
    _fields_ = [(f, C.c_double) for f in ("r_primal", "r_dual", "r_gap", "rel_kkt", "primal_obj",
                                          "dual_obj", "ax_inf", "b_inf", "qx_inf", "aty_inf",
                                          "c_inf", "xqx", "cx", "by")]


@dataclass
class OracleSettings:
    eps: float = 1e-6
    max_iter: int = 200000
    time_limit_s: float = 3600.0
    check_every: int = 64
    restart_mode: int = RESTART_ADAPTIVE
    fixed_K: int = 100
    beta_sufficient: float = 0.2
    beta_necessary: float = 0.8
    beta_artificial: float = 0.36
    pw_smoothing: float = 0.2
    eps_zero: float = 1e-10
    step_safety: float = 0.99
    norm_A: float = 0.0
    norm_Q: float = 0.0
    power_iter_max: int = 1000
    power_iter_rtol: float = 1e-7
    warm_fallback: int = 1
    detect_infeasibility: int = 0
    eps_infeasible: float = 1e-8
    momentum: int = 1

    def _c(self) -> _Settings:
        s = _Settings()
        for name, _ in _Settings._fields_:
            setattr(s, name, getattr(self, name))
        return s


_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from .build import build
            build()
        lib = C.CDLL(LIB_PATH)
        lib.orc_set_threads.argtypes = [C.c_int32]
        lib.orc_get_threads.restype = C.c_int32
        lib.orc_spmv.argtypes = [C.c_int64, _pi, _pi, _pd, _pd, _pd]
        lib.orc_spmv_t.argtypes = [C.c_int64, C.c_int64, _pi, _pi, _pd, _pd, _pd]
        lib.orc_rel_kkt.argtypes = [C.POINTER(_Problem), _pd, _pd, C.POINTER(_Kkt)]
        lib.orc_norm_A.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_double, _pi]
        lib.orc_norm_A.restype = C.c_double
        lib.orc_norm_Q.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_double, _pi]
        lib.orc_norm_Q.restype = C.c_double
        lib.orc_step_schedule.argtypes = [C.POINTER(_Settings), C.c_double, C.c_double,
                                          C.c_double, C.c_int64, _pd, _pd, _pd]
        lib.orc_run_inner.argtypes = [C.POINTER(_Problem), C.POINTER(_Settings), C.c_double,
                                      C.c_double, C.c_double, C.c_int64, _pd, _pd, _pd, _pd]
        lib.orc_solve.argtypes = [C.POINTER(_Problem), C.POINTER(_Settings), _pd, _pd, C.c_double,
                                  _pd, _pd, C.POINTER(_Result), C.POINTER(_CheckLog), C.c_int64,
                                  C.POINTER(C.c_int64)]
        lib.orc_solve.restype = C.c_int
        lib.orc_infeas_check.argtypes = [C.POINTER(_Problem), _pd, _pd, C.POINTER(_Infeas)]
        lib.orc_infeas_check.restype = None
        lib.orc_precondition.argtypes = [C.POINTER(_Problem), C.c_int32, C.c_int32, C.c_int32,
                                         _pd, _pd, _pd, _pd, _pd, _pd, _pd, _pd]
        lib.orc_precondition.restype = None
        lib.orc_solve_scaled.argtypes = [C.POINTER(_Problem), C.POINTER(_Problem), _pd, _pd,
                                         C.POINTER(_Settings), _pd, _pd, C.c_double, _pd, _pd,
                                         C.POINTER(_Result), C.POINTER(_CheckLog), C.c_int64,
                                         C.POINTER(C.c_int64)]
        lib.orc_solve_scaled.restype = C.c_int
        _lib = lib
    return _lib


def set_threads(t: int) -> None:
    """Host threads for the row loops of later solves (bitwise the one-thread results)."""
    load().orc_set_threads(int(t))


def get_threads() -> int:
    return int(load().orc_get_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, typ):
    return a.ctypes.data_as(typ)


class _ProblemRef:
    """Keeps the numpy arrays alive while the C struct points into them."""

    def __init__(self, qp):
        self.arrs = dict(
            q_rowptr=np.ascontiguousarray(qp.q_rowptr, dtype=np.int32),
            q_col=np.ascontiguousarray(qp.q_col, dtype=np.int32),
            q_val=_f64(qp.q_val),
            a_rowptr=np.ascontiguousarray(qp.a_rowptr, dtype=np.int32),
            a_col=np.ascontiguousarray(qp.a_col, dtype=np.int32),
            a_val=_f64(qp.a_val),
            c=_f64(qp.c), b=_f64(qp.b) if qp.m else np.zeros(1),
            l=_f64(qp.l), u=_f64(qp.u),
            row_type=np.ascontiguousarray(qp.row_type, dtype=np.uint8) if qp.m
            else np.zeros(1, np.uint8))
        if self.arrs["a_val"].size == 0:
            self.arrs["a_val"] = np.zeros(1)
            self.arrs["a_col"] = np.zeros(1, np.int32)
        a = self.arrs
        self.s = _Problem(qp.n, qp.m, _ptr(a["q_rowptr"], _pi), _ptr(a["q_col"], _pi),
                          _ptr(a["q_val"], _pd), _ptr(a["a_rowptr"], _pi), _ptr(a["a_col"], _pi),
                          _ptr(a["a_val"], _pd), _ptr(a["c"], _pd), _ptr(a["b"], _pd),
                          _ptr(a["l"], _pd), _ptr(a["u"], _pd), _ptr(a["row_type"], _pu8))


def spmv(rowptr, col, val, x):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = _f64(val)
    x = _f64(x)
    nrows = rowptr.size - 1
    y = np.zeros(max(nrows, 1))
    if col.size == 0:
        col = np.zeros(1, np.int32); val = np.zeros(1)
    load().orc_spmv(nrows, _ptr(rowptr, _pi), _ptr(col, _pi), _ptr(val, _pd), _ptr(x, _pd),
                    _ptr(y, _pd))
    return y[:nrows]


def spmv_t(rowptr, col, val, x, ncols):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = _f64(val)
    x = _f64(x) if x.size else np.zeros(1)
    if col.size == 0:
        col = np.zeros(1, np.int32); val = np.zeros(1)
    y = np.zeros(ncols)
    load().orc_spmv_t(rowptr.size - 1, ncols, _ptr(rowptr, _pi), _ptr(col, _pi), _ptr(val, _pd),
                      _ptr(x, _pd), _ptr(y, _pd))
    return y


def rel_kkt(qp, x, y) -> dict:
    pr = _ProblemRef(qp)
    x = _f64(x)
    y = _f64(y) if qp.m else np.zeros(1)
    out = _Kkt()
    load().orc_rel_kkt(C.byref(pr.s), _ptr(x, _pd), _ptr(y, _pd), C.byref(out))
    return {name: getattr(out, name) for name, _ in _Kkt._fields_}


def norm_A(qp, maxit=1000, rtol=1e-7):
    pr = _ProblemRef(qp)
    it = C.c_int32(0)
    v = load().orc_norm_A(C.byref(pr.s), maxit, rtol, C.byref(it))
    return v, it.value


def norm_Q(qp, maxit=1000, rtol=1e-7):
    pr = _ProblemRef(qp)
    it = C.c_int32(0)
    v = load().orc_norm_Q(C.byref(pr.s), maxit, rtol, C.byref(it))
    return v, it.value


def step_schedule(settings: OracleSettings, nA, nQ, omega, K):
    p = np.zeros(K); d = np.zeros(K); s = np.zeros(K)
    load().orc_step_schedule(C.byref(settings._c()), nA, nQ, omega, K, _ptr(p, _pd),
                             _ptr(d, _pd), _ptr(s, _pd))
    return p, d, s


def run_inner(qp, settings: OracleSettings, nA, nQ, omega, iters, x0=None, y0=None):
    pr = _ProblemRef(qp)
    x = _f64(x0 if x0 is not None else np.zeros(qp.n)).copy()
    y = _f64(y0 if y0 is not None else np.zeros(max(qp.m, 1))).copy()
    if y.size == 0:
        y = np.zeros(1)
    xb = np.zeros(qp.n); yb = np.zeros(max(qp.m, 1))
    load().orc_run_inner(C.byref(pr.s), C.byref(settings._c()), nA, nQ, omega, iters,
                         _ptr(x, _pd), _ptr(y, _pd), _ptr(xb, _pd), _ptr(yb, _pd))
    return x, y[:qp.m], xb, yb[:qp.m]


def infeas_check(qp, dx, dy) -> dict:
    """Certificate ratios of a direction (dx, dy): see orc_infeas_check."""
    pr = _ProblemRef(qp)
    dx = _f64(dx)
    dy = _f64(dy) if qp.m else np.zeros(1)
    out = _Infeas()
    load().orc_infeas_check(C.byref(pr.s), _ptr(dx, _pd), _ptr(dy, _pd), C.byref(out))
    return {"primal_ratio": out.primal_ratio, "dual_ratio": out.dual_ratio}


def precondition(qp, ruiz_iters=10, l2=True, pc=True):
    """Diagonal preconditioning of K = [[Q, A'], [A, 0]]; returns (scaled instance,
    D2 [n], D1 [m]) with Q~ = D2 Q D2, A~ = D1 A D2, c~ = D2 c, b~ = D1 b, bounds / D2."""
    import dataclasses
    pr = _ProblemRef(qp)
    qv = np.zeros(max(len(qp.q_val), 1))
    av = np.zeros(max(len(qp.a_val), 1))
    c = np.zeros(qp.n); l = np.zeros(qp.n); u = np.zeros(qp.n)
    b = np.zeros(max(qp.m, 1)); dv = np.zeros(qp.n); dr = np.zeros(max(qp.m, 1))
    load().orc_precondition(C.byref(pr.s), int(ruiz_iters), int(bool(l2)), int(bool(pc)),
                            _ptr(qv, _pd), _ptr(av, _pd), _ptr(c, _pd), _ptr(b, _pd),
                            _ptr(l, _pd), _ptr(u, _pd), _ptr(dv, _pd), _ptr(dr, _pd))
    scaled = dataclasses.replace(qp, q_val=qv[:len(qp.q_val)], a_val=av[:len(qp.a_val)], c=c,
                                 b=b[:qp.m], l=l, u=u)
    return scaled, dv, dr[:qp.m]


def solve_scaled(scaled, orig, d_var, d_row, settings: OracleSettings | None = None, x0=None,
                 y0=None, omega0=0.0, log_cap: int = 0):
    """Solve the preconditioned instance; relKKT, warm starts and outputs refer to orig."""
    return solve(scaled, settings, x0, y0, omega0, log_cap, _orig=(orig, d_var, d_row))


def solve(qp, settings: OracleSettings | None = None, x0=None, y0=None, omega0=0.0,
          log_cap: int = 0, _orig=None):
    """Run the oracle; returns (x, y, result dict, check log list)."""
    settings = settings or OracleSettings()
    pr = _ProblemRef(qp)
    x = np.zeros(qp.n)
    y = np.zeros(max(qp.m, 1))
    res = _Result()
    logs = (_CheckLog * max(log_cap, 1))()
    nlog = C.c_int64(0)
    x0p = _f64(x0) if x0 is not None else None
    y0p = _f64(y0) if y0 is not None else None
    if y0p is not None and y0p.size == 0:
        y0p = np.zeros(1)
    tail = (_ptr(x0p, _pd) if x0p is not None else None,
            _ptr(y0p, _pd) if y0p is not None else None,
            float(omega0), _ptr(x, _pd), _ptr(y, _pd), C.byref(res),
            logs if log_cap > 0 else None, log_cap, C.byref(nlog))
    if _orig is None:
        rc = load().orc_solve(C.byref(pr.s), C.byref(settings._c()), *tail)
    else:
        orig, dv, dr = _orig
        po = _ProblemRef(orig)
        dv = _f64(dv)
        dr = _f64(dr) if orig.m else np.ones(1)
        rc = load().orc_solve_scaled(C.byref(pr.s), C.byref(po.s), _ptr(dv, _pd), _ptr(dr, _pd),
                                     C.byref(settings._c()), *tail)
    if rc != 0:
        raise ValueError(f"oracle rejected the problem (rc={rc}, status={res.status})")
    r = {name: getattr(res, name) for name, _ in _Result._fields_}
    log = [{name: getattr(logs[i], name) for name, _ in _CheckLog._fields_}
           for i in range(min(nlog.value, log_cap))]
    return x, y[:qp.m], r, log
