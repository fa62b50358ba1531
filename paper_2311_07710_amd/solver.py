"""Python front end of the MI355X rAPDHG library (marshalling only).

``Solver`` wraps qp_create / qp_solve / qp_free for one QP, ``BatchSolver``
wraps qp_create / qp_batch_solve for many.  Problems are any object with the
attributes of ``qpgen.QPInstance`` (or ``qpgen.BatchInstances``); host arrays
are numpy, device arrays torch CUDA tensors.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, fields

import numpy as np

from . import _binding as B


@dataclass
class Settings:
    eps: float = 1e-6
    max_iter: int = 200000
    time_limit_s: float = 3600.0
    check_every: int = 64
    restart_mode: int = B.QP_RESTART_ADAPTIVE
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
    use_graph: int = 1
    profile: int = 0
    log_checks: int = 0
    device: int = 0
    panels_dual: int = 0
    panels_primal: int = 0
    momentum: int = 1
    precondition: int = 0
    ruiz_iters: int = 10
    detect_infeasibility: int = 0
    eps_infeasible: float = 1e-8
    check_symmetry: int = 0
    # called with a dict per relKKT evaluation of a single-QP solve (see qp_log_fn)
    log_cb: object = None

    def c_struct(self) -> B.qp_settings:
        """The C settings; a log_cb is wrapped in a C function pointer that the returned
        struct keeps alive (hold the struct as long as the handle)."""
        s = B.qp_settings()
        for f in fields(self):
            if f.name == "log_cb":
                continue
            setattr(s, f.name, getattr(self, f.name))
        if self.log_cb is not None:
            fn = self.log_cb
            s.log_cb = B.qp_log_fn(lambda p, _u: fn(
                {name: getattr(p.contents, name) for name, _ in B.qp_check_info._fields_}))
        return s


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


class _Keep:
    """Holds converted arrays alive while the library reads them."""

    def __init__(self, device: bool):
        self.device = device
        self.arrs = []

    def ptr(self, a, dtype):
        if a is None:
            return None
        if self.device:
            import torch
            tdt = {np.float64: torch.float64, np.int32: torch.int32, np.uint8: torch.uint8,
                   np.int64: torch.int64}[dtype]
            t = a if _is_torch(a) else torch.as_tensor(np.asarray(a))
            t = t.to(device="cuda", dtype=tdt).contiguous()
            self.arrs.append(t)
            return t.data_ptr() if t.numel() else None
        arr = np.ascontiguousarray(a, dtype=dtype)
        self.arrs.append(arr)
        return arr.ctypes.data if arr.size else None


def _result_dict(r: B.qp_result) -> dict:
    return {name: getattr(r, name) for name, _ in B.qp_result._fields_}


def _desc(qp, keep: _Keep, batch: bool) -> B.qp_problem_desc:
    d = B.qp_problem_desc()
    if batch:
        d.n = int(qp.var_off[-1])
        d.m = int(qp.row_off[-1])
        d.num_instances = int(qp.count)
    else:
        d.n = int(qp.n)
        d.m = int(qp.m)
        d.num_instances = 1
    d.mem_space = B.QP_MEM_DEVICE if keep.device else B.QP_MEM_HOST
    d.Q = B.qp_csr(keep.ptr(qp.q_rowptr, np.int32), keep.ptr(qp.q_col, np.int32),
                   keep.ptr(qp.q_val, np.float64), int(qp.q_rowptr[-1]))
    d.A = B.qp_csr(keep.ptr(qp.a_rowptr, np.int32), keep.ptr(qp.a_col, np.int32),
                   keep.ptr(qp.a_val, np.float64), int(qp.a_rowptr[-1]))
    d.c = keep.ptr(qp.c, np.float64)
    d.b = keep.ptr(qp.b, np.float64)
    d.l = keep.ptr(qp.l, np.float64)
    d.u = keep.ptr(qp.u, np.float64)
    d.row_type = keep.ptr(qp.row_type, np.uint8)
    if batch:
        host = _Keep(False)
        keep.arrs.append(host)
        d.var_off = host.ptr(qp.var_off, np.int64)
        d.row_off = host.ptr(qp.row_off, np.int64)
    if keep.device:
        import torch
        d.stream = torch.cuda.current_stream().cuda_stream
    return d


class Solver:
    """One convex QP on the GPU (qp_create / qp_solve)."""

    def __init__(self, qp, settings: Settings | None = None, device_arrays: bool = False):
        self.lib = B.load()
        self.settings = settings or Settings()
        self.device_arrays = device_arrays
        self.n, self.m = int(qp.n), int(qp.m)
        keep = _Keep(device_arrays)
        desc = _desc(qp, keep, batch=False)
        h = C.c_void_p()
        self._cs = self.settings.c_struct()  # keeps a log_cb thunk alive with the handle
        B.check(self.lib.qp_create(C.byref(desc), C.byref(self._cs), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.qp_free(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def norms(self):
        a, q = C.c_double(), C.c_double()
        B.check(self.lib.qp_get_norms(self.h, C.addressof(a), C.addressof(q)))
        return a.value, q.value

    def scaling(self):
        """(D2, D1) of the Sec. 5 preprocessing (ones when it is off)."""
        dv, dr = np.zeros(self.n), np.zeros(max(self.m, 1))
        B.check(self.lib.qp_get_scaling(self.h, dv.ctypes.data, dr.ctypes.data))
        return dv, dr[:self.m]

    def set_norms(self, norm_A: float, norm_Q: float):
        a, q = C.c_double(norm_A), C.c_double(norm_Q)
        B.check(self.lib.qp_set_norms(self.h, C.byref(a), C.byref(q)))

    def update_vectors(self, c=None, b=None):
        keep = _Keep(self.device_arrays)
        B.check(self.lib.qp_update_vectors(self.h, keep.ptr(c, np.float64), keep.ptr(b, np.float64)))

    def solve(self, x0=None, y0=None, omega0: float = 0.0):
        """Returns (x, y, result dict).  x, y are numpy (host mode) or torch (device mode)."""
        keep = _Keep(self.device_arrays)
        ws = None
        if x0 is not None or y0 is not None or omega0 > 0.0:
            ws = B.qp_warm_start(keep.ptr(x0, np.float64), keep.ptr(y0, np.float64), float(omega0))
        if self.device_arrays:
            import torch
            x = torch.empty(self.n, dtype=torch.float64, device="cuda")
            y = torch.empty(max(self.m, 1), dtype=torch.float64, device="cuda")
            torch.cuda.current_stream().synchronize()
            xp, yp = x.data_ptr(), y.data_ptr()
        else:
            x = np.zeros(self.n)
            y = np.zeros(max(self.m, 1))
            xp, yp = x.ctypes.data, y.ctypes.data
        res = B.qp_result()
        B.check(self.lib.qp_solve(self.h, C.byref(ws) if ws is not None else None, C.byref(res),
                                  xp, yp if self.m else None))
        return x, y[: self.m], _result_dict(res)

    def check_log(self):
        n = C.c_int64()
        B.check(self.lib.qp_get_check_log(self.h, None, 0, C.byref(n)))
        buf = (B.qp_check_info * max(n.value, 1))()
        B.check(self.lib.qp_get_check_log(self.h, buf, n.value, C.byref(n)))
        return [{name: getattr(buf[i], name) for name, _ in B.qp_check_info._fields_}
                for i in range(n.value)]

    def profile(self) -> dict:
        p = B.qp_profile()
        B.check(self.lib.qp_get_profile(self.h, C.byref(p)))
        return {name: getattr(p, name) for name, _ in B.qp_profile._fields_}


class BatchSolver:
    """Many independent QPs in one persistent launch (qp_create / qp_batch_solve)."""

    def __init__(self, batch, settings: Settings | None = None, device_arrays: bool = False):
        self.lib = B.load()
        self.settings = settings or Settings()
        self.device_arrays = device_arrays
        self.count = int(batch.count)
        self.var_off = np.asarray(batch.var_off, dtype=np.int64)
        self.row_off = np.asarray(batch.row_off, dtype=np.int64)
        keep = _Keep(device_arrays)
        desc = _desc(batch, keep, batch=True)
        h = C.c_void_p()
        self._cs = self.settings.c_struct()  # keeps a log_cb thunk alive with the handle
        B.check(self.lib.qp_create(C.byref(desc), C.byref(self._cs), C.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.qp_free(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    __del__ = close

    def update_vectors(self, c=None, b=None):
        keep = _Keep(self.device_arrays)
        B.check(self.lib.qp_update_vectors(self.h, keep.ptr(c, np.float64), keep.ptr(b, np.float64)))

    def norms(self):
        a = np.zeros(self.count)
        q = np.zeros(self.count)
        B.check(self.lib.qp_get_norms(self.h, a.ctypes.data, q.ctypes.data))
        return a, q

    def scaling(self):
        """(D2, D1) of the Sec. 5 preprocessing, all instances concatenated."""
        ntot, mtot = int(self.var_off[-1]), int(self.row_off[-1])
        dv, dr = np.zeros(max(ntot, 1)), np.zeros(max(mtot, 1))
        B.check(self.lib.qp_get_scaling(self.h, dv.ctypes.data, dr.ctypes.data))
        return dv[:ntot], dr[:mtot]

    def set_norms(self, norm_A=None, norm_Q=None):
        a = None if norm_A is None else np.ascontiguousarray(norm_A, dtype=np.float64)
        q = None if norm_Q is None else np.ascontiguousarray(norm_Q, dtype=np.float64)
        B.check(self.lib.qp_set_norms(self.h, a.ctypes.data if a is not None else None,
                                      q.ctypes.data if q is not None else None))

    def autotune(self, sample: int = 64, iters: int = 256):
        out = np.zeros(4, dtype=np.int32)
        B.check(self.lib.qp_batch_autotune(self.h, int(sample), int(iters), out.ctypes.data))
        return [int(v) for v in out]

    def set_threads(self, threads):
        t = np.ascontiguousarray(threads, dtype=np.int32)
        B.check(self.lib.qp_batch_set_threads(self.h, t.ctypes.data))

    def solve(self, x0=None, y0=None, omega0=None):
        """x0/y0: concatenated warm starts (or None); omega0: per-instance array or None."""
        keep = _Keep(self.device_arrays)
        ntot, mtot = int(self.var_off[-1]), int(self.row_off[-1])
        ws_arr = None
        if x0 is not None or y0 is not None or omega0 is not None:
            ws_arr = (B.qp_warm_start * self.count)()
            xb = keep.ptr(x0, np.float64)
            yb = keep.ptr(y0, np.float64)
            esz = 8
            for i in range(self.count):
                ws_arr[i].x0 = (xb + esz * int(self.var_off[i])) if xb else None
                ws_arr[i].y0 = (yb + esz * int(self.row_off[i])) if yb else None
                ws_arr[i].omega0 = float(omega0[i]) if omega0 is not None else 0.0
        if self.device_arrays:
            import torch
            x = torch.empty(ntot, dtype=torch.float64, device="cuda")
            y = torch.empty(max(mtot, 1), dtype=torch.float64, device="cuda")
            torch.cuda.current_stream().synchronize()
            xp, yp = x.data_ptr(), y.data_ptr()
        else:
            x = np.zeros(ntot)
            y = np.zeros(max(mtot, 1))
            xp, yp = x.ctypes.data, y.ctypes.data
        res = (B.qp_result * self.count)()
        B.check(self.lib.qp_batch_solve(self.h, ws_arr, res, xp, yp))
        return x, y[:mtot], [_result_dict(res[i]) for i in range(self.count)]
