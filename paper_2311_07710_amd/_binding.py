"""ctypes binding of ``lib/libqp_mi355x.so`` (declarations in include/qp.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Arrays are numpy (host memory) or torch CUDA tensors (device memory,
``mem_space = QP_MEM_DEVICE``); torch is used for nothing but memory and
streams.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libqp_mi355x.so")

QP_OK = 0
QP_ERR_INVALID_ARGUMENT = 1
QP_ERR_OUT_OF_MEMORY = 2
QP_ERR_DEVICE = 3
QP_ERR_BATCH_MISMATCH = 4
QP_ERR_UNSUPPORTED = 5

QP_OPTIMAL, QP_ITERATION_LIMIT, QP_TIME_LIMIT, QP_NUMERICAL_ERROR = 0, 1, 2, 3
QP_PRIMAL_INFEASIBLE, QP_DUAL_INFEASIBLE = 4, 5
QP_RESTART_ADAPTIVE, QP_RESTART_FIXED_K, QP_RESTART_HALVING, QP_RESTART_NONE = 0, 1, 2, 3
QP_MEM_HOST, QP_MEM_DEVICE = 0, 1

_vp = C.c_void_p


class qp_csr(C.Structure):
    _fields_ = [("row_ptr", _vp), ("col_idx", _vp), ("val", _vp), ("nnz", C.c_int64)]


class qp_problem_desc(C.Structure):
    _fields_ = [("n", C.c_int64), ("m", C.c_int64), ("num_instances", C.c_int32),
                ("mem_space", C.c_int32), ("Q", qp_csr), ("A", qp_csr), ("c", _vp), ("b", _vp),
                ("l", _vp), ("u", _vp), ("row_type", _vp), ("var_off", _vp), ("row_off", _vp),
                ("stream", _vp)]


class qp_check_info(C.Structure):
    _fields_ = [("total", C.c_int64), ("k", C.c_int64), ("r_cur", C.c_double),
                ("r_avg", C.c_double), ("candidate", C.c_int32), ("restarted", C.c_int32),
                ("omega", C.c_double)]


qp_log_fn = C.CFUNCTYPE(None, C.POINTER(qp_check_info), C.c_void_p)


class qp_settings(C.Structure):
    _fields_ = [("eps", C.c_double), ("max_iter", C.c_int64), ("time_limit_s", C.c_double),
                ("check_every", C.c_int32), ("restart_mode", C.c_int32), ("fixed_K", C.c_int32),
                ("beta_sufficient", C.c_double), ("beta_necessary", C.c_double),
                ("beta_artificial", C.c_double), ("pw_smoothing", C.c_double),
                ("eps_zero", C.c_double), ("step_safety", C.c_double), ("norm_A", C.c_double),
                ("norm_Q", C.c_double), ("power_iter_max", C.c_int32),
                ("power_iter_rtol", C.c_double), ("warm_fallback", C.c_int32),
                ("use_graph", C.c_int32), ("profile", C.c_int32), ("log_checks", C.c_int32),
                ("device", C.c_int32), ("panels_dual", C.c_int32), ("panels_primal", C.c_int32),
                ("momentum", C.c_int32), ("precondition", C.c_int32), ("ruiz_iters", C.c_int32),
                ("detect_infeasibility", C.c_int32), ("eps_infeasible", C.c_double),
                ("check_symmetry", C.c_int32), ("log_cb", qp_log_fn), ("log_user", _vp)]


class qp_warm_start(C.Structure):
    _fields_ = [("x0", _vp), ("y0", _vp), ("omega0", C.c_double)]


class qp_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("used_warm_start", C.c_int32), ("iterations", C.c_int64),
                ("restarts", C.c_int64), ("kkt_evals", C.c_int64), ("rel_kkt", C.c_double),
                ("r_primal", C.c_double), ("r_dual", C.c_double), ("r_gap", C.c_double),
                ("primal_obj", C.c_double), ("dual_obj", C.c_double), ("omega", C.c_double),
                ("norm_A", C.c_double), ("norm_Q", C.c_double), ("solve_time_s", C.c_double),
                ("start_s", C.c_double), ("end_s", C.c_double)]


class qp_profile(C.Structure):
    _fields_ = [("dual_launches", C.c_int64), ("primal_launches", C.c_int64),
                ("dual_ms", C.c_double), ("primal_ms", C.c_double),
                ("dual_bytes", C.c_double), ("primal_bytes", C.c_double)]


# every function declared in include/qp.h, with its ctypes signature
SIGNATURES = {
    "qp_default_settings": (None, [C.POINTER(qp_settings)]),
    "qp_create": (C.c_int, [C.POINTER(qp_problem_desc), C.POINTER(qp_settings), C.POINTER(_vp)]),
    "qp_solve": (C.c_int, [_vp, C.POINTER(qp_warm_start), C.POINTER(qp_result), _vp, _vp]),
    "qp_batch_solve": (C.c_int, [_vp, C.POINTER(qp_warm_start), C.POINTER(qp_result), _vp, _vp]),
    "qp_get_check_log": (C.c_int, [_vp, C.POINTER(qp_check_info), C.c_int64,
                                   C.POINTER(C.c_int64)]),
    "qp_get_profile": (C.c_int, [_vp, C.POINTER(qp_profile)]),
    "qp_get_norms": (C.c_int, [_vp, _vp, _vp]),
    "qp_get_scaling": (C.c_int, [_vp, _vp, _vp]),
    "qp_update_vectors": (C.c_int, [_vp, _vp, _vp]),
    "qp_set_norms": (C.c_int, [_vp, _vp, _vp]),
    "qp_batch_autotune": (C.c_int, [_vp, C.c_int32, C.c_int32, _vp]),
    "qp_batch_set_threads": (C.c_int, [_vp, _vp]),
    "qp_free": (None, [_vp]),
    "qp_last_error": (C.c_char_p, []),
    "qp_version": (C.c_int, []),
}

# every function declared in include/qp_mlp.h
MLP_SIGNATURES = {
    "qp_mlp_create": (C.c_int, [C.c_int32, _vp, C.c_int32, C.c_int32, C.POINTER(_vp)]),
    "qp_mlp_free": (None, [_vp]),
    "qp_mlp_num_params": (C.c_int64, [_vp]),
    "qp_mlp_set_params": (C.c_int, [_vp, _vp]),
    "qp_mlp_get_params": (C.c_int, [_vp, _vp]),
    "qp_mlp_get_grads": (C.c_int, [_vp, _vp]),
    "qp_mlp_set_grads": (C.c_int, [_vp, _vp]),
    "qp_mlp_forward": (C.c_int, [_vp, _vp, C.c_int32, _vp]),
    "qp_mlp_forward_rows": (C.c_int, [_vp, _vp, C.c_int64, _vp, C.c_int32, _vp]),
    "qp_mlp_forward_noalloc": (C.c_int, [_vp, _vp, C.c_int32, _vp]),
    "qp_mlp_backward": (C.c_int, [_vp, _vp, C.c_int32, C.POINTER(C.c_float)]),
    "qp_mlp_backward_rows": (C.c_int, [_vp, _vp, C.c_int64, _vp, C.c_int32,
                                       C.POINTER(C.c_float)]),
    "qp_mlp_adam_step": (C.c_int, [_vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32]),
}

_lib = None
ABI_VERSION = 2  # QP_ABI_VERSION of include/qp.h (qp_result gained start_s, end_s)


def load():
    """Load the HIP library; raises if it has not been built (no CPU fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in {**SIGNATURES, **MLP_SIGNATURES}.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        if lib.qp_version() != ABI_VERSION:
            raise RuntimeError(f"{LIB_PATH} has ABI version {lib.qp_version()}, this binding "
                               f"expects {ABI_VERSION}: rebuild the library")
        _lib = lib
    return _lib


class QPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc: int):
    if rc != QP_OK:
        raise QPError(rc, load().qp_last_error().decode())
