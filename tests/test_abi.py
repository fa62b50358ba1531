"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/qp.h, its struct layouts match the binding, defaults carry
the paper's constants, and malformed host input is rejected before any device
work (no compute call is made here)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import paper_2311_07710_amd as qpa
from paper_2311_07710_amd import _binding as B
from paper_2311_07710_amd.solver import Settings, _desc, _Keep
import qpgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qp.h")


def _declared_functions(header=HEADER):
    src = open(header).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qp_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = qpa.load()
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.SIGNATURES)
    mlp_names = _declared_functions(os.path.join(ROOT, "include", "qp_mlp.h"))
    assert set(mlp_names) == set(B.MLP_SIGNATURES)
    for n in mlp_names:
        assert hasattr(lib, n), n
    assert lib.qp_version() == B.ABI_VERSION == 2


def test_struct_layouts_match_header(tmp_path):
    structs = ["qp_csr", "qp_problem_desc", "qp_settings", "qp_warm_start", "qp_result",
               "qp_check_info", "qp_profile"]
    prog = tmp_path / "sz.c"
    body = "\n".join(f'printf("{s} %zu\\n", sizeof({s}));' for s in structs)
    offs = "\n".join(f'printf("off {s}.{f} %zu\\n", offsetof({s}, {f}));'
                     for s in ("qp_settings", "qp_result")
                     for f, _ in getattr(B, s)._fields_)
    prog.write_text(f'#include <stdio.h>\n#include <stddef.h>\n#include "{HEADER}"\n'
                    f"int main(void){{{body}\n{offs}\nreturn 0;}}\n")
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-std=c99", "-Wall", "-o", str(exe), str(prog)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        parts = line.split()
        if len(parts) == 2:
            got[parts[0]] = int(parts[1])
        elif len(parts) == 3:
            got[parts[1]] = int(parts[2])
    for s in structs:
        assert got[s] == C.sizeof(getattr(B, s)), s
    for s in ("qp_settings", "qp_result"):
        cls = getattr(B, s)
        for f, _ in cls._fields_:
            assert got[f"{s}.{f}"] == getattr(cls, f).offset, (s, f)


def test_default_settings_carry_paper_constants():
    lib = qpa.load()
    s = B.qp_settings()
    lib.qp_default_settings(C.byref(s))
    assert s.eps == 1e-6 and s.max_iter == 200000 and s.time_limit_s == 3600.0
    assert (s.beta_sufficient, s.beta_necessary, s.beta_artificial) == (0.2, 0.8, 0.36)
    assert s.pw_smoothing == 0.2 and s.step_safety == 0.99
    assert s.restart_mode == B.QP_RESTART_ADAPTIVE and s.check_every == 64
    py = Settings()
    for name, _ in B.qp_settings._fields_:
        if name in ("log_cb", "log_user"):
            assert not getattr(s, name), name   # NULL
            continue
        assert getattr(py, name) == getattr(s, name), name


def _create_rc(qp, **settings):
    lib = qpa.load()
    keep = _Keep(False)
    d = _desc(qp, keep, batch=False)
    h = C.c_void_p()
    rc = lib.qp_create(C.byref(d), C.byref(Settings(**settings).c_struct()), C.byref(h))
    if rc == 0:
        lib.qp_free(h)
    return rc, lib.qp_last_error().decode()


def _tiny():
    return qpgen.tiny_random_qp(1)


@pytest.mark.parametrize("mutate,needle", [
    (lambda q: q.a_rowptr.__setitem__(3, q.a_rowptr[4] + 1), "A.row_ptr decreases"),
    (lambda q: q.a_col.__setitem__(7, 100), "A.col_idx[7] = 100 out of range"),
    (lambda q: q.q_col.__setitem__(0, -1), "Q.col_idx[0] = -1"),
    (lambda q: q.row_type.__setitem__(2, 7), "row_type[2] = 7"),
    (lambda q: (q.l.__setitem__(5, 3.0), q.u.__setitem__(5, 2.0)), "invalid bounds at variable 5"),
    (lambda q: q.l.__setitem__(4, np.inf), "invalid bounds at variable 4"),
])
def test_malformed_input_rejected_on_host(mutate, needle):
    qp = _tiny()
    qp.a_rowptr = qp.a_rowptr.copy(); qp.a_col = qp.a_col.copy(); qp.q_col = qp.q_col.copy()
    qp.row_type = qp.row_type.copy(); qp.l = qp.l.copy(); qp.u = qp.u.copy()
    mutate(qp)
    rc, msg = _create_rc(qp)
    assert rc == B.QP_ERR_INVALID_ARGUMENT
    assert needle in msg


@pytest.mark.parametrize("kw,needle", [({"check_every": 0}, "check_every"),
                                       ({"restart_mode": 9}, "restart_mode"),
                                       ({"restart_mode": 1, "fixed_K": 0}, "fixed_K"),
                                       ({"eps": -1.0}, "eps"),
                                       ({"momentum": 2}, "momentum"),
                                       ({"beta_sufficient": 0.0}, "beta_sufficient"),
                                       ({"beta_necessary": 1.5}, "beta_necessary"),
                                       ({"beta_artificial": float("nan")}, "beta_artificial"),
                                       ({"pw_smoothing": -0.1}, "pw_smoothing"),
                                       ({"pw_smoothing": 1.01}, "pw_smoothing"),
                                       ({"eps_zero": -1.0}, "eps_zero"),
                                       ({"power_iter_max": 0}, "power_iter_max"),
                                       ({"power_iter_rtol": -1e-7}, "power_iter_rtol"),
                                       ({"step_safety": 0.0}, "step_safety"),
                                       ({"ruiz_iters": 101}, "ruiz_iters"),
                                       ({"eps_infeasible": 0.0}, "eps_infeasible")])
def test_bad_settings_rejected(kw, needle):
    rc, msg = _create_rc(_tiny(), **kw)
    assert rc == B.QP_ERR_INVALID_ARGUMENT and needle in msg


@pytest.mark.parametrize("field,value", [("n", 2**31 - 10), ("Q.nnz", 2**31), ("A.nnz", 2**31 - 1)])
def test_int32_index_range_rejected_before_reading(field, value):
    """Sizes beyond int32 indexing of P = [Q | -A'] are refused from the descriptor's
    sizes alone: the (small) arrays behind it are never read at those sizes."""
    lib = qpa.load()
    keep = _Keep(False)
    d = _desc(_tiny(), keep, batch=False)
    obj, _, attr = field.rpartition(".")
    setattr(getattr(d, obj) if obj else d, attr, value)
    h = C.c_void_p()
    rc = lib.qp_create(C.byref(d), C.byref(Settings().c_struct()), C.byref(h))
    assert rc == B.QP_ERR_INVALID_ARGUMENT
    assert "exceeds int32" in lib.qp_last_error().decode()


def test_null_arguments():
    lib = qpa.load()
    assert lib.qp_create(None, None, None) == B.QP_ERR_INVALID_ARGUMENT
    lib.qp_free(None)
    r = B.qp_result()
    assert lib.qp_solve(None, None, C.byref(r), None, None) == B.QP_ERR_INVALID_ARGUMENT
    assert "null" in lib.qp_last_error().decode()


@pytest.mark.parametrize("field", ["col_idx", "val"])
def test_null_matrix_arrays_rejected_on_host(field):
    """A null A.col_idx or A.val with A.nnz > 0 is an argument error, not a host crash."""
    lib = qpa.load()
    keep = _Keep(False)
    d = _desc(_tiny(), keep, batch=False)
    assert d.A.nnz > 0
    setattr(d.A, field, None)
    h = C.c_void_p()
    rc = lib.qp_create(C.byref(d), C.byref(Settings().c_struct()), C.byref(h))
    assert rc == B.QP_ERR_INVALID_ARGUMENT
    assert "A.col_idx and A.val are required" in lib.qp_last_error().decode()


def _batch_create_rc(batch, **settings):
    lib = qpa.load()
    keep = _Keep(False)
    d = _desc(batch, keep, batch=True)
    h = C.c_void_p()
    rc = lib.qp_create(C.byref(d), C.byref(Settings(**settings).c_struct()), C.byref(h))
    if rc == 0:
        lib.qp_free(h)
    return rc, lib.qp_last_error().decode()


def _small_batch():
    import dataclasses
    insts = [qpgen.tiny_random_qp(s, n=12, m=6, n_eq=3) for s in (1, 2, 3)]
    b = qpgen.concat_batch(insts)
    return dataclasses.replace(b, var_off=b.var_off.copy(), row_off=b.row_off.copy(),
                               a_col=b.a_col.copy(), q_col=b.q_col.copy(), l=b.l.copy(),
                               row_type=b.row_type.copy(), q_val=b.q_val.copy())


@pytest.mark.parametrize("mutate,code,needle", [
    (lambda b: b.var_off.__setitem__(1, b.var_off[2]), 4, "n_i > 0"),
    (lambda b: b.var_off.__setitem__(0, 1), 4, "do not span"),
    (lambda b: b.row_off.__setitem__(1, b.row_off[2] + 1), 4, "m_i >= 0"),
    (lambda b: b.a_col.__setitem__(0, 12), 1, "A column index outside its instance"),
    (lambda b: b.q_col.__setitem__(5, -1), 1, "Q column index outside its instance"),
    (lambda b: b.row_type.__setitem__(4, 3), 1, "row_type"),
    (lambda b: b.l.__setitem__(7, np.inf), 1, "invalid bounds at variable 7"),
])
def test_malformed_batch_rejected_on_host(mutate, code, needle):
    b = _small_batch()
    mutate(b)
    rc, msg = _batch_create_rc(b)
    assert rc == code and needle in msg, (rc, msg)


def test_asymmetric_q_rejected_when_checked():
    qp = _tiny()
    qp.q_val = qp.q_val.copy()
    # perturb one strictly off-diagonal entry only
    rows = np.repeat(np.arange(qp.n), np.diff(qp.q_rowptr))
    k = int(np.flatnonzero(rows != qp.q_col)[0])
    qp.q_val[k] += 1e-9
    rc, msg = _create_rc(qp, check_symmetry=1)
    assert rc == B.QP_ERR_INVALID_ARGUMENT and "not symmetric at" in msg
    b = _small_batch()
    rows = np.repeat(np.arange(int(b.var_off[-1])), np.diff(b.q_rowptr))
    loc = rows - np.repeat(b.var_off[:-1], np.diff(b.var_off))[rows]
    k = int(np.flatnonzero(loc != b.q_col)[-1])
    b.q_val[k] += 1.0
    rc, msg = _batch_create_rc(b, check_symmetry=1)
    assert rc == B.QP_ERR_INVALID_ARGUMENT and "instance 2 is not symmetric" in msg
