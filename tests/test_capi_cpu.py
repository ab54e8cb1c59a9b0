"""The C-ABI library loads on a GPU-less host and exports every entry point
that include/psl.h declares; argument checks that run before any device call
return PSL_ERR_INVALID. No compute call is made here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    text = open(os.path.join(ROOT, "include", "psl.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(psl_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("psl_presolve_create", "psl_presolve_run", "psl_postsolve", "psl_reduced_problem"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2609_16182_amd import psl
    if not os.path.exists(psl.LIB_PATH):
        pytest.fail("libpsl.so is not built: run `python -m paper_2609_16182_amd.build`")
    lib = psl.load()
    for name in declared():
        assert hasattr(lib, name), name


def test_struct_layouts():
    from paper_2609_16182_amd import psl
    assert psl.RECORD_DTYPE.itemsize == 48
    assert C.sizeof(psl.psl_lp) == 4 + 4 + 8 + 8 + 8 * 8 + 8
    s = psl.psl_settings_default()
    assert (s.max_rounds, s.max_outer, s.enable_parallel_rows) == (16, 4, 1)
    assert (s.feas_tol, s.fix_tol, s.min_improve, s.par_tol, s.inf_value, s.coef_tol) == \
        (1e-9, 1e-9, 1e-7, 1e-9, 1e20, 1e-9)


def test_defaults_match_the_oracle():
    from oracle import oracle as O
    from paper_2609_16182_amd import psl
    s = psl.psl_settings_default()
    for k, v in O.DEFAULTS.items():
        assert getattr(s, k) == v, k


def test_argument_errors_without_device():
    from paper_2609_16182_amd import psl
    lib = psl.load()
    h = C.c_void_p()
    s = psl.psl_settings_default()
    assert lib.psl_presolve_create(None, C.byref(s), C.byref(h)) == psl.PSL_ERR_INVALID
    lp = psl.psl_lp(-1, 2, 0, 0, None, None, None, None, None, None, None, None, 0.0)
    assert lib.psl_presolve_create(C.byref(lp), C.byref(s), C.byref(h)) == psl.PSL_ERR_INVALID
    assert "negative" in psl.psl_last_error(None)
    lp = psl.psl_lp(1, 1, 1, 0, None, None, None, None, None, None, None, None, 0.0)
    assert lib.psl_presolve_create(C.byref(lp), C.byref(s), C.byref(h)) == psl.PSL_ERR_INVALID
    # the size limits are checked before any array is read
    for dims, word in (((1, 1, 1 << 30), "nnz"), ((1 << 30, 1, 0), "m and n"), ((1, 1 << 30, 0), "m and n")):
        lp = psl.psl_lp(*dims, 0, None, None, None, None, None, None, None, None, 0.0)
        assert lib.psl_presolve_create(C.byref(lp), C.byref(s), C.byref(h)) == psl.PSL_ERR_INVALID
        assert psl.psl_last_error(None).startswith(word), psl.psl_last_error(None)
    lp = psl.psl_lp(1, 1, 1, 0, None, None, None, None, None, None, None, None, 0.0)
    assert lib.psl_presolve_create(C.byref(lp), C.byref(s), C.byref(h)) == psl.PSL_ERR_INVALID
    bad = psl.psl_settings_default()
    bad.max_rounds = 0
    arrs = []
    lp = psl.make_lp({"m": 0, "n": 0, **{k: np.zeros(1 if k == "row_ptr" else 0) for k in
                                          ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")}}, arrs)
    assert lib.psl_presolve_create(C.byref(lp), C.byref(bad), C.byref(h)) == psl.PSL_ERR_INVALID
    assert lib.psl_presolve_run(None, None, None) == psl.PSL_ERR_INVALID
