"""ctypes wrapper of the sequential CPU reference presolver (TEST INFRASTRUCTURE).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module; the GPU library never imports or links it. It compiles
``psl_oracle.c`` with gcc (-O2 -ffp-contract=off) when the shared object is
missing or older than its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "psl_oracle.c")
LIB = os.path.join(HERE, "libpsl_oracle.so")

RECORD_DTYPE = np.dtype([
    ("type", "u1"), ("side", "u1"), ("round", "<u2"),
    ("i", "<i4"), ("j", "<i4"), ("k", "<i4"), ("v", "<f8", (4,)),
])
assert RECORD_DTYPE.itemsize == 48

REC_NAMES = {1: "FIX_COL", 2: "EMPTY_COL", 3: "EMPTY_ROW", 4: "REDUNDANT_ROW",
             5: "SINGLETON_ROW", 6: "BOUND_CHANGE", 7: "PARALLEL_ROW", 8: "LEADER_SIDES",
             9: "DUAL_FIX", 10: "FREE_SINGLETON", 11: "PARALLEL_COL", 12: "LEADER_BOUNDS",
             13: "FORCING_ROW", 14: "DOUBLETON_ROW", 15: "DOMINATED_COL"}
REC = {v: k for k, v in REC_NAMES.items()}
RESULT_NAMES = {0: "REDUCED", 1: "UNCHANGED", 2: "INFEASIBLE", 3: "UNBOUNDED_OR_INFEASIBLE"}

# default settings (the round semantics depend on them; the GPU library uses
# the same defaults)
DEFAULTS = dict(max_rounds=16, max_outer=4, enable_parallel_rows=1,
                feas_tol=1e-9, fix_tol=1e-9, min_improve=1e-7, par_tol=1e-9,
                inf_value=1e20, coef_tol=1e-9, enable_dual_fix=0, enable_free_singletons=0,
                enable_parallel_cols=0, enable_forcing_rows=0, enable_doubletons=0, enable_dominated=0)


class _LP(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("lhs", C.c_void_p), ("rhs", C.c_void_p), ("lb", C.c_void_p),
                ("ub", C.c_void_p), ("c", C.c_void_p), ("obj_offset", C.c_double)]


class _Settings(C.Structure):
    _fields_ = [("max_rounds", C.c_int32), ("max_outer", C.c_int32),
                ("enable_parallel_rows", C.c_int32),
                ("feas_tol", C.c_double), ("fix_tol", C.c_double),
                ("min_improve", C.c_double), ("par_tol", C.c_double),
                ("inf_value", C.c_double), ("coef_tol", C.c_double),
                ("enable_dual_fix", C.c_int32), ("enable_free_singletons", C.c_int32),
                ("enable_parallel_cols", C.c_int32), ("enable_forcing_rows", C.c_int32),
                ("enable_doubletons", C.c_int32), ("enable_dominated", C.c_int32)]


def build(force=False, extra_flags=()):
    """Compile the oracle; ``extra_flags`` (e.g. -D defines) go to a separate
    output file so that the default library is never replaced by a variant."""
    out = LIB
    if extra_flags:
        tag = "_".join(f.strip("-").replace("=", "") for f in extra_flags)
        out = os.path.join(HERE, f"libpsl_oracle_{tag}.so")
    if (not force and os.path.exists(out)
            and os.path.getmtime(out) >= os.path.getmtime(SRC)
            and os.path.getmtime(out) >= os.path.getmtime(os.path.join(HERE, "psl_oracle.h"))):
        return out
    tmp = out + f".tmp{os.getpid()}"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
           "-shared", "-Wall", "-Wextra", *extra_flags, "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_libs = {}


def _load(path=None):
    path = path or build()
    if path in _libs:
        return _libs[path]
    lib = C.CDLL(path)
    lib.or_presolve.argtypes = [C.POINTER(_LP), C.POINTER(_Settings), C.POINTER(C.c_void_p)]
    lib.or_presolve.restype = C.c_int
    lib.or_free.argtypes = [C.c_void_p]
    lib.or_error.argtypes = [C.c_void_p]
    lib.or_error.restype = C.c_char_p
    for name in ("or_result", "or_rounds"):
        getattr(lib, name).argtypes = [C.c_void_p]
        getattr(lib, name).restype = C.c_int32
    lib.or_num_records.argtypes = [C.c_void_p]
    lib.or_num_records.restype = C.c_int64
    lib.or_records.argtypes = [C.c_void_p]
    lib.or_records.restype = C.c_void_p
    lib.or_reduced_dims.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                    C.POINTER(C.c_int64), C.POINTER(C.c_double)]
    lib.or_reduced_copy.argtypes = [C.c_void_p] + [C.c_void_p] * 15
    lib.or_postsolve.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
    lib.or_postsolve.restype = C.c_int
    lib.or_postsolve_dual.argtypes = [C.c_void_p] + [C.c_void_p] * 5
    lib.or_postsolve_dual.restype = C.c_int
    lib.or_pairwise_sum.argtypes = [C.c_void_p, C.c_int64]
    lib.or_pairwise_sum.restype = C.c_double
    lib.or_row_key.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
    lib.or_row_key.restype = C.c_uint64
    lib.or_activities.argtypes = [C.POINTER(_LP)] + [C.c_void_p] * 4
    lib.or_activities.restype = C.c_int
    _libs[path] = lib
    return lib


def _ptr(a):
    return a.ctypes.data if a is not None and a.size else None


class OracleError(RuntimeError):
    pass


class Result:
    """Outputs of one oracle presolve, copied into numpy arrays."""

    def __init__(self, lib, h):
        self.result = lib.or_result(h)
        self.result_name = RESULT_NAMES[self.result]
        self.rounds = lib.or_rounds(h)
        nrec = lib.or_num_records(h)
        if nrec:
            buf = (C.c_char * (nrec * 48)).from_address(lib.or_records(h))
            self.records = np.frombuffer(bytes(buf), dtype=RECORD_DTYPE).copy()
        else:
            self.records = np.zeros(0, RECORD_DTYPE)
        self.reduced = None
        if self.result in (0, 1):
            m, n, nnz, off = C.c_int32(), C.c_int32(), C.c_int64(), C.c_double()
            lib.or_reduced_dims(h, C.byref(m), C.byref(n), C.byref(nnz), C.byref(off))
            m, n, nnz = m.value, n.value, nnz.value
            r = dict(m=m, n=n, nnz=nnz, obj_offset=off.value,
                     row_ptr=np.zeros(m + 1, np.int32), col_idx=np.zeros(nnz, np.int32),
                     val=np.zeros(nnz), col_ptr=np.zeros(n + 1, np.int32),
                     row_idx=np.zeros(nnz, np.int32), cval=np.zeros(nnz),
                     lhs=np.zeros(m), rhs=np.zeros(m), lb=np.zeros(n), ub=np.zeros(n),
                     c=np.zeros(n), row_map=np.zeros(m, np.int32), col_map=np.zeros(n, np.int32),
                     row_class=np.zeros(m, np.uint8), col_class=np.zeros(n, np.uint8))
            keys = ["row_ptr", "col_idx", "val", "col_ptr", "row_idx", "cval", "lhs", "rhs",
                    "lb", "ub", "c", "row_map", "col_map", "row_class", "col_class"]
            lib.or_reduced_copy(h, *[r[k].ctypes.data for k in keys])
            self.reduced = r
        self._lib = lib
        self._h = h

    def postsolve(self, x_red):
        x_red = np.ascontiguousarray(x_red, np.float64)
        n = self.n_orig
        x = np.zeros(n)
        if self._lib.or_postsolve(self._h, _ptr(x_red), _ptr(x) if n else None):
            raise OracleError("postsolve needs a reduced problem")
        return x

    def postsolve_dual(self, x_red, y_red):
        """(x, y, z) of the original LP from the reduced problem's primal
        solution and row duals (z = c - A'y)."""
        x_red = np.ascontiguousarray(x_red, np.float64)
        y_red = np.ascontiguousarray(y_red, np.float64)
        n, m = self.n_orig, self.m_orig
        x, y, z = np.zeros(n), np.zeros(m), np.zeros(n)
        if self._lib.or_postsolve_dual(self._h, _ptr(x_red), _ptr(y_red), _ptr(x), _ptr(y), _ptr(z)):
            raise OracleError("postsolve needs a reduced problem")
        return x, y, z

    def close(self):
        if self._h:
            self._lib.or_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def presolve(lp, lib_path=None, **settings):
    """Run the oracle on an LP dict (see the generators) and return a Result."""
    lib = _load(lib_path)
    s = dict(DEFAULTS)
    s.update(settings)
    arrs = {
        "row_ptr": np.ascontiguousarray(lp["row_ptr"], np.int32),
        "col_idx": np.ascontiguousarray(lp["col_idx"], np.int32),
        "val": np.ascontiguousarray(lp["val"], np.float64),
        "lhs": np.ascontiguousarray(lp["lhs"], np.float64),
        "rhs": np.ascontiguousarray(lp["rhs"], np.float64),
        "lb": np.ascontiguousarray(lp["lb"], np.float64),
        "ub": np.ascontiguousarray(lp["ub"], np.float64),
        "c": np.ascontiguousarray(lp["c"], np.float64),
    }
    m, n = int(lp["m"]), int(lp["n"])
    nnz = int(arrs["row_ptr"][-1]) if m else 0
    clp = _LP(m, n, nnz, _ptr(arrs["row_ptr"]), _ptr(arrs["col_idx"]), _ptr(arrs["val"]),
              _ptr(arrs["lhs"]), _ptr(arrs["rhs"]), _ptr(arrs["lb"]), _ptr(arrs["ub"]),
              _ptr(arrs["c"]), float(lp.get("obj_offset", 0.0)))
    cs = _Settings(int(s["max_rounds"]), int(s["max_outer"]), int(s["enable_parallel_rows"]),
                   s["feas_tol"], s["fix_tol"], s["min_improve"], s["par_tol"],
                   s["inf_value"], s["coef_tol"], int(s["enable_dual_fix"]), int(s["enable_free_singletons"]),
                   int(s["enable_parallel_cols"]), int(s["enable_forcing_rows"]), int(s["enable_doubletons"]),
                   int(s["enable_dominated"]))
    h = C.c_void_p()
    st = lib.or_presolve(C.byref(clp), C.byref(cs), C.byref(h))
    if st != 0:
        msg = lib.or_error(h).decode()
        lib.or_free(h)
        raise OracleError(msg)
    res = Result(lib, h)
    res.n_orig = n
    res.m_orig = m
    return res


def _clp(lp):
    arrs = {k: np.ascontiguousarray(lp[k], np.int32 if k in ("row_ptr", "col_idx") else np.float64)
            for k in ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")}
    m, n = int(lp["m"]), int(lp["n"])
    nnz = int(arrs["row_ptr"][-1]) if m else 0
    clp = _LP(m, n, nnz, *[_ptr(arrs[k]) for k in ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")],
              float(lp.get("obj_offset", 0.0)))
    return clp, arrs


def activities(lp, lib_path=None):
    """Round-1 (minact, maxact, ninf_min, ninf_max) of every row."""
    clp, keep = _clp(lp)
    m = int(lp["m"])
    out = [np.zeros(m), np.zeros(m), np.zeros(m, np.int32), np.zeros(m, np.int32)]
    _load(lib_path).or_activities(C.byref(clp), *[_ptr(a) for a in out])
    return tuple(out)


def pairwise_sum(x, lib_path=None):
    x = np.ascontiguousarray(x, np.float64)
    return _load(lib_path).or_pairwise_sum(_ptr(x), len(x))


def row_key(cols, vals, lib_path=None):
    cols = np.ascontiguousarray(cols, np.int32)
    vals = np.ascontiguousarray(vals, np.float64)
    return _load(lib_path).or_row_key(_ptr(cols), _ptr(vals), len(cols))
