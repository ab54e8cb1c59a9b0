"""Thin ctypes binding of libpsl (include/psl.h): argument marshalling only.

Every presolve step runs in the library's HIP kernels. PyTorch, when used,
only provides device memory and the stream. Loading fails loudly when
libpsl.so has not been built (python -m paper_2609_16182_amd.build).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsl.so")

PSL_OK, PSL_ERR_INVALID, PSL_ERR_OOM, PSL_ERR_DEVICE, PSL_ERR_STATE, PSL_ERR_CAPACITY, PSL_ERR_UNSUPPORTED = range(7)
STATUS_NAMES = ["OK", "INVALID", "OOM", "DEVICE", "STATE", "CAPACITY", "UNSUPPORTED"]
RESULT_NAMES = {0: "REDUCED", 1: "UNCHANGED", 2: "INFEASIBLE", 3: "UNBOUNDED_OR_INFEASIBLE"}
PSL_MEM_HOST, PSL_MEM_DEVICE = 0, 1

RECORD_DTYPE = np.dtype([
    ("type", "u1"), ("side", "u1"), ("round", "<u2"),
    ("i", "<i4"), ("j", "<i4"), ("k", "<i4"), ("v", "<f8", (4,)),
])
REC_NAMES = {1: "FIX_COL", 2: "EMPTY_COL", 3: "EMPTY_ROW", 4: "REDUNDANT_ROW",
             5: "SINGLETON_ROW", 6: "BOUND_CHANGE", 7: "PARALLEL_ROW", 8: "LEADER_SIDES",
             9: "DUAL_FIX", 10: "FREE_SINGLETON", 11: "PARALLEL_COL", 12: "LEADER_BOUNDS",
             13: "FORCING_ROW", 14: "DOUBLETON_ROW", 15: "DOMINATED_COL"}


class psl_lp(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64), ("mem", C.c_int),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("lhs", C.c_void_p), ("rhs", C.c_void_p), ("lb", C.c_void_p), ("ub", C.c_void_p),
                ("c", C.c_void_p), ("obj_offset", C.c_double)]


class psl_settings(C.Structure):
    _fields_ = [("max_rounds", C.c_int32), ("max_outer", C.c_int32), ("enable_parallel_rows", C.c_int32),
                ("feas_tol", C.c_double), ("fix_tol", C.c_double), ("min_improve", C.c_double),
                ("par_tol", C.c_double), ("inf_value", C.c_double), ("coef_tol", C.c_double),
                ("bin_thresholds", C.c_void_p), ("n_bins", C.c_int32), ("device", C.c_int32),
                ("stream", C.c_void_p), ("split_sweep", C.c_int32), ("enable_dual_fix", C.c_int32),
                ("enable_free_singletons", C.c_int32), ("enable_parallel_cols", C.c_int32),
                ("enable_forcing_rows", C.c_int32), ("enable_doubletons", C.c_int32),
                ("device_records", C.c_int64), ("enable_dominated", C.c_int32)]


class psl_stats(C.Structure):
    _fields_ = [("rounds", C.c_int32), ("outer_cycles", C.c_int32), ("records", C.c_int64),
                ("nnz_in", C.c_int64), ("nnz_out", C.c_int64), ("m_out", C.c_int32), ("n_out", C.c_int32),
                ("ms_ingest", C.c_double), ("ms_sweep", C.c_double), ("ms_decide", C.c_double),
                ("ms_parallel", C.c_double), ("ms_compact", C.c_double), ("ms_total", C.c_double),
                ("sweep_launches", C.c_int64), ("sweep_bytes", C.c_double), ("ms_long", C.c_double),
                ("alg_bytes", C.c_double), ("ingest_bytes", C.c_double), ("sweep_nnz", C.c_int64),
                ("record_flushes", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class psl_reduced_view(C.Structure):
    _fields_ = [("m", C.c_int32), ("n", C.c_int32), ("nnz", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("cval", C.c_void_p),
                ("lhs", C.c_void_p), ("rhs", C.c_void_p), ("lb", C.c_void_p), ("ub", C.c_void_p),
                ("c", C.c_void_p), ("obj_offset", C.c_double),
                ("row_map", C.c_void_p), ("col_map", C.c_void_p),
                ("row_class", C.c_void_p), ("col_class", C.c_void_p)]


class psl_tuning(C.Structure):
    _fields_ = [("bin_thresholds", C.c_int32 * 3), ("split_sweep", C.c_int32), ("candidates", C.c_int32),
                ("ms_best", C.c_double), ("ms_default", C.c_double)]


class psl_server_config(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_size_t), ("slots", C.c_int32), ("threaded", C.c_int32),
                ("max_batch_lps", C.c_int32), ("max_batch_rows", C.c_int32), ("max_batch_cols", C.c_int32),
                ("max_batch_nnz", C.c_int64), ("keep_original", C.c_int32)]


class psl_ticket_info(C.Structure):
    _fields_ = [("status", C.c_int), ("result", C.c_int), ("queue_ms", C.c_double), ("latency_ms", C.c_double),
                ("batch_lps", C.c_int32), ("slot", C.c_int32), ("stats", psl_stats)]


class psl_noalloc_out(C.Structure):
    _fields_ = [("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val", C.c_void_p),
                ("col_ptr", C.c_void_p), ("row_idx", C.c_void_p), ("cval", C.c_void_p),
                ("lhs", C.c_void_p), ("rhs", C.c_void_p), ("lb", C.c_void_p), ("ub", C.c_void_p),
                ("c", C.c_void_p), ("row_map", C.c_void_p), ("col_map", C.c_void_p),
                ("row_class", C.c_void_p), ("col_class", C.c_void_p),
                ("records", C.c_void_p), ("records_cap", C.c_int64),
                ("m_out", C.c_int32), ("n_out", C.c_int32), ("nnz_out", C.c_int64),
                ("obj_offset", C.c_double), ("records_out", C.c_int64)]


class PslError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES[status] if 0 <= status < 7 else status}: {msg}")
        self.status = status


_lib = None
_hip = None


def load(path=None):
    """Load libpsl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2609_16182_amd.build`")
    lib = C.CDLL(path)
    lib.psl_settings_default.argtypes = [C.POINTER(psl_settings)]
    lib.psl_settings_default.restype = None
    lib.psl_presolve_create.argtypes = [C.POINTER(psl_lp), C.POINTER(psl_settings), C.POINTER(C.c_void_p)]
    lib.psl_presolve_reload.argtypes = [C.c_void_p, C.POINTER(psl_lp)]
    lib.psl_presolve_run.argtypes = [C.c_void_p, C.POINTER(C.c_int), C.POINTER(psl_stats)]
    lib.psl_reduced_problem.argtypes = [C.c_void_p, C.POINTER(psl_reduced_view)]
    lib.psl_records.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_void_p, C.c_int64]
    lib.psl_postsolve.argtypes = [C.c_void_p] + [C.c_void_p] * 6
    lib.psl_presolve_free.argtypes = [C.c_void_p]
    lib.psl_presolve_free.restype = None
    lib.psl_last_error.argtypes = [C.c_void_p]
    lib.psl_last_error.restype = C.c_char_p
    lib.psl_batch_create.argtypes = [C.c_int32, C.c_void_p, C.POINTER(psl_settings), C.POINTER(C.c_void_p)]
    lib.psl_batch_reload.argtypes = [C.c_void_p, C.c_int32, C.c_void_p]
    lib.psl_batch_run.argtypes = [C.c_void_p, C.c_void_p, C.POINTER(psl_stats)]
    lib.psl_batch_stats.argtypes = [C.c_void_p, C.c_int32, C.POINTER(psl_stats)]
    lib.psl_batch_reduced_problem.argtypes = [C.c_void_p, C.c_int32, C.POINTER(psl_reduced_view)]
    lib.psl_batch_records.argtypes = [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.c_void_p, C.c_int64]
    lib.psl_batch_postsolve.argtypes = [C.c_void_p, C.c_int32] + [C.c_void_p] * 6
    lib.psl_presolve_noalloc.argtypes = [C.POINTER(psl_lp), C.POINTER(psl_settings), C.POINTER(psl_noalloc_out),
                                         C.POINTER(C.c_int), C.POINTER(psl_stats)]
    lib.psl_presolve_noalloc.restype = C.c_int
    lib.psl_tune.argtypes = [C.c_int32, C.c_void_p, C.POINTER(psl_settings), C.c_int32, C.POINTER(psl_tuning)]
    lib.psl_tune.restype = C.c_int
    lib.psl_batch_free.argtypes = [C.c_void_p]
    lib.psl_batch_free.restype = None
    lib.psl_batch_last_error.argtypes = [C.c_void_p]
    lib.psl_batch_last_error.restype = C.c_char_p
    lib.psl_server_config_default.argtypes = [C.POINTER(psl_server_config)]
    lib.psl_server_config_default.restype = None
    lib.psl_server_create.argtypes = [C.POINTER(psl_server_config), C.POINTER(psl_settings), C.POINTER(C.c_void_p)]
    lib.psl_server_submit.argtypes = [C.c_void_p, C.POINTER(psl_lp), C.POINTER(C.c_uint64)]
    lib.psl_server_step.argtypes = [C.c_void_p, C.POINTER(C.c_int32)]
    lib.psl_server_poll.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_int32)]
    lib.psl_server_wait.argtypes = [C.c_void_p, C.c_uint64, C.c_double]
    lib.psl_server_info.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(psl_ticket_info)]
    lib.psl_server_reduced_problem.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(psl_reduced_view)]
    lib.psl_server_records.argtypes = [C.c_void_p, C.c_uint64, C.POINTER(C.c_int64), C.c_void_p, C.c_int64]
    lib.psl_server_postsolve.argtypes = [C.c_void_p, C.c_uint64] + [C.c_void_p] * 6
    lib.psl_server_release.argtypes = [C.c_void_p, C.c_uint64]
    lib.psl_server_drain.argtypes = [C.c_void_p]
    lib.psl_server_memory.argtypes = [C.c_void_p] + [C.POINTER(C.c_size_t)] * 4
    lib.psl_server_memory.restype = C.c_int
    lib.psl_server_free.argtypes = [C.c_void_p]
    lib.psl_server_free.restype = None
    lib.psl_server_last_error.argtypes = [C.c_void_p]
    lib.psl_server_last_error.restype = C.c_char_p
    for f in ("psl_presolve_create", "psl_presolve_reload", "psl_presolve_run", "psl_reduced_problem",
              "psl_records", "psl_postsolve", "psl_batch_create", "psl_batch_reload", "psl_batch_run",
              "psl_batch_stats", "psl_batch_reduced_problem", "psl_batch_records", "psl_batch_postsolve",
              "psl_server_create", "psl_server_submit", "psl_server_step", "psl_server_poll", "psl_server_wait",
              "psl_server_info", "psl_server_reduced_problem", "psl_server_records", "psl_server_postsolve",
              "psl_server_release", "psl_server_drain"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _hiprt():
    """HIP runtime (already loaded by libpsl) for device-to-host copies."""
    global _hip
    if _hip is None:
        _hip = C.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.hipMemcpy.restype = C.c_int
    return _hip


def _check(st, h=None):
    if st != PSL_OK:
        raise PslError(st, load().psl_last_error(h).decode())


def _bcheck(st, b=None):
    if st != PSL_OK:
        raise PslError(st, load().psl_batch_last_error(b).decode())


def _scheck(st, sv=None):
    if st != PSL_OK:
        raise PslError(st, load().psl_server_last_error(sv).decode())


# ---------------------------------------------------------------------------
# the C-ABI, one Python function per entry point
# ---------------------------------------------------------------------------

def psl_settings_default():
    s = psl_settings()
    load().psl_settings_default(C.byref(s))
    return s


def psl_presolve_create(lp: psl_lp, settings: psl_settings):
    h = C.c_void_p()
    _check(load().psl_presolve_create(C.byref(lp), C.byref(settings), C.byref(h)))
    return h


def psl_presolve_reload(h, lp: psl_lp):
    _check(load().psl_presolve_reload(h, C.byref(lp)), h)


def psl_presolve_run(h):
    res = C.c_int()
    st = psl_stats()
    _check(load().psl_presolve_run(h, C.byref(res), C.byref(st)), h)
    return res.value, st


def psl_reduced_problem(h):
    v = psl_reduced_view()
    _check(load().psl_reduced_problem(h, C.byref(v)), h)
    return v


def psl_records(h):
    cnt = C.c_int64()
    _check(load().psl_records(h, C.byref(cnt), None, 0), h)
    out = np.zeros(cnt.value, RECORD_DTYPE)
    if cnt.value:
        _check(load().psl_records(h, C.byref(cnt), out.ctypes.data, cnt.value), h)
    return out


def _post_args(x_red, y_red, m, n):
    """Host arrays of a postsolve call: the argument pointers (x_red, y_red,
    z_red, x, y, z) and the outputs (x, or x, y, z when y_red is given)."""
    x_red = np.ascontiguousarray(x_red, np.float64)
    x = np.zeros(n)
    keep = [x_red]
    args = [x_red.ctypes.data if x_red.size else None, None, None, x.ctypes.data if n else None, None, None]
    if y_red is None:
        return args, keep, (x,)
    y_red = np.ascontiguousarray(y_red, np.float64)
    y, z = np.zeros(m), np.zeros(n)
    keep.append(y_red)
    # a non-null y_red asks for the dual pass even when the reduced LP has no rows
    y_buf = y_red if y_red.size else np.zeros(1)
    keep.append(y_buf)
    args[1] = y_buf.ctypes.data
    args[4] = y.ctypes.data if m else None
    args[5] = z.ctypes.data if n else None
    return args, keep, (x, y, z)


def psl_postsolve(h, x_red, n, y_red=None, m=0):
    """x, or (x, y, z) with y_red (row duals of the reduced LP; m rows)."""
    args, keep, out = _post_args(x_red, y_red, m, n)
    _check(load().psl_postsolve(h, *args), h)
    return out[0] if len(out) == 1 else out


def psl_presolve_noalloc(lp: psl_lp, settings: psl_settings, out: psl_noalloc_out):
    """One presolve in the library's static device scratch; results go into
    the caller's device buffers named in `out`. Returns (result, stats)."""
    res = C.c_int(0)
    st = psl_stats()
    _check(load().psl_presolve_noalloc(C.byref(lp), C.byref(settings), C.byref(out), C.byref(res), C.byref(st)))
    return res.value, st


def psl_presolve_free(h):
    if h:
        load().psl_presolve_free(h)


def psl_last_error(h=None):
    return load().psl_last_error(h).decode()


def lp_array(lps):
    """ctypes array of psl_lp structs (reusable across reloads)."""
    if isinstance(lps, C.Array):
        return lps
    return (psl_lp * len(lps))(*lps)


def psl_batch_create(lps, settings: psl_settings):
    arr = lp_array(lps)
    b = C.c_void_p()
    _bcheck(load().psl_batch_create(len(arr), C.cast(arr, C.c_void_p), C.byref(settings), C.byref(b)))
    return b


def psl_batch_reload(b, lps):
    arr = lp_array(lps)
    _bcheck(load().psl_batch_reload(b, len(arr), C.cast(arr, C.c_void_p)), b)


def psl_batch_run(b, k):
    res = (C.c_int * k)()
    st = psl_stats()
    _bcheck(load().psl_batch_run(b, C.cast(res, C.c_void_p), C.byref(st)), b)
    return list(res), st


def psl_batch_stats(b, idx):
    st = psl_stats()
    _bcheck(load().psl_batch_stats(b, idx, C.byref(st)), b)
    return st


def psl_batch_reduced_problem(b, idx):
    v = psl_reduced_view()
    _bcheck(load().psl_batch_reduced_problem(b, idx, C.byref(v)), b)
    return v


def psl_batch_records(b, idx):
    cnt = C.c_int64()
    _bcheck(load().psl_batch_records(b, idx, C.byref(cnt), None, 0), b)
    out = np.zeros(cnt.value, RECORD_DTYPE)
    if cnt.value:
        _bcheck(load().psl_batch_records(b, idx, C.byref(cnt), out.ctypes.data, cnt.value), b)
    return out


def psl_batch_postsolve(b, idx, x_red, n, y_red=None, m=0):
    args, keep, out = _post_args(x_red, y_red, m, n)
    _bcheck(load().psl_batch_postsolve(b, idx, *args), b)
    return out[0] if len(out) == 1 else out


def psl_tune(lps, settings: psl_settings, reps=3):
    """Time candidate launch shapes on these LPs; returns a dict with the
    fastest (bin_thresholds, split_sweep) and the timings."""
    arr = lp_array(lps)
    t = psl_tuning()
    _bcheck(load().psl_tune(len(arr), C.cast(arr, C.c_void_p), C.byref(settings), reps, C.byref(t)))
    return {"bin_thresholds": tuple(t.bin_thresholds), "split_sweep": t.split_sweep,
            "candidates": t.candidates, "ms_best": t.ms_best, "ms_default": t.ms_default}


def psl_batch_free(b):
    if b:
        load().psl_batch_free(b)


def psl_batch_last_error(b=None):
    return load().psl_batch_last_error(b).decode()


def psl_server_config_default():
    c = psl_server_config()
    load().psl_server_config_default(C.byref(c))
    return c


def psl_server_create(cfg: psl_server_config, settings: psl_settings):
    sv = C.c_void_p()
    _scheck(load().psl_server_create(C.byref(cfg), C.byref(settings), C.byref(sv)))
    return sv


def psl_server_submit(sv, lp: psl_lp):
    t = C.c_uint64()
    _scheck(load().psl_server_submit(sv, C.byref(lp), C.byref(t)), sv)
    return t.value


def psl_server_step(sv):
    n = C.c_int32()
    _scheck(load().psl_server_step(sv, C.byref(n)), sv)
    return n.value


def psl_server_poll(sv, cap=1024):
    arr = (C.c_uint64 * cap)()
    n = C.c_int32()
    _scheck(load().psl_server_poll(sv, C.cast(arr, C.c_void_p), cap, C.byref(n)), sv)
    return list(arr[:n.value])


def psl_server_wait(sv, ticket, timeout_ms=-1.0):
    _scheck(load().psl_server_wait(sv, ticket, float(timeout_ms)), sv)


def psl_server_info(sv, ticket):
    i = psl_ticket_info()
    _scheck(load().psl_server_info(sv, ticket, C.byref(i)), sv)
    return i


def psl_server_reduced_problem(sv, ticket):
    v = psl_reduced_view()
    _scheck(load().psl_server_reduced_problem(sv, ticket, C.byref(v)), sv)
    return v


def psl_server_records(sv, ticket):
    cnt = C.c_int64()
    _scheck(load().psl_server_records(sv, ticket, C.byref(cnt), None, 0), sv)
    out = np.zeros(cnt.value, RECORD_DTYPE)
    if cnt.value:
        _scheck(load().psl_server_records(sv, ticket, C.byref(cnt), out.ctypes.data, cnt.value), sv)
    return out


def psl_server_postsolve(sv, ticket, x_red, n, y_red=None, m=0):
    args, keep, out = _post_args(x_red, y_red, m, n)
    _scheck(load().psl_server_postsolve(sv, ticket, *args), sv)
    return out[0] if len(out) == 1 else out


def psl_server_release(sv, ticket):
    _scheck(load().psl_server_release(sv, ticket), sv)


def psl_server_drain(sv):
    _scheck(load().psl_server_drain(sv), sv)


def psl_server_memory(sv):
    v = [C.c_size_t() for _ in range(4)]
    _scheck(load().psl_server_memory(sv, *[C.byref(x) for x in v]), sv)
    return dict(zip(("arena_bytes", "heap_bytes", "heap_used", "heap_peak"), [x.value for x in v]))


def reduced_footprint(m, n, nnz):
    """Bytes a request reserves in the server's result heap (its LP's sizes)."""
    def a(x):
        return (x + 255) // 256 * 256
    sizes = [(m + 1) * 4, nnz * 4, nnz * 8, (n + 1) * 4, nnz * 4, nnz * 8, m * 8, m * 8, n * 8, n * 8, n * 8,
             m * 4, n * 4, m, n]
    return sum(a(x) for x in sizes)


def psl_server_free(sv):
    if sv:
        load().psl_server_free(sv)


def psl_server_last_error(sv=None):
    return load().psl_server_last_error(sv).decode()


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

_LP_KEYS = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")


def _is_torch(a):
    return type(a).__module__.startswith("torch")


def make_lp(lp, keep):
    """psl_lp from a dict of numpy arrays (host) or torch CUDA tensors (device)."""
    arrs = {}
    dev = None
    for k in _LP_KEYS:
        a = lp[k]
        if _is_torch(a):
            d = a.is_cuda
            want = {"row_ptr": "int32", "col_idx": "int32"}.get(k, "float64")
            if str(a.dtype).split(".")[-1] != want or not a.is_contiguous():
                raise ValueError(f"{k}: needs a contiguous {want} tensor")
        else:
            d = False
            a = np.ascontiguousarray(a, np.int32 if k in ("row_ptr", "col_idx") else np.float64)
        if dev is None:
            dev = d
        elif dev != d:
            raise ValueError("all arrays must be on the host or all on the device")
        arrs[k] = a
    keep.append(arrs)

    def ptr(a):
        if _is_torch(a):
            return a.data_ptr() if a.numel() else None
        return a.ctypes.data if a.size else None

    m, n = int(lp["m"]), int(lp["n"])
    nnz = int(lp.get("nnz", int(arrs["row_ptr"][-1]) if m else 0))
    return psl_lp(m, n, nnz, PSL_MEM_DEVICE if dev else PSL_MEM_HOST,
                  *[ptr(arrs[k]) for k in _LP_KEYS], float(lp.get("obj_offset", 0.0)))


def tune(lps, reps=3, stream=None, **settings):
    """psl_tune on a list of LP dicts or an LpSet."""
    lset = lps if isinstance(lps, LpSet) else LpSet(lps)
    return psl_tune(lset.arr, make_settings(stream=stream, **settings), reps)


def make_settings(stream=None, **kw):
    s = psl_settings_default()
    names = {f for f, _ in psl_settings._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"unknown setting {k!r}")
        if k == "bin_thresholds":
            arr = (C.c_int32 * len(v))(*v)
            s.bin_thresholds = C.cast(arr, C.c_void_p)
            s.n_bins = len(v)
            s._thr = arr
        else:
            setattr(s, k, v)
    if stream is not None:
        s.stream = stream
    return s


def _d2h(ptr, count, dtype):
    out = np.zeros(count, dtype)
    if count:
        st = _hiprt().hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2)  # hipMemcpyDeviceToHost
        if st != 0:
            raise PslError(PSL_ERR_DEVICE, f"hipMemcpy failed ({st})")
    return out


def reduced_to_host(v):
    """Copy of a psl_reduced_view's arrays on the host (numpy)."""
    m, n, nnz = v.m, v.n, v.nnz
    return dict(
        m=m, n=n, nnz=nnz, obj_offset=v.obj_offset,
        row_ptr=_d2h(v.row_ptr, m + 1, np.int32), col_idx=_d2h(v.col_idx, nnz, np.int32),
        val=_d2h(v.val, nnz, np.float64), col_ptr=_d2h(v.col_ptr, n + 1, np.int32),
        row_idx=_d2h(v.row_idx, nnz, np.int32), cval=_d2h(v.cval, nnz, np.float64),
        lhs=_d2h(v.lhs, m, np.float64), rhs=_d2h(v.rhs, m, np.float64),
        lb=_d2h(v.lb, n, np.float64), ub=_d2h(v.ub, n, np.float64), c=_d2h(v.c, n, np.float64),
        row_map=_d2h(v.row_map, m, np.int32), col_map=_d2h(v.col_map, n, np.int32),
        row_class=_d2h(v.row_class, m, np.uint8), col_class=_d2h(v.col_class, n, np.uint8))


class Presolver:
    """One presolve handle: create (copies the LP to the device), run, read."""

    def __init__(self, lp, stream=None, **settings):
        self._keep = []
        self.n = int(lp["n"])
        self.m = int(lp["m"])
        self.settings = make_settings(stream=stream, **settings)
        self.h = psl_presolve_create(make_lp(lp, self._keep), self.settings)
        self._keep.clear()

    def reload(self, lp):
        keep = []
        psl_presolve_reload(self.h, make_lp(lp, keep))
        self.n = int(lp["n"])
        self.m = int(lp["m"])

    def run(self):
        res, st = psl_presolve_run(self.h)
        self.result = res
        self.result_name = RESULT_NAMES[res]
        self.stats = st.as_dict()
        return self.result_name

    def records(self):
        return psl_records(self.h)

    def view(self):
        return psl_reduced_problem(self.h)

    def reduced(self):
        """Copy of the reduced problem on the host (numpy)."""
        return reduced_to_host(self.view())

    def postsolve(self, x_red, y_red=None):
        """x of the original LP, or (x, y, z) when the reduced LP's row duals
        y_red are given."""
        return psl_postsolve(self.h, x_red, self.n, y_red, self.m)

    def close(self):
        if getattr(self, "h", None):
            psl_presolve_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def presolve(lp, **settings):
    """Create, run and collect everything on the host; returns a dict."""
    p = Presolver(lp, **settings)
    try:
        name = p.run()
        out = {"result_name": name, "records": p.records(), "stats": p.stats}
        out["reduced"] = p.reduced() if name in ("REDUCED", "UNCHANGED") else None
        return out, p
    except Exception:
        p.close()
        raise


class LpSet:
    """Prepared psl_lp descriptors of several LPs (arrays kept alive), for
    repeated batch reloads without rebuilding them."""

    def __init__(self, lps):
        self._keep = []
        self.ns = [int(lp["n"]) for lp in lps]
        self.ms = [int(lp["m"]) for lp in lps]
        self.arr = lp_array([make_lp(lp, self._keep) for lp in lps])

    def __len__(self):
        return len(self.ns)


class Batch:
    """A batch handle: K LPs presolved together, each with its own result."""

    def __init__(self, lps, stream=None, **settings):
        lset = lps if isinstance(lps, LpSet) else LpSet(lps)
        self.ns = list(lset.ns)
        self.ms = list(lset.ms)
        self.settings = make_settings(stream=stream, **settings)
        self.h = psl_batch_create(lset.arr, self.settings)

    def reload(self, lps):
        lset = lps if isinstance(lps, LpSet) else LpSet(lps)
        self.ns = list(lset.ns)
        self.ms = list(lset.ms)
        psl_batch_reload(self.h, lset.arr)

    def run(self):
        res, st = psl_batch_run(self.h, len(self.ns))
        self.results = [RESULT_NAMES[r] for r in res]
        self.stats = st.as_dict()
        return self.results

    def lp_stats(self, idx):
        return psl_batch_stats(self.h, idx).as_dict()

    def records(self, idx):
        return psl_batch_records(self.h, idx)

    def view(self, idx):
        return psl_batch_reduced_problem(self.h, idx)

    def reduced(self, idx):
        return reduced_to_host(self.view(idx))

    def postsolve(self, idx, x_red, y_red=None):
        return psl_batch_postsolve(self.h, idx, x_red, self.ns[idx], y_red, self.ms[idx])

    def close(self):
        if getattr(self, "h", None):
            psl_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching presolve server (psl_server_*). The arrays of a
    submitted LP are kept alive here until its ticket is released. With
    threaded=0 nothing runs between calls of step(), each of which admits
    waiting LPs into free slots and advances every resident batch by one
    round (psl_server_step)."""

    def __init__(self, stream=None, **config):
        settings = {k: config.pop(k) for k in list(config) if k in {f for f, _ in psl_settings._fields_}}
        self.cfg = psl_server_config_default()
        names = {f for f, _ in psl_server_config._fields_}
        for k, v in config.items():
            if k not in names:
                raise TypeError(f"unknown server setting {k!r}")
            setattr(self.cfg, k, v)
        self.settings = make_settings(**settings)
        self.h = psl_server_create(self.cfg, self.settings)
        self._keep = {}
        self._n = {}
        self._m = {}

    def submit(self, lp):
        keep = []
        t = psl_server_submit(self.h, make_lp(lp, keep))
        self._keep[t] = keep
        self._n[t] = int(lp["n"])
        self._m[t] = int(lp["m"])
        return t

    def step(self):
        return psl_server_step(self.h)

    def poll(self, cap=1024):
        return psl_server_poll(self.h, cap)

    def wait(self, ticket, timeout_ms=-1.0):
        psl_server_wait(self.h, ticket, timeout_ms)

    def info(self, ticket):
        i = psl_server_info(self.h, ticket)
        return {"status": i.status, "result_name": RESULT_NAMES.get(i.result, i.result), "queue_ms": i.queue_ms,
                "latency_ms": i.latency_ms, "batch_lps": i.batch_lps, "slot": i.slot, "stats": i.stats.as_dict()}

    def records(self, ticket):
        return psl_server_records(self.h, ticket)

    def view(self, ticket):
        return psl_server_reduced_problem(self.h, ticket)

    def reduced(self, ticket):
        return reduced_to_host(self.view(ticket))

    def postsolve(self, ticket, x_red, y_red=None):
        return psl_server_postsolve(self.h, ticket, x_red, self._n[ticket], y_red, self._m[ticket])

    def release(self, ticket):
        psl_server_release(self.h, ticket)
        self._keep.pop(ticket, None)
        self._n.pop(ticket, None)
        self._m.pop(ticket, None)

    def drain(self):
        psl_server_drain(self.h)

    def memory(self):
        return psl_server_memory(self.h)

    def close(self):
        if getattr(self, "h", None):
            psl_server_free(self.h)
            self.h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
