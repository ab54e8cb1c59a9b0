"""Element-by-element comparison of the GPU library with the CPU oracle."""
import numpy as np

from oracle import oracle as O


def _bits(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.float64:
        return a.view(np.uint64)
    return a


def first_record_mismatch(got, ref):
    n = min(len(got), len(ref))
    gb = got.view(np.uint8).reshape(len(got), 48)[:n] if len(got) else np.zeros((0, 48), np.uint8)
    rb = ref.view(np.uint8).reshape(len(ref), 48)[:n] if len(ref) else np.zeros((0, 48), np.uint8)
    bad = np.flatnonzero(np.any(gb != rb, axis=1))
    if len(bad) == 0:
        return None if len(got) == len(ref) else n
    return int(bad[0])


def describe(rec):
    return (f"type={O.REC_NAMES.get(int(rec['type']), rec['type'])} side={rec['side']} round={rec['round']} "
            f"i={rec['i']} j={rec['j']} k={rec['k']} v={list(rec['v'])}")


REDUCED_KEYS = ("row_ptr", "col_idx", "val", "col_ptr", "row_idx", "cval", "lhs", "rhs", "lb", "ub", "c",
                "row_map", "col_map", "row_class", "col_class")


def assert_same(got, ref, label=""):
    """got: output of psl.presolve; ref: oracle Result. Bit-exact on
    everything: result, record stream, reduced problem, offset."""
    assert got["result_name"] == ref.result_name, (label, got["result_name"], ref.result_name)
    g, r = got["records"], ref.records
    k = first_record_mismatch(g, r)
    if k is not None:
        msg = f"{label}: records differ at {k} of {len(g)} (gpu) / {len(r)} (oracle)"
        if k < len(g):
            msg += "\n gpu:    " + describe(g[k])
        if k < len(r):
            msg += "\n oracle: " + describe(r[k])
        raise AssertionError(msg)
    if ref.reduced is None:
        return
    gr, rr = got["reduced"], ref.reduced
    for key in ("m", "n", "nnz"):
        assert gr[key] == rr[key], (label, key, gr[key], rr[key])
    assert _bits(np.array([gr["obj_offset"]]))[0] == _bits(np.array([rr["obj_offset"]]))[0], \
        (label, "obj_offset", gr["obj_offset"], rr["obj_offset"])
    for key in REDUCED_KEYS:
        a, b = _bits(gr[key]), _bits(rr[key])
        if not np.array_equal(a, b):
            idx = np.flatnonzero(a != b)[:5]
            raise AssertionError(f"{label}: reduced {key} differs at {idx.tolist()}: "
                                 f"gpu {gr[key][idx].tolist()} oracle {rr[key][idx].tolist()}")
