"""Digests of a presolve result (outcome, record stream, reduced problem),
computed the same way from the oracle's and from the library's output.

Every array is hashed in a fixed dtype (records as 48-byte structs; indices
int32, values float64 bit patterns, classes uint8), so equal digests mean
bit-identical results.
"""
from __future__ import annotations

import hashlib

import numpy as np

ARRAYS = (("row_ptr", np.int32), ("col_idx", np.int32), ("val", np.float64), ("col_ptr", np.int32),
          ("row_idx", np.int32), ("cval", np.float64), ("lhs", np.float64), ("rhs", np.float64),
          ("lb", np.float64), ("ub", np.float64), ("c", np.float64), ("row_map", np.int32),
          ("col_map", np.int32), ("row_class", np.uint8), ("col_class", np.uint8))


def _sha(b):
    return hashlib.sha256(b).hexdigest()


def digest_of(result_name, records, reduced):
    """Per-part digests (dict of hex strings and sizes)."""
    rec = np.ascontiguousarray(records)
    out = {"result_name": result_name, "records": int(len(rec)), "records_sha256": _sha(rec.tobytes())}
    if reduced is not None:
        out["reduced"] = {"m": int(reduced["m"]), "n": int(reduced["n"]), "nnz": int(reduced["nnz"]),
                          "obj_offset_bits": int(np.array([reduced["obj_offset"]], np.float64).view(np.uint64)[0])}
        for key, dt in ARRAYS:
            out["reduced"][key + "_sha256"] = _sha(np.ascontiguousarray(reduced[key], dt).tobytes())
    return out


def lp_digest(result_name, records, reduced):
    """One short digest of a whole result."""
    return _sha(repr(sorted(_flat(digest_of(result_name, records, reduced)))).encode())[:24]


def _flat(d, prefix=""):
    for k, v in d.items():
        if isinstance(v, dict):
            yield from _flat(v, prefix + k + ".")
        else:
            yield (prefix + k, v)
