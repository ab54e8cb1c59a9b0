"""Test helpers: golden fixtures, dense LP views, an independent vertex
enumerator and a HiGHS (scipy) solve. None of this is presolve arithmetic."""
from __future__ import annotations

import itertools
import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _num(v):
    if isinstance(v, str):
        return float(v)
    return v


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        g = json.load(f)
    lp = g["lp"]
    out = {
        "m": lp["m"], "n": lp["n"],
        "row_ptr": np.array(lp["row_ptr"], np.int32),
        "col_idx": np.array(lp["col_idx"], np.int32),
        "val": np.array(lp["val"], np.float64),
        "obj_offset": 0.0,
    }
    for k in ("lhs", "rhs", "lb", "ub", "c"):
        out[k] = np.array([_num(v) for v in lp[k]], np.float64)
    return g, out


def make(m, n, rows, lhs, rhs, lb, ub, c):
    """LP dict from a list of rows [(col, val), ...]."""
    rp = [0]
    ci, va = [], []
    for r in rows:
        for j, a in sorted(r):
            ci.append(j)
            va.append(a)
        rp.append(len(ci))
    return {"m": m, "n": n, "row_ptr": np.array(rp, np.int32), "col_idx": np.array(ci, np.int32),
            "val": np.array(va, np.float64), "lhs": np.array(lhs, float), "rhs": np.array(rhs, float),
            "lb": np.array(lb, float), "ub": np.array(ub, float), "c": np.array(c, float),
            "obj_offset": 0.0}


def dense(lp):
    m, n = lp["m"], lp["n"]
    A = np.zeros((m, n))
    rp = lp["row_ptr"]
    for i in range(m):
        for k in range(rp[i], rp[i + 1]):
            A[i, lp["col_idx"][k]] = lp["val"][k]
    return A


def feasible(lp, x, tol=1e-7):
    A = dense(lp)
    ax = A @ x
    sc = np.maximum(1.0, np.abs(ax))
    ok = np.all(ax >= lp["lhs"] - tol * sc) and np.all(ax <= lp["rhs"] + tol * sc)
    scx = np.maximum(1.0, np.abs(x))
    ok &= np.all(x >= lp["lb"] - tol * scx) and np.all(x <= lp["ub"] + tol * scx)
    return bool(ok)


def vertices(lp, tol=1e-9):
    """All vertices of {lhs <= Ax <= rhs, lb <= x <= ub} for a tiny LP with
    finite bounds: every choice of n linearly independent active constraints,
    solved and kept if feasible."""
    A = dense(lp)
    m, n = A.shape
    if n == 0:
        return np.zeros((1, 0))
    planes, rhs_v = [], []
    for i in range(m):
        for s in {lp["lhs"][i], lp["rhs"][i]}:
            if np.isfinite(s):
                planes.append(A[i])
                rhs_v.append(s)
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        for s in {lp["lb"][j], lp["ub"][j]}:
            if np.isfinite(s):
                planes.append(e)
                rhs_v.append(s)
    planes = np.array(planes)
    rhs_v = np.array(rhs_v)
    combos = np.array(list(itertools.combinations(range(len(planes)), n)))
    if len(combos) == 0:
        return np.zeros((0, n))
    M = planes[combos]
    b = rhs_v[combos]
    det = np.linalg.det(M)
    good = np.abs(det) > 1e-12
    if not good.any():
        return np.zeros((0, n))
    X = np.linalg.solve(M[good], b[good][..., None])[..., 0]
    keep = [x for x in X if feasible(lp, x, tol=1e-9)]
    if not keep:
        return np.zeros((0, n))
    V = np.unique(np.round(np.array(keep), 12), axis=0)
    return V


def highs(lp):
    """Solve with scipy's HiGHS. Returns (status, objective, x) with status in
    {'optimal', 'infeasible', 'unbounded'}."""
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix
    m, n = lp["m"], lp["n"]
    if n == 0:
        ok = all((lp["lhs"][i] <= 1e-9 * max(1, abs(lp["lhs"][i]))) and
                 (lp["rhs"][i] >= -1e-9 * max(1, abs(lp["rhs"][i]))) for i in range(m))
        return ("optimal" if ok else "infeasible"), float(lp.get("obj_offset", 0.0)), np.zeros(0)
    A = csr_matrix((lp["val"], lp["col_idx"], lp["row_ptr"]), shape=(m, n))
    lhs, rhs = lp["lhs"], lp["rhs"]
    ub_rows = np.isfinite(rhs)
    lb_rows = np.isfinite(lhs)
    A_ub = []
    b_ub = []
    if ub_rows.any():
        A_ub.append(A[ub_rows])
        b_ub.append(rhs[ub_rows])
    if lb_rows.any():
        A_ub.append(-A[lb_rows])
        b_ub.append(-lhs[lb_rows])
    from scipy.sparse import vstack
    kw = {}
    if A_ub:
        kw["A_ub"] = vstack(A_ub).tocsr()
        kw["b_ub"] = np.concatenate(b_ub)
    bounds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u)
              for l, u in zip(lp["lb"], lp["ub"])]
    res = linprog(lp["c"], bounds=bounds, method="highs", **kw)
    off = float(lp.get("obj_offset", 0.0))
    if res.status == 0:
        return "optimal", float(res.fun) + off, res.x
    if res.status == 2:
        return "infeasible", None, None
    if res.status == 3:
        return "unbounded", None, None
    raise RuntimeError(f"HiGHS status {res.status}: {res.message}")


def reduced_lp(red):
    return {k: red[k] for k in ("m", "n", "row_ptr", "col_idx", "val", "lhs", "rhs",
                                "lb", "ub", "c", "obj_offset")}


def highs_duals(lp):
    """Solve with scipy's HiGHS and return (status, x, y): x the primal
    solution, y the row multipliers in the convention c - A'y - z = 0 with
    y_i >= 0 when row i is at lhs and <= 0 at rhs (from the marginals of the
    two one-sided inequalities of each row). Only 'optimal' carries x, y."""
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix, vstack
    m, n = lp["m"], lp["n"]
    if n == 0:
        return "empty", np.zeros(0), np.zeros(m)
    A = csr_matrix((lp["val"], lp["col_idx"], lp["row_ptr"]), shape=(m, n))
    lhs, rhs = lp["lhs"], lp["rhs"]
    up = np.flatnonzero(np.isfinite(rhs))
    lo = np.flatnonzero(np.isfinite(lhs))
    kw = {}
    if len(up) + len(lo):
        kw["A_ub"] = vstack([A[up], -A[lo]]).tocsr()
        kw["b_ub"] = np.concatenate([rhs[up], -lhs[lo]])
    bounds = [(None if not np.isfinite(l) else l, None if not np.isfinite(u) else u)
              for l, u in zip(lp["lb"], lp["ub"])]
    res = linprog(lp["c"], bounds=bounds, method="highs", **kw)
    if res.status != 0:
        return {2: "infeasible", 3: "unbounded"}.get(res.status, "other"), None, None
    y = np.zeros(m)
    if len(up) + len(lo):
        mu = res.ineqlin.marginals
        y[up] += mu[:len(up)]
        y[lo] -= mu[len(up):]
    return "optimal", res.x, y


def kkt_violations(lp, x, y, z, tol=1e-6):
    """Violations of the optimality conditions of lp at (x, y, z) with
    z = c - A'y: primal feasibility, the signs of y and z against the active
    sides and bounds (complementary slackness), and the duality gap. Returns
    a list of messages (empty when optimal within tol)."""
    A = dense(lp)
    out = []
    if not feasible(lp, x, tol=tol):
        out.append("primal infeasible")
    ax = A @ x
    st = lp["c"] - A.T @ y - z
    if np.max(np.abs(st), initial=0.0) > tol * max(1.0, np.max(np.abs(lp["c"]), initial=0.0)):
        out.append("stationarity")
    for i in range(lp["m"]):
        sc = tol * max(1.0, abs(ax[i]))
        ys = tol * max(1.0, np.max(np.abs(y), initial=0.0))
        if y[i] > ys and not (np.isfinite(lp["lhs"][i]) and abs(ax[i] - lp["lhs"][i]) <= sc):
            out.append(f"y[{i}]={y[i]:.3g} > 0 but row {i} not at lhs")
        if y[i] < -ys and not (np.isfinite(lp["rhs"][i]) and abs(ax[i] - lp["rhs"][i]) <= sc):
            out.append(f"y[{i}]={y[i]:.3g} < 0 but row {i} not at rhs")
    zs = tol * max(1.0, np.max(np.abs(z), initial=0.0))
    for j in range(lp["n"]):
        sc = tol * max(1.0, abs(x[j]))
        if z[j] > zs and not (np.isfinite(lp["lb"][j]) and abs(x[j] - lp["lb"][j]) <= sc):
            out.append(f"z[{j}]={z[j]:.3g} > 0 but x[{j}] not at lb")
        if z[j] < -zs and not (np.isfinite(lp["ub"][j]) and abs(x[j] - lp["ub"][j]) <= sc):
            out.append(f"z[{j}]={z[j]:.3g} < 0 but x[{j}] not at ub")
    # duality gap: c'x against the dual objective of the active sides and bounds
    # (multipliers within the tolerance of zero count as zero)
    ys = tol * max(1.0, np.max(np.abs(y), initial=0.0))
    dual = 0.0
    for i in range(lp["m"]):
        if y[i] > ys:
            dual += y[i] * lp["lhs"][i]
        elif y[i] < -ys:
            dual += y[i] * lp["rhs"][i]
    for j in range(lp["n"]):
        if z[j] > zs:
            dual += z[j] * lp["lb"][j]
        elif z[j] < -zs:
            dual += z[j] * lp["ub"][j]
    primal = float(lp["c"] @ x)
    if abs(primal - dual) > 1e-5 * max(1.0, abs(primal)):
        out.append(f"duality gap {primal - dual:.3g}")
    return out
