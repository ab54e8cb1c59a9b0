"""The oracle against brute force and an independent LP solver.

Tiny LPs: vertex enumeration (finite bounds) and scipy's HiGHS give the
optimum of the original and of the reduced problem; presolve must keep the
optimum (after the objective offset), postsolve must return a feasible,
optimal point, and every vertex of the original must stay feasible for the
reduced problem (the tightened bounds and merged rows keep the feasible set;
section 2.1 'Explorers', primal explorers preserve the feasible set).
Medium LPs (the small synthetic workload): HiGHS on original vs reduced.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import feasible, highs, reduced_lp, vertices

R = O.REC


def _removed_fixed(res):
    """Columns fixed by primal reasoning (input or propagation), with values."""
    out = {}
    for r in res.records:
        if r["type"] == R["FIX_COL"]:
            out[int(r["j"])] = r["v"][0]
    return out


def _check(lp, res, tol=1e-7):
    st, obj, _ = highs(lp)
    if res.result_name == "INFEASIBLE":
        assert st == "infeasible"
        return st
    if res.result_name == "UNBOUNDED_OR_INFEASIBLE":
        assert st in ("unbounded", "infeasible")
        return st
    red = reduced_lp(res.reduced)
    st2, obj2, xr = highs(red)
    assert st2 == st, (st, st2)
    if st == "optimal":
        assert abs(obj2 - obj) <= tol * max(1.0, abs(obj)), (obj, obj2)
        x = res.postsolve(xr)
        assert feasible(lp, x, tol=1e-6)
        assert abs(float(lp["c"] @ x) - obj) <= 1e-6 * max(1.0, abs(obj))
    return st


@pytest.mark.parametrize("seed", range(150))
def test_tiny_finite_bounds_vertices(seed):
    lp = lpgen.tiny(seed, finite_bounds=True)
    res = O.presolve(lp)
    V = vertices(lp)
    st = _check(lp, res)
    if len(V) == 0:
        assert st == "infeasible"
        return
    # optimum by enumeration agrees with HiGHS
    assert st == "optimal"
    vopt = min(float(lp["c"] @ v) for v in V)
    _, hobj, _ = highs(lp)
    assert abs(vopt - hobj) <= 1e-7 * max(1.0, abs(vopt))
    if res.result_name not in ("REDUCED", "UNCHANGED"):
        return
    # every vertex of the original satisfies the reduced problem (primal
    # reductions keep the feasible set; empty columns are not in kept rows)
    red = reduced_lp(res.reduced)
    fixed = _removed_fixed(res)
    for v in V:
        for j, val in fixed.items():
            assert abs(v[j] - val) <= 1e-7 * max(1.0, abs(val))
        assert feasible(red, v[res.reduced["col_map"]], tol=1e-7)
    # and the reduced optimum, lifted, is optimal for the original
    Vr = vertices(red) if red["n"] > 0 else np.zeros((1, 0))
    assert len(Vr) > 0
    best = min(float(red["c"] @ v) for v in Vr) + red["obj_offset"]
    assert abs(best - vopt) <= 1e-7 * max(1.0, abs(vopt))


@pytest.mark.parametrize("seed", range(150, 350))
def test_tiny_mixed_bounds_highs(seed):
    lp = lpgen.tiny(seed)
    res = O.presolve(lp)
    _check(lp, res)


@pytest.mark.parametrize("seed", range(6))
def test_medium_highs(seed):
    lp = lpgen.make_lp(300, 450, seed=100 + seed, row_len=(2, 7), singleton=10, empty=5,
                       doubleton=20, duplicate=10, fixed_cols=15)
    res = O.presolve(lp)
    assert res.result_name == "REDUCED"
    _check(lp, res)


def test_small_workload_highs():
    lp = lpgen.single_small()
    res = O.presolve(lp)
    assert res.result_name == "REDUCED"
    st = _check(lp, res)
    assert st == "optimal"
    # the planted feasible point satisfies the reduced problem's bounds
    r = res.reduced
    x0 = lp["x0"][r["col_map"]]
    sc = np.maximum(1, np.abs(x0))
    assert np.all(x0 >= r["lb"] - 1e-9 * sc) and np.all(x0 <= r["ub"] + 1e-9 * sc)
