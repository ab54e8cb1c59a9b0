"""Dual postsolve of the oracle against the optimality conditions of the
original LP (section 2.1, "Postsolver"; section 3.3 returns primal and dual
solutions of the original problem).

For each LP: presolve, solve the REDUCED problem with scipy's HiGHS (a basic
optimal solution with its row marginals), postsolve (x, y, z), and check in
the ORIGINAL problem primal feasibility, z = c - A'y, the signs of y and z
against the active sides and bounds, and a zero duality gap. HiGHS never sees
the original problem's duals, so a wrong transfer rule (a dropped bound
change, a wrong sign of a tightened bound, a parallel row's lambda) shows as
a sign or gap violation. Tiny LPs mix every row and bound kind with planted
singleton, duplicate, empty rows and fixed columns; the small workload adds
doubletons and propagation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import highs_duals, kkt_violations, make, reduced_lp

R = O.REC


def _check_dual(lp, tol=1e-6):
    res = O.presolve(lp)
    if res.result_name not in ("REDUCED", "UNCHANGED"):
        return None
    red = reduced_lp(res.reduced)
    st, xr, yr = highs_duals(red)
    if st == "empty":
        xr, yr = np.zeros(0), np.zeros(red["m"])
    elif st != "optimal":
        return None
    x, y, z = res.postsolve_dual(xr, yr)
    bad = kkt_violations(lp, x, y, z, tol=tol)
    assert not bad, bad[:5]
    return res


@pytest.mark.parametrize("seed", range(300))
def test_tiny_dual_postsolve_kkt(seed):
    _check_dual(lpgen.tiny(seed, finite_bounds=seed % 2 == 0))


def test_dual_moves_into_source_row():
    """x1 + x2 <= 4 (row 0) with x >= 0 and min -x1: round 1 tightens x1 <= 4
    and x2 <= 4 from row 0; the reduced LP keeps the row (not redundant), the
    optimum x1 = 4 sits at the tightened bound with reduced cost -1, which the
    postsolve moves into row 0: y0 = -1, z = 0 for x1 and z = 1 for x2."""
    inf = np.inf
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-inf], [4.0], [0, 0], [inf, inf], [-1.0, 0.0])
    res = O.presolve(lp)
    red = reduced_lp(res.reduced)
    st, xr, yr = highs_duals(red)
    assert st == "optimal"
    x, y, z = res.postsolve_dual(xr, yr)
    assert np.allclose(x, [4, 0]) and np.allclose(y, [-1.0]) and np.allclose(z, [0.0, 1.0])
    assert not kkt_violations(lp, x, y, z)


def test_dual_through_singleton_row():
    """A singleton row 2 <= 2 x0 <= 6 becomes the bounds 1 <= x0 <= 3 and is
    removed; with min x0 the optimum x0 = 1 is at the bound the row gave, so
    the row gets y = z / a = 1 / 2 and x0's reduced cost returns to 0."""
    inf = np.inf
    lp = make(2, 2, [[(0, 2.0)], [(0, 1.0), (1, 1.0)]], [2.0, -inf], [6.0, 10.0], [-inf, 0], [inf, inf],
              [1.0, 0.0])
    res = O.presolve(lp)
    types = set(int(t) for t in res.records["type"])
    assert R["SINGLETON_ROW"] in types
    red = reduced_lp(res.reduced)
    st, xr, yr = highs_duals(red)
    assert st == "optimal"
    x, y, z = res.postsolve_dual(xr, yr)
    assert np.isclose(x[0], 1.0) and np.isclose(y[0], 0.5) and np.isclose(z[0], 0.0)
    assert not kkt_violations(lp, x, y, z)


def test_dual_through_parallel_rows():
    """Row 1 = -2 x row 0 (parallel, lambda = -2): 1 <= x0 + x1 and
    -2 x0 - 2 x1 <= -3 (i.e. x0 + x1 >= 1.5) merge into the leader row 0 with
    lhs 1.5 from row 1. With min x0 + 2 x1 the merged lhs is active; its dual
    belongs to row 1: y1 = y_leader / lambda < 0 (row 1 at its rhs), y0 = 0."""
    inf = np.inf
    lp = make(2, 2, [[(0, 1.0), (1, 1.0)], [(0, -2.0), (1, -2.0)]], [1.0, -inf], [inf, -3.0], [0, 0],
              [10, 10], [1.0, 2.0])
    res = O.presolve(lp)
    types = set(int(t) for t in res.records["type"])
    assert R["PARALLEL_ROW"] in types and R["LEADER_SIDES"] in types
    red = reduced_lp(res.reduced)
    st, xr, yr = highs_duals(red)
    assert st == "optimal"
    x, y, z = res.postsolve_dual(xr, yr)
    assert np.isclose(x @ lp["c"], 1.5)
    assert y[0] == 0.0 and np.isclose(y[1], -0.5)
    assert not kkt_violations(lp, x, y, z)


@pytest.mark.parametrize("seed", range(6))
def test_medium_dual_postsolve(seed):
    lp = lpgen.make_lp(300, 450, seed=200 + seed, row_len=(2, 7), singleton=10, empty=5, doubleton=20,
                       duplicate=10, fixed_cols=15)
    _check_dual(lp, tol=1e-6)


def test_small_workload_dual_postsolve():
    lp = lpgen.single_small()
    res = _check_dual(lp, tol=1e-6)
    assert res is not None and res.result_name == "REDUCED"
