"""Dominated columns through implied dual bounds in the oracle (a dual
explorer, section 2.1: a reduction that keeps at least one optimal solution;
the bounds on the row duals come from the row sides and from column
singletons, as the locks come from the rows in section 3.2).

Pins that do not reuse the oracle's arithmetic:
  * closed forms on hand LPs: a column priced out by a cheaper singleton in
    its row (fixed at its lower bound, which dual fixing alone does not do: the
    row locks it), the mirror at the upper bound, an infinite preferred bound
    (the LP is unbounded), crossing dual bounds (nothing happens), a column of
    zero reduced-cost range (kept);
  * optimality: HiGHS on the original vs the reduced LP, the postsolved x
    feasible and optimal, and the dual postsolve satisfying the original KKT
    conditions, on tiny LPs with planted cheap singleton columns, alone and
    with every other optional reduction; medium LPs likewise.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import feasible, highs, highs_duals, kkt_violations, make, reduced_lp

INF = np.inf
DC = dict(enable_dominated=1)
ALL = dict(enable_dominated=1, enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1,
           enable_forcing_rows=1, enable_doubletons=1)


def _recs(res, name):
    return [r for r in res.records if O.REC_NAMES[int(r["type"])] == name]


def _check_optimal(lp, res):
    st, obj, _ = highs(lp)
    if res.result_name == "INFEASIBLE":
        assert st == "infeasible"
        return
    if res.result_name == "UNBOUNDED_OR_INFEASIBLE":
        assert st in ("unbounded", "infeasible")
        return
    red = reduced_lp(res.reduced)
    st2, obj2, xr = highs(red)
    if st2 == "empty":
        obj2, xr, st2 = red["obj_offset"], np.zeros(0), "optimal"
    assert st2 == st, (st, st2)
    if st != "optimal":
        return
    assert abs(obj2 - obj) <= 1e-7 * max(1.0, abs(obj)), (obj, obj2)
    x = res.postsolve(xr)
    assert feasible(lp, x, tol=1e-6)
    assert abs(float(lp["c"] @ x) - obj) <= 1e-6 * max(1.0, abs(obj))
    dst, xr2, yr = highs_duals(red)
    if dst == "empty":
        xr2, yr = np.zeros(0), np.zeros(red["m"])
    elif dst != "optimal":
        return
    x2, y, z = res.postsolve_dual(xr2, yr)
    bad = kkt_violations(lp, x2, y, z, tol=1e-6)
    assert not bad, bad[:5]


def test_off_by_default():
    assert O.DEFAULTS["enable_dominated"] == 0
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [1.0], [INF], [0, 0], [INF, 5], [1.0, 2.0])
    assert not _recs(O.presolve(lp), "DOMINATED_COL")


def test_priced_out_by_a_cheaper_singleton():
    """min x0 + 2 x1 s.t. x0 + x1 >= 1, x0 in [0, inf), x1 in [0, 5]: the row
    has y >= 0 and the singleton x0 (no upper bound) gives y <= c0 / 1 = 1,
    so z1 >= 2 - 1 = 1 > 0 and x1 goes to 0. Dual fixing does not: the row
    keeps x1 from decreasing. Then the row is a singleton row, x0 >= 1, and
    x0 leaves at 1: optimum 1."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [1.0], [INF], [0, 0], [INF, 5], [1.0, 2.0])
    assert not _recs(O.presolve(lp, enable_dual_fix=1), "DUAL_FIX")
    res = O.presolve(lp, **DC)
    dc = _recs(res, "DOMINATED_COL")
    assert [(int(r["j"]), int(r["side"]), float(r["v"][0]), float(r["v"][1])) for r in dc] == [(1, 0, 0.0, 2.0)]
    assert res.reduced["n"] == 0 and res.reduced["obj_offset"] == 1.0
    assert np.array_equal(res.postsolve(np.zeros(0)), [1.0, 0.0])
    _check_optimal(lp, res)


def test_mirror_at_the_upper_bound():
    """min -x0 - 3 x1 s.t. x0 + x1 <= 5, x0 in (-inf, 3], x1 in [0, 4]: the
    row has y <= 0, the singleton x0 (no lower bound) gives y >= -1, so
    z1 <= -3 + 1 = -2 < 0 and x1 goes to 4; optimum -13 at (1, 4)."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [5.0], [-INF, 0], [3, 4], [-1.0, -3.0])
    res = O.presolve(lp, **DC)
    dc = _recs(res, "DOMINATED_COL")
    assert [(int(r["j"]), int(r["side"]), float(r["v"][0])) for r in dc] == [(1, 1, 4.0)]
    _check_optimal(lp, res)
    st, obj, _ = highs(lp)
    assert st == "optimal" and obj == pytest.approx(-13.0)


def test_infinite_preferred_bound_is_unbounded():
    """min x0 + 2 x1 s.t. x0 + x1 >= 1 (y0 >= 0), x1 - x2 <= 3 (y1 <= 0),
    x0 in [0, inf), x1 in (-inf, 5], x2 in [0, 1]: the singleton x0 gives
    y0 <= 1, so z1 >= 2 - 1 - 0 = 1 > 0 and x1 would go to -inf: the LP is
    unbounded (x0 = 1 - x1 keeps it feasible at a cost 1 + x1)."""
    lp = make(2, 3, [[(0, 1.0), (1, 1.0)], [(1, 1.0), (2, -1.0)]], [1.0, -INF], [INF, 3.0], [0, -INF, 0],
              [INF, 5, 1], [1.0, 2.0, 0.0])
    res = O.presolve(lp, **DC)
    assert res.result_name == "UNBOUNDED_OR_INFEASIBLE"
    assert highs(lp)[0] == "unbounded"


def test_crossing_dual_bounds_mean_unbounded():
    """Two singletons in one equality row: x0 >= 0 with cost 1 gives y <= 1,
    x1 <= 0 (no lower bound) with cost 3 gives y >= 3: the bounds cross, the
    dual has no solution and the LP is unbounded (x1 falls, x0 = 2 - x1 - x2
    rises, the cost 2 + 2 x1 + 4 x2 falls)."""
    lp = make(1, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)]], [2.0], [2.0], [0, -INF, 0], [INF, 0, 1], [1.0, 3.0, 5.0])
    res = O.presolve(lp, **DC)
    assert not _recs(res, "DOMINATED_COL")
    assert res.result_name == "UNBOUNDED_OR_INFEASIBLE"
    assert highs(lp)[0] == "unbounded"


def test_zero_range_kept():
    """min x0 + x1 s.t. x0 + x1 >= 1, x0 >= 0 free above, x1 in [0, 5]: y <= 1
    from the singleton, so z1 >= 1 - 1 = 0: not strictly positive, x1 stays."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [1.0], [INF], [0, 0], [INF, 5], [1.0, 1.0])
    assert not _recs(O.presolve(lp, **DC), "DOMINATED_COL")


def with_cheap_singletons(lp, seed, count=2):
    """The LP with `count` new singleton columns (one row each; either in
    [0, inf) with a small positive cost or in (-inf, 0] with a small negative
    one, so that the cost keeps them bounded) that price other columns of
    their rows out."""
    rng = np.random.default_rng(seed)
    m, n = lp["m"], lp["n"]
    if m == 0:
        return lp
    rows = [[(int(lp["col_idx"][k]), float(lp["val"][k])) for k in range(lp["row_ptr"][i], lp["row_ptr"][i + 1])]
            for i in range(m)]
    lb, ub, c = list(lp["lb"]), list(lp["ub"]), list(lp["c"])
    for t in range(count):
        i = int(rng.integers(m))
        rows[i].append((n + t, float(rng.choice([1.0, -1.0, 2.0]))))
        up = rng.random() < 0.5
        lb.append(0.0 if up else -INF)
        ub.append(INF if up else 0.0)
        c.append(float(rng.choice([0.25, 0.5])) * (1.0 if up else -1.0))
    return make(m, n + count, rows, lp["lhs"], lp["rhs"], lb, ub, c)


@pytest.mark.parametrize("seed", range(300))
def test_tiny_optimal_and_kkt(seed):
    lp = with_cheap_singletons(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), seed)
    _check_optimal(lp, O.presolve(lp, **DC))
    _check_optimal(lp, O.presolve(lp, **ALL))


def test_tiny_fires():
    total = sides = 0
    seen = set()
    for seed in range(300):
        lp = with_cheap_singletons(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), seed)
        dc = _recs(O.presolve(lp, **DC), "DOMINATED_COL")
        total += len(dc)
        seen |= {int(r["side"]) for r in dc}
    assert total >= 40 and seen == {0, 1}, (total, seen)


@pytest.mark.parametrize("seed", range(4))
def test_medium(seed):
    lp = with_cheap_singletons(lpgen.make_lp(300, 450, seed=700 + seed, row_len=(2, 7), singleton=10, empty=5,
                                             doubleton=20, duplicate=10, fixed_cols=15), seed, count=300)
    for extra in (DC, ALL):
        res = O.presolve(lp, **extra)
        assert len(_recs(res, "DOMINATED_COL")) >= 1
        _check_optimal(lp, res)
