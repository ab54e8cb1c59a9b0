"""Free column singletons with zero cost in the oracle (section 3.2, "Column
singletons": a variable in one constraint, free or with bounds implied by
that constraint, can be eliminated; with c_j = 0 the objective substitution
is zero, so the row and the column simply leave and postsolve takes x_j from
the row).

Pins that do not reuse the oracle's arithmetic:
  * closed forms on hand LPs (a bound implied by the column's own row keeps it
    eligible; a finite input bound, a bound from another row or a nonzero cost
    do not; two candidates in one row: the lowest column goes, the other is
    empty next round);
  * a replay of every FREE_SINGLETON record against the original LP and the
    record stream: c_j = 0, a_ij and the sides as recorded, row i the only
    row of j alive after that round's decisions, and every tightening of j's
    bounds sourced by row i from an infinite input bound;
  * optimality: HiGHS on the original vs the reduced LP, the postsolved x
    feasible and optimal, and the dual postsolve satisfying the original KKT
    conditions; also with dual fixing on.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import feasible, highs, highs_duals, kkt_violations, make, reduced_lp

R = O.REC
INF = np.inf
FS = dict(enable_free_singletons=1)


def _fs(res):
    return [r for r in res.records if r["type"] == R["FREE_SINGLETON"]]


def _recs(res):
    return [(O.REC_NAMES[int(r["type"])], int(r["i"]), int(r["j"]), int(r["round"])) for r in res.records]


def replay_free_singletons(lp, res):
    rp, ci, va = lp["row_ptr"], lp["col_idx"], lp["val"]
    rec = res.records
    row_removed = {}  # row -> round its removal record (other than FREE_SINGLETON) was written
    for r in rec:
        if r["type"] in (R["EMPTY_ROW"], R["REDUNDANT_ROW"], R["SINGLETON_ROW"], R["PARALLEL_ROW"]):
            row_removed.setdefault(int(r["i"]), int(r["round"]))
    fs_removed = {int(r["i"]): int(r["round"]) for r in _fs(res)}
    n = 0
    for r in _fs(res):
        rd, i, j = int(r["round"]), int(r["i"]), int(r["j"])
        side, cj = int(r["side"]), r["v"][3]
        # the side the cost prefers (lhs for c_j / a_ij > 0), finite; 0 for no cost
        if cj == 0:
            assert side == 0
        else:
            assert side == (1 if cj / r["v"][0] > 0 else 2)
            assert np.isfinite(r["v"][side])
        cols = ci[rp[i]:rp[i + 1]]
        assert j in cols
        assert va[rp[i] + int(np.nonzero(cols == j)[0][0])] == r["v"][0]
        # sides as they were: the input, replaced by earlier merges
        lhs, rhs = float(lp["lhs"][i]), float(lp["rhs"][i])
        for q in rec:
            if q["type"] == R["LEADER_SIDES"] and int(q["i"]) == i and int(q["round"]) < rd:
                lhs, rhs = q["v"][2], q["v"][3]
        lhs = -INF if lhs <= -1e20 else lhs
        rhs = INF if rhs >= 1e20 else rhs
        assert (lhs, rhs) == (r["v"][1], r["v"][2])
        # alive rows of j after this round's decisions
        alive = []
        for k in range(lp["m"]):
            if j not in ci[rp[k]:rp[k + 1]]:
                continue
            gone = row_removed.get(k, 10**9) <= rd or fs_removed.get(k, 10**9) < rd
            if not gone:
                alive.append(k)
        assert alive == [i], (i, j, alive)
        # bounds: infinite, or tightened only from row i
        for side, key in ((0, "lb"), (1, "ub")):
            ch = [q for q in rec if q["type"] == R["BOUND_CHANGE"] and int(q["j"]) == j and int(q["side"]) == side
                  and int(q["round"]) <= rd]
            assert abs(lp[key][j]) >= 1e20 or np.isinf(lp[key][j])
            assert all(int(q["k"]) == i for q in ch), (i, j, side)
        n += 1
    return n


def _feasible_status(lp):
    """HiGHS on the LP with a zero objective: whether it is feasible (HiGHS
    may label a feasible unbounded LP infeasible when it has an objective)."""
    z = dict(lp)
    z["c"] = np.zeros(lp["n"])
    return highs(z)[0]


def _check_optimal(lp, res, **settings):
    st, obj, _ = highs(lp)
    if res.result_name == "INFEASIBLE":
        assert _feasible_status(lp) == "infeasible"
        return
    if res.result_name == "UNBOUNDED_OR_INFEASIBLE":
        assert st in ("unbounded", "infeasible")
        return
    red = reduced_lp(res.reduced)
    st2, obj2, xr = highs(red)
    assert _feasible_status(red) == _feasible_status(lp)
    assert (st == "optimal") == (st2 == "optimal"), (st, st2)
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
    assert O.DEFAULTS["enable_free_singletons"] == 0
    lp = make(2, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [-INF, 1.0], [4.0, INF],
              [-INF, 0, 0], [INF, 5, 5], [0.0, 1.0, 1.0])
    assert "FREE_SINGLETON" not in [t for t, *_ in _recs(O.presolve(lp))]


def test_bound_implied_by_its_own_row_keeps_it_free():
    """x0 free, c0 = 0, only in row 0 (x0 + x1 + x2 <= 4): round 1 tightens
    x0 <= 4 from row 0 itself, which keeps x0 eligible; row 0 leaves with x0
    in round 1; row 1 (x1 + x2 >= 1) remains; postsolve puts x0 at 0 when
    x1 + x2 is within row 0's sides."""
    lp = make(2, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [-INF, 1.0], [4.0, INF],
              [-INF, 0, 0], [INF, 5, 5], [0.0, 1.0, 1.0])
    res = O.presolve(lp, **FS)
    got = _recs(res)
    assert ("BOUND_CHANGE", -1, 0, 1) in got
    assert ("FREE_SINGLETON", 0, 0, 1) in got
    r = _fs(res)[0]
    assert (r["v"][0], r["v"][1], r["v"][2]) == (1.0, -INF, 4.0)
    assert res.reduced["m"] == 1 and list(res.reduced["row_map"]) == [1]
    x = res.postsolve(np.array([1.0, 0.0]))
    assert np.array_equal(x, [0.0, 1.0, 0.0])
    # rest above the rhs: x0 takes the difference
    x = res.postsolve(np.array([5.0, 2.0]))
    assert np.array_equal(x, [-3.0, 5.0, 2.0])


def test_finite_input_bound_cost_or_foreign_bound_excludes():
    base = [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]]
    # finite input lower bound
    lp = make(2, 3, base, [-INF, 1.0], [4.0, INF], [0, 0, 0], [INF, 5, 5], [0.0, 1.0, 1.0])
    assert not _fs(O.presolve(lp, **FS))
    # nonzero cost towards an infinite side: unbounded, nothing eliminated
    lp = make(2, 3, base, [-INF, 1.0], [4.0, INF], [-INF, 0, 0], [INF, 5, 5], [1.0, 1.0, 1.0])
    res = O.presolve(lp, **FS)
    assert res.result_name == "UNBOUNDED_OR_INFEASIBLE" and not _fs(res)
    assert highs(lp)[0] == "unbounded"
    # the lower bound comes from another row (a singleton row x0 >= -3, removed)
    lp = make(3, 3, base + [[(0, 1.0)]], [-INF, 1.0, -3.0], [4.0, INF, INF], [-INF, 0, 0], [INF, 5, 5],
              [0.0, 1.0, 1.0])
    res = O.presolve(lp, **FS)
    assert ("SINGLETON_ROW", 2, 0, 1) in _recs(res)
    assert not _fs(res)


def test_two_candidates_in_one_row():
    """x0 and x1 both free, zero-cost singletons of row 0: x0 leaves with the
    row; x1 is then an empty column (c = 0: value 0) in round 2."""
    lp = make(2, 4, [[(0, 1.0), (1, 2.0), (2, 1.0)], [(2, 1.0), (3, 1.0)]], [-INF, 1.0], [4.0, INF],
              [-INF, -INF, 0, 0], [INF, INF, 5, 5], [0.0, 0.0, 1.0, 1.0])
    res = O.presolve(lp, **FS)
    got = _recs(res)
    assert ("FREE_SINGLETON", 0, 0, 1) in got
    assert ("EMPTY_COL", -1, 1, 2) in got
    _check_optimal(lp, res)


def zero_cost_free(lp):
    """The LP with c_j = 0 on every column that has no finite input bound (as
    the workload generator does), so free singletons are frequent."""
    out = dict(lp)
    c = np.array(lp["c"], float)
    c[np.isinf(lp["lb"]) & np.isinf(lp["ub"])] = 0.0
    out["c"] = c
    return out


@pytest.mark.parametrize("seed", range(300))
def test_tiny_replay_and_optimal(seed):
    lp = zero_cost_free(lpgen.tiny(seed, finite_bounds=False))
    for df in (0, 1):
        res = O.presolve(lp, **FS, enable_dual_fix=df)
        replay_free_singletons(lp, res)
        _check_optimal(lp, res)


@pytest.mark.parametrize("seed", range(4))
def test_medium(seed):
    lp = lpgen.make_lp(300, 450, seed=400 + seed, row_len=(2, 7), singleton=10, empty=5, doubleton=20,
                       duplicate=10, fixed_cols=15)
    res = O.presolve(lp, **FS)
    assert replay_free_singletons(lp, res) > 0
    _check_optimal(lp, res)


def test_tiny_family_fires():
    total = sum(len(_fs(O.presolve(zero_cost_free(lpgen.tiny(s)), **FS))) for s in range(300))
    assert total > 30


def test_substitution_into_the_objective():
    """min 2 x0 + x1 with x0 free in row 0 (x0 + x1 + x2 = 4) and row 1
    (x1 + x2 >= 1), x1, x2 in [0, 5]: x0 = 4 - x1 - x2 leaves with row 0
    (r = 2 > 0: the row at its lhs 4); the reduced costs are c1 = 1 - 2 = -1,
    c2 = 0 - 2 = -2 and the offset 2 * 4 = 8; optimum -7 at x1 = x2 = 5,
    x0 = -6."""
    lp = make(2, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [4.0, 1.0], [4.0, INF],
              [-INF, 0, 0], [INF, 5, 5], [2.0, 1.0, 0.0])
    res = O.presolve(lp, **FS)
    r = _fs(res)[0]
    assert (int(r["i"]), int(r["j"]), int(r["side"]), int(r["round"])) == (0, 0, 1, 1)
    red = res.reduced
    assert list(red["c"]) == [-1.0, -2.0] and red["obj_offset"] == 8.0
    x = res.postsolve(np.array([5.0, 5.0]))
    assert np.array_equal(x, [-6.0, 5.0, 5.0])
    _check_optimal(lp, res)


def test_dual_of_a_substituted_row_in_later_rounds():
    """min 2 x0 - x1 + 2 x2 s.t. 0.25 <= x0 + 2 x1 <= 1.75 (row 0), x2 = 0.25
    (row 1), 3 x0 - 2 x2 = -2.75 (row 2), 0.5 x0 - x2 = -0.625 (row 3),
    x0 in [-2, 2], x1 free, x2 in [0, 1]. Round 1 fixes x2 = 0.25 and
    substitutes the free x1 out of row 0 (y0 = -1/2, c0 becomes 2.5); round 2
    fixes x0 = -0.75 from rows 2 and 3, whose dual must carry x0's cost as it
    was then (2.5). The optimum x = (-0.75, 1.25, 0.25) has every column
    strictly inside its bounds, so z = 0, and y0 = c1 / 2 = -1/2."""
    lp = make(4, 3, [[(0, 1.0), (1, 2.0)], [(2, 1.0)], [(0, 3.0), (2, -2.0)], [(0, 0.5), (2, -1.0)]],
              [0.25, 0.25, -2.75, -0.625], [1.75, 0.25, -2.75, -0.625], [-2.0, -INF, 0.0], [2.0, INF, 1.0],
              [2.0, -1.0, 2.0])
    res = O.presolve(lp, **FS)
    fs = _fs(res)
    assert [(int(r["i"]), int(r["j"]), int(r["side"]), int(r["round"])) for r in fs] == [(0, 1, 2, 1)]
    assert res.reduced["n"] == 0
    x, y, z = res.postsolve_dual(np.zeros(0), np.zeros(0))
    assert np.allclose(x, [-0.75, 1.25, 0.25], rtol=0, atol=1e-12)
    assert y[0] == -0.5
    assert np.allclose(z, 0.0, rtol=0, atol=1e-12), z
    assert not kkt_violations(lp, x, y, z)


def test_rows_sharing_a_column_take_turns():
    """x0 (row 0: x0 + x2 = 3) and x1 (row 1: x1 + x2 = 5) are free with cost
    1; both substitutions would change c2, so row 0 (the lowest) goes in
    round 1 and row 1 in round 2: c2 = 0 - 1 - 1 = -2, offset 3 + 5 = 8; x2,
    now in no row with cost -2, is fixed at its upper bound 10 in round 3:
    offset 8 - 20 = -12 (min of x0 + x1 = 8 - 2 x2 over x2 in [0, 10])."""
    lp = make(2, 3, [[(0, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [3.0, 5.0], [3.0, 5.0], [-INF, -INF, 0],
              [INF, INF, 10], [1.0, 1.0, 0.0])
    res = O.presolve(lp, **FS)
    got = [(int(r["i"]), int(r["round"])) for r in _fs(res)]
    assert got == [(0, 1), (1, 2)]
    empty = [r for r in res.records if r["type"] == R["EMPTY_COL"]]
    assert [(int(r["j"]), float(r["v"][0]), float(r["v"][1]), int(r["round"])) for r in empty] == [(2, 10.0, -2.0, 3)]
    red = res.reduced
    assert red["n"] == 0 and red["obj_offset"] == -12.0
    x = res.postsolve(np.zeros(0))
    assert np.array_equal(x, [-7.0, -5.0, 10.0])
    _check_optimal(lp, res)


@pytest.mark.parametrize("seed", range(300))
def test_tiny_with_costs_replay_and_optimal(seed):
    """The tiny family as generated: free columns with costs."""
    lp = lpgen.tiny(seed, finite_bounds=False)
    for df in (0, 1):
        res = O.presolve(lp, **FS, enable_dual_fix=df)
        replay_free_singletons(lp, res)
        _check_optimal(lp, res)


def test_tiny_with_costs_fire():
    total = 0
    for seed in range(300):
        res = O.presolve(lpgen.tiny(seed, finite_bounds=False), **FS)
        total += sum(1 for r in _fs(res) if r["v"][3] != 0)
    assert total > 20


def test_three_rows_sharing_a_column_substitute_one_round_each():
    """Rows i = 0, 1, 2: x_i + x_3 = s_i (3, 5, 7), x_i free with cost c_i
    (1, 2, -1), x_3 in [0, 10] without cost. The rows share x_3, so one row
    substitutes per round, lowest first: rounds 1, 2, 3. x_3's cost becomes
    0 - 1 - 2 + 1 = -2 and it leaves empty at its upper bound 10. The offset is
    1*3 + 2*5 + (-1)*7 (the rows at the sides their costs prefer) - 2*10 = -14."""
    lp = make(3, 4, [[(0, 1.0), (3, 1.0)], [(1, 1.0), (3, 1.0)], [(2, 1.0), (3, 1.0)]], [3.0, 5.0, 7.0],
              [3.0, 5.0, 7.0], [-INF, -INF, -INF, 0.0], [INF, INF, INF, 10.0], [1.0, 2.0, -1.0, 0.0])
    res = O.presolve(lp, enable_free_singletons=1)
    fs = [r for r in res.records if O.REC_NAMES[int(r["type"])] == "FREE_SINGLETON"]
    assert [(int(r["i"]), int(r["j"]), int(r["round"]), int(r["side"])) for r in fs] == [(0, 0, 1, 1), (1, 1, 2, 1),
                                                                                          (2, 2, 3, 2)]
    ec = [r for r in res.records if O.REC_NAMES[int(r["type"])] == "EMPTY_COL"]
    assert [(int(r["j"]), float(r["v"][0]), float(r["v"][1])) for r in ec] == [(3, 10.0, -2.0)]
    assert res.reduced["obj_offset"] == -14.0
