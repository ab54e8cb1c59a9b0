"""Dual fixing in the oracle: the lock-based dual reduction (section 2.1,
"Explorers": dual explorers keep at least one optimal solution; section 3.2,
"Internal data structures": variable locks count the rows that keep a
variable from increasing or decreasing, recomputed on demand).

Pins that do not reuse the oracle's arithmetic:
  * closed forms on hand LPs: the fixed side, value and round (c > 0 at lb,
    c < 0 at ub, c = 0 at a finite bound, an infinite bound => unbounded, a
    lock dropped by a row removed in the same round, locks both ways => kept);
  * a replay of every DUAL_FIX record against the ORIGINAL LP and the record
    stream: the rows alive after that round, their sides at that point and
    the column's bound at that point are rebuilt in Python; the lock in the
    cost direction must be zero and the value must be that bound (a swapped
    side or sign in the lock rule fails here);
  * completeness: no column of the reduced LP is still lock-free towards its
    cost-preferred finite bound (a missed fixing fails here);
  * optimality: HiGHS on the original vs the reduced LP (objective offset
    included), the postsolved x feasible and optimal, and the dual postsolve
    (x, y, z) satisfying the original LP's KKT conditions.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import feasible, highs, highs_duals, kkt_violations, make, reduced_lp

R = O.REC
INF = np.inf


def _df_records(res):
    return [r for r in res.records if r["type"] == R["DUAL_FIX"]]


def _locks(rows, lhs, rhs, alive, j):
    """(down, up) locks of column j over the alive rows (rows: list of
    {col: coefficient})."""
    down = up = 0
    for i, row in enumerate(rows):
        if not alive[i] or j not in row:
            continue
        a = row[j]
        lfin, rfin = np.isfinite(lhs[i]), np.isfinite(rhs[i])
        if a > 0:
            down += lfin
            up += rfin
        else:
            down += rfin
            up += lfin
    return down, up


def _rows_of(lp):
    rp, ci, va = lp["row_ptr"], lp["col_idx"], lp["val"]
    return [{int(ci[k]): float(va[k]) for k in range(rp[i], rp[i + 1])} for i in range(lp["m"])]


def replay_dual_fixes(lp, res):
    """Check every DUAL_FIX record against the LP and the earlier records."""
    rows = _rows_of(lp)
    m = lp["m"]
    rec = res.records
    removed_at = np.full(m, np.iinfo(np.int64).max)
    for r in rec:
        if r["type"] in (R["EMPTY_ROW"], R["REDUNDANT_ROW"], R["SINGLETON_ROW"], R["PARALLEL_ROW"]):
            removed_at[r["i"]] = min(removed_at[r["i"]], int(r["round"]))
    n_checked = 0
    for r in _df_records(res):
        rd, j, side, v, cj = int(r["round"]), int(r["j"]), int(r["side"]), r["v"][0], r["v"][1]
        assert cj == lp["c"][j]
        alive = removed_at > rd  # rows removed up to this round no longer lock
        lhs = np.array(lp["lhs"], float)
        rhs = np.array(lp["rhs"], float)
        lhs[np.abs(lhs) >= 1e20] = -INF
        rhs[np.abs(rhs) >= 1e20] = INF
        lo, up = float(lp["lb"][j]), float(lp["ub"][j])
        for q in rec:
            if q["type"] == R["LEADER_SIDES"] and int(q["round"]) < rd:
                lhs[q["i"]], rhs[q["i"]] = q["v"][2], q["v"][3]
            if q["type"] == R["BOUND_CHANGE"] and int(q["j"]) == j and int(q["round"]) <= rd:
                if q["side"] == 0:
                    lo = q["v"][1]
                else:
                    up = q["v"][1]
        down, upl = _locks(rows, lhs, rhs, alive, j)
        if cj > 0:
            assert side == 0 and down == 0 and v == lo, (j, rd, down, v, lo)
        elif cj < 0:
            assert side == 1 and upl == 0 and v == up, (j, rd, upl, v, up)
        else:
            assert (side == 0 and down == 0 and v == lo) or (side == 1 and upl == 0 and v == up), (j, rd)
        assert np.isfinite(v)
        n_checked += 1
    return n_checked


def assert_complete(res):
    """No kept column of the reduced LP is lock-free towards its cost-preferred
    finite bound."""
    red = res.reduced
    rows = _rows_of(red)
    alive = np.ones(red["m"], bool)
    for j in range(red["n"]):
        down, upl = _locks(rows, red["lhs"], red["rhs"], alive, j)
        c, lo, up = red["c"][j], red["lb"][j], red["ub"][j]
        assert not (c > 0 and down == 0), j
        assert not (c < 0 and upl == 0), j
        assert not (c == 0 and down == 0 and np.isfinite(lo)), j
        assert not (c == 0 and upl == 0 and np.isfinite(up)), j


def _types(res):
    return [O.REC_NAMES[int(t)] for t in res.records["type"]]


def test_off_by_default():
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [10.0], [0, 0], [8, 8], [1.0, 2.0])
    assert O.DEFAULTS["enable_dual_fix"] == 0
    assert "DUAL_FIX" not in _types(O.presolve(lp))


def test_cost_positive_fixes_at_lower_bound():
    """x1 + x2 <= 10 with x in [0, 8]^2 and c = (1, 2): no row keeps either
    variable from decreasing, so round 1 fixes both at 0; round 2 removes the
    then empty row; the reduced LP is empty with optimum 0."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [10.0], [0, 0], [8, 8], [1.0, 2.0])
    res = O.presolve(lp, enable_dual_fix=1)
    df = _df_records(res)
    assert [(int(r["j"]), int(r["side"]), float(r["v"][0]), int(r["round"])) for r in df] == [(0, 0, 0.0, 1),
                                                                                             (1, 0, 0.0, 1)]
    assert "EMPTY_ROW" in _types(res)
    assert res.reduced["m"] == 0 and res.reduced["n"] == 0 and res.reduced["obj_offset"] == 0.0


def test_cost_negative_fixes_at_upper_bound():
    """min -x1 + x2 s.t. x1 + x2 >= 1, x in [0, 3]^2: nothing keeps x1 from
    increasing (the row has no finite rhs), so x1 = 3 (side 1); x2 has the
    row's lhs as a down-lock and stays until the row is redundant."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [1.0], [INF], [0, 0], [3, 3], [-1.0, 1.0])
    res = O.presolve(lp, enable_dual_fix=1)
    df = _df_records(res)
    assert (int(df[0]["j"]), int(df[0]["side"]), float(df[0]["v"][0]), int(df[0]["round"])) == (0, 1, 3.0, 1)
    assert all(int(r["j"]) != 1 for r in df)
    st, obj, _ = highs(lp)
    st2, obj2, _ = highs(reduced_lp(res.reduced))
    assert st == st2 == "optimal" and obj == pytest.approx(obj2) and obj == pytest.approx(-3.0)


def test_infinite_preferred_bound_is_unbounded():
    """min x1 s.t. x1 + x2 <= 4, x1 <= 5 (no lower bound), x2 in [0, 1]:
    decreasing x1 never violates the row, so the LP is unbounded."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [4.0], [-INF, 0], [5, 1], [1.0, 0.0])
    res = O.presolve(lp, enable_dual_fix=1)
    assert res.result_name == "UNBOUNDED_OR_INFEASIBLE"
    assert highs(lp)[0] == "unbounded"


def test_zero_cost_fixes_at_finite_lock_free_bound():
    """min x2 s.t. x1 - x2 <= 2, x1 in [1, 4], x2 in [0, 10]: x1 (c = 0) has
    no down-lock and a finite lower bound: x1 = 1; x2 keeps its down-lock."""
    lp = make(1, 2, [[(0, 1.0), (1, -1.0)]], [-INF], [2.0], [1, 0], [4, 10], [0.0, 1.0])
    res = O.presolve(lp, enable_dual_fix=1)
    df = _df_records(res)
    assert [(int(r["j"]), int(r["side"]), float(r["v"][0])) for r in df] == [(0, 0, 1.0)]


def test_lock_dropped_by_a_row_removed_in_the_same_round():
    """Row 0 (x1 + x2 >= -100) is redundant in round 1 and holds x1's only
    down-lock; the locks are those of the rows alive after the round's
    removals, so x1 is fixed at 0 in round 1, and x2 (c < 0, no up-lock) at
    10 in the same round."""
    lp = make(2, 2, [[(0, 1.0), (1, 1.0)], [(0, 1.0), (1, -1.0)]], [-100.0, -INF], [INF, 5.0], [0, 0],
              [10, 10], [1.0, -1.0])
    res = O.presolve(lp, enable_dual_fix=1)
    got = [(O.REC_NAMES[int(r["type"])], int(r["i"]), int(r["j"]), int(r["round"])) for r in res.records]
    assert ("REDUNDANT_ROW", 0, -1, 1) in got
    assert ("DUAL_FIX", -1, 0, 1) in got and ("DUAL_FIX", -1, 1, 1) in got
    x = res.postsolve(np.zeros(res.reduced["n"]))
    assert np.array_equal(x, [0.0, 10.0])


def test_locks_both_ways_keep_the_column():
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [3.0], [3.0], [0, 0], [5, 5], [1.0, 0.0])
    res = O.presolve(lp, enable_dual_fix=1)
    assert "DUAL_FIX" not in _types(res)
    assert_complete(res)


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


@pytest.mark.parametrize("seed", range(300))
def test_tiny_dual_fix_replay_complete_optimal(seed):
    lp = lpgen.tiny(seed, finite_bounds=seed % 2 == 0)
    res = O.presolve(lp, enable_dual_fix=1)
    replay_dual_fixes(lp, res)
    if res.result_name in ("REDUCED", "UNCHANGED"):
        assert_complete(res)
    _check_optimal(lp, res)


@pytest.mark.parametrize("seed", range(4))
def test_medium_dual_fix(seed):
    lp = lpgen.make_lp(300, 450, seed=300 + seed, row_len=(2, 7), singleton=10, empty=5, doubleton=20,
                       duplicate=10, fixed_cols=15)
    res = O.presolve(lp, enable_dual_fix=1)
    assert replay_dual_fixes(lp, res) > 0
    if res.result_name in ("REDUCED", "UNCHANGED"):
        assert_complete(res)
    _check_optimal(lp, res)


def test_tiny_dual_fix_fires_often():
    """The tiny family exercises the rule: fixings on both sides happen."""
    sides = set()
    for seed in range(300):
        res = O.presolve(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), enable_dual_fix=1)
        sides |= {int(r["side"]) for r in _df_records(res)}
    assert sides == {0, 1}
