"""Pins of the CPU oracle against values the paper or the mathematics fix.

Every expected value here is derived by hand (in the docstring) or comes from
an independent source (exact rational arithmetic, math.fsum, a golden
fixture citing the paper); none is produced by re-running the oracle's own
formula.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import load_golden, make

INF = np.inf
R = O.REC


def recs(res, name):
    return res.records[res.records["type"] == R[name]]


# --------------------------------------------------------------------------
# canonical pairwise summation
# --------------------------------------------------------------------------

def test_pairwise_tree_shape_four_leaves():
    """[2^53, 1, 1, -2^53]: the tree is (2^53 + 1) + (1 - 2^53).
    2^53 + 1 is a tie and rounds to the even 2^53; 1 - 2^53 = -(2^53 - 1) is
    exact; the root is 1. Left-to-right summation gives 0, the exact sum is 2."""
    assert O.pairwise_sum([2.0 ** 53, 1.0, 1.0, -(2.0 ** 53)]) == 1.0


def test_pairwise_padding_odd_length():
    """Length 3 pads to 4 leaves: (x0 + x1) + (x2 + 0). With [1, 2^53, -2^53]:
    1 + 2^53 rounds to 2^53, minus 2^53 is 0. A tree split at len//2 would
    give 1 + (2^53 - 2^53) = 1."""
    assert O.pairwise_sum([1.0, 2.0 ** 53, -(2.0 ** 53)]) == 0.0


def test_pairwise_padding_length_five():
    """[2^53, 1, 1, 1, 1] pads to 8: ((2^53+1) + (1+1)) + ((1+0) + 0) =
    (2^53 + 2) + 1 = 2^53 + 3, a tie between 2^53+2 (odd significand) and
    2^53+4 (even), so 2^53 + 4. Left to right gives 2^53."""
    assert O.pairwise_sum([2.0 ** 53, 1.0, 1.0, 1.0, 1.0]) == 2.0 ** 53 + 4


def test_pairwise_empty_and_single():
    assert O.pairwise_sum([]) == 0.0
    assert O.pairwise_sum([-3.25]) == -3.25


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 65, 1000, 4097])
def test_pairwise_error_bound(n):
    """Pairwise summation error is at most gamma_k * sum|x|, k = ceil(log2 n),
    gamma_k = k u / (1 - k u), u = 2^-53 (Higham, Accuracy and Stability of
    Numerical Algorithms, sec. 4.2). Reference: math.fsum (correctly rounded)."""
    rng = np.random.default_rng(n)
    x = rng.normal(size=n) * np.exp(rng.uniform(-20, 20, size=n))
    s = O.pairwise_sum(x)
    exact = math.fsum(x)
    k = max(1, math.ceil(math.log2(n))) if n > 1 else 0
    u = 2.0 ** -53
    bound = k * u / (1 - k * u) * float(np.sum(np.abs(x))) + abs(exact) * u
    assert abs(s - exact) <= bound


def test_pairwise_integers_exact():
    x = np.arange(-500, 1500, dtype=np.float64)
    assert O.pairwise_sum(x) == float(sum(range(-500, 1500)))


# --------------------------------------------------------------------------
# activities with infinite-bound counts
# --------------------------------------------------------------------------

def test_activities_against_exact_rationals():
    """Min/max activity of each row of a random LP: the count of infinite
    contributions is exact, and the finite part is within the pairwise bound
    of the exact rational sum of a*lb (a>0) / a*ub (a<0) (min) and the reverse
    (max)."""
    lp = lpgen.power_law(seed=5, scale=0.002)
    mn, mx, nmin, nmax = O.activities(lp)
    rp, ci, va, lb, ub = lp["row_ptr"], lp["col_idx"], lp["val"], lp["lb"], lp["ub"]
    u = 2.0 ** -53
    for i in range(lp["m"]):
        tmin, tmax, cmin, cmax, absmin, absmax = Fraction(0), Fraction(0), 0, 0, 0.0, 0.0
        for k in range(rp[i], rp[i + 1]):
            a, j = va[k], ci[k]
            bmin = lb[j] if a > 0 else ub[j]
            bmax = ub[j] if a > 0 else lb[j]
            if np.isinf(bmin):
                cmin += 1
            else:
                p = a * bmin  # one rounding per product
                tmin += Fraction(p)
                absmin += abs(p)
            if np.isinf(bmax):
                cmax += 1
            else:
                p = a * bmax
                tmax += Fraction(p)
                absmax += abs(p)
        L = rp[i + 1] - rp[i]
        kk = max(1, math.ceil(math.log2(L))) if L > 1 else 0
        g = kk * u / (1 - kk * u)
        assert nmin[i] == cmin and nmax[i] == cmax
        assert abs(Fraction(mn[i]) - tmin) <= Fraction(g * absmin + 1e-300)
        assert abs(Fraction(mx[i]) - tmax) <= Fraction(g * absmax + 1e-300)


def test_redundant_row_activities_recorded():
    """0.5 x1 + 0.25 x2 <= 10 with x1 in [0, 4], x2 in [-2, 8]:
    min activity 0 - 0.5 = -0.5, max activity 2 + 2 = 4 <= 10, so the row is
    redundant in round 1 and its record carries (-0.5, 4, -inf, 10)."""
    lp = make(1, 2, [[(0, 0.5), (1, 0.25)]], [-INF], [10.0], [0, -2], [4, 8], [1, 1])
    res = O.presolve(lp)
    r = recs(res, "REDUNDANT_ROW")
    assert len(r) == 1 and r[0]["i"] == 0 and r[0]["round"] == 1
    assert list(r[0]["v"]) == [-0.5, 4.0, -INF, 10.0]


def test_redundant_with_infinite_min():
    """x1 - x2 <= 5, x1 in [0, 3], x2 in [0, inf): the max activity 3 - 0 = 3
    is finite and <= 5, the min activity is -inf (one infinite contribution):
    redundant; record v = (-inf, 3, -inf, 5)."""
    lp = make(1, 2, [[(0, 1.0), (1, -1.0)]], [-INF], [5.0], [0, 0], [3, INF], [1, 1])
    res = O.presolve(lp)
    r = recs(res, "REDUNDANT_ROW")
    assert len(r) == 1 and list(r[0]["v"]) == [-INF, 3.0, -INF, 5.0]


# --------------------------------------------------------------------------
# propagation (section 3.1)
# --------------------------------------------------------------------------

def test_paper_worked_example():
    g, lp = load_golden("worked_example_propagation.json")
    res = O.presolve(lp, max_rounds=1, enable_parallel_rows=0)
    bc = recs(res, "BOUND_CHANGE")
    bc = bc[bc["round"] == 1]
    ub = {int(r["j"]): r["v"][1] for r in bc if r["side"] == 1}
    assert ub == {0: g["expected_round1_upper_bounds"][0], 1: g["expected_round1_upper_bounds"][1]}
    assert all(r["k"] == 0 for r in bc)
    assert [r["v"][2] for r in bc if r["side"] == 1] == [1.0, 2.0]  # a_src,j


def test_negative_coefficient_lower_side():
    """-x1 + x2 >= -3 (lhs = -3, rhs = inf), x1 >= 0, x2 in [0, 2]:
    -x1 >= -3 - x2 >= -5, so x1 <= 5; x2 >= -3 + x1 >= -3 gives nothing."""
    lp = make(1, 2, [[(0, -1.0), (1, 1.0)]], [-3.0], [INF], [0, 0], [INF, 2], [1, 1])
    res = O.presolve(lp, max_rounds=1, enable_parallel_rows=0)
    bc = recs(res, "BOUND_CHANGE")
    assert [(int(r["j"]), int(r["side"]), r["v"][1]) for r in bc] == [(0, 1, 5.0)]


def test_one_infinite_contribution():
    """x1 + x2 <= 4, x1 in [0, inf), x2 free: the min activity has exactly one
    infinite contribution (x2's lower bound), so only x2 gets a bound:
    x2 <= 4 - min(x1) = 4. x1's residual contains x2's -inf, no bound."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [4.0], [0, -INF], [INF, INF], [1, 0])
    res = O.presolve(lp, max_rounds=1, enable_parallel_rows=0)
    bc = recs(res, "BOUND_CHANGE")
    assert [(int(r["j"]), int(r["side"]), r["v"][1]) for r in bc] == [(1, 1, 4.0)]


def test_min_improve_threshold():
    """x1 + x2 <= 1 - 1e-8, x1 in [0, 1], x2 in [0, 5]. For x1 the candidate
    1 - 1e-8 improves by 1e-8 < 1e-7 * max(1, 1): rejected. For x2 it improves
    by about 4: accepted, x2 <= 1 - 1e-8."""
    rhs = 1 - 1e-8
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [rhs], [0, 0], [1, 5], [1, 1])
    res = O.presolve(lp, max_rounds=1, enable_parallel_rows=0)
    bc = recs(res, "BOUND_CHANGE")
    assert [(int(r["j"]), int(r["side"]), r["v"][1]) for r in bc] == [(1, 1, rhs)]


def test_singleton_rows_become_bounds():
    """An LP made only of singleton rows reduces to pure bounds:
    2 x1 <= 6 -> x1 <= 3; -x2 <= 4 -> x2 >= -4; 3 <= 0.5 x3 <= 5 -> x3 in [6, 10].
    Every row is removed in round 1."""
    lp = make(3, 3, [[(0, 2.0)], [(1, -1.0)], [(2, 0.5)]], [-INF, -INF, 3.0], [6.0, 4.0, 5.0],
              [-INF, -INF, -INF], [INF, INF, INF], [-1.0, 1.0, 1.0])
    res = O.presolve(lp, enable_parallel_rows=0)
    s = recs(res, "SINGLETON_ROW")
    assert sorted(s["i"].tolist()) == [0, 1, 2] and set(s["round"].tolist()) == {1}
    red = res.reduced
    assert red["m"] == 0
    # the columns are empty once their rows are gone: fixed by cost sign
    # (c = -1 -> upper bound 3; c = 1 -> lower bounds -4 and 6)
    e = recs(res, "EMPTY_COL")
    assert {int(r["j"]): r["v"][0] for r in e} == {0: 3.0, 1: -4.0, 2: 6.0}
    bc = recs(res, "BOUND_CHANGE")
    got = {(int(r["j"]), int(r["side"])): r["v"][1] for r in bc}
    assert got == {(0, 1): 3.0, (1, 0): -4.0, (2, 0): 6.0, (2, 1): 10.0}


def test_empty_column_by_cost_sign_and_unbounded():
    """Columns in no row: c > 0 -> lb, c < 0 -> ub, c = 0 -> clamp(0, lb, ub);
    c < 0 with ub = inf is unbounded (or infeasible)."""
    lp = make(1, 4, [[]], [-1.0], [1.0], [1, -2, -3, 2], [5, 7, 4, 9], [2.0, -1.0, 0.0, 0.0])
    res = O.presolve(lp)
    e = recs(res, "EMPTY_COL")
    assert {int(r["j"]): r["v"][0] for r in e} == {0: 1.0, 1: 7.0, 2: 0.0, 3: 2.0}
    lp2 = make(1, 1, [[]], [-1.0], [1.0], [0.0], [INF], [-1.0])
    assert O.presolve(lp2).result_name == "UNBOUNDED_OR_INFEASIBLE"


def test_input_fixings_round_zero():
    """lb = ub on input: FIX_COL in round 0, ascending column index."""
    lp = make(1, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)]], [-INF], [10.0], [2, 0, 3], [2, 1, 3], [1, 1, 1])
    res = O.presolve(lp)
    f = recs(res, "FIX_COL")
    f0 = f[f["round"] == 0]
    assert f0["j"].tolist() == [0, 2] and [r["v"][0] for r in f0] == [2.0, 3.0]


def test_infeasibility_detection():
    """Empty row with 1 <= 0 <= 2 is infeasible; crossed bounds are infeasible;
    x1 + x2 >= 5 with x in [0, 1]^2 is infeasible (max activity 2 < 5)."""
    assert O.presolve(make(1, 1, [[]], [1.0], [2.0], [0], [1], [0])).result_name == "INFEASIBLE"
    assert O.presolve(make(0, 1, [], [], [], [2.0], [1.0], [0])).result_name == "INFEASIBLE"
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [5.0], [INF], [0, 0], [1, 1], [0, 0])
    assert O.presolve(lp).result_name == "INFEASIBLE"


def test_invalid_input_rejected():
    bad = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [1.0], [0, 0], [1, 1], [0, 0])
    bad["col_idx"] = np.array([1, 0], np.int32)
    with pytest.raises(O.OracleError):
        O.presolve(bad)
    bad = make(1, 2, [[(0, 0.0)]], [-INF], [1.0], [0, 0], [1, 1], [0, 0])
    with pytest.raises(O.OracleError):
        O.presolve(bad)
    bad = make(1, 1, [[(0, 1.0)]], [np.nan], [1.0], [0], [1], [0])
    with pytest.raises(O.OracleError):
        O.presolve(bad)


# --------------------------------------------------------------------------
# parallel rows (section 3.2)
# --------------------------------------------------------------------------

def test_parallel_rows_golden():
    g, lp = load_golden("parallel_rows_merge.json")
    res = O.presolve(lp)
    e = g["expected"]
    p = recs(res, "PARALLEL_ROW")
    assert p["i"].tolist() == e["removed"]
    assert all(int(r["k"]) == e["leader"] for r in p)
    assert {str(int(r["i"])): r["v"][0] for r in p} == e["lambda"]
    ls = recs(res, "LEADER_SIDES")
    assert len(ls) == 1 and ls[0]["i"] == e["leader"]
    assert ls[0]["v"][2] == e["new_lhs"] and ls[0]["v"][3] == e["new_rhs"]
    assert ls[0]["j"] == e["src_lhs"] and ls[0]["k"] == e["src_rhs"]
    assert res.reduced["m"] == 1
    assert res.reduced["lhs"][0] == -1.0 and res.reduced["rhs"][0] == 3.0


def test_parallel_leader_prefers_equality():
    """Rows 0 and 2 are inequalities, row 1 an equality, all parallel: the
    leader is row 1 (first equality); rows 0 and 2 are removed."""
    rows = [[(0, 1.0), (1, 1.0)], [(0, 2.0), (1, 2.0)], [(0, -1.0), (1, -1.0)]]
    lp = make(3, 2, rows, [-INF, 4.0, -10.0], [5.0, 4.0, INF], [-INF] * 2, [INF] * 2, [0, 0])
    res = O.presolve(lp)
    p = recs(res, "PARALLEL_ROW")
    assert p["i"].tolist() == [0, 2] and set(p["k"].tolist()) == {1}


def test_parallel_near_miss_not_merged():
    """Coefficient ratios differing by 1e-6 relative exceed par_tol = 1e-9."""
    rows = [[(0, 1.0), (1, 2.0)], [(0, 1.0), (1, 2.0 * (1 + 1e-6))]]
    lp = make(2, 2, rows, [-INF, -INF], [4.0, 5.0], [-INF] * 2, [INF] * 2, [0, 0])
    res = O.presolve(lp)
    assert len(recs(res, "PARALLEL_ROW")) == 0


def test_row_key_scale_invariant():
    """The key normalises by the first coefficient, so scaling a row by any
    lambda (including negative) whose products are exact leaves it unchanged;
    a different pattern changes it."""
    cols = np.array([3, 7, 11], np.int32)
    v = np.array([1.5, -0.75, 2.0])
    k = O.row_key(cols, v)
    for lam in (-2.0, 0.5, 4.0, -0.25):
        assert O.row_key(cols, v * lam) == k
    assert O.row_key(np.array([3, 7, 12], np.int32), v) != k
    assert O.row_key(cols, np.array([1.5, -0.75, 2.5])) != k


# --------------------------------------------------------------------------
# compaction (section 3.3)
# --------------------------------------------------------------------------

def test_compaction_invariants_small():
    lp = lpgen.single_small()
    res = O.presolve(lp)
    r = res.reduced
    m, n = r["m"], r["n"]
    # CSR and CSC describe the same matrix
    A = np.zeros((m, n))
    for i in range(m):
        for k in range(r["row_ptr"][i], r["row_ptr"][i + 1]):
            A[i, r["col_idx"][k]] = r["val"][k]
    B = np.zeros((m, n))
    for j in range(n):
        for k in range(r["col_ptr"][j], r["col_ptr"][j + 1]):
            B[r["row_idx"][k], j] = r["cval"][k]
    assert np.array_equal(A, B)
    assert r["nnz"] == r["row_ptr"][-1] == r["col_ptr"][-1]
    assert np.all(np.diff(r["row_map"]) > 0) and np.all(np.diff(r["col_map"]) > 0)
    # kept entries are the original coefficients of kept rows and columns
    Ao = np.zeros((lp["m"], lp["n"]))
    for i in range(lp["m"]):
        for k in range(lp["row_ptr"][i], lp["row_ptr"][i + 1]):
            Ao[i, lp["col_idx"][k]] = lp["val"][k]
    assert np.array_equal(Ao[np.ix_(r["row_map"], r["col_map"])], A)
    # every kept row still has an active column
    assert np.all(np.diff(r["row_ptr"]) >= 1)


def test_offset_collects_removed_costs():
    """x1 fixed at 2 (cost 3), x2 empty with cost -1 on [0, 4] -> 4. The row
    x1 + x3 <= 10 becomes the singleton x3 <= 8, x3 (cost 1) is then empty and
    goes to its lower bound 0: offset = 3*2 + (-1)*4 + 1*0 = 2, nothing kept."""
    lp = make(1, 3, [[(0, 1.0), (2, 1.0)]], [-INF], [10.0], [2, 0, 0], [2, 4, 20], [3.0, -1.0, 1.0])
    res = O.presolve(lp, enable_parallel_rows=0)
    r = res.reduced
    assert r["obj_offset"] == 2.0
    assert r["m"] == 0 and r["n"] == 0
