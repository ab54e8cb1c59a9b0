"""Parallel columns in the oracle (section 3.2, "Parallel columns": columns
with a_j = lambda a_k and c_j = lambda c_k merge into one variable whose
bounds follow from both; found as parallel rows of [c A']).

Pins that do not reuse the oracle's arithmetic:
  * closed forms: merged intervals for lambda > 0 and < 0 and for a group of
    three (summed in ascending column order), costs that are not
    proportional, columns stored with 300 entries (no length limit), and
    the postsolve split of a merged value;
  * completeness on tiny LPs with planted scaled copies: no two active
    columns of the reduced LP are parallel (a group lost to a key collision
    or to a length limit fails here);
  * a replay of every PARALLEL_COL record against the original LP: on the
    rows alive at that pass the column equals lambda times its leader's, and
    so does its cost (within the tolerance); each LEADER_BOUNDS interval is
    the sum of the old one and the members' scaled intervals;
  * optimality: HiGHS on the original vs the reduced LP, the postsolved x
    feasible and optimal, the dual postsolve satisfying the original KKT
    conditions, on tiny LPs with planted scaled copies of columns.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import feasible, highs, highs_duals, kkt_violations, make, reduced_lp

R = O.REC
INF = np.inf
PC = dict(enable_parallel_cols=1)


def _recs(res, *types):
    return [r for r in res.records if O.REC_NAMES[int(r["type"])] in types]


def _cols(lp):
    """column j -> {row: coefficient}"""
    cols = [dict() for _ in range(lp["n"])]
    rp, ci, va = lp["row_ptr"], lp["col_idx"], lp["val"]
    for i in range(lp["m"]):
        for k in range(rp[i], rp[i + 1]):
            cols[int(ci[k])][i] = float(va[k])
    return cols


def with_parallel_copies(lp, seed, copies=3):
    """The LP with `copies` new columns, each lambda times an existing one
    (coefficients and cost), with bounds of its own."""
    rng = np.random.default_rng(seed)
    m, n = lp["m"], lp["n"]
    rows = [[(int(lp["col_idx"][k]), float(lp["val"][k])) for k in range(lp["row_ptr"][i], lp["row_ptr"][i + 1])]
            for i in range(m)]
    lb, ub, c = list(lp["lb"]), list(lp["ub"]), list(lp["c"])
    srcs = rng.choice(n, size=min(copies, n), replace=False)
    for t, j in enumerate(srcs):
        lam = float(rng.choice([-2.0, -0.5, 0.5, 1.0, 3.0]))
        newj = n + t
        for i in range(m):
            for (col, a) in list(rows[i]):
                if col == j:
                    rows[i].append((newj, lam * a))
        lo = float(rng.choice([0.0, -1.0, -INF]))
        hi = float(rng.choice([2.0, 5.0, INF]))
        lb.append(lo)
        ub.append(hi)
        c.append(lam * c[j])
    return make(m, n + len(srcs), rows, lp["lhs"], lp["rhs"], lb, ub, c)


def replay_parallel_cols(lp, res, tol=1e-9):
    cols = _cols(lp)
    rec = res.records
    removed = {}
    for r in rec:
        if r["type"] in (R["EMPTY_ROW"], R["REDUNDANT_ROW"], R["SINGLETON_ROW"], R["PARALLEL_ROW"],
                         R["FREE_SINGLETON"]):
            removed.setdefault(int(r["i"]), int(r["round"]))
    n = 0
    groups = {}
    for r in rec:
        if r["type"] == R["PARALLEL_COL"]:
            rd, j, k, lam = int(r["round"]), int(r["j"]), int(r["k"]), r["v"][0]
            # rows alive at the column pass: not removed up to this pass (the
            # pass's parallel rows leave before its columns are compared)
            cj = {i: a for i, a in cols[j].items() if removed.get(i, 10**9) > rd}
            ck = {i: a for i, a in cols[k].items() if removed.get(i, 10**9) > rd}
            assert set(cj) == set(ck), (j, k)
            for i in cj:
                assert abs(cj[i] - lam * ck[i]) <= 1e-7 * max(1.0, abs(cj[i])), (j, k, i)
            assert abs(lp["c"][j] - lam * lp["c"][k]) <= 1e-7 * max(1.0, abs(lp["c"][j]))
            groups.setdefault((rd, k), []).append(r)
            n += 1
    for r in rec:
        if r["type"] == R["LEADER_BOUNDS"]:
            lo, up = r["v"][0], r["v"][1]
            for q in groups[(int(r["round"]), int(r["j"]))]:
                lam, l, u = q["v"][0], q["v"][1], q["v"][2]
                a, b = (lam * l, lam * u) if lam > 0 else (lam * u, lam * l)
                lo, up = lo + a, up + b
                lo = -INF if lo <= -1e20 else lo
                up = INF if up >= 1e20 else up
            assert (lo, up) == (r["v"][2], r["v"][3]), (r["j"], lo, up, r["v"])
    return n


def _check_optimal(lp, res):
    def feas(p):
        z = dict(p)
        z["c"] = np.zeros(p["n"])
        return highs(z)[0]
    st, obj, _ = highs(lp)
    if res.result_name == "INFEASIBLE":
        assert feas(lp) == "infeasible"
        return
    if res.result_name == "UNBOUNDED_OR_INFEASIBLE":
        assert st in ("unbounded", "infeasible")
        return
    red = reduced_lp(res.reduced)
    st2, obj2, xr = highs(red)
    assert feas(red) == feas(lp)
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


# rows 0, 1 hold x0 and x1 = 2 x0 (and x2); costs proportional
BASE_ROWS = [[(0, 1.0), (1, 2.0), (2, 1.0)], [(0, -1.0), (1, -2.0), (2, 3.0)]]


def test_off_by_default():
    assert O.DEFAULTS["enable_parallel_cols"] == 0
    lp = make(2, 3, BASE_ROWS, [1.0, -INF], [10.0, 4.0], [0, 1, 0], [3, 2, 5], [1.0, 2.0, 1.0])
    assert not _recs(O.presolve(lp), "PARALLEL_COL")


def test_merge_positive_lambda():
    """x1 = 2 x0 in every row and c1 = 2 c0: x0' = x0 + 2 x1 in [0 + 2, 3 + 4]."""
    lp = make(2, 3, BASE_ROWS, [1.0, -INF], [10.0, 4.0], [0, 1, 0], [3, 2, 5], [1.0, 2.0, 1.0])
    res = O.presolve(lp, **PC, enable_parallel_rows=0)
    lb_rec = _recs(res, "LEADER_BOUNDS")
    pc = _recs(res, "PARALLEL_COL")
    assert [(int(r["j"]), int(r["k"]), float(r["v"][0])) for r in pc] == [(1, 0, 2.0)]
    assert [(int(r["j"]), *map(float, r["v"])) for r in lb_rec][0][3:] == (2.0, 7.0)
    # postsolve split: merged value 5 -> x1 from its lower bound 1 (5 - 2*1 = 3 in [0, 3]), x0 = 3
    red = res.reduced
    k = list(red["col_map"]).index(0)
    xr = np.zeros(red["n"])
    xr[k] = 5.0
    x = res.postsolve(xr)
    assert (x[0], x[1]) == (3.0, 1.0)
    # merged value 2.5: x1 = 1 would leave 0.5 (fine), so x1 = 1, x0 = 0.5
    xr[k] = 2.5
    x = res.postsolve(xr)
    assert (x[0], x[1]) == (0.5, 1.0)
    # merged value 6: x1 must rise to 1.5 so that x0 = 3
    xr[k] = 6.0
    x = res.postsolve(xr)
    assert (x[0], x[1]) == (3.0, 1.5)


def test_merge_negative_lambda_and_group_of_three():
    rows = [[(0, 1.0), (1, -1.0), (2, 0.5), (3, 1.0)], [(0, 2.0), (1, -2.0), (2, 1.0), (3, -1.0)]]
    lp = make(2, 4, rows, [1.0, -INF], [10.0, 4.0], [0, 1, -2, 0], [3, 2, 4, 5], [1.0, -1.0, 0.5, 1.0])
    res = O.presolve(lp, **PC, enable_parallel_rows=0)
    pc = _recs(res, "PARALLEL_COL")
    assert [(int(r["j"]), int(r["k"]), float(r["v"][0])) for r in pc] == [(1, 0, -1.0), (2, 0, 0.5)]
    lbr = _recs(res, "LEADER_BOUNDS")[0]
    # [0, 3] + (-1)[1, 2] = [-2, 2]; + 0.5 [-2, 4] = [-3, 4]
    assert (float(lbr["v"][2]), float(lbr["v"][3])) == (-3.0, 4.0)
    _check_optimal(lp, res)


def test_not_proportional():
    lp = make(2, 3, BASE_ROWS, [1.0, -INF], [10.0, 4.0], [0, 1, 0], [3, 2, 5], [1.0, 3.0, 1.0])
    assert not _recs(O.presolve(lp, **PC), "PARALLEL_COL")


def test_long_columns_merge():
    """No length limit: x0 and x1 = 2 x0 in 300 rows x0 + 2 x1 + (1 + i % 3)
    x2 >= 5 + i / 100 (no bound tightens: the residual maxima are too large),
    costs 1 and 2: one PARALLEL_COL (1, 0, lambda 2), interval [0, 3] + 2 [1, 2]."""
    rows = [[(0, 1.0), (1, 2.0), (2, 1.0 + i % 3)] for i in range(300)]
    lp = make(300, 3, rows, [5.0 + i / 100 for i in range(300)], [INF] * 300, [0, 1, 0], [3, 2, 5],
              [1.0, 2.0, 1.0])
    res = O.presolve(lp, **PC, enable_parallel_rows=0)
    pc = _recs(res, "PARALLEL_COL")
    assert [(int(r["j"]), int(r["k"]), float(r["v"][0])) for r in pc] == [(1, 0, 2.0)]
    lbr = _recs(res, "LEADER_BOUNDS")[0]
    assert (float(lbr["v"][2]), float(lbr["v"][3])) == (2.0, 7.0)
    _check_optimal(lp, res)


def test_merged_interval_past_inf_value_is_not_merged():
    """x0, x1 = 2 x0, x2 = 3 x0 (coefficients and costs): the scaled bounds
    sum to a lower bound of 4e19 + 2 * 3e19 = 1e20 = inf_value, infinite under
    the convention, which no finite value satisfies: the group stays as it is.
    With bounds a thousand times smaller the same group merges, to the sum of
    the scaled intervals."""
    rows = [[(0, 1.0), (1, 2.0), (2, 3.0), (3, 1.0)], [(0, 2.0), (1, 4.0), (2, 6.0), (3, -1.0)]]
    c = [1.0, 2.0, 3.0, 0.5]
    lp = make(2, 4, rows, [-1e19, -INF], [INF, 1e19], [4e19, 3e19, -9e19, -1], [5e19, 4e19, 1.0, 1], c)
    res = O.presolve(lp, **PC, enable_parallel_rows=0)
    assert not _recs(res, "PARALLEL_COL", "LEADER_BOUNDS")
    assert res.result_name == "REDUCED" and res.reduced["n"] == 4
    # the mirror: bounds negated, the upper sum's partial -4e19 + 2 * -3e19 = -1e20
    lp = make(2, 4, rows, [-INF, -1e19], [1e19, INF], [-5e19, -4e19, -1.0, -1], [-4e19, -3e19, 9e19, 1], c)
    res = O.presolve(lp, **PC, enable_parallel_rows=0)
    assert not _recs(res, "PARALLEL_COL", "LEADER_BOUNDS")
    assert res.result_name == "REDUCED" and res.reduced["n"] == 4
    # sides that keep both rows and tighten no bound (the merge sees the input bounds)
    lp = make(2, 4, rows, [-1.6e17, -INF], [INF, 2.5e17], [4e16, 3e16, -9e16, -1], [5e16, 4e16, 1.0, 1], c)
    res = O.presolve(lp, **PC, enable_parallel_rows=0)
    assert [(int(r["j"]), int(r["k"]), float(r["v"][0])) for r in _recs(res, "PARALLEL_COL")] == [(1, 0, 2.0),
                                                                                                   (2, 0, 3.0)]
    lbr = _recs(res, "LEADER_BOUNDS")[0]
    assert (float(lbr["v"][2]), float(lbr["v"][3])) == (4e16 + 2 * 3e16 + 3 * -9e16, 5e16 + 2 * 4e16 + 3 * 1.0)


def nan_cases():
    """Groups x0, x1 = 2 x0, x2 = 3 x0 (coefficients and costs) whose partial
    sum reaches inf_value on the wrong side before an infinite member term:
    lower: 4e19 + 2 * 3e19 = 1e20 -> +inf, then 3 * -inf; upper: the mirror.
    x2 is free and x4 (not proportional) is free too, so every row has two
    infinite contributions on each side and no bound is tightened first."""
    rows = [[(0, 1.0), (1, 2.0), (2, 3.0), (3, 1.0), (4, 1.0)],
            [(0, 2.0), (1, 4.0), (2, 6.0), (3, -1.0), (4, -1.0)]]
    c = [1.0, 2.0, 3.0, 0.5, 0.25]
    lower = make(2, 5, rows, [-1e19, -INF], [INF, 1e19], [4e19, 3e19, -INF, -1, -INF], [5e19, 4e19, INF, 1, INF], c)
    upper = make(2, 5, rows, [-1e19, -INF], [INF, 1e19], [-5e19, -4e19, -INF, -1, -INF], [-4e19, -3e19, INF, 1, INF],
                 c)
    return {"lower": lower, "upper": upper}


def test_wrong_side_then_infinite_member_not_merged():
    """The partial sum is +inf (-inf for the upper side) when the infinite
    member's term comes: +inf + -inf is NaN, and the group is not merged
    (no NaN bound may reach the reduced problem)."""
    for name, lp in nan_cases().items():
        res = O.presolve(lp, **PC, enable_parallel_rows=0)
        assert not _recs(res, "PARALLEL_COL", "LEADER_BOUNDS"), name
        assert res.result_name == "REDUCED" or res.result_name == "UNCHANGED", name
        red = res.reduced
        assert red["n"] == 5 and not np.isnan(red["lb"]).any() and not np.isnan(red["ub"]).any(), name


@pytest.mark.parametrize("seed", range(300))
def test_tiny_planted_replay_optimal(seed):
    lp = with_parallel_copies(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), seed)
    for extra in ({}, dict(enable_dual_fix=1, enable_free_singletons=1)):
        res = O.presolve(lp, **PC, **extra)
        replay_parallel_cols(lp, res)
        _check_optimal(lp, res)


def with_long_parallel(seed, m=400, n=600, dense=6, copies=4):
    """A random LP whose first `dense` columns sit in about half of the rows
    (stored with far more than 64 entries), plus `copies` columns that are
    lambda times dense ones (some of them, with a few of their entries on
    rows that then get removed, in fewer alive rows than stored). Rows have
    feasible sides around a random point."""
    rng = np.random.default_rng(seed)
    x0 = rng.uniform(-1, 1, n + copies)
    rows = []
    for i in range(m):
        cols = set(rng.choice(np.arange(dense, n), size=int(rng.integers(2, 6)), replace=False).tolist())
        cols |= {j for j in range(dense) if rng.random() < 0.5}
        rows.append({int(j): float(rng.choice([-2.0, -1.0, 1.0, 1.5, 3.0])) for j in cols})
    srcs = rng.choice(dense, size=copies, replace=True)
    c = list(rng.choice([0.0, 1.0, -1.0, 2.0], size=n))
    lb = [-1.0 - rng.random() * 2 for _ in range(n)]
    ub = [1.0 + rng.random() * 2 for _ in range(n)]
    for t, j in enumerate(srcs):
        lam = float(rng.choice([-2.0, 0.5, 3.0]))
        for r in rows:
            if int(j) in r:
                r[n + t] = lam * r[int(j)]
        c.append(lam * c[int(j)])
        lb.append(float(rng.choice([-1.0, -INF])))
        ub.append(float(rng.choice([2.0, INF])))
    lhs, rhs = [], []
    for r in rows:
        act = sum(a * x0[j] for j, a in r.items())
        kind = rng.random()
        lhs.append(act - 1.0 if kind < 0.7 else -INF)
        rhs.append(act + 1.0 if kind > 0.3 else INF)
    return make(m, n + copies, [sorted(r.items()) for r in rows], lhs, rhs, lb, ub, c)


@pytest.mark.parametrize("seed", range(12))
def test_long_parallel_family(seed):
    lp = with_long_parallel(seed)
    for extra in ({}, dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_rows=0)):
        res = O.presolve(lp, **PC, **extra)
        assert replay_parallel_cols(lp, res) >= 1
        assert any(lp["row_ptr"][-1] and int(r["k"]) < 6 for r in _recs(res, "PARALLEL_COL"))
        if res.result_name in ("REDUCED", "UNCHANGED"):
            assert_no_parallel_left(res)
        _check_optimal(lp, res)


def assert_no_parallel_left(res):
    """No two active columns of the reduced LP (each in at least one row)
    are parallel: same rows, a_j = lambda a_k, c_j = lambda c_k."""
    red = res.reduced
    cols = _cols(red)
    c = red["c"]
    for j in range(red["n"]):
        if not cols[j]:
            continue
        for k in range(j):
            if set(cols[j]) != set(cols[k]) or (c[j] != 0) != (c[k] != 0):
                continue
            fj = c[j] if c[j] != 0 else cols[j][min(cols[j])]
            fk = c[k] if c[k] != 0 else cols[k][min(cols[k])]
            lam = fj / fk
            same = all(abs(cols[j][i] - lam * cols[k][i]) <= 1e-12 * max(1.0, abs(cols[j][i])) for i in cols[j])
            assert not same, (j, k, lam)


@pytest.mark.parametrize("seed", range(300))
def test_tiny_planted_complete(seed):
    lp = with_parallel_copies(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), seed)
    res = O.presolve(lp, **PC)
    if res.result_name in ("REDUCED", "UNCHANGED"):
        assert_no_parallel_left(res)


def test_tiny_planted_fire():
    total = 0
    for seed in range(300):
        lp = with_parallel_copies(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), seed)
        total += len(_recs(O.presolve(lp, **PC), "PARALLEL_COL"))
    assert total > 200


@pytest.mark.parametrize("seed", range(3))
def test_medium(seed):
    lp = with_parallel_copies(lpgen.make_lp(300, 450, seed=500 + seed, row_len=(2, 7), singleton=10, empty=5,
                                            doubleton=20, duplicate=10, fixed_cols=15), seed, copies=20)
    res = O.presolve(lp, **PC)
    n = replay_parallel_cols(lp, res)
    if res.result_name in ("REDUCED", "UNCHANGED"):
        assert n > 0
    _check_optimal(lp, res)
