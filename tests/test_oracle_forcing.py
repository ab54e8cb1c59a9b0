"""Forcing rows in the oracle (optional, enable_forcing_rows): a primal
explorer (section 2.1, "Explorers"; the explorers of Andersen & Andersen
1995 that the paper builds on). A row whose finite min activity reaches its
rhs holds only with every active column at the bound of its min contribution
(a > 0: lb, a < 0: ub); a max activity reaching the lhs, the other way round.
The row leaves (FORCING_ROW) and its columns are fixed at those bounds in
the same round.

Pins that do not reuse the oracle's arithmetic:
  * closed forms on hand LPs: the row's side, the fixed values and the round,
    precedence of infeasible and redundant rows, tiny coefficients excluded;
  * exactness: coefficients whose residual-activity bounds round away from
    the bounds still fix the columns at exactly their bounds;
  * a replay of every FORCING_ROW record against the ORIGINAL LP: at that
    round the row's min (max) activity over the columns' bounds then reaches
    its side, and every active column is then fixed at the forced bound;
  * brute force on tiny LPs with planted forcing rows: every vertex of the
    original stays feasible for the reduced LP, the optimum is unchanged
    (vertex enumeration and HiGHS), and the dual postsolve satisfies the
    original LP's optimality conditions (HiGHS duals of the reduced LP only).
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import feasible, highs, highs_duals, kkt_violations, make, reduced_lp, vertices

R = O.REC
INF = np.inf
FR = dict(enable_forcing_rows=1)


def _recs(res, *names):
    return res.records[np.isin(res.records["type"], [R[n] for n in names])]


def test_off_by_default():
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [0.0], [0, 0], [5, 4], [1, 1])
    assert not len(_recs(O.presolve(lp), "FORCING_ROW"))
    assert len(_recs(O.presolve(lp, **FR), "FORCING_ROW")) == 1


def test_min_side_closed_form():
    """x0 + x1 <= 0 with x in [0,5] x [0,4]: min activity 0 = rhs, so both
    columns sit at 0; round 1 removes the row and fixes both at 0."""
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [0.0], [0, 0], [5, 4], [1, 1])
    res = O.presolve(lp, **FR)
    f = _recs(res, "FORCING_ROW")
    assert f["i"].tolist() == [0] and f["side"].tolist() == [0] and f["round"].tolist() == [1]
    assert f["v"][0].tolist() == [0.0, -INF, 0.0, 0.0]
    fx = _recs(res, "FIX_COL")
    assert fx["j"].tolist() == [0, 1] and fx["v"][:, 0].tolist() == [0.0, 0.0]
    assert res.reduced["m"] == 0 and res.reduced["n"] == 0


def test_max_side_negative_coefficient():
    """-x0 + 2 x1 >= 10 with x0 in [-2, 3], x1 in [0, 4]: max activity
    2 + 8 = 10 = lhs, so x0 = -2 (a < 0: its lb gives the max contribution)
    and x1 = 4."""
    lp = make(1, 2, [[(0, -1.0), (1, 2.0)]], [10.0], [INF], [-2, 0], [3, 4], [1, 1])
    res = O.presolve(lp, **FR)
    f = _recs(res, "FORCING_ROW")
    assert f["side"].tolist() == [1] and f["v"][0][0] == 10.0
    bc = _recs(res, "BOUND_CHANGE")
    assert [(int(r["j"]), int(r["side"]), float(r["v"][1]), int(r["k"])) for r in bc] == [(0, 1, -2.0, 0),
                                                                                         (1, 0, 4.0, 0)]
    fx = _recs(res, "FIX_COL")
    assert fx["v"][:, 0].tolist() == [-2.0, 4.0]


def test_exact_bounds_despite_rounding():
    """0.1 x0 + 0.2 x1 + 0.3 x2 <= 0.6, x in [1, 10]: the min activity is
    fl(0.1 + 0.2 + 0.3) = 0.6000000000000001, within tol of the rhs. The
    residual bounds round below 1 (a crossing), while the forcing row fixes
    every column at exactly 1."""
    lp = make(1, 3, [[(0, 0.1), (1, 0.2), (2, 0.3)]], [-INF], [0.6], [1, 1, 1], [10, 10, 10], [1, 1, 1])
    res = O.presolve(lp, **FR)
    assert res.result_name == "REDUCED"
    assert _recs(res, "FIX_COL")["v"][:, 0].tolist() == [1.0, 1.0, 1.0]
    assert len(_recs(res, "FORCING_ROW")) == 1


def test_precedence_and_exclusions():
    # min activity above rhs + tol: infeasible, not forcing
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [-1e-3], [0, 0], [5, 4], [1, 1])
    assert O.presolve(lp, **FR).result_name == "INFEASIBLE"
    # both sides hold for every point: redundant, not forcing
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [9.0], [0, 0], [5, 4], [1, 1])
    res = O.presolve(lp, **FR)
    assert len(_recs(res, "REDUNDANT_ROW")) == 1 and not len(_recs(res, "FORCING_ROW"))
    # an infinite contribution on the forced side: not forcing
    lp = make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [0.0], [0, -INF], [5, 4], [1, 1])
    assert not len(_recs(O.presolve(lp, **FR), "FORCING_ROW"))
    # a tiny active coefficient (below coef_tol): not forcing
    lp = make(1, 2, [[(0, 1.0), (1, 1e-12)]], [-INF], [0.0], [0, 0], [5, 4], [1, 1])
    assert not len(_recs(O.presolve(lp, **FR), "FORCING_ROW"))
    # one active column: the singleton rule applies instead
    lp = make(1, 2, [[(0, 1.0), (1, 2.0)]], [-INF], [2.0], [0, 1], [5, 1], [1, 1])
    res = O.presolve(lp, **FR)
    assert not len(_recs(res, "FORCING_ROW")) and len(_recs(res, "SINGLETON_ROW")) == 1


def _activity_bounds(rows, lb, ub, i):
    lo = hi = 0.0
    for j, a in rows[i].items():
        lo += a * (lb[j] if a > 0 else ub[j])
        hi += a * (ub[j] if a > 0 else lb[j])
    return lo, hi


def replay(lp, res):
    """Every FORCING_ROW against the ORIGINAL LP and the record stream: the
    columns' bounds and the row's sides at that round are rebuilt from the
    records; the forced activity must be within tol of the side, and every
    active column of the row must be fixed (in that round) at the forced
    bound."""
    m, n = lp["m"], lp["n"]
    rows = [dict() for _ in range(m)]
    for i in range(m):
        for q in range(lp["row_ptr"][i], lp["row_ptr"][i + 1]):
            rows[i][int(lp["col_idx"][q])] = float(lp["val"][q])
    lb, ub = np.array(lp["lb"], float).copy(), np.array(lp["ub"], float).copy()
    lhs, rhs = np.array(lp["lhs"], float).copy(), np.array(lp["rhs"], float).copy()
    active = np.ones(n, bool)
    active[lb == ub] = False
    recs = res.records
    seen = 0
    for t, r in enumerate(recs):
        typ = int(r["type"])
        if typ == R["FORCING_ROW"]:
            i = int(r["i"])
            cols = [j for j in rows[i] if active[j]]
            assert len(cols) >= 2
            lo, hi = _activity_bounds(rows, lb, ub, i)
            side = int(r["side"])
            target = rhs[i] if side == 0 else lhs[i]
            got = lo if side == 0 else hi
            assert abs(got - target) <= 1e-9 * max(1.0, abs(target)) + 1e-12, (got, target)
            # the same round's column records fix every active column there
            fixed = {int(q["j"]): q["v"][0] for q in recs[t:] if q["round"] == r["round"]
                     and int(q["type"]) == R["FIX_COL"]}
            for j in cols:
                a = rows[i][j]
                want = lb[j] if (side == 0) == (a > 0) else ub[j]
                assert j in fixed and fixed[j] == want, (j, fixed.get(j), want)
            seen += 1
        elif typ == R["BOUND_CHANGE"]:
            (lb if int(r["side"]) == 0 else ub)[int(r["j"])] = r["v"][1]
        elif typ in (R["FIX_COL"], R["EMPTY_COL"], R["DUAL_FIX"]):
            j = int(r["j"])
            lb[j] = ub[j] = r["v"][0]
            active[j] = False
        elif typ == R["LEADER_SIDES"]:
            lhs[int(r["i"])], rhs[int(r["i"])] = r["v"][2], r["v"][3]
    return seen


def with_forcing_rows(lp, seed, k=2):
    """lp (finite bounds) with k planted forcing rows: random columns and
    coefficients, one side set to the min (or max) activity."""
    rng = np.random.default_rng(50_000 + seed)
    n = lp["n"]
    rows = [[(int(lp["col_idx"][q]), float(lp["val"][q])) for q in range(lp["row_ptr"][i], lp["row_ptr"][i + 1])]
            for i in range(lp["m"])]
    lhs, rhs = list(lp["lhs"]), list(lp["rhs"])
    lb, ub = np.array(lp["lb"], float), np.array(lp["ub"], float)
    fin = [j for j in range(n) if np.isfinite(lb[j]) and np.isfinite(ub[j]) and lb[j] < ub[j]]
    for _ in range(k):
        if len(fin) < 2:
            break
        cols = sorted(rng.choice(fin, size=int(rng.integers(2, min(4, len(fin)) + 1)), replace=False))
        vals = rng.choice([-2.0, -1.0, -0.5, 0.5, 1.0, 3.0], size=len(cols))
        lo = sum(a * (lb[j] if a > 0 else ub[j]) for j, a in zip(cols, vals))
        hi = sum(a * (ub[j] if a > 0 else lb[j]) for j, a in zip(cols, vals))
        rows.append([(int(j), float(a)) for j, a in zip(cols, vals)])
        if rng.random() < 0.5:
            lhs.append(-INF if rng.random() < 0.5 else lo - 1.0)
            rhs.append(lo)
        else:
            lhs.append(hi)
            rhs.append(INF if rng.random() < 0.5 else hi + 1.0)
    out = make(len(rows), n, rows, lhs, rhs, lb, ub, lp["c"])
    return out


@pytest.mark.parametrize("seed", range(150))
def test_tiny_planted_bruteforce_and_kkt(seed):
    lp = with_forcing_rows(lpgen.tiny(seed, finite_bounds=True), seed)
    res = O.presolve(lp, **FR)
    V = vertices(lp)
    if res.result_name == "INFEASIBLE":
        assert len(V) == 0 and highs(lp)[0] == "infeasible"
        return
    replay(lp, res)
    assert len(V) > 0
    vopt = min(float(lp["c"] @ v) for v in V)
    red = reduced_lp(res.reduced)
    fixed = {int(r["j"]): r["v"][0] for r in res.records if r["type"] == R["FIX_COL"]}
    for v in V:
        for j, val in fixed.items():
            assert abs(v[j] - val) <= 1e-7 * max(1.0, abs(val))
        assert feasible(red, v[res.reduced["col_map"]], tol=1e-7)
    st, xr, yr = highs_duals(red)
    if st == "empty":
        xr, yr = np.zeros(0), np.zeros(red["m"])
        obj = red["obj_offset"]
    else:
        assert st == "optimal"
        obj = float(red["c"] @ xr) + red["obj_offset"]
    assert abs(obj - vopt) <= 1e-7 * max(1.0, abs(vopt))
    x, y, z = res.postsolve_dual(xr, yr)
    assert feasible(lp, x, tol=1e-6)
    assert abs(float(lp["c"] @ x) - vopt) <= 1e-6 * max(1.0, abs(vopt))
    bad = kkt_violations(lp, x, y, z)
    assert not bad, bad[:5]


def test_tiny_planted_fire():
    fired = sum(len(_recs(O.presolve(with_forcing_rows(lpgen.tiny(s, finite_bounds=True), s), **FR),
                          "FORCING_ROW")) for s in range(150))
    assert fired >= 100


@pytest.mark.parametrize("seed", range(4))
def test_medium_with_other_reductions(seed):
    """A 300 x 450 LP with planted forcing rows (bounded columns), with the
    other optional reductions on and off: replay, HiGHS optimum and KKT."""
    base = lpgen.make_lp(300, 450, seed=200 + seed, row_len=(2, 7), singleton=10, empty=5, doubleton=20,
                         duplicate=10, fixed_cols=15)
    base = dict(base)
    rng = np.random.default_rng(seed)
    lb, ub = np.array(base["lb"]), np.array(base["ub"])
    inf_ub = ~np.isfinite(ub)
    ub = np.where(inf_ub, np.where(np.isfinite(lb), lb, 0.0) + rng.uniform(1, 10, len(ub)), ub)
    lb = np.where(np.isfinite(lb), lb, ub - 20.0)
    base["lb"], base["ub"] = lb, ub
    lp = with_forcing_rows(base, seed, k=30)
    for extra in ({}, dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1)):
        res = O.presolve(lp, **FR, **extra)
        if res.result_name == "INFEASIBLE":
            assert highs(lp)[0] == "infeasible"
            continue
        assert replay(lp, res) >= 10
        st, obj, _ = highs(lp)
        red = reduced_lp(res.reduced)
        st2, xr, yr = highs_duals(red)
        assert st == "optimal" and st2 == "optimal"
        obj2 = float(red["c"] @ xr) + red["obj_offset"]
        assert abs(obj2 - obj) <= 1e-7 * max(1.0, abs(obj))
        x, y, z = res.postsolve_dual(xr, yr)
        bad = kkt_violations(lp, x, y, z)
        assert not bad, bad[:5]
