"""Doubleton-equality substitution in the oracle (optional,
enable_doubletons): the doubleton-row explorer of section 2.1 ("Explorers":
an equality with two nonzeros eliminates one of its variables; "Postsolver":
the substitution keeps what recovers the eliminated variable). Once per outer
cycle, after the parallel passes, an equality a_j x_j + a_k x_k = b with two
active columns removes x_k = (b - a_j x_j) / a_k from every other row
(fill-in on column j), from the costs and from the bounds (x_k's bounds move
to x_j).

Pins that do not reuse the oracle's arithmetic:
  * closed forms: the reduced LP after one substitution, the choice of the
    eliminated column, fill-in and the in-place row (dead entry) layout, a
    cancelling coefficient, the lowest-row claim between two doubletons that
    share a column, transferred bounds (including an infeasible transfer);
  * brute force on tiny LPs with planted doubleton equalities: every vertex
    of the original, projected, is feasible for the reduced LP; the optimum
    is unchanged (vertex enumeration and HiGHS); postsolve returns a
    feasible, optimal x, and its duals satisfy the original LP's optimality
    conditions (HiGHS duals of the reduced LP only);
  * medium LPs with the other optional reductions: HiGHS optimum and KKT.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import dense, feasible, highs, highs_duals, kkt_violations, make, reduced_lp, vertices

R = O.REC
INF = np.inf
DB = dict(enable_doubletons=1)


def _recs(res, *names):
    return res.records[np.isin(res.records["type"], [R[n] for n in names])]


def test_off_by_default():
    lp = make(2, 3, [[(0, 1.0), (1, 2.0)], [(0, 1.0), (1, 1.0), (2, 1.0)]], [4.0, -INF], [4.0, 5.0],
              [0, 0, 0], [10, 3, 4], [1.0, -1.0, -2.0])
    assert not len(_recs(O.presolve(lp), "DOUBLETON_ROW"))
    assert len(_recs(O.presolve(lp, **DB), "DOUBLETON_ROW")) == 1


def test_closed_form_substitution():
    """x0 + 2 x1 = 4 (row 0), x0 + x1 + x2 <= 5 (row 1), x in [0,10]x[0,3]x[0,4],
    c = (1, -1, -2), one round. Both columns have two rows and |2| > |1|, so
    x1 = (4 - x0) / 2 leaves: row 1 becomes 0.5 x0 + x2 <= 5 - 2 = 3, the cost
    of x0 becomes 1 - (-1/2) 1 = 1.5, the offset gains -1 * 4 / 2 = -2."""
    lp = make(2, 3, [[(0, 1.0), (1, 2.0)], [(0, 1.0), (1, 1.0), (2, 1.0)]], [4.0, -INF], [4.0, 5.0],
              [0, 0, 0], [10, 3, 4], [1.0, -1.0, -2.0])
    res = O.presolve(lp, **DB, max_rounds=1, max_outer=1)
    d = _recs(res, "DOUBLETON_ROW")
    assert [(int(r["i"]), int(r["j"]), int(r["k"])) for r in d] == [(0, 0, 1)]
    assert d[0]["v"].tolist() == [1.0, 2.0, 4.0, -1.0]
    red = res.reduced
    assert red["m"] == 1 and red["col_map"].tolist() == [0, 2]
    assert red["val"].tolist() == [0.5, 1.0] and red["rhs"].tolist() == [3.0]
    assert red["c"].tolist() == [1.5, -2.0] and red["obj_offset"] == -2.0
    # x1 = (4 - x0) / 2 in [0, 2] (the round tightened its ub to 2): x0 in [0, 4]
    assert red["lb"].tolist() == [0.0, 0.0] and red["ub"].tolist() == [4.0, 4.0]
    x = res.postsolve(np.array([0.0, 3.0]))
    assert x.tolist() == [0.0, 2.0, 3.0]


def test_eliminated_column_choice():
    """The column in fewer alive rows leaves; on a tie the larger |a|; on a
    tie of both the lower index."""
    # x1 is in one row, x0 in two: x1 leaves
    lp = make(2, 3, [[(0, 1.0), (1, 1.0)], [(0, 3.0), (2, 1.0)]], [2.0, -INF], [2.0, 9.0], [-INF] * 3, [INF] * 3,
              [0, 0, 0])
    d = _recs(O.presolve(lp, **DB, max_rounds=1, max_outer=1), "DOUBLETON_ROW")
    assert (int(d[0]["j"]), int(d[0]["k"])) == (0, 1)
    # same rows each, |-3| > |1|: x1 leaves
    lp = make(1, 2, [[(0, 1.0), (1, -3.0)]], [2.0], [2.0], [-INF] * 2, [INF] * 2, [1, 1])
    d = _recs(O.presolve(lp, **DB, max_rounds=1, max_outer=1), "DOUBLETON_ROW")
    assert (int(d[0]["j"]), int(d[0]["k"])) == (0, 1)
    # full tie: the lower index (x0) leaves
    lp = make(1, 2, [[(0, 2.0), (1, -2.0)]], [2.0], [2.0], [-INF] * 2, [INF] * 2, [1, 1])
    d = _recs(O.presolve(lp, **DB, max_rounds=1, max_outer=1), "DOUBLETON_ROW")
    assert (int(d[0]["j"]), int(d[0]["k"])) == (1, 0)


def test_fill_in_and_dead_entries():
    """Row 0: x0 + x3 = 1; x3 is in rows 0-2, x0 in rows 0, 1, 3, 4, so x3 = 1 - x0
    leaves. Row 1 holds both: x0's coefficient 2 - 1 = 1, x3's entry becomes a
    dead +0 entry, rhs 10 - 1 = 9. Row 2 lacks x0: x0 takes x3's place at its
    sorted position (the entries between move) with coefficient 0 - 4 = -4,
    rhs 20 - 4 = 16. Rows 3, 4 do not hold x3 and stay."""
    rows = [[(0, 1.0), (3, 1.0)], [(0, 2.0), (1, 1.0), (3, 1.0)], [(1, 1.0), (2, 1.0), (3, 4.0)],
            [(0, 1.0), (4, 1.0)], [(0, 1.0), (2, 1.0)]]
    lp = make(5, 5, rows, [1.0] + [-INF] * 4, [1.0, 10.0, 20.0, 30.0, 40.0], [-INF] * 5, [INF] * 5, [0] * 5)
    res = O.presolve(lp, **DB, max_rounds=1, max_outer=1, enable_parallel_rows=0)
    d = _recs(res, "DOUBLETON_ROW")
    assert [(int(r["i"]), int(r["j"]), int(r["k"])) for r in d] == [(0, 0, 3)]
    red = res.reduced
    assert red["row_map"].tolist() == [1, 2, 3, 4] and red["col_map"].tolist() == [0, 1, 2, 4]
    assert dense(reduced_lp(red)).tolist() == [[1.0, 1.0, 0.0, 0.0], [-4.0, 1.0, 1.0, 0.0],
                                                [1.0, 0.0, 0.0, 1.0], [1.0, 0.0, 1.0, 0.0]]
    assert red["rhs"].tolist() == [9.0, 16.0, 30.0, 40.0]
    # reduced row 2's CSR keeps x0 first (inserted at its sorted place)
    q0, q1 = red["row_ptr"][1], red["row_ptr"][2]
    assert red["col_idx"][q0:q1].tolist() == [0, 1, 2] and red["val"][q0:q1].tolist() == [-4.0, 1.0, 1.0]


def test_cancellation_skips_the_substitution():
    """Row 1 has x0 with 2 and x1 with 2; eliminating x1 = 1 - x0 gives
    2 - 2 * 1 = 0 on x0: the candidate is dropped."""
    rows = [[(0, 1.0), (1, 1.0)], [(0, 2.0), (1, 2.0), (2, 1.0)]]
    lp = make(2, 3, rows, [1.0, -INF], [1.0, 5.0], [-INF] * 3, [INF] * 3, [0, 0, 0])
    res = O.presolve(lp, **DB, max_rounds=1, max_outer=1, enable_parallel_rows=0)
    assert not len(_recs(res, "DOUBLETON_ROW"))


def test_claims_between_two_doubletons():
    """Rows 0 and 1 are doubleton equalities sharing x1: in the first cycle row
    0 (the lower index) substitutes; row 1 is then x0 - x2 ... and, still a
    doubleton equality over two columns of which x0 was kept (its entries
    rewritten), it is not substituted again."""
    rows = [[(0, 1.0), (1, 1.0)], [(1, 1.0), (2, 1.0)], [(0, 1.0), (2, 1.0), (3, 1.0)]]
    lp = make(3, 4, rows, [1.0, 2.0, -INF], [1.0, 2.0, 9.0], [-INF] * 4, [INF] * 4, [0, 0, 0, 0])
    res = O.presolve(lp, **DB, enable_parallel_rows=0)
    d = _recs(res, "DOUBLETON_ROW")
    assert int(d[0]["i"]) == 0
    assert all(int(r["i"]) != 1 or int(r["round"]) > int(d[0]["round"]) for r in d)


def test_bounds_move_to_the_kept_column():
    """x0 - 2 x1 = 0 with x1 in [1, 2] (x1 is in one row, x0 in two): x1 = x0 / 2
    leaves, x0 in [2, 4] (BOUND_CHANGE from row 0, both sides). An
    incompatible x0 in [5, 9] makes the LP infeasible."""
    rows = [[(0, 1.0), (1, -2.0)], [(0, 1.0), (2, 1.0)]]
    lp = make(2, 3, rows, [0.0, -INF], [0.0, 50.0], [-INF, 1, -INF], [INF, 2, INF], [1, 0, 0])
    res = O.presolve(lp, **DB, max_rounds=1, max_outer=1, enable_parallel_rows=0)
    bc = [(int(r["j"]), int(r["side"]), float(r["v"][1]), int(r["k"])) for r in _recs(res, "BOUND_CHANGE")]
    assert (0, 0, 2.0, 0) in bc and (0, 1, 4.0, 0) in bc
    lp = make(2, 3, rows, [0.0, -INF], [0.0, 50.0], [5, 1, -INF], [9, 2, INF], [1, 0, 0])
    res = O.presolve(lp, **DB, enable_parallel_rows=0)
    assert res.result_name == "INFEASIBLE"


def with_doubletons(lp, seed, k=2):
    """lp with k planted doubleton equalities through its feasible point x0."""
    rng = np.random.default_rng(60_000 + seed)
    n = lp["n"]
    if n < 2:
        return lp
    x0 = np.array(lp["x0"], float)
    rows = [[(int(lp["col_idx"][q]), float(lp["val"][q])) for q in range(lp["row_ptr"][i], lp["row_ptr"][i + 1])]
            for i in range(lp["m"])]
    lhs, rhs = list(lp["lhs"]), list(lp["rhs"])
    for _ in range(k):
        j, kk = sorted(rng.choice(n, 2, replace=False).tolist())
        a = rng.choice([-2.0, -1.0, 0.5, 1.0, 3.0], 2)
        b = float(a[0] * x0[j] + a[1] * x0[kk])
        rows.append([(j, float(a[0])), (kk, float(a[1]))])
        lhs.append(b)
        rhs.append(b)
    out = make(len(rows), n, rows, lhs, rhs, lp["lb"], lp["ub"], lp["c"])
    out["x0"] = x0
    return out


@pytest.mark.parametrize("seed", range(200))
def test_tiny_planted_bruteforce_and_kkt(seed):
    lp = with_doubletons(lpgen.tiny(seed, finite_bounds=seed < 120), seed)
    res = O.presolve(lp, **DB)
    st, obj, _ = highs(lp)
    if res.result_name == "INFEASIBLE":
        assert st == "infeasible"
        return
    if res.result_name == "UNBOUNDED_OR_INFEASIBLE":
        assert st in ("unbounded", "infeasible")
        return
    red = reduced_lp(res.reduced)
    if seed < 120:
        V = vertices(lp)
        assert len(V) > 0
        for v in V:
            assert feasible(red, v[res.reduced["col_map"]], tol=1e-7)
    st2, xr, yr = highs_duals(red)
    if st2 == "empty":
        xr, yr = np.zeros(0), np.zeros(red["m"])
        obj2 = red["obj_offset"]
        st2 = "optimal"
    elif st2 == "optimal":
        obj2 = float(red["c"] @ xr) + red["obj_offset"]
    assert st2 == st
    if st != "optimal":
        return
    assert abs(obj2 - obj) <= 1e-7 * max(1.0, abs(obj))
    x, y, z = res.postsolve_dual(xr, yr)
    assert feasible(lp, x, tol=1e-6)
    assert abs(float(lp["c"] @ x) - obj) <= 1e-6 * max(1.0, abs(obj))
    bad = kkt_violations(lp, x, y, z)
    assert not bad, bad[:5]


ALL = dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1, enable_forcing_rows=1)


@pytest.mark.parametrize("seed", range(200))
def test_tiny_planted_every_reduction_kkt(seed):
    """The planted family with every optional reduction: the postsolved
    (x, y, z) of a HiGHS optimum of the reduced LP is optimal for the input
    (the doubleton rows often become singleton rows after a substitution into
    the objective, so the dual of a substituted row has to reach them)."""
    lp = with_doubletons(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), seed)
    res = O.presolve(lp, **DB, **ALL)
    if res.result_name not in ("REDUCED", "UNCHANGED"):
        assert highs(lp)[0] in ("infeasible", "unbounded")
        return
    red = reduced_lp(res.reduced)
    st, xr, yr = highs_duals(red)
    if st == "empty":
        xr, yr = np.zeros(0), np.zeros(red["m"])
    elif st != "optimal":
        return
    x, y, z = res.postsolve_dual(xr, yr)
    bad = kkt_violations(lp, x, y, z)
    assert not bad, bad[:5]


def test_tiny_planted_fire():
    fired = sum(len(_recs(O.presolve(with_doubletons(lpgen.tiny(s, finite_bounds=s < 120), s), **DB),
                          "DOUBLETON_ROW")) for s in range(200))
    assert fired >= 60


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("extra", [{}, dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1,
                                             enable_forcing_rows=1)])
def test_medium(seed, extra):
    lp = lpgen.make_lp(300, 450, seed=400 + seed, row_len=(2, 7), singleton=10, empty=5, doubleton=40,
                       duplicate=10, fixed_cols=15)
    res = O.presolve(lp, **DB, **extra)
    assert len(_recs(res, "DOUBLETON_ROW")) >= 10
    st, obj, _ = highs(lp)
    assert st == "optimal" and res.result_name == "REDUCED"
    red = reduced_lp(res.reduced)
    st2, xr, yr = highs_duals(red)
    assert st2 == "optimal"
    assert abs(float(red["c"] @ xr) + red["obj_offset"] - obj) <= 1e-7 * max(1.0, abs(obj))
    x, y, z = res.postsolve_dual(xr, yr)
    assert feasible(lp, x, tol=1e-6)
    bad = kkt_violations(lp, x, y, z)
    assert not bad, bad[:5]
