"""Pins of the parallel-row pass on the current problem (section 3.2,
'Parallel rows' with the inactive columns of 'Internal data structures'),
of the key's quantiser, and of what a second presolve may still change.

The parallel-row pass keys and verifies rows over their ACTIVE entries
(columns not fixed or removed), normalised by the first active coefficient;
the merged sides are compared after the removed columns' constant
contribution is moved out of them.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import feasible, highs, load_golden, make, reduced_lp, vertices

INF = np.inf
R = O.REC


def recs(res, name):
    return res.records[res.records["type"] == R[name]]


def test_active_parts_parallel_golden():
    """Hand-derived: the stored rows differ only in fixed columns."""
    g, lp = load_golden("parallel_rows_active.json")
    e = g["expected"]
    res = O.presolve(lp)
    p = recs(res, "PARALLEL_ROW")
    assert p["i"].tolist() == e["removed"] and p["k"].tolist() == [e["leader"]]
    assert p["v"][0][0] == e["lambda"]
    ls = recs(res, "LEADER_SIDES")
    assert len(ls) == 1 and ls[0]["i"] == e["leader"] and ls[0]["k"] == e["src_rhs"]
    assert ls[0]["v"][3] == e["stored_new_rhs"] and ls[0]["v"][2] == -INF
    assert res.reduced["m"] == e["reduced_m"]
    assert res.reduced["rhs"].tolist() == [e["reduced_rhs"]]
    assert res.reduced["lhs"].tolist() == [-INF]


def test_active_parts_negative_lambda_both_sides():
    """Row 0: x0 - 2 x1 + 4 x2 in [-1, 6] with x2 = 0.5 (constant 2): active
    part in [-3, 4]. Row 1: 3 x3 - 2 x0 + 4 x1 in [-10, 2] with x3 = 2
    (constant 6): active part in [-16, -4]; lambda = -2 maps it to
    [-4 / -2, -16 / -2] = [2, 8]. Merged effective sides [max(-3, 2),
    min(4, 8)] = [2, 4]: lhs from row 1, rhs kept by row 0 (stored 6);
    stored lhs 2 + 2 = 4."""
    rows = [[(0, 1.0), (1, -2.0), (2, 4.0)], [(0, -2.0), (1, 4.0), (3, 3.0)]]
    lp = make(2, 4, rows, [-1.0, -10.0], [6.0, 2.0], [-INF, -INF, 0.5, 2.0], [INF, INF, 0.5, 2.0], [0] * 4)
    res = O.presolve(lp)
    p = recs(res, "PARALLEL_ROW")
    assert p["i"].tolist() == [1] and p["k"].tolist() == [0] and p["v"][0][0] == -2.0
    ls = recs(res, "LEADER_SIDES")
    assert len(ls) == 1
    assert (int(ls[0]["j"]), int(ls[0]["k"])) == (1, 0)
    assert ls[0]["v"].tolist() == [-1.0, 6.0, 4.0, 6.0]
    assert res.reduced["lhs"].tolist() == [2.0] and res.reduced["rhs"].tolist() == [4.0]


def test_active_parts_fixed_column_not_in_key():
    """A fixed column breaks the stored pattern but not the active one; a
    column that is only in one row and NOT fixed keeps the rows apart."""
    rows = [[(0, 1.0), (1, 3.0), (2, 5.0)], [(0, 2.0), (1, 6.0)]]
    fixed = make(2, 3, rows, [-INF, -INF], [9.0, 8.0], [-INF, -INF, 1.0], [INF, INF, 1.0], [0] * 3)
    free = make(2, 3, rows, [-INF, -INF], [9.0, 8.0], [-INF, -INF, -INF], [INF, INF, INF], [0] * 3)
    assert len(recs(O.presolve(fixed), "PARALLEL_ROW")) == 1
    assert len(recs(O.presolve(free), "PARALLEL_ROW")) == 0


def test_active_parts_normalised_by_first_active():
    """The first stored coefficient belongs to a fixed column: lambda is the
    ratio of the first ACTIVE coefficients, 3 / 1."""
    rows = [[(0, 7.0), (1, 1.0), (2, 2.0)], [(1, 3.0), (2, 6.0), (3, -5.0)]]
    lp = make(2, 4, rows, [-INF, -INF], [10.0, 9.0], [1.0, -INF, -INF, 0.0], [1.0, INF, INF, 0.0], [0] * 4)
    res = O.presolve(lp)
    p = recs(res, "PARALLEL_ROW")
    assert p["i"].tolist() == [1] and p["v"][0][0] == 3.0
    # effective sides: row 0 <= 10 - 7 = 3, row 1 <= 9 - (-0) = 9 -> 9 / 3 = 3:
    # a tie, kept by the leader (lowest row) with its stored side unchanged
    assert len(recs(res, "LEADER_SIDES")) == 0
    assert res.reduced["rhs"].tolist() == [3.0]


def _bits(x):
    return int(np.array([x]).view(np.uint64)[0])


def _from_bits(b):
    return float(np.array([b], np.uint64).view(np.float64)[0])


def test_quantiser_rounds_bit_19():
    """The key keeps sign, exponent and the top 32 mantissa bits ROUNDED to
    nearest. 1.5 with its low 20 mantissa bits 0x80000 (bit 19 set) rounds up
    to the same 32-bit prefix as the next multiple of 2^20; with 0x7FFFF it
    rounds down. A truncating quantiser gives the opposite answer for both."""
    base = _bits(1.5)
    up = _from_bits(base | 0x80000)
    nxt = _from_bits(base + 0x100000)
    down = _from_bits(base | 0x7FFFF)
    cols = np.array([0, 1], np.int32)
    k_up = O.row_key(cols, np.array([1.0, up]))
    assert k_up == O.row_key(cols, np.array([1.0, nxt]))
    assert k_up != O.row_key(cols, np.array([1.0, down]))
    assert O.row_key(cols, np.array([1.0, down])) == O.row_key(cols, np.array([1.0, 1.5]))


def test_quantiser_decides_which_rows_meet():
    """Rows [1, up] and [1, nxt] share a key and are within par_tol
    (relative difference 2^-32 / 1.5 < 1e-9): merged. Rows [1, up] and
    [1, down] are as close but have different keys: never compared, so not
    merged (quantisation can only miss a pair)."""
    base = _bits(1.5)
    up = _from_bits(base | 0x80000)
    nxt = _from_bits(base + 0x100000)
    down = _from_bits(base | 0x7FFFF)
    for other, merged in ((nxt, 1), (down, 0)):
        rows = [[(0, 1.0), (1, up)], [(0, 1.0), (1, other)]]
        lp = make(2, 2, rows, [-INF, -INF], [4.0, 5.0], [-INF] * 2, [INF] * 2, [0, 0])
        assert len(recs(O.presolve(lp), "PARALLEL_ROW")) == merged


def _fixed_family(seed):
    """Tiny LP with finite bounds where row 1 is lambda times row 0 on the
    active columns and each row also holds a fixed column of its own."""
    rng = np.random.default_rng(70_000 + seed)
    n_act = int(rng.integers(2, 4))
    n = n_act + 2
    lb = np.concatenate([-rng.integers(0, 3, n_act).astype(float), [0.0, 0.0]])
    ub = np.concatenate([rng.integers(1, 5, n_act).astype(float), [0.0, 0.0]])
    fv = rng.choice([-1.0, 0.5, 1.0, 2.0], 2)
    lb[n_act:] = fv
    ub[n_act:] = fv
    base = rng.choice([-2.0, -1.0, 0.5, 1.0, 2.0, 3.0], n_act)
    lam = float(rng.choice([-3.0, -0.5, 0.5, 2.0, 4.0]))
    f0, f1 = rng.choice([-2.0, 1.0, 3.0], 2)
    r0 = [(j, float(base[j])) for j in range(n_act)] + [(n_act, float(f0))]
    r1 = [(j, float(lam * base[j])) for j in range(n_act)] + [(n_act + 1, float(f1))]
    x0 = lb + (ub - lb) * rng.random(n)
    a0 = sum(v * x0[j] for j, v in r0)
    a1 = sum(v * x0[j] for j, v in r1)
    rows = [r0, r1]
    lhs = [a0 - float(rng.integers(0, 3)), -INF]
    rhs = [a0 + float(rng.integers(0, 3)), a1 + float(rng.integers(0, 2))]
    if rng.random() < 0.5:
        j = int(rng.integers(0, n_act))
        k = (j + 1) % n_act
        rows.append([(j, 1.0), (k, -1.0)])
        lhs.append(-INF)
        rhs.append(float(x0[j] - x0[k]) + 1.0)
    c = rng.choice([-2.0, -1.0, 0.0, 1.0, 2.0], n)
    return make(len(rows), n, rows, lhs, rhs, lb, ub, c)


@pytest.mark.parametrize("seed", range(60))
def test_fixed_family_bruteforce(seed):
    """Merging over active parts keeps the feasible set: every vertex of the
    original is feasible for the reduced LP, and the optimum is unchanged
    (vertex enumeration and HiGHS)."""
    lp = _fixed_family(seed)
    res = O.presolve(lp, max_rounds=1)
    V = vertices(lp)
    if res.result_name == "INFEASIBLE":
        assert len(V) == 0 and highs(lp)[0] == "infeasible"
        return
    assert len(V) > 0
    vopt = min(float(lp["c"] @ v) for v in V)
    red = reduced_lp(res.reduced)
    fixed = {int(r["j"]): r["v"][0] for r in res.records if r["type"] == R["FIX_COL"]}
    for v in V:
        for j, val in fixed.items():
            assert abs(v[j] - val) <= 1e-7 * max(1.0, abs(val))
        assert feasible(red, v[res.reduced["col_map"]], tol=1e-7)
    st, obj, xr = highs(red)
    assert st == "optimal" and abs(obj - vopt) <= 1e-7 * max(1.0, abs(vopt))
    x = res.postsolve(xr)
    assert feasible(lp, x, tol=1e-6)


def test_fixed_family_merges():
    """Across the family row 1 is merged into row 0 whenever both rows are
    still alive at the parallel pass (they cannot be redundant and stay)."""
    merged = 0
    for seed in range(60):
        res = O.presolve(_fixed_family(seed), max_rounds=1)
        p = recs(res, "PARALLEL_ROW")
        merged += len(p)
        for r in p:
            assert (int(r["i"]), int(r["k"])) == (1, 0)
    assert merged >= 20


@pytest.mark.parametrize("seed", range(0, 350, 7))
def test_second_presolve_fixpoint(seed):
    """A presolve run to its fixpoint (round caps never reached) leaves
    nothing for a second one: the reduced LP comes back UNCHANGED."""
    lp = lpgen.tiny(seed, finite_bounds=seed < 150)
    res = O.presolve(lp, max_rounds=1000, max_outer=60)
    if res.result_name not in ("REDUCED", "UNCHANGED"):
        return
    again = O.presolve(reduced_lp(res.reduced), max_rounds=1000, max_outer=60)
    assert again.result_name == "UNCHANGED" and len(again.records) == 0


def test_second_presolve_small_workload():
    """The 2000 x 3000 workload: with the default caps (16 rounds, 4 cycles)
    the propagation chains are cut off, so a second presolve only tightens
    more bounds (BOUND_CHANGE records, no row or column removed); run to its
    fixpoint, a second presolve changes nothing."""
    lp = lpgen.single_small()
    res = O.presolve(lp)
    again = O.presolve(reduced_lp(res.reduced))
    assert again.result_name == "REDUCED"
    assert set(again.records["type"].tolist()) == {R["BOUND_CHANGE"]}
    full = O.presolve(lp, max_rounds=1000, max_outer=60)
    again = O.presolve(reduced_lp(full.reduced), max_rounds=1000, max_outer=60)
    assert again.result_name == "UNCHANGED"
