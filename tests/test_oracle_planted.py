"""Planted reductions of the small synthetic workload are all found by the
oracle; a down-scaled large workload needs at least 5 Jacobi rounds (its
planted 8-row chains move a finite bound one row per round)."""
import numpy as np

from oracle import oracle as O
from paper_2609_16182_amd import lpgen

R = O.REC


def _removed_rows(res):
    t = res.records["type"]
    row_types = [R[k] for k in ("EMPTY_ROW", "REDUNDANT_ROW", "SINGLETON_ROW", "PARALLEL_ROW")]
    return set(res.records["i"][np.isin(t, row_types)].tolist())


def test_planted_small_workload():
    lp = lpgen.single_small()
    res = O.presolve(lp)
    pl = lp["planted"]
    rec = res.records
    empty = set(rec["i"][rec["type"] == R["EMPTY_ROW"]].tolist())
    assert set(pl["empty_rows"].tolist()) <= empty
    fix0 = rec[(rec["type"] == R["FIX_COL"]) & (rec["round"] == 0)]
    assert fix0["j"].tolist() == sorted(pl["fixed_cols"].tolist())
    assert np.array_equal(fix0["v"][:, 0], lp["x0"][np.sort(pl["fixed_cols"])])
    removed = _removed_rows(res)
    assert set(pl["singleton_rows"].tolist()) <= removed
    # of each duplicate pair (row, scaled copy) at least one row is gone
    for d, s in pl["duplicate_pairs"].T:
        assert d in removed or s in removed
    assert int((rec["type"] == R["PARALLEL_ROW"]).sum()) >= 40
    # doubleton equalities that survive are listed as such in the reduced problem
    r = res.reduced
    kept = dict(zip(r["row_map"].tolist(), r["row_class"].tolist()))
    for i in pl["doubleton_rows"]:
        if i in kept and np.diff(r["row_ptr"])[r["row_map"].tolist().index(i)] == 2:
            assert kept[i] == 2


def test_duplicate_pairs_resolved():
    """Generate with known pairs: every duplicate row or its source is removed."""
    lp = lpgen.make_lp(600, 900, seed=77, row_len=(3, 6), duplicate=30)
    res = O.presolve(lp)
    removed = _removed_rows(res)
    par = set(res.records["i"][res.records["type"] == R["PARALLEL_ROW"]].tolist())
    for d, s in lp["planted"]["duplicate_pairs"].T:
        assert d in removed or s in removed
        assert d in par or s in par or (d in removed and s in removed)


def test_large_chains_need_five_rounds():
    lp = lpgen.large(scale=0.0005)
    res = O.presolve(lp, enable_parallel_rows=0)
    assert res.result_name == "REDUCED"
    assert res.rounds >= 5
    rec = res.records
    ch = set(lp["planted"]["chain_rows"].tolist())
    # the chain's upper bounds arrive one round after another
    ub_rounds = sorted(set(rec["round"][(rec["type"] == R["BOUND_CHANGE"]) & np.isin(rec["k"], list(ch))].tolist()))
    assert len(ub_rounds) >= 5
