"""Parallel columns on the GPU against the oracle, bit for bit (result,
records, reduced problem), with enable_parallel_cols = 1, alone and with the
other optional reductions.

The library keys the candidate columns, sorts them stably by key (and by LP
in a batch) and lets each group's first column verify and merge the others
in order; the oracle sorts (key, column) pairs on the host. Also: primal and
dual postsolve bit for bit against the oracle (the server too: the split
needs no original rows), batches of more than 256 LPs (two sort passes by
LP), and the parallel pass with rows off and columns on.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import make
from tests.parity_util import assert_same
from tests.test_oracle_parcols import BASE_ROWS, with_long_parallel, with_parallel_copies

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")

INF = np.inf
PC = dict(enable_parallel_cols=1)
ALL = dict(enable_parallel_cols=1, enable_dual_fix=1, enable_free_singletons=1)


def run_both(lp, **settings):
    s = {**PC, **settings}
    ref = O.presolve(lp, **{k: v for k, v in s.items() if k in O.DEFAULTS})
    got, p = psl.presolve(lp, **s)
    p.close()
    return got, ref


def _n_pc(records):
    return int((records["type"] == O.REC["PARALLEL_COL"]).sum())


@pytest.mark.parametrize("seed", range(0, 120))
def test_tiny_planted(seed):
    lp = with_parallel_copies(lpgen.tiny(seed, finite_bounds=seed % 2 == 0), seed)
    got, ref = run_both(lp, **(ALL if seed % 3 == 0 else {}))
    assert_same(got, ref, f"tiny {seed}")


@pytest.mark.parametrize("seed", range(12))
def test_long_columns(seed):
    """Columns stored with about 200 entries and their scaled copies: keyed
    and verified by wavefronts."""
    lp = with_long_parallel(seed)
    for extra in ({}, dict(ALL, enable_parallel_rows=0)):
        got, ref = run_both(lp, **extra)
        assert _n_pc(ref.records) >= 1
        assert_same(got, ref, f"long {seed} {extra}")


def test_long_hand_case():
    rows = [[(0, 1.0), (1, 2.0), (2, 1.0 + i % 3)] for i in range(300)]
    lp = make(300, 3, rows, [5.0 + i / 100 for i in range(300)], [INF] * 300, [0, 1, 0], [3, 2, 5], [1.0, 2.0, 1.0])
    got, ref = run_both(lp, enable_parallel_rows=0)
    assert _n_pc(ref.records) == 1
    assert_same(got, ref, "long hand case")


def test_hand_cases():
    cases = [
        make(2, 3, BASE_ROWS, [1.0, -INF], [10.0, 4.0], [0, 1, 0], [3, 2, 5], [1.0, 2.0, 1.0]),
        make(2, 4, [[(0, 1.0), (1, -1.0), (2, 0.5), (3, 1.0)], [(0, 2.0), (1, -2.0), (2, 1.0), (3, -1.0)]],
             [1.0, -INF], [10.0, 4.0], [0, 1, -2, 0], [3, 2, 4, 5], [1.0, -1.0, 0.5, 1.0]),
        make(2, 3, BASE_ROWS, [1.0, -INF], [10.0, 4.0], [0, 1, 0], [3, 2, 5], [1.0, 3.0, 1.0]),
    ]
    for k, lp in enumerate(cases):
        for rows_on in (0, 1):
            got, ref = run_both(lp, enable_parallel_rows=rows_on)
            assert_same(got, ref, f"hand {k} rows {rows_on}")


def test_wrong_side_then_infinite_member():
    from tests.test_oracle_parcols import nan_cases
    for name, lp in nan_cases().items():
        for rows_on in (0, 1):
            got, ref = run_both(lp, enable_parallel_cols=1, enable_parallel_rows=rows_on)
            assert not (ref.records["type"] == O.REC["PARALLEL_COL"]).any()
            assert_same(got, ref, f"{name} rows {rows_on}")


@pytest.mark.parametrize("seed", range(3))
def test_medium_planted(seed):
    lp = with_parallel_copies(lpgen.make_lp(300, 450, seed=500 + seed, row_len=(2, 7), singleton=10, empty=5,
                                            doubleton=20, duplicate=10, fixed_cols=15), seed, copies=20)
    got, ref = run_both(lp)
    assert_same(got, ref, f"medium {seed}")


@pytest.mark.parametrize("seed", [0, 1])
def test_single_small(seed):
    got, ref = run_both(lpgen.single_small(seed=seed))
    assert _n_pc(ref.records) > 0
    assert_same(got, ref, f"small {seed}")


@pytest.mark.parametrize("scale", [0.003, 0.02])
def test_power_law_scaled(scale):
    for extra in ({}, ALL):
        got, ref = run_both(lpgen.power_law(scale=scale), **extra)
        assert_same(got, ref, f"power-law {scale} {extra}")


def test_large_scaled():
    got, ref = run_both(lpgen.large(scale=0.0005), **ALL)
    assert_same(got, ref, "large 0.0005")


def test_postsolve_matches_oracle():
    lps = [lpgen.single_small(seed=7)] + [with_parallel_copies(lpgen.tiny(s), s) for s in range(30)]
    for seed, lp in enumerate(lps):
        ref = O.presolve(lp, **ALL)
        got, p = psl.presolve(lp, **ALL)
        try:
            if ref.result_name not in ("REDUCED", "UNCHANGED"):
                continue
            rng = np.random.default_rng(seed)
            xr = rng.normal(size=got["reduced"]["n"]) * 3
            yr = rng.normal(size=got["reduced"]["m"])
            assert np.array_equal(p.postsolve(xr).view(np.uint64), ref.postsolve(xr).view(np.uint64)), seed
            for a, b in zip(p.postsolve(xr, yr), ref.postsolve_dual(xr, yr)):
                assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), seed
        finally:
            p.close()


def test_batch_equals_alone_many_lps():
    """300 LPs: the sort by LP takes two 8-bit passes."""
    lps = [with_parallel_copies(lpgen.tiny(s % 150, finite_bounds=s % 2 == 0), s) for s in range(300)]
    lps += [lpgen.single_small(seed=6)]
    for extra in (PC, ALL):
        b = psl.Batch(lps, **extra)
        try:
            b.run()
            for idx, lp in enumerate(lps):
                ref = O.presolve(lp, **extra)
                name = b.results[idx]
                got = {"result_name": name, "records": b.records(idx),
                       "reduced": b.reduced(idx) if name in ("REDUCED", "UNCHANGED") else None}
                assert_same(got, ref, f"batch LP {idx} {extra}")
                if name in ("REDUCED", "UNCHANGED") and extra is PC:
                    xr = np.random.default_rng(idx).normal(size=got["reduced"]["n"])
                    assert np.array_equal(b.postsolve(idx, xr).view(np.uint64), ref.postsolve(xr).view(np.uint64))
        finally:
            b.close()


def test_server_postsolve_of_merged_columns():
    lp = with_parallel_copies(lpgen.single_small(seed=12), 12, copies=20)
    sv = psl.Server(hbm_budget_bytes=2 << 30, max_batch_lps=4, max_batch_rows=20_000, max_batch_cols=30_000,
                    max_batch_nnz=200_000, **PC)
    try:
        t = sv.submit(lp)
        sv.drain()
        sv.wait(t, 60_000)
        ref = O.presolve(lp, **PC)
        got = {"result_name": sv.info(t)["result_name"], "records": sv.records(t), "reduced": sv.reduced(t)}
        assert_same(got, ref, "server")
        assert _n_pc(got["records"]) > 0
        xr = np.random.default_rng(3).normal(size=got["reduced"]["n"])
        assert np.array_equal(sv.postsolve(t, xr).view(np.uint64), ref.postsolve(xr).view(np.uint64))
        sv.release(t)
    finally:
        sv.close()


def test_setting_validated():
    with pytest.raises(psl.PslError) as ei:
        psl.Presolver(lpgen.tiny(0), enable_parallel_cols=2)
    assert ei.value.status == psl.PSL_ERR_INVALID


def proportional_group(size, seed, infinite=True):
    """`size` columns proportional to one pattern in two rows (scales of both
    signs, costs scaled alike) beside one other column; bounds mix ordinary,
    huge (near 1e20) and infinite values, so that partial sums of the merged
    interval cross inf_value and infinite terms enter it."""
    rng = np.random.default_rng(seed)
    lam = rng.choice([0.5, 1.0, 2.0, 3.0, -1.0, -2.5], size=size)
    rows = [[(j, 1.0 * lam[j]) for j in range(size)] + [(size, 1.0)],
            [(j, 2.0 * lam[j]) for j in range(size)] + [(size, -1.0)]]
    lb, ub = [], []
    for _ in range(size):
        kind = rng.integers(0, 4 if infinite else 2)
        if kind == 0:
            a = float(rng.uniform(-5, 5)); lb.append(a); ub.append(a + float(rng.uniform(0, 3)))
        elif kind == 1:
            a = float(rng.uniform(3e19, 9e19)) * rng.choice([-1, 1]); lb.append(min(a, 0.0)); ub.append(max(a, 0.0))
        elif kind == 2:
            lb.append(-INF); ub.append(float(rng.uniform(0, 5)))
        else:
            lb.append(float(rng.uniform(-5, 0))); ub.append(INF)
    return make(2, size + 1, rows, [-1e19, -INF], [INF, 1e19], lb + [-1.0], ub + [1.0],
                [float(l) for l in lam] + [0.5])


def test_merged_intervals_crossing_inf_value():
    """Groups whose merged interval passes inf_value part way (the canonical
    fold turns it infinite for good) or meets infinite terms, in groups longer
    than one batch of loads of the accumulation."""
    cases = [make(2, 4, [[(0, 1.0), (1, 2.0), (2, 3.0), (3, 1.0)], [(0, 2.0), (1, 4.0), (2, 6.0), (3, -1.0)]],
                  [-1e19, -INF], [INF, 1e19], [4e19, 3e19, -9e19, -1], [5e19, 4e19, 1.0, 1], [1.0, 2.0, 3.0, 0.5]),
             make(2, 4, [[(0, 1.0), (1, 2.0), (2, 3.0), (3, 1.0)], [(0, 2.0), (1, 4.0), (2, 6.0), (3, -1.0)]],
                  [-INF, -1e19], [1e19, INF], [-5e19, -4e19, -1.0, -1], [-4e19, -3e19, 9e19, 1], [1.0, 2.0, 3.0, 0.5])]
    cases += [proportional_group(size, seed) for seed, size in enumerate((3, 5, 17, 40, 40, 40))]
    cases += [proportional_group(size, 10 + seed, infinite=False) for seed, size in enumerate((4, 17, 33, 40))]
    merged = 0
    for k, lp in enumerate(cases):
        got, ref = run_both(lp)
        assert_same(got, ref, f"group case {k}")
        merged += int((ref.records["type"] == O.REC["LEADER_BOUNDS"]).sum())
    assert merged >= 3
