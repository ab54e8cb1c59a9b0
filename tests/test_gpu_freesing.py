"""Free column singletons on the GPU against the oracle, bit for bit
(result, records, reduced problem), with enable_free_singletons = 1, alone
and with dual fixing: zero-cost eliminations, and substitutions of columns
with a cost (cost updates, the lowest-index turns of rows sharing a column,
long rows through the chunked claim and update kernels).

The library flags a column when it comes down to one row (and every column
in the first round), finds its alive row on the transposed copy, tracks per
bound side whether every tightening came from one row, and emits the
eliminations after the round's decision records; the oracle checks every
column of every alive row each round. Also: primal and dual postsolve (bit
for bit against the oracle), batches, the server's refusal (it keeps no
original rows) and the setting's validation.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import make
from tests.parity_util import assert_same

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")

INF = np.inf
FS = dict(enable_free_singletons=1)


def zero_cost_free(lp):
    out = dict(lp)
    c = np.array(lp["c"], float)
    c[np.isinf(lp["lb"]) & np.isinf(lp["ub"])] = 0.0
    out["c"] = c
    return out


def run_both(lp, **settings):
    s = {**FS, **settings}
    ref = O.presolve(lp, **{k: v for k, v in s.items() if k in O.DEFAULTS})
    got, p = psl.presolve(lp, **s)
    p.close()
    return got, ref


def _n_fs(records):
    return int((records["type"] == O.REC["FREE_SINGLETON"]).sum())


@pytest.mark.parametrize("seed", range(0, 120))
def test_tiny(seed):
    lp = zero_cost_free(lpgen.tiny(seed, finite_bounds=False))
    got, ref = run_both(lp, enable_dual_fix=seed % 2)
    assert_same(got, ref, f"tiny {seed}")


def test_hand_cases():
    cases = [
        make(2, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [-INF, 1.0], [4.0, INF],
             [-INF, 0, 0], [INF, 5, 5], [0.0, 1.0, 1.0]),
        make(2, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [-INF, 1.0], [4.0, INF],
             [0, 0, 0], [INF, 5, 5], [0.0, 1.0, 1.0]),
        make(3, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)], [(0, 1.0)]], [-INF, 1.0, -3.0],
             [4.0, INF, INF], [-INF, 0, 0], [INF, 5, 5], [0.0, 1.0, 1.0]),
        make(2, 4, [[(0, 1.0), (1, 2.0), (2, 1.0)], [(2, 1.0), (3, 1.0)]], [-INF, 1.0], [4.0, INF],
             [-INF, -INF, 0, 0], [INF, INF, 5, 5], [0.0, 0.0, 1.0, 1.0]),
    ]
    for k, lp in enumerate(cases):
        got, ref = run_both(lp)
        assert_same(got, ref, f"hand {k}")


@pytest.mark.parametrize("seed", range(4))
def test_medium(seed):
    lp = lpgen.make_lp(300, 450, seed=400 + seed, row_len=(2, 7), singleton=10, empty=5, doubleton=20,
                       duplicate=10, fixed_cols=15)
    got, ref = run_both(lp)
    assert _n_fs(ref.records) > 0
    assert_same(got, ref, f"medium {seed}")


@pytest.mark.parametrize("seed", [0, 1])
def test_single_small(seed):
    got, ref = run_both(lpgen.single_small(seed=seed))
    assert _n_fs(ref.records) > 0
    assert_same(got, ref, f"small {seed}")


@pytest.mark.parametrize("scale", [0.003, 0.02])
def test_power_law_scaled(scale):
    for df in (0, 1):
        got, ref = run_both(lpgen.power_law(scale=scale), enable_dual_fix=df)
        assert _n_fs(ref.records) > 0
        assert_same(got, ref, f"power-law {scale} dual fix {df}")


def test_large_scaled_with_chains_and_dense_lines():
    got, ref = run_both(lpgen.large(scale=0.0005))
    assert_same(got, ref, "large 0.0005")


def test_split_sweep_and_bins_do_not_change_results():
    lp = lpgen.single_small(seed=4)
    ref = O.presolve(lp, **FS)
    for extra in (dict(split_sweep=1), dict(bin_thresholds=[16, 2048, 4])):
        got, p = psl.presolve(lp, **FS, **extra)
        p.close()
        assert_same(got, ref, str(extra))


def test_postsolve_matches_oracle():
    for seed, lp in enumerate([lpgen.single_small(seed=7)] +
                              [zero_cost_free(lpgen.tiny(s, finite_bounds=False)) for s in range(30)]):
        ref = O.presolve(lp, **FS)
        got, p = psl.presolve(lp, **FS)
        try:
            if ref.result_name not in ("REDUCED", "UNCHANGED"):
                continue
            rng = np.random.default_rng(seed)
            xr = rng.normal(size=got["reduced"]["n"])
            yr = rng.normal(size=got["reduced"]["m"])
            assert np.array_equal(p.postsolve(xr).view(np.uint64), ref.postsolve(xr).view(np.uint64)), seed
            for a, b in zip(p.postsolve(xr, yr), ref.postsolve_dual(xr, yr)):
                assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), seed
        finally:
            p.close()


def test_batch_equals_alone():
    lps = [zero_cost_free(lpgen.tiny(s, finite_bounds=False)) for s in range(24)]
    lps += [lpgen.single_small(seed=6),
            lpgen.make_lp(300, 450, seed=405, row_len=(2, 7), singleton=10, empty=5, doubleton=20, duplicate=10,
                          fixed_cols=15)]
    for df in (0, 1):
        b = psl.Batch(lps, **FS, enable_dual_fix=df)
        try:
            b.run()
            for idx, lp in enumerate(lps):
                ref = O.presolve(lp, **FS, enable_dual_fix=df)
                name = b.results[idx]
                got = {"result_name": name, "records": b.records(idx),
                       "reduced": b.reduced(idx) if name in ("REDUCED", "UNCHANGED") else None}
                assert_same(got, ref, f"batch LP {idx} dual fix {df}")
                if name in ("REDUCED", "UNCHANGED"):
                    xr = np.random.default_rng(idx).normal(size=got["reduced"]["n"])
                    assert np.array_equal(b.postsolve(idx, xr).view(np.uint64), ref.postsolve(xr).view(np.uint64))
        finally:
            b.close()


def test_server_refuses_postsolve_of_eliminations():
    lp = lpgen.single_small(seed=12)
    sv = psl.Server(hbm_budget_bytes=2 << 30, max_batch_lps=4, max_batch_rows=20_000, max_batch_cols=30_000,
                    max_batch_nnz=200_000, **FS)
    try:
        t = sv.submit(lp)
        sv.drain()
        sv.wait(t, 60_000)
        ref = O.presolve(lp, **FS)
        got = {"result_name": sv.info(t)["result_name"], "records": sv.records(t), "reduced": sv.reduced(t)}
        assert_same(got, ref, "server")
        assert _n_fs(got["records"]) > 0
        with pytest.raises(psl.PslError) as ei:
            sv.postsolve(t, np.zeros(got["reduced"]["n"]))
        assert ei.value.status == psl.PSL_ERR_UNSUPPORTED
        sv.release(t)
    finally:
        sv.close()


def test_setting_validated():
    with pytest.raises(psl.PslError) as ei:
        psl.Presolver(lpgen.tiny(0), enable_free_singletons=3)
    assert ei.value.status == psl.PSL_ERR_INVALID


# ---- substitution of singletons with a cost ---------------------------------

@pytest.mark.parametrize("seed", range(0, 120))
def test_tiny_with_costs(seed):
    lp = lpgen.tiny(seed, finite_bounds=False)
    got, ref = run_both(lp, enable_dual_fix=seed % 2)
    assert_same(got, ref, f"tiny with costs {seed}")


def long_rows_sharing_columns(seed, m=6, width=80):
    """Equality rows of `width` entries, each with one free column with a cost
    and columns shared with the next row, so that long rows claim, lose and
    substitute over rounds."""
    rng = np.random.default_rng(seed)
    n_shared = width - 1
    n = m + n_shared * m // 2 + n_shared
    rows, lhs, rhs = [], [], []
    for i in range(m):
        shared = list(range(m + (i * n_shared) // 2, m + (i * n_shared) // 2 + n_shared))
        cols = [i] + shared
        vals = rng.choice([-2.0, -1.0, 0.5, 1.0, 3.0], size=len(cols))
        rows.append(list(zip(cols, vals)))
        s = float(rng.uniform(1, 5))
        lhs.append(s)
        rhs.append(s)
    lb = [-INF] * m + [0.0] * (n - m)
    ub = [INF] * m + [2.0] * (n - m)
    c = list(rng.choice([-1.0, 1.0, 2.0], size=m)) + list(rng.uniform(-1, 1, size=n - m))
    return make(m, n, rows, lhs, rhs, lb, ub, c)


def test_substitution_cases_and_long_rows():
    cases = [
        make(2, 3, [[(0, 1.0), (1, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [4.0, 1.0], [4.0, INF],
             [-INF, 0, 0], [INF, 5, 5], [2.0, 1.0, 0.0]),
        make(2, 3, [[(0, 1.0), (2, 1.0)], [(1, 1.0), (2, 1.0)]], [3.0, 5.0], [3.0, 5.0], [-INF, -INF, 0],
             [INF, INF, 10], [1.0, 1.0, 0.0]),
        make(3, 4, [[(0, 1.0), (3, 1.0)], [(1, 1.0), (3, 1.0)], [(2, 1.0), (3, 1.0)]], [3.0, 5.0, 7.0],
             [3.0, 5.0, 7.0], [-INF, -INF, -INF, 0.0], [INF, INF, INF, 10.0], [1.0, 2.0, -1.0, 0.0]),
    ] + [long_rows_sharing_columns(s) for s in range(6)]
    for k, lp in enumerate(cases):
        ref = O.presolve(lp, **FS)
        if k >= 3:
            assert _n_fs(ref.records) > 0, k
        got, ref = run_both(lp)
        assert_same(got, ref, f"substitution case {k}")
        if ref.result_name in ("REDUCED", "UNCHANGED"):
            p = psl.Presolver(lp, **FS)
            p.run()
            rng = np.random.default_rng(k)
            xr = rng.normal(size=got["reduced"]["n"])
            yr = rng.normal(size=got["reduced"]["m"])
            for a, b in zip(p.postsolve(xr, yr), ref.postsolve_dual(xr, yr)):
                assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), k
            p.close()


def test_batch_with_costs_equals_alone():
    lps = [lpgen.tiny(s, finite_bounds=False) for s in range(40)] + [long_rows_sharing_columns(s) for s in range(4)]
    b = psl.Batch(lps, **FS, enable_dual_fix=1)
    try:
        b.run()
        for idx, lp in enumerate(lps):
            ref = O.presolve(lp, **FS, enable_dual_fix=1)
            name = b.results[idx]
            got = {"result_name": name, "records": b.records(idx),
                   "reduced": b.reduced(idx) if name in ("REDUCED", "UNCHANGED") else None}
            assert_same(got, ref, f"batch LP {idx}")
    finally:
        b.close()


def dense_column_down_to_one_row(rows, cost, seed=0):
    """`rows` scaled copies of x0 + x1 (inequalities, removed as parallel to
    the leader) and, last, the equality x0 + x1 = 5 that leads them: the free
    column x0, stored with `rows` entries, keeps one alive row, its last."""
    rng = np.random.default_rng(seed)
    lam = rng.uniform(0.5, 3.0, size=rows - 1) * rng.choice([-1.0, 1.0], size=rows - 1)
    body = [[(0, l), (1, l)] for l in lam] + [[(0, 1.0), (1, 1.0)]]
    lhs = [(-INF if l > 0 else 7.0 * l) for l in lam] + [5.0]
    rhs = [(7.0 * l if l > 0 else INF) for l in lam] + [5.0]
    return make(rows, 3, body + [], lhs, rhs, [-INF, 0.0, 0.0], [INF, 10.0, 1.0], [cost, 1.0, -1.0])


def test_dense_column_down_to_one_row():
    """A free column stored with up to 5000 entries becomes a singleton after
    the parallel-row pass; its row is found by the wavefront walk."""
    for rows in (65, 200, 5000):
        for cost in (0.0, 2.0, -1.0):
            lp = dense_column_down_to_one_row(rows, cost, seed=rows)
            got, ref = run_both(lp)
            assert _n_fs(ref.records) == 1, (rows, cost)
            assert_same(got, ref, f"dense column {rows} cost {cost}")
