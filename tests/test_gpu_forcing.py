"""Forcing rows on the GPU against the oracle, bit for bit (result, records,
reduced problem), with enable_forcing_rows = 1: planted forcing rows on
their min and max sides in tiny and medium LPs (with and without the other
optional reductions), the generators' workloads, long rows, every launch
shape, batches (each LP as alone), the dual postsolve, and the setting's
validation."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import highs_duals, kkt_violations, make, reduced_lp
from tests.parity_util import assert_same
from tests.test_oracle_forcing import with_forcing_rows

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")

INF = np.inf
FR = dict(enable_forcing_rows=1)
ALL = dict(enable_forcing_rows=1, enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1)


def run_both(lp, **settings):
    s = {**FR, **settings}
    ref = O.presolve(lp, **{k: v for k, v in s.items() if k in O.DEFAULTS})
    got, p = psl.presolve(lp, **s)
    p.close()
    return got, ref


def _n_fr(records):
    return int((records["type"] == O.REC["FORCING_ROW"]).sum())


@pytest.mark.parametrize("seed", range(0, 150))
def test_tiny_planted(seed):
    lp = with_forcing_rows(lpgen.tiny(seed, finite_bounds=True), seed)
    got, ref = run_both(lp, **(ALL if seed % 3 == 0 else {}))
    assert_same(got, ref, f"tiny {seed}")


def test_hand_cases():
    cases = [
        make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [0.0], [0, 0], [5, 4], [1, 1]),
        make(1, 2, [[(0, -1.0), (1, 2.0)]], [10.0], [INF], [-2, 0], [3, 4], [1, 1]),
        make(1, 3, [[(0, 0.1), (1, 0.2), (2, 0.3)]], [-INF], [0.6], [1, 1, 1], [10, 10, 10], [1, 1, 1]),
        make(1, 2, [[(0, 1.0), (1, 1e-12)]], [-INF], [0.0], [0, 0], [5, 4], [1, 1]),
        make(1, 2, [[(0, 1.0), (1, 1.0)]], [-INF], [-1e-3], [0, 0], [5, 4], [1, 1]),
    ]
    for k, lp in enumerate(cases):
        got, ref = run_both(lp)
        assert_same(got, ref, f"hand {k}")


def bounded_medium(seed, m=300, n=450, k=30):
    """The 300 x 450 generator with every bound made finite around its
    feasible point x0, plus k forcing rows that keep x0 feasible: each
    planted row puts x0 at the bound its side forces (that bound is moved to
    x0_j) and takes the forced activity as its side."""
    base = dict(lpgen.make_lp(m, n, seed=200 + seed, row_len=(2, 7), singleton=10, empty=5, doubleton=20,
                              duplicate=10, fixed_cols=15))
    rng = np.random.default_rng(seed)
    x0 = np.array(base["x0"], float)
    lb, ub = np.array(base["lb"], float), np.array(base["ub"], float)
    lb = np.where(np.isfinite(lb), lb, np.minimum(x0, 0.0) - 20.0)
    ub = np.where(np.isfinite(ub), ub, np.maximum(x0, lb) + rng.uniform(1, 10, n))
    rows = [[(int(base["col_idx"][q]), float(base["val"][q]))
             for q in range(base["row_ptr"][i], base["row_ptr"][i + 1])] for i in range(base["m"])]
    lhs, rhs = list(base["lhs"]), list(base["rhs"])
    free = [j for j in range(n) if lb[j] < ub[j]]
    used = set()
    for _ in range(k):
        cand = [j for j in free if j not in used]
        cols = sorted(rng.choice(cand, size=int(rng.integers(2, 6)), replace=False).tolist())
        used.update(cols)
        vals = rng.choice([-2.0, -1.0, -0.5, 0.5, 1.0, 3.0], size=len(cols))
        side_min = rng.random() < 0.5
        act = 0.0
        for j, a in zip(cols, vals):
            if side_min == (a > 0):
                lb[j] = x0[j]  # x0 sits at lb
            else:
                ub[j] = x0[j]  # x0 sits at ub
            act += a * x0[j]
        rows.append(list(zip(cols, vals.tolist())))
        lhs.append(-INF if side_min else act)
        rhs.append(act if side_min else INF)
    return make(len(rows), n, rows, lhs, rhs, lb, ub, base["c"])


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("extra", [{}, ALL])
def test_medium_planted(seed, extra):
    lp = bounded_medium(seed)
    got, ref = run_both(lp, **extra)
    assert _n_fr(ref.records) >= 10
    assert_same(got, ref, f"medium {seed} {extra}")


def with_long_forcing_rows(seed):
    """A bounded LP with forcing rows of 600 and 5000 entries (wavefront and
    multi-workgroup bins) and one of 3000 with a tiny coefficient (not
    forcing), over a point x0 that every row keeps feasible."""
    rng = np.random.default_rng(77 + seed)
    n = 12000
    lb = -rng.integers(0, 3, n).astype(float)
    ub = rng.integers(1, 5, n).astype(float)
    x0 = lb + (ub - lb) * rng.random(n)
    rows, lhs, rhs = [], [], []
    free = np.arange(n)
    rng.shuffle(free)
    at = 0
    for L, tiny in ((600, False), (5000, False), (3000, True), (40, False), (9, False)):
        cols = np.sort(free[at:at + L])
        at += L
        vals = rng.choice([-2.0, -1.0, 0.5, 1.0, 3.0], L)
        if tiny:
            vals[L // 2] = 1e-12
        side_min = rng.random() < 0.5
        for j, a in zip(cols, vals):
            if side_min == (a > 0):
                lb[j] = x0[j]
            else:
                ub[j] = x0[j]
        act = float(np.dot(vals, x0[cols]))
        rows.append(list(zip(cols.tolist(), vals.tolist())))
        lhs.append(-INF if side_min else act)
        rhs.append(act if side_min else INF)
    for _ in range(3000):  # ordinary short rows over all columns, x0 feasible
        cols = np.sort(rng.choice(n, 5, replace=False))
        vals = rng.choice([-1.0, 1.0, 2.0], 5)
        rows.append(list(zip(cols.tolist(), vals.tolist())))
        lhs.append(-INF)
        rhs.append(float(np.dot(vals, x0[cols])) + 1.0)
    c = rng.choice([-1.0, 0.0, 1.0], n)
    return make(len(rows), n, rows, lhs, rhs, lb, ub, c)


@pytest.mark.parametrize("thr", [None, (16, 2048), (512, 4096, 4)])
def test_long_rows_and_shapes(thr):
    lp = with_long_forcing_rows(0)
    kw = {} if thr is None else dict(bin_thresholds=thr)
    got, ref = run_both(lp, **kw)
    assert _n_fr(ref.records) >= 4
    assert_same(got, ref, f"long {thr}")
    got, ref = run_both(lp, split_sweep=1)
    assert_same(got, ref, "long split")


@pytest.mark.parametrize("wl", ["small", "power", "large"])
def test_workloads(wl):
    lp = {"small": lambda: lpgen.single_small(seed=3), "power": lambda: lpgen.power_law(scale=0.01),
          "large": lambda: lpgen.large(scale=0.0005)}[wl]()
    for extra in ({}, ALL):
        got, ref = run_both(lp, **extra)
        assert_same(got, ref, f"{wl} {extra}")


def test_dual_postsolve():
    for seed in range(30):
        lp = with_forcing_rows(lpgen.tiny(seed, finite_bounds=True), seed)
        got, p = psl.presolve(lp, **FR)
        try:
            if got["result_name"] not in ("REDUCED", "UNCHANGED"):
                continue
            red = reduced_lp(got["reduced"])
            st, xr, yr = highs_duals(red)
            if st == "empty":
                xr, yr = np.zeros(0), np.zeros(red["m"])
            elif st != "optimal":
                continue
            x, y, z = p.postsolve(xr, yr)
            ref = O.presolve(lp, **FR)
            for a, b in zip((x, y, z), ref.postsolve_dual(xr, yr)):
                assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), seed
            bad = kkt_violations(lp, x, y, z, tol=1e-6)
            assert not bad, (seed, bad[:5])
        finally:
            p.close()


def test_batch_equals_alone():
    lps = [with_forcing_rows(lpgen.tiny(s, finite_bounds=True), s) for s in range(20)]
    lps += [bounded_medium(7), with_long_forcing_rows(1)]
    b = psl.Batch(lps, **FR)
    try:
        b.run()
        for idx, lp in enumerate(lps):
            ref = O.presolve(lp, **FR)
            name = b.results[idx]
            got = {"result_name": name, "records": b.records(idx),
                   "reduced": b.reduced(idx) if name in ("REDUCED", "UNCHANGED") else None}
            assert_same(got, ref, f"batch LP {idx}")
    finally:
        b.close()


def test_setting_validated():
    with pytest.raises(psl.PslError) as ei:
        psl.Presolver(lpgen.tiny(0), enable_forcing_rows=2)
    assert ei.value.status == psl.PSL_ERR_INVALID
