"""GPU parity of the parallel-row pass on the current problem: rows parallel
only over their active entries (fixed columns of their own, fixed first
entries, negative lambda, long rows split over workgroups, the quantiser's
rounding), bit for bit against the oracle through the C-ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from tests.lp_utils import load_golden, make
from tests.parity_util import assert_same
from tests.test_oracle_parallel_active import _bits, _fixed_family, _from_bits

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")

INF = np.inf


def run_both(lp, **settings):
    ref = O.presolve(lp, **{k: v for k, v in settings.items() if k in O.DEFAULTS})
    got, p = psl.presolve(lp, **settings)
    p.close()
    return got, ref


def test_golden_active_parts():
    _, lp = load_golden("parallel_rows_active.json")
    got, ref = run_both(lp)
    assert (ref.records["type"] == O.REC["PARALLEL_ROW"]).sum() == 1
    assert_same(got, ref, "active golden")


def test_hand_cases():
    cases = {
        "negative lambda": make(2, 4, [[(0, 1.0), (1, -2.0), (2, 4.0)], [(0, -2.0), (1, 4.0), (3, 3.0)]],
                                [-1.0, -10.0], [6.0, 2.0], [-INF, -INF, 0.5, 2.0], [INF, INF, 0.5, 2.0], [0] * 4),
        "first entry fixed": make(2, 4, [[(0, 7.0), (1, 1.0), (2, 2.0)], [(1, 3.0), (2, 6.0), (3, -5.0)]],
                                  [-INF, -INF], [10.0, 9.0], [1.0, -INF, -INF, 0.0], [1.0, INF, INF, 0.0], [0] * 4),
    }
    for name, lp in cases.items():
        got, ref = run_both(lp)
        assert (ref.records["type"] == O.REC["PARALLEL_ROW"]).sum() == 1, name
        assert_same(got, ref, name)


def test_quantiser_rows():
    base = _bits(1.5)
    up = _from_bits(base | 0x80000)
    for other in (_from_bits(base + 0x100000), _from_bits(base | 0x7FFFF)):
        rows = [[(0, 1.0), (1, up)], [(0, 1.0), (1, other)]]
        lp = make(2, 2, rows, [-INF, -INF], [4.0, 5.0], [-INF] * 2, [INF] * 2, [0, 0])
        got, ref = run_both(lp)
        assert_same(got, ref, f"quantiser {other!r}")


@pytest.mark.parametrize("seed", range(60))
def test_fixed_family(seed):
    got, ref = run_both(_fixed_family(seed), max_rounds=1)
    assert_same(got, ref, f"fixed family {seed}")


def parallel_mix(seed, groups=300, long_rows=6, long_len=3000):
    """Rows in groups of 2-4 that are scaled copies over their active columns,
    each row also holding fixed columns of its own at random places (also
    before its first active entry); a few groups have long rows (more than
    one workgroup chunk). Columns: free active ones, then fixed ones. Sides
    come from a point x0 (activity +- a slack), so the LP stays feasible."""
    rng = np.random.default_rng(900 + seed)
    n_act = 4000
    n_fix = 3000
    n = n_act + n_fix
    fixv = rng.choice([-1.0, 0.0, 0.5, 2.0], n_fix)
    lb = np.concatenate([np.full(n_act, -INF), fixv])
    ub = np.concatenate([np.full(n_act, INF), fixv])
    x0 = np.concatenate([rng.uniform(-1, 1, n_act), fixv])
    rows, lhs, rhs = [], [], []
    for g in range(groups + long_rows):
        L = int(rng.integers(2, 9)) if g < groups else long_len
        act = np.sort(rng.choice(n_act, L, replace=False))
        base = rng.choice([-2.0, -1.0, 0.5, 1.0, 1.5, 3.0], L)
        for r in range(int(rng.integers(2, 5))):
            lam = 1.0 if r == 0 else float(rng.choice([-4.0, -1.0, 0.5, 2.0, 8.0]))
            nf = int(rng.integers(0, 4)) if g < groups else int(rng.integers(50, 200))
            fx = n_act + rng.choice(n_fix, nf, replace=False)
            if g >= groups and r > 0:  # a fixed column before the first active one
                fx = np.concatenate([fx, [n_act + int(rng.integers(0, 8))]])
            ent = {int(j): float(lam * v) for j, v in zip(act, base)}
            for j in np.unique(fx):
                ent[int(j)] = float(rng.choice([-3.0, 1.0, 2.5]))
            a = sum(v * x0[j] for j, v in ent.items())
            kind = rng.integers(0, 3)
            rows.append(sorted(ent.items()))
            lhs.append(-INF if kind == 1 else a - float(rng.uniform(0, 2)))
            rhs.append(INF if kind == 2 else a + float(rng.uniform(0, 2)))
    order = rng.permutation(len(rows))
    rows = [rows[i] for i in order]
    lhs = [lhs[i] for i in order]
    rhs = [rhs[i] for i in order]
    c = np.zeros(n)
    return make(len(rows), n, rows, lhs, rhs, lb, ub, c)


@pytest.mark.parametrize("seed", range(3))
@pytest.mark.parametrize("thr", [None, (16, 2048), (64, 2048, 4)])
def test_parallel_mix(seed, thr):
    lp = parallel_mix(seed)
    kw = {} if thr is None else dict(bin_thresholds=thr)
    got, ref = run_both(lp, **kw)
    assert (ref.records["type"] == O.REC["PARALLEL_ROW"]).sum() > 300
    assert_same(got, ref, f"mix {seed} {thr}")


def test_parallel_mix_batch():
    """The same LPs in one batch: each LP's outcome equals its alone result."""
    lps = [parallel_mix(s, groups=80, long_rows=2) for s in range(4)]
    refs = [O.presolve(lp) for lp in lps]
    b = psl.Batch(psl.LpSet(lps))
    b.run()
    for k, (lp, ref) in enumerate(zip(lps, refs)):
        got = {"result_name": b.results[k], "records": b.records(k), "reduced": b.reduced(k)}
        assert_same(got, ref, f"batch lp {k}")
    b.close()
