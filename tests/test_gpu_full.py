"""Full-size power-law LP (m = 1e6, n = 1.5e6, about 9.2e6 nonzeros), in the
launch configuration the benchmark times (default bins): every output of the
GPU library equals the oracle's, bit for bit. The oracle finishes this size in
seconds, so nothing needs sampling."""
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.parity_util import assert_same

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")


@pytest.fixture(scope="module")
def power_lp():
    t0 = time.time()
    lp = lpgen.power_law(seed=1, scale=1.0)
    print(f"generated nnz={lpgen.nnz(lp)} in {time.time() - t0:.1f}s", flush=True)
    return lp


def test_power_law_full_size(power_lp):
    lp = power_lp
    t0 = time.time()
    ref = O.presolve(lp)
    print(f"oracle {ref.result_name} rounds={ref.rounds} records={len(ref.records)} in {time.time() - t0:.1f}s",
          flush=True)
    got, p = psl.presolve(lp)
    print(f"gpu stats {got['stats']}", flush=True)
    p.close()
    assert_same(got, ref, "power-law full size")
    # the planted feasible point satisfies the reduced bounds (primal reductions)
    r = got["reduced"]
    x0 = lp["x0"][r["col_map"]]
    sc = np.maximum(1.0, np.abs(x0))
    assert np.all(x0 >= r["lb"] - 1e-9 * sc) and np.all(x0 <= r["ub"] + 1e-9 * sc)


EVERY = dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1, enable_forcing_rows=1,
             enable_doubletons=1, enable_dominated=1)


@pytest.mark.parametrize("extra", [dict(enable_dual_fix=1), dict(enable_free_singletons=1),
                                   dict(enable_parallel_cols=1),
                                   dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1),
                                   dict(enable_forcing_rows=1), dict(enable_doubletons=1), dict(enable_dominated=1),
                                   EVERY],
                         ids=["dual_fix", "free_singletons", "parallel_cols", "all", "forcing_rows", "doubletons",
                              "dominated", "every"])
def test_power_law_full_size_next_reductions(power_lp, extra):
    """The same LP with the optional reductions on (the benchmark's legs)."""
    lp = power_lp
    t0 = time.time()
    ref = O.presolve(lp, **extra)
    kinds = {name: int((ref.records["type"] == O.REC[name]).sum())
             for name in ("DUAL_FIX", "FREE_SINGLETON", "PARALLEL_COL", "FORCING_ROW", "DOUBLETON_ROW",
                          "DOMINATED_COL")}
    print(f"oracle {ref.result_name} rounds={ref.rounds} records={len(ref.records)} {kinds} "
          f"in {time.time() - t0:.1f}s", flush=True)
    if extra.get("enable_dual_fix"):
        assert kinds["DUAL_FIX"] > 0
    if extra.get("enable_free_singletons"):
        assert kinds["FREE_SINGLETON"] > 0
    if extra.get("enable_parallel_cols"):
        assert kinds["PARALLEL_COL"] > 0
    if extra.get("enable_doubletons"):
        assert kinds["DOUBLETON_ROW"] > 0
    if extra.get("enable_dominated"):
        assert kinds["DOMINATED_COL"] > 0
    got, p = psl.presolve(lp, **extra)
    print(f"gpu stats {got['stats']}", flush=True)
    p.close()
    assert_same(got, ref, f"power-law full size, {extra}")


def _load_digests(name):
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_digests.py)")
    with open(path) as f:
        return json.load(f)


@pytest.mark.timeout(900)
def test_large_full_size_digest():
    """The large LP (m = 1e7, n = 1.5e7, ~9.7e7 nnz with 20 dense rows of 1e6
    entries and 20 dense columns of 1e5, planted chains): outcome, record
    stream and reduced problem equal the oracle's bit for bit, compared
    through SHA-256 digests written by tests/golden/make_digests.py (the oracle
    needs minutes at this size)."""
    from tests.golden.digest import digest_of
    ref = _load_digests("large_1e7_digest.json")
    t0 = time.time()
    lp = lpgen.large(seed=2, scale=1.0)
    print(f"generated nnz={lpgen.nnz(lp)} in {time.time() - t0:.1f}s", flush=True)
    assert (lp["m"], lp["n"], lpgen.nnz(lp)) == (ref["m"], ref["n"], ref["nnz"])
    got, p = psl.presolve(lp)
    print(f"gpu stats {got['stats']}", flush=True)
    p.close()
    assert got["stats"]["rounds"] == ref["rounds"]
    dg = digest_of(got["result_name"], got["records"], got["reduced"])
    for key in ("result_name", "records", "records_sha256"):
        assert dg[key] == ref[key], key
    for key, v in ref["reduced"].items():
        assert dg["reduced"][key] == v, key
    # the chains need at least 5 Jacobi rounds
    assert ref["rounds"] >= 5
    r = got["reduced"]
    x0 = lp["x0"][r["col_map"]]
    sc = np.maximum(1.0, np.abs(x0))
    assert np.all(x0 >= r["lb"] - 1e-9 * sc) and np.all(x0 <= r["ub"] + 1e-9 * sc)


@pytest.mark.timeout(600)
def test_batch_4096_digests():
    """All 4096 LPs of the batched workload, presolved in one batch from
    device-resident inputs, in the benchmark's launch configuration: each
    LP's result equals the oracle's (digests by tests/golden/make_digests.py)."""
    from concurrent.futures import ProcessPoolExecutor
    import os

    import torch
    from tests.golden.digest import lp_digest
    ref = _load_digests("batch_4096_digests.json")
    with ProcessPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        lps = list(ex.map(lpgen.batch_member, range(4096), chunksize=64))
    keys = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")
    dev = []
    for lp in lps:
        d = {k: torch.from_numpy(np.ascontiguousarray(lp[k])).cuda() for k in keys}
        d.update(m=lp["m"], n=lp["n"], nnz=lpgen.nnz(lp))
        dev.append(d)
    torch.cuda.synchronize()
    b = psl.Batch(dev)
    b.run()
    bad = []
    for i in range(4096):
        name = b.results[i]
        red = b.reduced(i) if name in ("REDUCED", "UNCHANGED") else None
        if lp_digest(name, b.records(i), red) != ref["digests"][i] or b.lp_stats(i)["rounds"] != ref["rounds"][i]:
            bad.append(i)
    b.close()
    assert not bad, f"{len(bad)} LPs differ, first {bad[:10]}"


@pytest.fixture(scope="module")
def power_lp_reordered(power_lp):
    """The same LP with its dense columns first (empty ones last, in one run of
    hundreds of thousands) and its longest rows first."""
    from tests.test_gpu_parity import by_popularity, rows_by_length
    return rows_by_length(by_popularity(power_lp))


@pytest.mark.parametrize("extra", [{}, EVERY],
                         ids=["default", "all"])
def test_power_law_full_size_reordered(power_lp_reordered, extra):
    lp = power_lp_reordered
    t0 = time.time()
    ref = O.presolve(lp, **extra)
    print(f"oracle {ref.result_name} rounds={ref.rounds} records={len(ref.records)} in {time.time() - t0:.1f}s",
          flush=True)
    got, p = psl.presolve(lp, **extra)
    p.close()
    assert_same(got, ref, f"power-law full size reordered, {extra}")
