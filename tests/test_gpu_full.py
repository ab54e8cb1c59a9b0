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


def test_power_law_full_size():
    t0 = time.time()
    lp = lpgen.power_law(seed=1, scale=1.0)
    print(f"generated nnz={lpgen.nnz(lp)} in {time.time() - t0:.1f}s", flush=True)
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
