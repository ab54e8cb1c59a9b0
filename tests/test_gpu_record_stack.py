"""The postsolve stack with a host flush (section 3.3: the device stack is
flushed to the host when it nears capacity): settings.device_records = R
keeps a fixed device stack of R records. Outcome, records, reduced problem and
postsolve (primal and dual) must be those of the growing buffer, bit for bit,
and the oracle's; the smallest R (one phase's worst case) forces flushes
between rounds and passes. Sizes below that minimum, and the entry points that
keep no handle (batches, servers, the no-allocation call), are refused."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.parity_util import assert_same
from tests.test_oracle_doubleton import with_doubletons

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")

ALL = dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1, enable_forcing_rows=1,
           enable_doubletons=1)


def _phase(lp, doubletons):
    m, n = int(lp["m"]), int(lp["n"])
    return max(m + 3 * n + 16, (2 * m + 3 * n if doubletons else m + n) + 16)


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


def _check(lp, extra, min_flushes=1):
    ref_o = O.presolve(lp, **{k: v for k, v in extra.items() if k in O.DEFAULTS})
    got0, p0 = psl.presolve(lp, **extra)
    R = _phase(lp, extra.get("enable_doubletons", 0))
    got1, p1 = psl.presolve(lp, device_records=R, **extra)
    try:
        assert got1["stats"]["record_flushes"] >= min_flushes, got1["stats"]["record_flushes"]
        assert got0["stats"]["record_flushes"] == 0
        assert_same(got1, ref_o, "flushed stack vs oracle")
        assert np.array_equal(got0["records"], got1["records"])
        if got1["result_name"] in ("REDUCED", "UNCHANGED"):
            n_red = got1["reduced"]["n"]
            m_red = got1["reduced"]["m"]
            rng = np.random.default_rng(1)
            xr = rng.uniform(-1, 1, n_red)
            yr = rng.uniform(-1, 1, m_red)
            assert np.array_equal(_bits(p0.postsolve(xr)), _bits(p1.postsolve(xr)))
            for a, b in zip(p0.postsolve(xr, yr), p1.postsolve(xr, yr)):
                assert np.array_equal(_bits(a), _bits(b))
    finally:
        p0.close()
        p1.close()
    return got1


def test_small_workload_flushes():
    _check(lpgen.single_small(seed=3), {})


@pytest.mark.parametrize("seed", range(6))
def test_every_reduction(seed):
    lp = with_doubletons(lpgen.make_lp(400, 600, seed=600 + seed, row_len=(2, 7), singleton=10, empty=5,
                                       doubleton=40, duplicate=10, fixed_cols=15), seed)
    _check(lp, ALL)


def test_power_law_scaled():
    _check(lpgen.power_law(scale=0.01, seed=2), {})


def test_reload_resets_the_stack():
    a = lpgen.single_small(seed=4)
    b = dict(a)
    b["c"] = 2.0 * a["c"] - 1.0  # same shape, other costs (reload keeps m, n and nnz)
    R = _phase(a, 0)
    p = psl.Presolver(a, device_records=R)
    try:
        for lp in (a, b, a):
            p.reload(lp)
            p.run()
            ref = O.presolve(lp)
            got = {"result_name": p.result_name, "records": p.records(),
                   "reduced": p.reduced() if p.result_name in ("REDUCED", "UNCHANGED") else None}
            assert_same(got, ref, "reload")
            assert p.stats["record_flushes"] >= 1
    finally:
        p.close()


def test_refusals():
    lp = lpgen.single_small(seed=3)
    with pytest.raises(psl.PslError) as ei:
        psl.Presolver(lp, device_records=_phase(lp, 0) - 1)
    assert ei.value.status == psl.PSL_ERR_INVALID
    with pytest.raises(psl.PslError) as ei:
        psl.Presolver(lp, device_records=-1)
    assert ei.value.status == psl.PSL_ERR_INVALID
    with pytest.raises(psl.PslError) as ei:
        psl.Batch([lp, lp], device_records=10 ** 6)
    assert ei.value.status == psl.PSL_ERR_UNSUPPORTED
    with pytest.raises(psl.PslError) as ei:
        psl.Server(device_records=10 ** 6)
    assert ei.value.status == psl.PSL_ERR_UNSUPPORTED
