"""psl_presolve_noalloc (the entry point for callers that cannot allocate
device memory) against psl_presolve_create + psl_presolve_run: the same
outcome, records and reduced problem, bit for bit, on two calls in a row
through the C-ABI, the second with a smaller LP (the static scratch then
holds the first call's contents, laid out for another LP)."""
import numpy as np
import pytest

from paper_2609_16182_amd import lpgen
from tests.parity_util import assert_same

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")
torch = pytest.importorskip("torch")

KEYS = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")


class _Ref:
    """The existing entry points' result in the shape assert_same expects."""

    def __init__(self, got):
        self.result_name = got["result_name"]
        self.records = got["records"]
        self.reduced = got["reduced"]


def _device_lp(lp):
    d = {k: torch.from_numpy(np.ascontiguousarray(lp[k])).cuda() for k in KEYS}
    d.update(m=lp["m"], n=lp["n"], nnz=int(lp["row_ptr"][-1]) if lp["m"] else 0)
    return d


def _noalloc(lp_dev, records_cap, **settings):
    m, n, nnz = lp_dev["m"], lp_dev["n"], lp_dev["nnz"]
    dev = "cuda"
    buf = dict(row_ptr=torch.zeros(m + 1, dtype=torch.int32, device=dev),
               col_idx=torch.zeros(max(nnz, 1), dtype=torch.int32, device=dev),
               val=torch.zeros(max(nnz, 1), dtype=torch.float64, device=dev),
               col_ptr=torch.zeros(n + 1, dtype=torch.int32, device=dev),
               row_idx=torch.zeros(max(nnz, 1), dtype=torch.int32, device=dev),
               cval=torch.zeros(max(nnz, 1), dtype=torch.float64, device=dev),
               lhs=torch.zeros(max(m, 1), dtype=torch.float64, device=dev),
               rhs=torch.zeros(max(m, 1), dtype=torch.float64, device=dev),
               lb=torch.zeros(max(n, 1), dtype=torch.float64, device=dev),
               ub=torch.zeros(max(n, 1), dtype=torch.float64, device=dev),
               c=torch.zeros(max(n, 1), dtype=torch.float64, device=dev),
               row_map=torch.zeros(max(m, 1), dtype=torch.int32, device=dev),
               col_map=torch.zeros(max(n, 1), dtype=torch.int32, device=dev),
               row_class=torch.zeros(max(m, 1), dtype=torch.uint8, device=dev),
               col_class=torch.zeros(max(n, 1), dtype=torch.uint8, device=dev),
               records=torch.zeros(max(records_cap, 1) * 48, dtype=torch.uint8, device=dev))
    out = psl.psl_noalloc_out()
    for k, t in buf.items():
        setattr(out, k, t.data_ptr())
    out.records_cap = records_cap
    keep = []
    res, _ = psl.psl_presolve_noalloc(psl.make_lp(lp_dev, keep),
                                      psl.make_settings(stream=torch.cuda.current_stream().cuda_stream,
                                                        **settings), out)
    torch.cuda.synchronize()
    name = psl.RESULT_NAMES[res]
    rec = buf["records"][: out.records_out * 48].cpu().numpy().view(psl.RECORD_DTYPE).copy()
    red = None
    if name in ("REDUCED", "UNCHANGED"):
        mo, no, zo = out.m_out, out.n_out, out.nnz_out

        def h(k, cnt, dt):
            return buf[k][:cnt].cpu().numpy().view(dt).copy() if cnt else np.zeros(0, dt)
        red = dict(m=mo, n=no, nnz=zo, obj_offset=out.obj_offset,
                   row_ptr=h("row_ptr", mo + 1, np.int32), col_idx=h("col_idx", zo, np.int32),
                   val=h("val", zo, np.float64), col_ptr=h("col_ptr", no + 1, np.int32),
                   row_idx=h("row_idx", zo, np.int32), cval=h("cval", zo, np.float64),
                   lhs=h("lhs", mo, np.float64), rhs=h("rhs", mo, np.float64), lb=h("lb", no, np.float64),
                   ub=h("ub", no, np.float64), c=h("c", no, np.float64), row_map=h("row_map", mo, np.int32),
                   col_map=h("col_map", no, np.int32), row_class=h("row_class", mo, np.uint8),
                   col_class=h("col_class", no, np.uint8))
    return {"result_name": name, "records": rec, "reduced": red}


def _existing(lp_dev, **settings):
    got, p = psl.presolve(lp_dev, stream=torch.cuda.current_stream().cuda_stream, **settings)
    p.close()
    return _Ref(got)


@pytest.mark.parametrize("settings", [{}, dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1)])
def test_noalloc_matches_create_run_twice(settings):
    big = _device_lp(lpgen.single_small(seed=0))
    small = _device_lp(lpgen.make_lp(300, 450, seed=105, row_len=(2, 7), singleton=10, empty=5, doubleton=20,
                                     duplicate=10, fixed_cols=15))
    for lp in (big, small):
        ref = _existing(lp, **settings)
        got = _noalloc(lp, records_cap=200000, **settings)
        assert got["result_name"] == "REDUCED"
        assert_same(got, ref, f"noalloc m={lp['m']}")


def test_noalloc_rejects_beyond_limits():
    lp = _device_lp(lpgen.single_small(seed=1))
    with pytest.raises(psl.PslError) as e:
        _noalloc(lp, records_cap=10)
    assert e.value.status == psl.PSL_ERR_CAPACITY
    big = lpgen.power_law(scale=0.3)  # working set above the static scratch
    with pytest.raises(psl.PslError) as e:
        _noalloc(_device_lp(big), records_cap=1 << 20)
    assert e.value.status == psl.PSL_ERR_CAPACITY
    # and a good call afterwards still matches
    small = _device_lp(lpgen.single_small(seed=2))
    assert_same(_noalloc(small, records_cap=200000), _existing(small), "after rejections")
