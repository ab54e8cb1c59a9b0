"""Serving: every request's result is the same alone and in the mix.

LPs are submitted from another thread at random moments while batches are
on the device, so they land in batches of varying composition on both
slots; each ticket's outcome, records and reduced problem are compared bit
for bit with the CPU oracle run on that LP alone. Also: manual stepping,
admission by the result-heap budget (the queue head waits for releases),
invalid LPs failing alone, device-resident inputs, postsolve.
"""
import threading
import time

import numpy as np
import pytest

from oracle import oracle as O
from paper_2609_16182_amd import lpgen
from tests.lp_utils import make
from tests.parity_util import assert_same

pytestmark = pytest.mark.gpu

psl = pytest.importorskip("paper_2609_16182_amd.psl")

INF = np.inf
SMALL = dict(hbm_budget_bytes=6 << 30, max_batch_lps=16, max_batch_rows=60_000, max_batch_cols=90_000,
             max_batch_nnz=600_000)


def got_of(sv, t):
    info = sv.info(t)
    assert info["status"] == psl.PSL_OK, info
    name = info["result_name"]
    out = {"result_name": name, "records": sv.records(t)}
    out["reduced"] = sv.reduced(t) if name in ("REDUCED", "UNCHANGED") else None
    return out, info


def mix_lps():
    lps = [lpgen.tiny(s, finite_bounds=s % 3 == 0) for s in range(24)]
    lps += [lpgen.batch_member(i, m=200 + 173 * i) for i in range(12)]
    lps += [lpgen.single_small(seed=11)]
    lps.append(make(1, 2, [[(0, 1.0), (1, 1.0)]], [5.0], [INF], [0, 0], [1, 1], [1.0, 1.0]))  # infeasible
    lps.append(make(1, 2, [[(0, 1.0)]], [0.0], [4.0], [0, 0], [10, INF], [1.0, -1.0]))      # unbounded
    rng = np.random.default_rng(5)
    order = rng.permutation(len(lps))
    return [lps[i] for i in order]


def test_server_mix_equals_alone():
    lps = mix_lps()
    # two slots: arrivals come faster than two slots finish, so LPs share batches
    sv = psl.Server(slots=2, **SMALL)
    tickets = [None] * len(lps)
    rng = np.random.default_rng(1)
    delays = rng.exponential(0.002, len(lps))

    def producer():
        for i, lp in enumerate(lps):
            time.sleep(delays[i])
            tickets[i] = sv.submit(lp)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    sv.drain()
    batch_sizes, slots = [], set()
    for i, lp in enumerate(lps):
        sv.wait(tickets[i], 60_000)
        got, info = got_of(sv, tickets[i])
        assert_same(got, O.presolve(lp), f"ticket {i}")
        assert info["latency_ms"] >= info["queue_ms"] >= 0
        batch_sizes.append(info["batch_lps"])
        slots.add(info["slot"])
        if got["reduced"] is not None:
            x_red = np.random.default_rng(i).uniform(-1, 1, got["reduced"]["n"])
            x = sv.postsolve(tickets[i], x_red)
            p = psl.Presolver(lp)
            p.run()
            assert np.array_equal(x, p.postsolve(x_red))
            p.close()
        sv.release(tickets[i])
    assert max(batch_sizes) > 1, batch_sizes  # LPs were presolved together
    assert len(set(sv.poll())) == len(lps)
    sv.close()


def test_server_manual_steps_and_invalid_member():
    lps = [lpgen.batch_member(i, m=300 + 50 * i) for i in range(5)]
    bad = dict(lpgen.tiny(2))
    bad["col_idx"] = np.array(bad["col_idx"], np.int32).copy()
    bad["col_idx"][-1] = bad["n"] + 5
    lps.insert(2, bad)
    sv = psl.Server(slots=1, threaded=0, **SMALL)
    ts = [sv.submit(lp) for lp in lps]
    with pytest.raises(psl.PslError):
        sv.info(ts[0])  # not done yet
    steps = 0
    while sv.step() > 0:  # one unit of the batch's run per step
        steps += 1
    assert steps >= 3  # round 0, at least one round, the compaction
    for i, (t, lp) in enumerate(zip(ts, lps)):
        info = sv.info(t)
        if i == 2:
            assert info["status"] == psl.PSL_ERR_INVALID
            continue
        got, _ = got_of(sv, t)
        assert_same(got, O.presolve(lp), f"manual {i}")
    assert sv.step() == 0
    sv.close()


def test_stepped_server_admits_between_rounds():
    """A stepped server with three slots: LPs submitted while other batches
    are between their rounds are admitted at the next step on a free slot and
    run beside them; every ticket equals the oracle's presolve of its LP."""
    lps = mix_lps()
    sv = psl.Server(slots=3, threaded=0, **SMALL)
    tickets, pending = [], list(range(len(lps)))
    arrival = {}
    rng = np.random.default_rng(4)
    steps = 0
    while True:
        for _ in range(int(rng.integers(0, 3))):  # arrivals between steps
            if pending:
                i = pending.pop(0)
                t = sv.submit(lps[i])
                arrival[t] = time.perf_counter()
                tickets.append((i, t))
        n = sv.step()
        steps += 1
        assert steps < 10_000
        if not pending and n == 0:
            break
    assert len(set(sv.poll())) == len(lps)
    spans = []
    for i, t in tickets:
        got, info = got_of(sv, t)
        assert_same(got, O.presolve(lps[i]), f"stepped ticket {i}")
        start = arrival[t] + info["queue_ms"] * 1e-3
        spans.append((info["slot"], start, arrival[t] + info["latency_ms"] * 1e-3))
        sv.release(t)
    assert len({sl for sl, _, _ in spans}) >= 2
    # batches on different slots were resident at the same time
    assert any(a[0] != b[0] and a[1] < b[2] and b[1] < a[2] for a in spans for b in spans)
    assert sv.step() == 0
    sv.close()


def test_stepped_server_drain_and_invalid_members():
    """drain() steps a stepped server with two slots until every ticket is
    done; an invalid LP fails its own ticket only, in whichever batch it
    lands."""
    lps = [lpgen.batch_member(30 + i, m=200 + 40 * i) for i in range(9)]
    bad = dict(lpgen.tiny(5))
    bad["val"] = np.array(bad["val"], np.float64).copy()
    bad["val"][0] = 0.0  # a stored zero coefficient is rejected
    lps.insert(4, bad)
    sv = psl.Server(slots=2, threaded=0, **{**SMALL, "max_batch_lps": 3})
    ts = [sv.submit(lp) for lp in lps]
    sv.drain()
    assert len(set(sv.poll())) == len(lps)
    for i, (t, lp) in enumerate(zip(ts, lps)):
        info = sv.info(t)
        if i == 4:
            assert info["status"] == psl.PSL_ERR_INVALID
            continue
        assert info["batch_lps"] <= 3
        got, _ = got_of(sv, t)
        assert_same(got, O.presolve(lp), f"drained {i}")
    assert sv.step() == 0
    sv.close()


def test_stepped_server_waits_for_memory():
    """A stepped server whose result heap holds two reservations: the third LP
    is not admitted while the first two results stay resident (drain reports
    it), and is admitted at the next step once they are released."""
    lps = [lpgen.batch_member(20 + i, m=4000) for i in range(3)]
    foot = max(psl.reduced_footprint(lp["m"], lp["n"], lpgen.nnz(lp)) for lp in lps)
    probe = psl.Server(slots=2, threaded=0, **SMALL)
    arena = probe.memory()["arena_bytes"]
    probe.close()
    sv = psl.Server(slots=2, threaded=0, **{**SMALL, "hbm_budget_bytes": arena + int(2.5 * foot)})
    ts = [sv.submit(lp) for lp in lps]
    while sv.step() > 0:
        pass
    done = list(sv.poll())
    assert sorted(done) == ts[:2]
    for i in range(2):
        got, _ = got_of(sv, ts[i])
        assert_same(got, O.presolve(lps[i]), f"resident {i}")
    with pytest.raises(psl.PslError) as e:
        sv.drain()
    assert e.value.status == psl.PSL_ERR_CAPACITY
    sv.release(ts[0])
    sv.release(ts[1])
    sv.drain()
    assert list(sv.poll()) == [ts[2]]
    got, _ = got_of(sv, ts[2])
    assert_same(got, O.presolve(lps[2]), "admitted after a release")
    sv.close()


def test_server_admission_waits_for_memory():
    lps = [lpgen.batch_member(20 + i, m=4000) for i in range(8)]
    foot = max(psl.reduced_footprint(lp["m"], lp["n"], lpgen.nnz(lp)) for lp in lps)
    probe = psl.Server(slots=1, **SMALL)
    arena = probe.memory()["arena_bytes"]
    probe.close()
    # a result heap that holds two reservations at a time, not three
    sv = psl.Server(slots=1, **{**SMALL, "hbm_budget_bytes": arena + int(2.5 * foot)})
    heap = sv.memory()["heap_bytes"]
    assert 2 * foot <= heap < 3 * foot
    ts = [sv.submit(lp) for lp in lps]
    left = set(ts)
    deadline = time.time() + 120
    while left and time.time() < deadline:
        for t in sv.poll():
            idx = ts.index(t)
            got, info = got_of(sv, t)
            assert info["batch_lps"] <= 2, info
            assert_same(got, O.presolve(lps[idx]), f"budget {idx}")
            sv.release(t)
            left.discard(t)
        time.sleep(0.001)
    assert not left, "not every request completed"
    mem = sv.memory()
    assert mem["heap_peak"] <= heap and mem["heap_used"] == 0
    with pytest.raises(psl.PslError) as e:
        sv.submit(lpgen.batch_member(99, m=20000))  # its reservation can never fit the heap
    assert e.value.status == psl.PSL_ERR_CAPACITY
    sv.close()


def test_server_device_inputs():
    torch = pytest.importorskip("torch")
    lps = [lpgen.batch_member(i, m=500 + 90 * i) for i in range(6)] + [lpgen.tiny(9)]
    keys = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")
    sv = psl.Server(**SMALL)
    ts = []
    for lp in lps:
        d = {k: torch.from_numpy(np.ascontiguousarray(lp[k])).cuda() for k in keys}
        d.update(m=lp["m"], n=lp["n"], nnz=lpgen.nnz(lp))
        ts.append(sv.submit(d))
    sv.drain()
    for t, lp in zip(ts, lps):
        got, _ = got_of(sv, t)
        assert_same(got, O.presolve(lp), "device")
        sv.release(t)
    sv.close()


class _Alone:
    """psl.presolve's result in the shape assert_same expects."""

    def __init__(self, got):
        self.result_name = got["result_name"]
        self.records = got["records"]
        self.reduced = got["reduced"]


def test_server_serving_sizes():
    """LPs of the serving pool's sizes, up to m = 1e6 (about 1.2e7 nonzeros),
    mixed with small ones on the default server (four slots): each ticket
    equals the LP presolved alone, bit for bit; the one of m near 2e5 also
    equals the oracle."""
    big = [lpgen.serving_member(0, m_lo=900_000, m_hi=1_000_000), lpgen.serving_member(1, m_lo=150_000,
                                                                                       m_hi=250_000)]
    lps = [big[0], lpgen.tiny(3), big[1], lpgen.batch_member(2, m=500), lpgen.single_small(seed=12)]
    sv = psl.Server()
    try:
        tickets = [sv.submit(lp) for lp in lps]
        for t in tickets:
            sv.wait(t, 120_000)
        for k, (lp, t) in enumerate(zip(lps, tickets)):
            got, info = got_of(sv, t)
            alone, p = psl.presolve(lp)
            p.close()
            assert_same(got, _Alone(alone), f"serving size LP {k} (m = {lp['m']})")
        got, _ = got_of(sv, tickets[2])
        assert_same(got, O.presolve(lps[2]), "m near 2e5 against the oracle")
    finally:
        sv.close()
