"""Host logic of bench.py on the CPU: the one-GPU guard and the serving
replay's accounting (against a stand-in server that completes every request
on its next poll)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


class _InstantServer:
    """Completes each request at its next poll, with a fixed latency."""

    def __init__(self):
        self.next, self.waiting, self.released = 1, [], []

    def submit(self, lp):
        t = self.next
        self.next += 1
        self.waiting.append(t)
        return t

    def poll(self):
        done, self.waiting = self.waiting, []
        return done

    def info(self, t):
        return {"latency_ms": 2.0 + (t % 5), "queue_ms": 0.5, "batch_lps": 1}

    def release(self, t):
        self.released.append(t)


def test_replay_counts_and_percentiles():
    sv = _InstantServer()
    r = bench._replay(None, sv, [{"m": 1}] * 4, rate=400.0, seconds=0.5, seed=3)
    rng = np.random.default_rng(3)
    arrivals = np.cumsum(rng.exponential(1.0 / 400.0, int(400.0 * 0.5 * 1.5) + 16))
    assert r["requests"] == int((arrivals < 0.5).sum())
    assert len(sv.released) == r["requests"]  # every ticket released
    assert 2.0 <= r["p50_ms"] <= 6.0 and 2.0 <= r["p99_ms"] <= 6.0
    assert r["mean_queue_ms"] == 0.5 and r["mean_batch_lps"] == 1.0
