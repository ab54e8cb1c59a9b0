"""Benchmark: presolve throughput on one MI355X.

A step is one full pass of the hot path over one LP already resident in HBM:
ingest (validation, transposed copy, bins; psl_presolve_reload) followed by
psl_presolve_run (all propagation rounds, parallel rows, compaction). The
workload is the power-law LP (m = 1e6, n = 1.5e6, row lengths 2 + Zipf(2)
capped at 1e5, power-law column choice, about 9.2e6 nonzeros, FP64 values,
int32 indices).

Prints one JSON line. `value` = input nonzeros x steps / wall time of the
timed steps (nnz/s). `roofline` describes the row-sweep kernel: algorithmic
bytes of its launches / its device time (HIP events on the library's stream).
`cpu_baseline` times the sequential CPU oracle on the same LP.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "presolve nnz/s and % HBM peak vs CPU oracle; batched LPs/s + p99 latency"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1.0 = the full power-law LP)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    return ap.parse_args()


def measured_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary,
    or None when the sweep's sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "powerlaw_1e6_k_sweep_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    src = b"".join(open(os.path.join(ROOT, x), "rb").read() for x in t["sources"])
    if hashlib.sha256(src).hexdigest() != t["source_sha256"]:
        return None
    return t["traffic_bytes_per_launch"]


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(see DESIGN.md for how the presolve would shard).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2609_16182_amd import lpgen, psl

    torch.cuda.set_device(0)
    t0 = time.time()
    lp = lpgen.power_law(seed=1, scale=args.scale)
    nnz = lpgen.nnz(lp)
    print(f"[bench] workload m={lp['m']} n={lp['n']} nnz={nnz} generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    keys = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")
    dev = {k: torch.from_numpy(np.ascontiguousarray(lp[k])).cuda() for k in keys}
    dev.update(m=lp["m"], n=lp["n"], nnz=nnz)
    stream = torch.cuda.current_stream()
    p = psl.Presolver(dev, stream=stream.cuda_stream)
    p.run()
    first = p.stats
    for _ in range(args.warmup):
        p.reload(dev)
        p.run()
    torch.cuda.synchronize()

    sweep_ms = 0.0
    sweep_bytes = 0.0
    sweep_launches = 0
    step_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        p.reload(dev)
        p.run()
        step_ms.append((time.perf_counter() - ts) * 1e3)
        st = p.stats
        sweep_ms += st["ms_sweep"]
        sweep_bytes += st["sweep_bytes"]
        sweep_launches += st["sweep_launches"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    stats = p.stats
    p.close()

    value = nnz * args.steps / elapsed
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else 0.0
    per_launch_bytes = sweep_bytes / max(1, sweep_launches)
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(),
        "kernel": "k_sweep<0> (row sweep: activities, decisions, implied bounds)",
        "launches": sweep_launches, "avg_launch_us": round(sweep_ms * 1e3 / max(1, sweep_launches), 2),
        "alg_bytes_per_launch": round(per_launch_bytes),
    }

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        t = time.perf_counter()
        ref = O.presolve(lp)
        dt = time.perf_counter() - t
        cpu = {"value": round(nnz / dt, 1), "unit": "nnz/s", "cores": 1, "kind": "oracle",
               "sample": f"one full sequential presolve of the same LP ({nnz} nnz, {ref.rounds} rounds), "
                         f"{dt:.2f}s on one host core"}
        if ref.records.shape[0] != stats["records"]:
            print("[bench] WARNING: record counts differ from the oracle", file=sys.stderr)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "nnz/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "power-law LP: m=1e6, n=1.5e6, rows 2+Zipf(2) capped 1e5, "
                               "power-law columns, planted 2% singleton/doubleton/duplicate rows",
                   "m": lp["m"], "n": lp["n"], "nnz": nnz, "scale": args.scale,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "detail": {"rounds": stats["rounds"], "records": stats["records"], "nnz_out": stats["nnz_out"],
                   "ms_ingest": round(stats["ms_ingest"], 3), "ms_run_device": round(stats["ms_total"], 3),
                   "ms_sweep": round(stats["ms_sweep"], 3), "ms_decide": round(stats["ms_decide"], 3),
                   "ms_parallel": round(stats["ms_parallel"], 3), "ms_compact": round(stats["ms_compact"], 3),
                   "step_ms_p50": round(float(np.median(step_ms)), 3),
                   "first_run_ms": round(first["ms_total"], 3)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
