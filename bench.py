"""Benchmark: presolve throughput on one MI355X.

A step is one full pass of the hot path over one LP already resident in HBM:
ingest (validation, transposed copy, bins; psl_presolve_reload) followed by
psl_presolve_run (all propagation rounds, parallel rows, compaction). The
headline workload is the large LP (m = 1e7, n = 1.5e7, U{3..12} nnz/row,
20 dense rows of 1e6 entries, 20 dense columns in 1e5 rows, 1% planted
reductions with 8-row propagation chains; about 9.7e7 nonzeros, FP64 values,
int32 indices), the largest single-GPU configuration.

Prints one JSON line. `value` = input nonzeros x steps / wall time of the
timed steps (nnz/s). `roofline` describes the row-sweep kernel: algorithmic
bytes of its launches / its device time (HIP events on the library's
stream); `hbm_whole_run` the algorithmic bytes of every pass of a step
(ingest, rounds, parallel passes, compaction) over the step's wall time.
`cpu_baseline` times the sequential CPU oracle on a bounded sample of the
workload (the same generator at 5% scale), in a child process that runs
beside the GPU legs. The batched (4096 LPs) and served workloads follow.
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
    ap.add_argument("--scale", type=float, default=1.0, help="workload scale (1.0 = the full-size LP)")
    ap.add_argument("--workload", choices=("powerlaw", "large"), default="large",
                    help="single-LP workload: the large LP (default) or the power-law LP")
    ap.add_argument("--cpu-sample-scale", type=float, default=0.05,
                    help="scale of the workload instance the CPU oracle presolves (bounded sample)")
    ap.add_argument("--cpu-baseline-child", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--reduction-steps", type=int, default=10,
                    help="timed steps of the same LP with each optional reduction on (0 = skip)")
    ap.add_argument("--batch-lps", type=int, default=4096, help="LPs of the batched workload (0 = skip it)")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--only-batch", action="store_true", help="run the batched workload only")
    ap.add_argument("--batch-no-seq", action="store_true", help="skip the sequential single-LP baseline")
    ap.add_argument("--serve-pool", type=int, default=256, help="LPs in the serving pool (0 = skip serving)")
    ap.add_argument("--serve-rates", default="50,200,1000,2000")
    ap.add_argument("--serve-seconds", type=float, default=6.0)
    ap.add_argument("--serve-slots", type=int, default=4, help="batch engines of the continuous-batching server")
    ap.add_argument("--serve-fifo-max-rate", type=float, default=float("inf"),
                    help="skip the one-LP-per-launch server above this rate (its queue only grows there)")
    ap.add_argument("--only-serving", action="store_true", help="run the serving workload only")
    return ap.parse_args()


def _workload(name, scale):
    from paper_2609_16182_amd import lpgen
    return lpgen.power_law(seed=1, scale=scale) if name == "powerlaw" else lpgen.large(seed=2, scale=scale)


def cpu_baseline_child(args):
    """The CPU oracle on a bounded sample of the workload (no GPU is touched
    here): prints one JSON line."""
    from oracle import oracle as O
    from paper_2609_16182_amd import lpgen
    lp = _workload(args.workload, args.cpu_sample_scale)
    nnz = lpgen.nnz(lp)
    t = time.perf_counter()
    ref = O.presolve(lp)
    dt = time.perf_counter() - t
    print(json.dumps({"value": round(nnz / dt, 1), "unit": "nnz/s", "cores": 1, "kind": "oracle",
                      "sample": f"one sequential presolve of the same generator at {args.cpu_sample_scale:g} scale "
                                f"(m={lp['m']}, n={lp['n']}, {nnz} nnz, {ref.rounds} rounds), {dt:.2f}s on one "
                                f"host core"}), flush=True)


def start_cpu_baseline(args):
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", "--workload", args.workload,
           "--cpu-sample-scale", str(args.cpu_sample_scale)]
    return subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                            env=dict(os.environ, OMP_NUM_THREADS="1"))


def finish_cpu_baseline(proc):
    out, err = proc.communicate(timeout=900)
    if proc.returncode != 0:
        print(f"[bench] CPU baseline failed: {err[-2000:]}", file=sys.stderr, flush=True)
        return None
    return json.loads(out.strip().splitlines()[-1])


def _member(i):
    from paper_2609_16182_amd import lpgen
    return lpgen.batch_member(i)


def _pool_warm(i):
    from oracle import oracle as O  # noqa: F401 (loads the oracle in the worker)
    return i


def _member_generated(i):
    _member(i)
    return 0


def _member_presolved(i):
    from oracle import oracle as O
    O.presolve(_member(i))
    return 0


def _serving_member(i):
    from paper_2609_16182_amd import lpgen
    return lpgen.serving_member(i)


def _replay(psl, sv, pool, rate, seconds, seed):
    """Submit pool LPs at Poisson arrivals of `rate`/s for `seconds`, release
    each result once done; returns per-request latencies and the span."""
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, int(rate * seconds * 1.5) + 16))
    arrivals = arrivals[arrivals < seconds]
    picks = rng.integers(0, len(pool), len(arrivals))
    lat, qms, bsz, arr_of = [], [], [], {}
    t0 = time.perf_counter()
    k = 0
    last_done = t0
    pending = 0
    while k < len(arrivals) or pending:
        now = time.perf_counter() - t0
        while k < len(arrivals) and arrivals[k] <= now:
            t = sv.submit(pool[picks[k]])
            arr_of[t] = arrivals[k]
            k += 1
            pending += 1
        for t in sv.poll():
            info = sv.info(t)
            if arr_of[t] >= 0.1 * seconds:  # warm-up arrivals are not counted
                lat.append(info["latency_ms"])
                qms.append(info["queue_ms"])
                bsz.append(info["batch_lps"])
            sv.release(t)
            pending -= 1
            last_done = time.perf_counter()
        if now > seconds + 120:
            raise RuntimeError("serving run did not drain")
        time.sleep(0.0002)
    span = last_done - t0
    lat = np.array(lat)
    return {"rate": rate, "requests": int(len(arrivals)), "lps_per_s": round(len(arrivals) / span, 1),
            "p50_ms": round(float(np.percentile(lat, 50)), 3), "p99_ms": round(float(np.percentile(lat, 99)), 3),
            "mean_queue_ms": round(float(np.mean(qms)), 3), "mean_batch_lps": round(float(np.mean(bsz)), 2)}


def serving_leg(args, torch, psl):
    """Poisson arrivals of LPs from a device-resident pool (m log-uniform in
    [1e3, 1e6], n = 1.5m, U{4..20} nnz/row); latency = submit -> reduced LP
    ready on the device. The continuous-batching server (--serve-slots) is compared
    with a one-LP-per-launch FIFO server (1 slot, batches of 1) at each rate."""
    from concurrent.futures import ProcessPoolExecutor

    t0 = time.time()
    workers = min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(workers) as ex:
        lps = list(ex.map(_serving_member, range(args.serve_pool)))
    keys = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")
    pool = []
    for lp in lps:
        d = {k: torch.from_numpy(np.ascontiguousarray(lp[k])).cuda() for k in keys}
        d.update(m=lp["m"], n=lp["n"], nnz=int(lp["row_ptr"][-1]))
        pool.append(d)
    del lps
    torch.cuda.synchronize()
    pool_nnz = [d["nnz"] for d in pool]
    print(f"[bench] serving pool of {len(pool)} LPs (mean nnz {np.mean(pool_nnz):.0f}, max {max(pool_nnz)}) "
          f"in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    rates = [float(r) for r in args.serve_rates.split(",")]
    out = {"metric": "serving LPs/s and latency", "pool": len(pool), "mean_nnz": round(float(np.mean(pool_nnz))),
           "seconds_per_rate": args.serve_seconds, "batched": [], "fifo_one_lp_per_launch": []}
    out["slots"] = args.serve_slots
    # each slot's arena holds a batch of up to 2.6e6 rows / 3e7 nonzeros (about
    # 9.5 GB); the rest of the budget is the heap of device-resident results
    budget = (24 + 10 * args.serve_slots) << 30
    for kind, cfg in (("batched", dict(slots=args.serve_slots, hbm_budget_bytes=budget)),
                      ("fifo_one_lp_per_launch", dict(slots=1, max_batch_lps=1))):
        sv = psl.Server(**cfg)
        for lp in pool[:2]:  # warm up
            sv.wait(sv.submit(lp))
        for t in sv.poll():
            sv.release(t)
        for i, rate in enumerate(rates):
            if kind != "batched" and rate > args.serve_fifo_max_rate:
                out[kind].append({"rate": rate, "skipped": "above --serve-fifo-max-rate"})
                continue
            r = _replay(psl, sv, pool, rate, args.serve_seconds, seed=100 + i)
            out[kind].append(r)
            print(f"[bench] serving {kind} rate {rate}: {r}", file=sys.stderr, flush=True)
        sv.close()
    out["config"] = {"workload": "Poisson arrivals over a pool of LPs with m log-uniform in [1e3, 1e6], n = 1.5m, "
                                 "U{4..20} nnz/row, small-LP planting ratios; inputs device-resident",
                     "rates": rates}
    return out


def batch_leg(args, torch, psl):
    """4096 LPs (m log-uniform in [100, 20000], n = 1.5m, U{4..10} nnz/row),
    device-resident. A batched step = psl_batch_reload + psl_batch_run of all
    of them; the sequential baseline = psl_presolve_reload + psl_presolve_run
    of each LP on its own handle, one after the other on the same stream."""
    from concurrent.futures import ProcessPoolExecutor

    K = args.batch_lps
    t0 = time.time()
    workers = min(16, os.cpu_count() or 1)
    with ProcessPoolExecutor(workers) as ex:
        lps = list(ex.map(_member, range(K), chunksize=64))
    keys = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")
    dev = []
    for lp in lps:
        d = {k: torch.from_numpy(np.ascontiguousarray(lp[k])).cuda() for k in keys}
        d.update(m=lp["m"], n=lp["n"], nnz=int(lp["row_ptr"][-1]))
        dev.append(d)
    total_nnz = sum(d["nnz"] for d in dev)
    print(f"[bench] batch of {K} LPs, {total_nnz} nnz, generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream().cuda_stream
    lset = psl.LpSet(dev)
    # launch shapes picked by the tuner on the batch itself: the fastest shape
    # of a smaller sample (fewer waves per launch) need not be the batch's
    t0 = time.time()
    tuned = psl.tune(lset, reps=2, stream=stream)
    print(f"[bench] tuner: {tuned} in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    shape = dict(bin_thresholds=tuned["bin_thresholds"], split_sweep=tuned["split_sweep"])
    b = psl.Batch(lset, stream=stream, **shape)
    b.run()
    b.reload(lset)
    b.run()
    torch.cuda.synchronize()
    ms = []
    stats = None
    for _ in range(args.batch_steps):
        torch.cuda.synchronize()
        ts = time.perf_counter()
        b.reload(lset)
        b.run()
        ms.append((time.perf_counter() - ts) * 1e3)
        stats = b.stats
    torch.cuda.synchronize()
    batch_ms = float(np.median(ms))
    bres = list(b.results)
    brec = [b.lp_stats(i)["records"] for i in range(K)]
    bout = [b.lp_stats(i)["nnz_out"] for i in range(K)]
    print(f"[bench] batched step {batch_ms:.1f} ms", file=sys.stderr, flush=True)

    if args.batch_no_seq:
        b.close()
        return {"metric": "batched LPs/s", "value": round(K / (batch_ms * 1e-3), 1), "ms_per_batch": batch_ms,
                "tuned_shape": tuned,
                "device_ms": {k: round(stats[k], 3) for k in ("ms_ingest", "ms_sweep", "ms_long", "ms_decide",
                                                             "ms_parallel", "ms_compact", "ms_total")},
                "rounds": stats["rounds"]}
    # sequential single-LP runs on the same stream
    t0 = time.time()
    hs = [psl.Presolver(d, stream=stream, **shape) for d in dev]
    print(f"[bench] {K} single-LP handles created in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    for p in hs[:64]:
        p.run()
    torch.cuda.synchronize()
    ts = time.perf_counter()
    for p, d in zip(hs, dev):
        p.reload(d)
        p.run()
    torch.cuda.synchronize()
    seq_ms = (time.perf_counter() - ts) * 1e3
    same = all(p.result_name == r and p.stats["records"] == rc and p.stats["nnz_out"] == no
               for p, r, rc, no in zip(hs, bres, brec, bout))
    sample = list(range(0, K, max(1, K // 16)))
    same_bytes = all(hs[i].records().tobytes() == b.records(i).tobytes() for i in sample)
    for p in hs:
        p.close()
    b.close()
    print(f"[bench] sequential {seq_ms:.1f} ms, equal outputs: {same and same_bytes}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        n_s = min(K, 256)
        nnz_s = sum(int(lp["row_ptr"][-1]) for lp in lps[:n_s])
        ts = time.perf_counter()
        for lp in lps[:n_s]:
            O.presolve(lp)
        dt = time.perf_counter() - ts
        one = {"value": round(n_s / dt, 1), "unit": "LPs/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {n_s} LPs of the batch ({nnz_s} nnz, already generated), one after the "
                         f"other on one host core, {dt:.2f}s"}
        # LP-parallel: a pool of processes over the first LPs, each task one
        # LP generated then presolved; the generation alone is timed the same
        # way and taken off
        n_p = min(K, 1024)
        with ProcessPoolExecutor(workers) as ex:
            list(ex.map(_pool_warm, range(4 * workers), chunksize=1))  # workers started, oracle loaded
            ts = time.perf_counter()
            list(ex.map(_member_generated, range(n_p), chunksize=8))
            t_gen = time.perf_counter() - ts
            ts = time.perf_counter()
            list(ex.map(_member_presolved, range(n_p), chunksize=8))
            t_all = time.perf_counter() - ts
        cpu = {"value": round(n_p / max(t_all - t_gen, 1e-9), 1), "unit": "LPs/s", "cores": workers,
               "kind": "oracle",
               "sample": f"the first {n_p} LPs of the batch, LP-parallel over {workers} processes (one task = "
                         f"generate and presolve one LP, {t_all:.2f}s, less the same pool generating them, "
                         f"{t_gen:.2f}s)", "one_core": one}
    return {
        "metric": "batched LPs/s", "lps": K, "nnz": total_nnz,
        "value": round(K / (batch_ms * 1e-3), 1), "unit": "LPs/s",
        "ms_per_batch": round(batch_ms, 3), "nnz_per_s": round(total_nnz / (batch_ms * 1e-3), 1),
        "sequential": {"value": round(K / (seq_ms * 1e-3), 1), "unit": "LPs/s", "ms_total": round(seq_ms, 1)},
        "speedup_vs_sequential": round(seq_ms / batch_ms, 2),
        "tuned_shape": tuned,
        "equal_outputs": bool(same and same_bytes),
        "device_ms": {k: round(stats[k], 3) for k in ("ms_ingest", "ms_sweep", "ms_long", "ms_decide",
                                                     "ms_parallel", "ms_compact", "ms_total")},
        "rounds": stats["rounds"], "sweep_launches": stats["sweep_launches"],
        "config": {"workload": "4096 LPs, m log-uniform [100, 20000], n = 1.5m, U{4..10} nnz/row, "
                               "small-LP planting ratios", "steps": args.batch_steps},
        "cpu_baseline": cpu,
    }


def measured_traffic(workload):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    of the workload, or None when there is none or the sweep's sources changed
    since the counters were taken."""
    import hashlib
    name = {"powerlaw": "powerlaw_1e6", "large": "large_1e7"}[workload]
    path = os.path.join(ROOT, "profiles", f"{name}_k_sweep_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    src = b"".join(open(os.path.join(ROOT, x), "rb").read() for x in t["sources"])
    if hashlib.sha256(src).hexdigest() != t["source_sha256"]:
        return None
    return t["traffic_bytes_per_launch"]


def gather_ceiling(entries, sweep_rate):
    """The sweep's gathers against what this GPU serves for its pattern:
    random 16-byte gathers from a table of the workload's column count, with
    a streamed index and coefficient per gather (libpsl_probe.so). None when
    the probe is not built."""
    import ctypes
    path = os.path.join(ROOT, "paper_2609_16182_amd", "libpsl_probe.so")
    if not os.path.exists(path):
        return None
    lib = ctypes.CDLL(path)
    lib.psl_probe_gather.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
    rate = ctypes.c_double(0.0)
    if lib.psl_probe_gather(int(entries), 100_000_000, 4, ctypes.byref(rate)) != 0:
        return None
    return {"gathers_per_s": round(rate.value), "table_entries": int(entries), "bytes_per_gather": 16,
            "sweep_gathers_per_s": round(sweep_rate), "frac": round(sweep_rate / rate.value, 4),
            "note": "random 16-byte gathers (one cache line each) beside a streamed 12 B per gather: the "
                    "practical ceiling of the sweep's bound gathers; frac = the sweep's swept nonzeros per "
                    "second of sweep time over that rate"}


def main():
    args = parse()
    if args.cpu_baseline_child:
        cpu_baseline_child(args)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the presolve has no multi-GPU path "
              "(batched and served LPs would shard across GPUs as whole LPs).", file=sys.stderr)
        sys.exit(2)

    # the CPU oracle's bounded sample runs in a child process beside the GPU
    # legs (started before anything touches the GPU)
    cpu_proc = None
    if not args.no_cpu_baseline and not (args.only_batch or args.only_serving):
        cpu_proc = start_cpu_baseline(args)

    import torch

    from paper_2609_16182_amd import lpgen, psl

    torch.cuda.set_device(0)
    if args.only_batch:
        print(json.dumps(batch_leg(args, torch, psl)), flush=True)
        return
    if args.only_serving:
        print(json.dumps(serving_leg(args, torch, psl)), flush=True)
        return
    t0 = time.time()
    lp = _workload(args.workload, args.scale)
    nnz = lpgen.nnz(lp)
    print(f"[bench] workload m={lp['m']} n={lp['n']} nnz={nnz} generated in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)
    keys = ("row_ptr", "col_idx", "val", "lhs", "rhs", "lb", "ub", "c")
    dev = {k: torch.from_numpy(np.ascontiguousarray(lp[k])).cuda() for k in keys}
    dev.update(m=lp["m"], n=lp["n"], nnz=nnz)
    m_in, n_in = lp["m"], lp["n"]
    del lp
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
    sweep_nnz = 0
    run_bytes = 0.0
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
        sweep_nnz += st["sweep_nnz"]
        run_bytes += st["alg_bytes"] + st["ingest_bytes"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    stats = p.stats
    p.close()
    print(f"[bench] {args.steps} steps in {elapsed:.3f}s", file=sys.stderr, flush=True)

    value = nnz * args.steps / elapsed
    achieved = sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else 0.0
    per_launch_bytes = sweep_bytes / max(1, sweep_launches)
    whole = run_bytes / elapsed / 1e9
    roofline = {
        "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(args.workload) if args.scale == 1.0 else None,
        "kernel": "k_sweep (row sweep: activities, decisions, implied bounds)",
        "launches": sweep_launches, "avg_launch_us": round(sweep_ms * 1e3 / max(1, sweep_launches), 2),
        "alg_bytes_per_launch": round(per_launch_bytes),
    }
    hbm_whole = {"achieved": round(whole, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(whole / HBM_PEAK_GBS, 4), "alg_bytes_per_step": round(run_bytes / args.steps),
                 "note": "algorithmic bytes of every pass of a step (ingest, rounds, parallel passes, compaction) "
                         "over the step's wall time"}

    # the same workload with the optional reductions switched on
    reductions = None
    if args.reduction_steps > 0:
        reductions = {}
        every = dict(enable_dual_fix=1, enable_free_singletons=1, enable_parallel_cols=1, enable_forcing_rows=1,
                     enable_doubletons=1, enable_dominated=1)
        for name, extra in (("dual_fix", dict(enable_dual_fix=1)),
                            ("free_singletons", dict(enable_free_singletons=1)),
                            ("parallel_cols", dict(enable_parallel_cols=1)),
                            ("forcing_rows", dict(enable_forcing_rows=1)),
                            ("doubletons", dict(enable_doubletons=1)),
                            ("dominated_cols", dict(enable_dominated=1)),
                            ("all", every)):
            q = psl.Presolver(dev, stream=stream.cuda_stream, **extra)
            for _ in range(2):
                q.reload(dev)
                q.run()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(args.reduction_steps):
                q.reload(dev)
                q.run()
            torch.cuda.synchronize()
            dt = time.perf_counter() - t
            qs = q.stats
            recs = q.records()
            q.close()
            reductions[name] = {
                "value": round(nnz * args.reduction_steps / dt, 1), "unit": "nnz/s", "steps": args.reduction_steps,
                "ms_per_step": round(dt * 1e3 / args.reduction_steps, 3), "rounds": qs["rounds"],
                "records": qs["records"], "dual_fixes": int((recs["type"] == 9).sum()),
                "free_singletons": int((recs["type"] == 10).sum()),
                "parallel_cols": int((recs["type"] == 11).sum()),
                "forcing_rows": int((recs["type"] == 13).sum()), "doubletons": int((recs["type"] == 14).sum()),
                "dominated_cols": int((recs["type"] == 15).sum()), "nnz_out": qs["nnz_out"],
                "m_out": qs["m_out"], "n_out": qs["n_out"], "ms_decide": round(qs["ms_decide"], 3),
                "ms_run_device": round(qs["ms_total"], 3)}
            print(f"[bench] reductions {name}: {reductions[name]['ms_per_step']} ms/step", file=sys.stderr,
                  flush=True)
    del dev
    torch.cuda.empty_cache()
    ceiling = gather_ceiling(n_in, sweep_nnz / (sweep_ms * 1e-3) if sweep_ms > 0 else 0.0)

    batch = batch_leg(args, torch, psl) if args.batch_lps > 0 else None
    serving = serving_leg(args, torch, psl) if args.serve_pool > 0 else None
    cpu = finish_cpu_baseline(cpu_proc) if cpu_proc is not None else None

    desc = {"powerlaw": "power-law LP: m=1e6, n=1.5e6, rows 2+Zipf(2) capped 1e5, power-law columns, planted 2% "
                        "singleton/doubleton/duplicate rows",
            "large": "large LP: m=1e7, n=1.5e7, rows U{3..12}, 20 dense rows of 1e6, 20 dense columns of 1e5, "
                     "1% planted reductions with 8-row propagation chains"}[args.workload]
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "nnz/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": desc, "m": m_in, "n": n_in, "nnz": nnz, "scale": args.scale,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "hbm_whole_run": hbm_whole,
        "gather_ceiling": ceiling,
        "cpu_baseline": cpu,
        "detail": {"rounds": stats["rounds"], "records": stats["records"], "nnz_out": stats["nnz_out"],
                   "ms_ingest": round(stats["ms_ingest"], 3), "ms_run_device": round(stats["ms_total"], 3),
                   "ms_sweep": round(stats["ms_sweep"], 3), "ms_long": round(stats["ms_long"], 3),
                   "ms_decide": round(stats["ms_decide"], 3),
                   "ms_parallel": round(stats["ms_parallel"], 3), "ms_compact": round(stats["ms_compact"], 3),
                   "step_ms_p50": round(float(np.median(step_ms)), 3),
                   "first_run_ms": round(first["ms_total"], 3),
                   "m_out": stats["m_out"], "n_out": stats["n_out"]},
        "reductions": reductions,
        "batch": batch,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
