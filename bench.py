#!/usr/bin/env python3
"""Benchmark of the whole method on one MI355X.

One step = one pass of the hot path over the workload: ingest of the CSR
graph already resident in HBM (validation, weighted degrees, 2W), then the
full multi-level method (level set-up, degree bucketing, synchronous local
moving sweeps with the exact acceptance test, renumbering, contraction),
with the final labels written to device memory.

value = local-move GTEPS of the whole job: the method's executed sweeps
(including each phase's final discarded one) times the edge entries of
their level's graph, divided by the wall time of the step.  Per-kernel
device times come from HIP events recorded around every launch on the
library's stream during the timed steps.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local-move GTEPS + full-Louvain seconds; batched/served vs plain, 1 GPU"
HBM_PEAK_GBS = 8000.0


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chunglu1m")
    ap.add_argument("--pass-batch", type=int, default=0)
    ap.add_argument("--no-timing", action="store_true", help="time steps without per-kernel events")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "graphs shard across GPUs only by design, see the sharding notes", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import graphgen as gg
    import paper_1805_10904_amd as L

    log(f"generating {args.workload}")
    t = time.time()
    g = gg.config(args.workload)
    log(f"generated n={g.n} nnz={g.nnz} in {time.time() - t:.1f}s")
    dev = torch.device("cuda", 0)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ctx = L.Context(0)
    timing = not args.no_timing

    def step(tm):
        G = ctx.graph_create(rp, col, w)
        r = ctx.run(G, timing=tm, pass_batch=args.pass_batch, labels_out=out)
        G.destroy()
        return r

    for k in range(args.warmup):
        step(timing)
        log(f"warmup {k + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        results.append(step(timing))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"timed {args.steps} steps")
    ms_per_step = (t1 - t0) * 1000.0 / max(1, args.steps)
    r = results[-1]
    levels = r.stats["levels"]
    edges = sum(lv["sweeps_executed"] * lv["nnz"] for lv in levels)
    sweeps = sum(lv["sweeps_executed"] for lv in levels)
    value = edges / (ms_per_step / 1000.0) / 1e9

    roofline = None
    sweep_gteps = None
    if timing:
        agg = {}
        for res in results:
            for name, k in res.stats["kernels"].items():
                a = agg.setdefault(name, dict(launches=0, ms=0.0, alg_bytes=0.0))
                for key in a:
                    a[key] += k[key]
        sweep_ms = sum(lv["ms_sweep"] for res in results for lv in res.stats["levels"]) / len(results)
        sweep_gteps = edges / (sweep_ms / 1000.0) / 1e9 if sweep_ms > 0 else None
        dom_name, dom = max(agg.items(), key=lambda kv: kv[1]["ms"])
        achieved = dom["alg_bytes"] / (dom["ms"] / 1000.0) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom_name,
                    "avg_launch_us": round(dom["ms"] * 1000.0 / dom["launches"], 2),
                    "launches_per_step": dom["launches"] / len(results)}
        top = sorted(agg.items(), key=lambda kv: -kv[1]["ms"])[:8]
        log("kernel time per step: " + ", ".join(f"{n} {a['ms'] / len(results):.3f} ms" for n, a in top))

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        import oracle
        log("timing the CPU oracle on the same graph")
        runs = 0
        spent = 0.0
        ref = None
        while runs < 3 and (runs == 0 or spent < 10.0):
            c0 = time.perf_counter()
            ref = oracle.louvain(g.row_ptr, g.col, g.w)
            spent += time.perf_counter() - c0
            runs += 1
        ref_edges = sum(lv["sweeps_executed"] * lv["nnz"] for lv in ref.levels)
        cpu = {"value": round(ref_edges / (spent / runs) / 1e9, 5), "unit": "GTEPS", "cores": 1, "kind": "oracle",
               "sample": f"{runs} full single-threaded oracle run(s) of {args.workload}, "
                         f"{spent / runs:.2f} s each"}
        labels = out.cpu().numpy()
        parity = bool(np.array_equal(labels, ref.labels) and r.q_int == ref.q_int)
        log(f"oracle {spent / runs:.2f} s per run, parity {parity}")

    line = {
        "metric": METRIC, "value": round(value, 4), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "nnz": g.nnz, "levels": len(levels), "sweeps": sweeps,
                   "edges_swept": edges, "parallelism": "single GPU"},
        "full_louvain_s": round(ms_per_step / 1000.0, 6),
        "sweep_gteps": None if sweep_gteps is None else round(sweep_gteps, 3),
        "q": r.q,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_vs_oracle": parity,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
