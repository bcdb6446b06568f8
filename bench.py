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
device times come from HIP events that the kernel dispatches themselves
fill (hipExtLaunchKernel) on the library's stream: every launch in the last
warm-up step, the dominant kernel's launches in the last timed step (the
events add a few microseconds around each timed kernel, so the other timed
steps carry none).

Beside the plain run, the line reports the run that keeps the dendrogram
(per-level maps and the last level's graph), a run checkpointed after its
first level and resumed, with their wall times and whether their labels
equal the plain run's, and the run with the optional final merge after
every phase (time, Q, merge kernels' device time); skip these with
--no-dendro.  --shards N (default 8) times one GPU's share of the workload
split into N entry-balanced vertex ranges (sweep kernels per pass, ghosts
read in place; no exchange) against the whole graph.

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


def recorded_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summaries (FETCH_SIZE and WRITE_SIZE, calibrated
    against a plain copy), or None when none covers it or the sources it was
    measured on have changed since."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*_pmc.md"))):
        with open(path) as f:
            m = re.search(r"```traffic\n(.*?)```", f.read(), re.S)
        if not m:
            continue
        rec = json.loads(m.group(1))
        if rec["workload"] != workload or rec["kernel"].replace(" ", "") != kernel.replace(" ", ""):
            continue
        h = hashlib.sha256()
        try:
            for src in rec["sources"]:
                with open(os.path.join(ROOT, src), "rb") as f:
                    h.update(f.read())
        except OSError:
            return None
        return int(rec["bytes_per_launch"]) if h.hexdigest() == rec["sha256"] else None
    return None


def log(msg):
    sys.stderr.write(f"[bench] {msg}\n")
    sys.stderr.flush()


def _gen_chunk(args):
    import graphgen as gg
    kind, first, count, kw = args
    fn = gg.batch_sbm if kind == "batch" else gg.served_chunglu
    return fn(count, first=first, **kw)


def generate(kind: str, count: int, workers: int, **kw) -> list:
    """Seeded graphs generated in worker processes (forked before any GPU use)."""
    import multiprocessing as mp
    chunk = max(1, min(64, (count + 4 * workers - 1) // (4 * workers)))
    jobs = [(kind, f, min(chunk, count - f), kw) for f in range(0, count, chunk)]
    if workers <= 1:
        parts = [_gen_chunk(j) for j in jobs]
    else:
        with mp.get_context("fork").Pool(workers) as pool:
            parts = pool.map(_gen_chunk, jobs, chunksize=1)
    return [g for part in parts for g in part]


def percentile(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def bench_batched(L, torch, graphs, warmup: int, profile: bool = False, tuning=None):
    """One louvain_run_batch call against the plain louvain_run loop on the
    same device-resident graphs; outputs must be identical.  The plain loop
    runs with the plain workload's launch shapes (`tuning`), the batched
    call with shapes tuned on the batched workload itself (a batched call
    over every 16th graph, coordinate descent over the shape fields)."""
    ctx = L.Context(0)
    if tuning:
        ctx.set_tuning(**tuning)
    dev = torch.device("cuda", 0)
    Gs = [ctx.graph_create(g.row_ptr, g.col, g.w) for g in graphs]
    out_p = [torch.empty(g.n, dtype=torch.int32, device=dev) for g in graphs]
    out_b = [torch.empty(g.n, dtype=torch.int32, device=dev) for g in graphs]
    torch.cuda.synchronize()
    for G, o in zip(Gs[:64], out_p):      # warm-up of the plain path
        ctx.run(G, labels_out=o, device=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain = [ctx.run(G, labels_out=o, device=True) for G, o in zip(Gs, out_p)]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    t = time.time()
    sample = Gs[::16] if len(Gs) >= 64 else Gs
    best = ctx.autotune_batch(sample)
    tuned = ctx.get_tuning()
    tune_s = time.time() - t
    log(f"batched: autotuned on {len(sample)} graphs in {tune_s:.1f}s: {tuned} ({best['ms']:.2f} ms per call)")
    for _ in range(warmup):
        ctx.run_batch(Gs, labels_out=out_b, stats=False, device=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = ctx.run_batch(Gs, labels_out=out_b, stats=True, device=True)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t1
    same = all(torch.equal(a, b) for a, b in zip(out_p, out_b)) and \
        all(p.q_int == r.q_int for p, r in zip(plain, res))
    edges = sum(lv["sweeps_executed"] * lv["nnz"] for r in res for lv in r.stats["levels"])
    if profile:
        pr = ctx.run_batch(Gs, labels_out=out_b, stats=True, timing=True, device=True)
        ks = sorted(pr[0].stats["kernels"].items(), key=lambda kv: -kv[1]["ms"])
        log(f"batched call with kernel timing: {pr[0].stats['ms_total']:.1f} ms device, kernels " +
            ", ".join(f"{n} {k['ms']:.1f} ms/{k['launches']}" for n, k in ks[:14]))
        passes = {}
        for r in res:
            for lvl, lv in enumerate(r.stats["levels"]):
                passes[lvl] = max(passes.get(lvl, 0), lv["gpu_passes"])
        log(f"max device passes per level: {passes}")
    for G in Gs:
        G.destroy()
    ctx.close()
    return {"graphs": len(graphs), "n_total": int(sum(g.n for g in graphs)),
            "nnz_total": int(sum(g.nnz for g in graphs)), "edges_swept": int(edges),
            "plain_s": round(tp, 4), "batched_s": round(tb, 4), "speedup": round(tp / tb, 3),
            "batched_gteps": round(edges / tb / 1e9, 4), "plain_gteps": round(edges / tp / 1e9, 4),
            "launch_shapes": tuned, "plain_launch_shapes": tuning, "autotune_s": round(tune_s, 2),
            "autotune_sample_graphs": len(sample), "identical_outputs": bool(same)}


def bench_served(L, torch, pool, requests: int, load: float, seed: int = 1005, tuning=None,
                 budget: int = 200 * 10 ** 9):
    """Request loop on Poisson traces against the plain path on the same
    traces, both measured on the device.

    A served request takes its device CSR in (copy, validation, degrees) and
    runs the method; so does a plain request (graph_create, run, destroy),
    one at a time in arrival order.  The saturating trace (every request at
    time 0) gives graphs/s; the Poisson trace at `load` x the plain path's
    measured capacity gives p50/p99 latency (arrival to result).  The
    request loop's memory budget is `budget` bytes.  The plain path's device
    busy time (its kernels' summed device time over its wall time) bounds
    what any batching can gain over it."""
    import numpy as np
    ctx = L.Context(0)
    if tuning:
        ctx.set_tuning(**tuning)
    ctx.serve_budget(budget)
    dev = torch.device("cuda", 0)
    res_in = [(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev), torch.from_numpy(g.w).to(dev))
              for g in pool]
    outs = [torch.empty(g.n, dtype=torch.int32, device=dev) for g in pool]
    torch.cuda.synchronize()
    ref_q = []
    kernel_ms = []
    for t, o in zip(res_in, outs):     # warm-up, reference outputs and device time per graph
        G = ctx.graph_create(*t)
        r = ctx.run(G, labels_out=o, timing=True)
        G.destroy()
        ref_q.append(r.q_int)
        kernel_ms.append(sum(k["ms"] for k in r.stats["kernels"].values()))
    trace = [k % len(pool) for k in range(requests)]
    rng = np.random.default_rng([seed, 7])

    def plain_trace(arrivals):
        """The plain path over the trace, first come first served, on the device."""
        lat = []
        labels = [torch.empty(pool[k].n, dtype=torch.int32, device=dev) for k in trace]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i, k in enumerate(trace):
            wait = t0 + arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            G = ctx.graph_create(*res_in[k])
            ctx.run(G, labels_out=labels[i])
            G.destroy()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - t0 - arrivals[i])
        span = time.perf_counter() - t0
        ok = all(torch.equal(labels[i], outs[k]) for i, k in enumerate(trace))
        return lat, span, ok

    def served_trace(arrivals):
        labels = [torch.empty(pool[k].n, dtype=torch.int32, device=dev) for k in trace]
        torch.cuda.synchronize()
        tickets = []
        t0 = time.perf_counter()
        for i, k in enumerate(trace):
            wait = t0 + arrivals[i] - time.perf_counter()
            if wait > 0:
                time.sleep(wait)
            rp, cl, w = res_in[k]
            tickets.append(ctx.submit(rp, cl, w, labels_out=labels[i]))
        done = {}
        while len(done) < len(tickets):
            for t in tickets:
                if t not in done:
                    r = ctx.poll(t, wait_us=1000)
                    if r is not None:
                        done[t] = r
        lat = [(done[t].t_done_us - done[t].t_submit_us) / 1e6 for t in tickets]
        span = (max(done[t].t_done_us for t in tickets) - min(done[t].t_submit_us for t in tickets)) / 1e6
        ok = all(done[t].status in (0, -6) and done[t].q_int == ref_q[k] for t, k in zip(tickets, trace))
        ok = ok and all(torch.equal(labels[i], outs[k]) for i, k in enumerate(trace))
        return lat, span, ok

    zero = np.zeros(len(trace))
    _, plain_span, ok_p0 = plain_trace(zero)
    capacity = len(trace) / plain_span
    lat_sat, span_sat, ok_sat = served_trace(zero)
    qps = load * capacity
    arrivals = np.cumsum(rng.exponential(1.0 / qps, len(trace)))
    lat, span, ok = served_trace(arrivals)
    plain_lat, _, ok_p1 = plain_trace(arrivals)
    busy = sum(kernel_ms[k] for k in trace) / 1000.0 / plain_span
    ctx.close()
    return {"distinct_graphs": len(pool), "requests": requests, "budget_bytes": budget,
            "mean_nnz": int(np.mean([pool[k].nnz for k in trace])),
            "plain_capacity_gps": round(capacity, 3),
            "saturated_gps": round(len(trace) / span_sat, 3),
            "saturated_speedup": round(len(trace) / span_sat / capacity, 3),
            "plain_device_busy": round(busy, 3), "speedup_bound_from_plain_idle": round(1.0 / busy, 3),
            "trace_qps": round(qps, 3), "load": load,
            "p50_s": round(percentile(lat, 50), 5), "p99_s": round(percentile(lat, 99), 5),
            "plain_p50_s": round(percentile(plain_lat, 50), 5), "plain_p99_s": round(percentile(plain_lat, 99), 5),
            "plain_latency": "measured: the plain path replayed on the device over the same trace",
            "identical_outputs": bool(ok and ok_sat and ok_p0 and ok_p1)}


def shard_bounds(row_ptr, nshards: int):
    """nshards + 1 vertex bounds of contiguous ranges balanced by entries."""
    import numpy as np
    n, nnz = row_ptr.shape[0] - 1, int(row_ptr[-1])
    b = np.searchsorted(row_ptr, np.linspace(0, nnz, nshards + 1).astype(np.int64), side="left")
    b[0], b[-1] = 0, n
    return b


def shard_csr(row_ptr, col, w, lo: int, hi: int):
    """One GPU's share of vertices [lo, hi): its rows renumbered from 0 (columns
    ascending), then one empty row per ghost (a neighbour outside the range,
    numbered after the local vertices in ascending ID order).  Returns
    (row_ptr, col, w, ghost IDs, fraction of entries to ghosts)."""
    import numpy as np
    a, b = int(row_ptr[lo]), int(row_ptr[hi])
    c = col[a:b].astype(np.int64)
    outside = (c < lo) | (c >= hi)
    ghost_ids = np.unique(c[outside])
    nl, ng = hi - lo, int(ghost_ids.shape[0])
    colk = np.where(outside, nl + np.searchsorted(ghost_ids, c), c - lo)
    rpk = np.full(nl + ng + 1, b - a, np.int64)
    rpk[:nl + 1] = row_ptr[lo:hi + 1] - a
    # columns ascend inside every row again after renumbering
    rows = np.repeat(np.arange(nl, dtype=np.int64), np.diff(rpk[:nl + 1]))
    order = np.argsort(rows * (nl + ng) + colk, kind="stable")
    frac = float(outside.mean()) if b > a else 0.0
    return rpk, colk[order].astype(np.int32), w[a:b][order], ghost_ids, frac


def bench_shards(torch, ctx, g, nshards: int) -> dict:
    """One GPU's share of a sharded run, at its real shape: the vertices are
    split into nshards contiguous ranges balanced by entries; shard k holds
    the rows of its range (renumbered from 0) plus one empty row per ghost
    (a neighbour outside the range, numbered after the local vertices), so
    its per-vertex state covers local vertices and ghost copies, as a GPU's
    would.  Each shard's level-0 phase runs alone; its sweep kernels' device
    time per pass and its renumbering and contraction time are compared with
    the whole graph's (the exchange of ghost labels and community deltas
    between GPUs, and of contracted entries, is not part of it).  The labels
    of a shard alone mean nothing: only the timing is reported."""
    import numpy as np
    dev = torch.device("cuda", 0)
    rp, col, w = g.row_ptr, g.col, g.w
    bounds = shard_bounds(rp, nshards)

    def per_pass(rpk, colk, wk):
        # level 0's phase, then its renumbering and contraction (a second
        # level is started so that the first one is contracted)
        G = ctx.graph_create(torch.from_numpy(rpk).to(dev), torch.from_numpy(colk).to(dev),
                             torch.from_numpy(wk).to(dev))
        ctx.run(G, max_levels=2)   # warm-up
        r = ctx.run(G, max_levels=2, timing=True)
        G.destroy()
        lv = r.stats["levels"][0]
        return lv["ms_sweep"] / max(1, lv["gpu_passes"]), lv["gpu_passes"], lv["ms_contract"]

    full_ms, full_passes, full_contract = per_pass(rp, col, w)
    shards = []
    for k in range(nshards):
        lo, hi = int(bounds[k]), int(bounds[k + 1])
        rpk, colk, wk, ghost_ids, frac = shard_csr(rp, col, w, lo, hi)
        ms, passes, contract_ms = per_pass(rpk, colk, wk)
        shards.append({"vertices": hi - lo, "ghosts": int(ghost_ids.shape[0]), "entries": int(rpk[-1]),
                       "ghost_entry_fraction": round(frac, 4), "sweep_ms_per_pass": round(ms, 4),
                       "passes": passes, "contract_ms": round(contract_ms, 4)})
    worst = max(x["sweep_ms_per_pass"] for x in shards)
    worst_c = max(x["contract_ms"] for x in shards)
    return {"shards": nshards, "whole_graph_sweep_ms_per_pass": round(full_ms, 4),
            "max_shard_sweep_ms_per_pass": round(worst, 4), "speedup_per_pass": round(full_ms / worst, 3),
            "whole_graph_contract_ms": round(full_contract, 4), "max_shard_contract_ms": round(worst_c, 4),
            "per_shard": shards}


def bench_dendro(torch, ctx, rp, col, w, ref_labels, plain_ms: float, runs: int = 3) -> dict:
    """The run that keeps the dendrogram (per-level maps and the last level's
    graph), and a run resumed from the first level's state, against the
    plain run on the same graph: wall time per run, identical outputs."""
    def one():
        G = ctx.graph_create(rp, col, w)
        res, D = ctx.run(G, dendrogram=True)
        Gl = D.graph()
        G.destroy()
        return res, D, Gl

    for r in one()[1:]:
        r.destroy()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        res, D, Gl = one()
        levels, sizes = D.levels, D.n
        D.destroy()
        Gl.destroy()
    torch.cuda.synchronize()
    dendro_ms = (time.perf_counter() - t0) * 1000.0 / runs
    same = bool(torch.equal(res.labels, ref_labels))
    # checkpoint after the first level, then resume: both parts timed
    G = ctx.graph_create(rp, col, w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    part, D = ctx.run(G, max_levels=1, dendrogram=True)
    Gl = D.graph()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rest = ctx.resume(Gl, 1, part.labels)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    same = same and bool(torch.equal(rest.labels, ref_labels))
    D.destroy()
    Gl.destroy()
    G.destroy()
    return {"ms_per_run": round(dendro_ms, 3), "plain_ms_per_run": round(plain_ms, 3),
            "overhead": round(dendro_ms / plain_ms, 3), "levels": levels, "map_entries": int(sum(sizes[:-1])),
            "checkpoint_level1_ms": round((t1 - t0) * 1000.0, 3), "resume_ms": round((t2 - t1) * 1000.0, 3),
            "identical_outputs": same}


def bench_merge(torch, ctx, rp, col, w, plain_ms: float, plain_q: float, runs: int = 3) -> dict:
    """The run with the final merge after every phase against the plain run:
    wall time per run, Q, and the merge kernels' device time (one timed run)."""
    def one(timing=False):
        G = ctx.graph_create(rp, col, w)
        r = ctx.run(G, merge=True, timing=timing)
        G.destroy()
        return r

    one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(runs):
        r = one()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1000.0 / runs
    k = one(timing=True).stats["kernels"]
    merge_ms = sum(v["ms"] for n, v in k.items() if n in ("k_comm_state", "k_merge_lone"))
    return {"ms_per_run": round(ms, 3), "plain_ms_per_run": round(plain_ms, 3), "overhead": round(ms / plain_ms, 3),
            "q": r.q, "q_plain": plain_q, "levels": len(r.stats["levels"]),
            "merge_kernels_ms": round(merge_ms, 4)}


def time_oracle_runs(oracle, g, threads: int, min_s: float, max_runs: int):
    """Full oracle runs on the host: (result, runs, seconds per run)."""
    oracle.set_threads(threads)
    runs, spent, res = 0, 0.0, None
    while runs < max_runs and (runs == 0 or spent < min_s):
        c0 = time.perf_counter()
        res = oracle.louvain(g.row_ptr, g.col, g.w)
        spent += time.perf_counter() - c0
        runs += 1
    oracle.set_threads(1)
    return res, runs, spent / runs


def cpu_full_runs(np, g, workload: str, r, out, threads: int):
    """The oracle on the whole workload (OpenMP variant, then single-threaded
    when it stays short), in GTEPS of the method's executed sweeps; parity of
    the GPU run's labels and Q_int with it."""
    import oracle
    ref, runs, per = time_oracle_runs(oracle, g, threads, 10.0, 3)
    ref_edges = sum(lv["sweeps_executed"] * lv["nnz"] for lv in ref.levels)
    cpu = {"value": round(ref_edges / per / 1e9, 5), "unit": "GTEPS", "cores": threads, "kind": "oracle",
           "sample": f"{runs} full oracle run(s) of {workload} with its OpenMP variant on {threads} "
                     f"threads, {per:.3f} s each"}
    same = True
    if threads > 1 and per < 20.0:   # the single-threaded oracle too, when it stays within the sample
        ref1, runs1, per1 = time_oracle_runs(oracle, g, 1, 5.0, 2)
        cpu["single_thread_value"] = round(ref_edges / per1 / 1e9, 5)
        cpu["sample"] += f" (single-threaded: {runs1} run(s), {per1:.3f} s each)"
        same = bool(np.array_equal(ref1.labels, ref.labels))
    labels = out.cpu().numpy()
    parity = bool(np.array_equal(labels, ref.labels) and r.q_int == ref.q_int and same)
    return cpu, parity


def cpu_sweep_sample(np, g, workload: str, threads: int):
    """For a workload whose whole oracle run takes many minutes: level-0
    sweeps of the oracle (OpenMP variant), from singletons and from a
    4,096-community labelling, in GTEPS (entries per second of sweeps)."""
    import graphgen as gg
    import oracle
    oracle.set_threads(threads)
    t = 0.0
    sweeps = 0
    for labels in (None, gg.random_labels(g.n, 4096, 11)):
        c0 = time.perf_counter()
        oracle.local_move(g.row_ptr, g.col, g.w, labels)
        t += time.perf_counter() - c0
        sweeps += 1
    oracle.set_threads(1)
    return {"value": round(sweeps * g.nnz / t / 1e9, 5), "unit": "GTEPS", "cores": threads, "kind": "oracle",
            "sample": f"{sweeps} level-0 sweeps of {workload} (from singletons and from 4,096 random "
                      f"communities) with the oracle's OpenMP variant on {threads} threads, {t / sweeps:.2f} s "
                      f"each; a whole oracle run of this graph takes about ten minutes"}


def golden_parity(np, workload: str, r, out):
    """Labels, Q_int and level records of the GPU run against the oracle's
    results stored as digests (tests/golden/<workload>_expected.json, written
    by a script that calls only the oracle and the generators)."""
    import hashlib
    path = os.path.join(ROOT, "tests", "golden", f"{workload}_expected.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        exp = json.load(f)["run"]
    labels = np.ascontiguousarray(out.cpu().numpy(), dtype=np.int32)
    same = hashlib.sha256(labels.tobytes()).hexdigest() == exp["labels"] and str(r.q_int) == exp["q_int"]
    lv = [(x["n"], x["nnz"], x["sweeps_executed"], x["sweeps_accepted"], str(x["q_int"])) for x in r.stats["levels"]]
    lv_exp = [(x["n"], x["nnz"], x["sweeps_executed"], x["sweeps_accepted"], x["q_int"]) for x in exp["levels"]]
    return bool(same and lv == lv_exp)


def _gather_lib():
    import ctypes as C
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "paper_1805_10904_amd", "libgather_ref.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run paper_1805_10904_amd/build.py")
    lib = C.CDLL(path)
    lib.gather_ref_us.argtypes = [C.c_void_p, C.c_int64, C.c_int64, C.c_int, C.POINTER(C.c_float)]
    lib.gather_ref_us.restype = C.c_int
    return lib


def _gather_only_us(lib, idx_ptr: int, m: int, n: int, reps: int) -> float:
    import ctypes as C
    us = C.c_float(0)
    rc = lib.gather_ref_us(idx_ptr, int(m), int(n), int(reps), C.byref(us))
    if rc != 0:
        raise RuntimeError(f"gather_ref_us failed ({rc})")
    return float(us.value)


def gather_reference(torch, np, g, ctx, rp, col, w, dominant: str, tuning: dict):
    """The sweep at level 0 against a plain gather of the same words: every
    swept entry reads one 8-byte published word at its column, in a random
    order over the level's n words.  libgather_ref times a kernel that does
    those reads and nothing else (same count, same columns, same order of
    rows, one store per 4 or 16 reads), which is what the memory system gives
    that pattern; the sweep does them plus its table work.
    Compact levels (dominant kernel k_cpt_groups): that kernel's level-0
    launches against the reads of the rows it sweeps (small_max < d <= 341,
    loops excluded).  General levels (2W >= 2^31, whatever kernel
    dominates): the level-0 passes (every sweep kernel, level 0 in input
    order) against the reads of every entry (the workloads have no loops).
    None otherwise."""
    if not dominant:
        return None
    lib = _gather_lib()
    if dominant.startswith("k_cpt_groups"):
        d = np.diff(g.row_ptr)
        rows = np.nonzero((d > tuning["small_max"]) & (3 * d <= 2 * 512) & (d <= tuning["block_max"]))[0]
        lens = d[rows]
        first = np.repeat(g.row_ptr[rows] - np.concatenate(([0], np.cumsum(lens)[:-1])), lens)
        ent = first + np.arange(int(lens.sum()), dtype=np.int64)
        cols = g.col[ent]
        cols = cols[cols != np.repeat(rows, lens)].astype(np.int32)
        if cols.size == 0 or cols.min() < 0 or cols.max() >= g.n:
            return None
        G = ctx.graph_create(rp, col, w)
        r = ctx.run(G, max_levels=1, timing=dominant)
        G.destroy()
        k = r.stats["kernels"].get(dominant)
        if not k or k["launches"] == 0:
            return None
        sweep_us = k["ms"] * 1000.0 / k["launches"]
        dev_cols = torch.from_numpy(cols).to(torch.device("cuda", 0))
        us = _gather_only_us(lib, dev_cols.data_ptr(), cols.size, g.n, 20)
        m = int(cols.size)
        return {"what": "level-0 launches of the packed-class sweep vs a kernel that only reads the same published "
                        "words (8 B at each swept entry's column, same rows, same order)",
                "rows": int(rows.size), "gathers": m, "words": int(g.n),
                "sweep_launch_us": round(sweep_us, 2), "sweep_launches": int(k["launches"]),
                "gather_only_us": round(us, 2),
                "sweep_gathers_per_s": round(m / (sweep_us * 1e-6), 1),
                "gather_only_per_s": round(m / (us * 1e-6), 1),
                "sweep_over_gather_only": round(sweep_us / us, 3)}
    if g.nnz == 0 or int(g.w.sum(dtype=np.int64)) < (1 << 31):
        return None   # compact levels: only the packed-class comparison above
    keys = ("small_max", "block_max", "pass_batch", "group_slots", "group_vertices", "overlap", "reorder",
            "group_tiles")
    ctx.set_tuning(*[2 if k == "reorder" else int(tuning[k]) for k in keys])   # level 0 in input order
    try:
        G = ctx.graph_create(rp, col, w)
        r = ctx.run(G, max_levels=1, timing=True)
        G.destroy()
    finally:
        ctx.set_tuning(*[int(tuning[k]) for k in keys])
    lv0 = r.stats["levels"][0]
    if lv0["gpu_passes"] <= 0 or lv0["ms_sweep"] <= 0:
        return None
    pass_us = lv0["ms_sweep"] * 1000.0 / lv0["gpu_passes"]
    us = _gather_only_us(lib, col.data_ptr(), g.nnz, g.n, 5)
    return {"what": "level-0 sweep passes (every sweep kernel, level 0 in input order) vs a kernel that only reads "
                    "one 8-byte word at every entry's column (the passes' neighbour reads, same order)",
            "gathers": int(g.nnz), "words": int(g.n), "passes": int(lv0["gpu_passes"]),
            "pass_us": round(pass_us, 1), "gather_only_us": round(us, 1),
            "pass_gathers_per_s": round(g.nnz / (pass_us * 1e-6), 1),
            "gather_only_per_s": round(g.nnz / (us * 1e-6), 1),
            "pass_over_gather_only": round(pass_us / us, 3)}


def measure_plain(L, torch, np, g, workload: str, steps: int, warmup: int, timing: bool, pass_batch: int,
                  shapes=None, autotune: bool = True, cpu: str = "full"):
    """The plain method on one workload: W warm-up steps (the last one times
    every launch), K timed steps (the last one times the dominant kernel's
    launches), the roofline of the dominant kernel, the CPU oracle beside it
    (cpu: "full" whole runs, "sweeps" level-0 sweeps, "none") and parity.
    A step = graph_create from the device-resident CSR + run + destroy."""
    dev = torch.device("cuda", 0)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    out = torch.empty(g.n, dtype=torch.int32, device=dev)
    ctx = L.Context(0)

    def step(tm):
        G = ctx.graph_create(rp, col, w)
        r = ctx.run(G, timing=tm, pass_batch=pass_batch, labels_out=out)
        G.destroy()
        return r

    if shapes:
        ctx.set_tuning(*[int(x) for x in shapes.split(",")])
    tuning = ctx.get_tuning()
    if autotune and not shapes:
        G = ctx.graph_create(rp, col, w)
        t = time.time()
        best = ctx.autotune(G)
        G.destroy()
        tuning = ctx.get_tuning()
        log(f"{workload}: autotuned launch shapes in {time.time() - t:.2f}s: {tuning} ({best['ms']:.3f} ms per run)")

    # warm-up steps; the last one records every kernel to find the dominant
    # one, whose launches alone are timed in the last timed step
    dominant = table = table_levels = None
    nwarm = max(2, warmup) if timing else warmup
    for k in range(nwarm):
        full = timing and k == nwarm - 1
        r0 = step(full)
        if full:
            table = r0.stats["kernels"]
            table_levels = r0.stats["levels"]
            dominant = max(table.items(), key=lambda kv: kv[1]["ms"])[0]
        log(f"{workload}: warmup {k + 1}/{nwarm} done")
    torch.cuda.synchronize()
    results = []
    t0 = time.perf_counter()
    # the dominant kernel's launches carry dispatch events in the last timed
    # step only: each event adds a few microseconds before and after its
    # kernel, which would otherwise weigh on every step's wall time
    for k in range(steps):
        results.append(step(dominant if timing and k == steps - 1 else False))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    log(f"{workload}: timed {steps} steps")
    ms_per_step = (t1 - t0) * 1000.0 / max(1, steps)
    r = results[-1]
    levels = r.stats["levels"]
    edges = sum(lv["sweeps_executed"] * lv["nnz"] for lv in levels)
    sweeps = sum(lv["sweeps_executed"] for lv in levels)
    res = {"value": round(edges / (ms_per_step / 1000.0) / 1e9, 4), "unit": "GTEPS", "steps": steps,
           "warmup": warmup, "ms_per_step": round(ms_per_step, 4), "full_louvain_s": round(ms_per_step / 1000.0, 6),
           "config": {"workload": workload, "n": g.n, "nnz": g.nnz, "levels": len(levels), "sweeps": sweeps,
                      "edges_swept": edges, "launch_shapes": tuning},
           "q": r.q, "sweep_gteps": None, "level0_sweep_gteps": None, "kernel_ms_per_step": None,
           "roofline": None, "cpu_baseline": None, "parity_vs_oracle": None}
    if timing:
        dom = dict(launches=0, ms=0.0, alg_bytes=0.0)
        k = r.stats["kernels"].get(dominant)
        if k:
            for key in dom:
                dom[key] += k[key]
        achieved = dom["alg_bytes"] / (dom["ms"] / 1000.0) / 1e9
        sweep_ms = sum(v["ms"] for n, v in table.items() if n.startswith(("k_cpt_", "k_sweep", "k_hub", "k_commit",
                                                                             "k_qsum", "k_finalize")))
        lv0 = table_levels[0] if table_levels else None
        traffic = recorded_traffic(workload, dominant)
        alg_per_launch = dom["alg_bytes"] / max(1, dom["launches"])
        res["sweep_gteps"] = round(edges / (sweep_ms / 1000.0) / 1e9, 3) if sweep_ms > 0 else None
        res["level0_sweep_gteps"] = (round(lv0["sweeps_executed"] * lv0["nnz"] / (lv0["ms_sweep"] / 1000.0) / 1e9, 3)
                                     if lv0 and lv0["ms_sweep"] > 0 else None)
        res["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dominant,
                           "avg_launch_us": round(dom["ms"] * 1000.0 / max(1, dom["launches"]), 2),
                           "launches_per_step": dom["launches"], "traffic_unit": "bytes per launch",
                           "alg_bytes_per_launch": round(alg_per_launch),
                           "traffic_over_alg": round(traffic / alg_per_launch, 3) if traffic else None}
        res["roofline"]["gather_ref"] = gather_reference(torch, np, g, ctx, rp, col, w, dominant, tuning)
        if res["roofline"]["gather_ref"]:
            log(f"{workload}: level-0 gathers: {res['roofline']['gather_ref']}")
        top = sorted(table.items(), key=lambda kv: -kv[1]["ms"])[:20]
        log(f"{workload}: kernel time of one step (all launches timed): " +
            ", ".join(f"{n} {a['ms']:.3f} ms" for n, a in top))
        kernel_ms = sum(a["ms"] for a in table.values())
        res["kernel_ms_per_step"] = round(kernel_ms, 4)
        res["launches_per_step"] = int(sum(a["launches"] for a in table.values()))
        log(f"{workload}: all kernels {kernel_ms:.3f} ms per step ({res['launches_per_step']} launches); timed "
            f"step {ms_per_step:.3f} ms; dominant {dominant} "
            f"{dom['ms'] * 1000.0 / max(1, dom['launches']):.2f} us per launch in the last timed step")
    threads = max(1, min(16, os.cpu_count() or 1))
    if cpu == "full":
        log(f"{workload}: timing the CPU oracle on the same graph")
        res["cpu_baseline"], res["parity_vs_oracle"] = cpu_full_runs(np, g, workload, r, out, threads)
        log(f"{workload}: oracle: {res['cpu_baseline']['sample']}, parity {res['parity_vs_oracle']}")
    elif cpu == "sweeps":
        log(f"{workload}: timing level-0 sweeps of the CPU oracle")
        res["cpu_baseline"] = cpu_sweep_sample(np, g, workload, threads)
        res["parity_vs_oracle"] = golden_parity(np, workload, r, out)
        log(f"{workload}: oracle: {res['cpu_baseline']['sample']}; parity with the stored oracle results "
            f"{res['parity_vs_oracle']}")
    return res, dict(ctx=ctx, rp=rp, col=col, w=w, out=out, r=r, tuning=tuning)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="chunglu1m")
    ap.add_argument("--pass-batch", type=int, default=0)
    ap.add_argument("--no-timing", action="store_true", help="time steps without per-kernel events")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (skip the autotuner)")
    ap.add_argument("--shapes", default=None,
                    help="fixed launch shapes: small_max,block_max,pass_batch[,group_slots[,group_vertices"
                         "[,overlap[,reorder[,group_tiles]]]]]")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rmat24", type=int, default=1,
                    help="also measure the R-MAT scale-24 workload (its own roofline, level-0 oracle sweeps, "
                         "parity with the stored oracle results); 0 = skip")
    ap.add_argument("--rmat24-steps", type=int, default=3)
    ap.add_argument("--sbm1k", type=int, default=1, help="also time the 1,000-vertex SBM workload; 0 = skip")
    ap.add_argument("--batched", type=int, default=4096,
                    help="graphs of the batched comparison (0 = skip)")
    ap.add_argument("--batched-nmax", type=int, default=100_000)
    ap.add_argument("--batched-profile", action="store_true", help="log the batched call's kernel table")
    ap.add_argument("--served", type=int, default=48,
                    help="distinct request graphs of the served comparison (0 = skip)")
    ap.add_argument("--served-requests", type=int, default=0, help="trace length (default 3x the graphs)")
    ap.add_argument("--served-load", type=float, default=0.7, help="trace QPS as a fraction of plain capacity")
    ap.add_argument("--no-dendro", action="store_true",
                    help="skip the dendrogram / resume and final-merge comparisons")
    ap.add_argument("--shards", type=int, default=8,
                    help="time one GPU's share of this many vertex shards (0 or 1 = skip)")
    ap.add_argument("--gen-workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "graphs shard across GPUs only by design, see the sharding notes", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    # graphs of the batched and served workloads, generated before any GPU use
    batch_graphs = served_pool = None
    if args.batched > 0:
        t = time.time()
        batch_graphs = generate("batch", args.batched, args.gen_workers, n_hi=args.batched_nmax)
        log(f"generated {len(batch_graphs)} batched graphs, {sum(g.nnz for g in batch_graphs)} entries, "
            f"in {time.time() - t:.1f}s")
    if args.served > 0:
        t = time.time()
        served_pool = generate("served", args.served, args.gen_workers)
        log(f"generated {len(served_pool)} request graphs, {sum(g.nnz for g in served_pool)} entries, "
            f"in {time.time() - t:.1f}s")

    import torch

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {args.copy_calibration_mib} MiB three times")
        return

    import graphgen as gg
    import paper_1805_10904_amd as L

    timing = not args.no_timing
    log(f"generating {args.workload}")
    t = time.time()
    g = gg.config(args.workload)
    log(f"generated n={g.n} nnz={g.nnz} in {time.time() - t:.1f}s")
    head_cpu = "none" if args.no_cpu_baseline else ("sweeps" if args.workload == "rmat24" else "full")
    head, ctxs = measure_plain(L, torch, np, g, args.workload, args.steps, args.warmup, timing, args.pass_batch,
                               shapes=args.shapes, autotune=not args.no_autotune, cpu=head_cpu)
    ctx, rp, col, w, out, r, tuning = (ctxs[k] for k in ("ctx", "rp", "col", "w", "out", "r", "tuning"))
    ms_per_step = head["ms_per_step"]

    dendro = merged = None
    if not args.no_dendro:
        log("dendrogram and resume vs plain")
        try:
            dendro = bench_dendro(torch, ctx, rp, col, w, out.clone(), ms_per_step)
        except Exception as e:  # the main measurement stands on its own
            dendro = {"error": f"{type(e).__name__}: {e}"}
        log(f"dendrogram: {dendro}")
        log("final merge vs plain")
        try:
            merged = bench_merge(torch, ctx, rp, col, w, ms_per_step, r.q)
        except Exception as e:
            merged = {"error": f"{type(e).__name__}: {e}"}
        log(f"merge: {merged}")

    shards = None
    if args.shards > 1:
        log(f"one GPU's share of {args.shards} shards")
        try:
            shards = bench_shards(torch, ctx, g, args.shards)
        except Exception as e:  # the main measurement stands on its own
            shards = {"error": f"{type(e).__name__}: {e}"}
        log(f"shards: {shards}")
    ctx.close()
    del ctxs, rp, col, w, out

    others = {}
    for name, on in (("sbm1k", args.sbm1k), ("rmat24", args.rmat24)):
        if not on or name == args.workload:
            continue
        log(f"generating {name}")
        t = time.time()
        gx = gg.config(name)
        log(f"generated n={gx.n} nnz={gx.nnz} in {time.time() - t:.1f}s")
        cpu_mode = "none" if args.no_cpu_baseline else ("sweeps" if name == "rmat24" else "full")
        steps = args.rmat24_steps if name == "rmat24" else max(args.steps, 20)
        warm = 2 if name == "rmat24" else max(args.warmup, 5)
        try:
            resx, cx = measure_plain(L, torch, np, gx, name, steps, warm, timing, args.pass_batch,
                                     shapes=args.shapes, autotune=not args.no_autotune and name != "rmat24",
                                     cpu=cpu_mode)
            cx["ctx"].close()
            del cx
        except Exception as e:  # the headline stands on its own
            resx = {"error": f"{type(e).__name__}: {e}"}
        others[name] = resx
        log(f"{name}: {resx}")
        del gx

    batched = served = None
    if batch_graphs is not None:
        log("batched vs plain")
        try:
            batched = bench_batched(L, torch, batch_graphs, warmup=1, profile=args.batched_profile, tuning=tuning)
        except Exception as e:  # the main measurement stands on its own
            batched = {"error": f"{type(e).__name__}: {e}"}
        log(f"batched: {batched}")
        del batch_graphs
    if served_pool is not None:
        log("served vs plain")
        try:
            served = bench_served(L, torch, served_pool, args.served_requests or 3 * len(served_pool),
                                  args.served_load, tuning=tuning)
        except Exception as e:
            served = {"error": f"{type(e).__name__}: {e}"}
        log(f"served: {served}")

    cfg = dict(head["config"])
    cfg["parallelism"] = "single GPU"
    line = {
        "metric": METRIC, "value": head["value"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": cfg,
        "full_louvain_s": head["full_louvain_s"],
        "sweep_gteps": head["sweep_gteps"],
        "level0_sweep_gteps": head["level0_sweep_gteps"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "launches_per_step": head.get("launches_per_step"),
        "q": head["q"],
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
        "parity_vs_oracle": head["parity_vs_oracle"],
    }
    if "rmat24" in others:
        line["c3_rmat24"] = others["rmat24"]
    if "sbm1k" in others:
        line["c1_sbm1k"] = others["sbm1k"]
    if dendro is not None:
        line["dendrogram"] = dendro
    if merged is not None:
        line["final_merge"] = merged
    if shards is not None:
        line["one_gpu_share"] = shards
    if batched is not None:
        line["batched"] = batched
    if served is not None:
        line["served"] = served
    print(json.dumps(line))


if __name__ == "__main__":
    main()
