"""GPU tests of the served form (louvain_submit / louvain_poll).

Each request's result in the mix equals the oracle's and the plain call's
for that graph alone; admission keeps the admitted footprint within the
budget; a failing request does not disturb the others.
"""
import sys
import threading
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture()
def L():
    import paper_1805_10904_amd as L
    return L


def _levels(levels):
    return [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"]) for lv in levels]


def _ref_levels(ref):
    return [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"]) for lv in ref.levels]


def _check(g, r, tag, **kw):
    ref = oracle.louvain(g.row_ptr, g.col, g.w, **kw)
    labels = r.labels.cpu().numpy() if hasattr(r.labels, "cpu") else r.labels
    assert r.status in (0, -6), f"{tag}: status {r.status} {r.error}"
    assert np.array_equal(labels, ref.labels), f"{tag}: labels differ"
    assert r.q_int == ref.q_int, f"{tag}: Q_int differs"
    assert abs(r.q - ref.q) <= 1e-12 * max(abs(ref.q), 1e-3)
    assert _levels(r.levels) == _ref_levels(ref), f"{tag}: level records differ"
    assert (r.status == 0) == (ref.status == 0)


def _drain(ctx, tickets, timeout_s=120.0):
    out = {}
    t_end = time.time() + timeout_s
    while len(out) < len(tickets):
        assert time.time() < t_end, "served requests did not finish in time"
        for t in tickets:
            if t in out:
                continue
            r = ctx.poll(t, wait_us=2000)
            if r is not None:
                out[t] = r
    return out


def test_served_mix_equals_alone(L):
    """Arrivals spread over time join the running batch at level boundaries."""
    ctx = L.Context(0)
    graphs = gg.batch_sbm(24, n_hi=20_000, first=200) + [gg.config("sbm1k"), gg.config("chunglu_n20000")]
    tickets = []

    def producer():
        for k, g in enumerate(graphs):
            tickets.append(ctx.submit(g.row_ptr, g.col, g.w))
            if k % 3 == 2:
                time.sleep(0.002)

    th = threading.Thread(target=producer)
    th.start()
    th.join()
    _say(f"submitted {len(tickets)} requests")
    res = _drain(ctx, tickets)
    for k, (g, t) in enumerate(zip(graphs, tickets)):
        r = res[t]
        _check(g, r, f"request {k}")
        assert r.t_submit_us <= r.t_admit_us <= r.t_done_us
    # the same graphs alone through the plain call
    for k in (0, 5, len(graphs) - 1):
        g = graphs[k]
        G = ctx.graph_create(g.row_ptr, g.col, g.w)
        a = ctx.run(G)
        assert np.array_equal(a.labels, res[tickets[k]].labels) and a.q_int == res[tickets[k]].q_int
        G.destroy()
    ctx.close()


def test_served_device_pointers_and_params(L):
    import torch
    ctx = L.Context(0)
    dev = torch.device("cuda", 0)
    graphs = gg.batch_sbm(6, n_hi=5000, first=300)
    kws = [dict(), dict(max_levels=1), dict(singlet_rule=False), dict(), dict(max_sweeps=1), dict()]
    tickets = []
    for g, kw in zip(graphs, kws):
        rp = torch.from_numpy(g.row_ptr).to(dev)
        cl = torch.from_numpy(g.col).to(dev)
        w = torch.from_numpy(g.w).to(dev)
        torch.cuda.synchronize()
        tickets.append(ctx.submit(rp, cl, w, **kw))
    res = _drain(ctx, tickets)
    for k, (g, kw, t) in enumerate(zip(graphs, kws, tickets)):
        assert res[t].labels.is_cuda
        _check(g, res[t], f"request {k} {kw}", **kw)
    ctx.close()


def test_served_budget_admission(L):
    """With a budget of about three graphs, the admitted footprint never exceeds it."""
    ctx = L.Context(0)
    graphs = gg.batch_sbm(12, n_lo=2000, n_hi=8000, first=400)
    sizes = [L.workspace_bytes(g.n, g.nnz) for g in graphs]
    budget = 3 * max(sizes)
    ctx.serve_budget(budget)
    tickets = [ctx.submit(g.row_ptr, g.col, g.w) for g in graphs]
    res = _drain(ctx, tickets)
    for k, (g, t) in enumerate(zip(graphs, tickets)):
        _check(g, res[t], f"request {k}")
    # at every admission instant the requests resident then fit the budget
    spans = [(res[t].t_admit_us, res[t].t_done_us, b) for t, b in zip(tickets, sizes)]
    for a, _, _ in spans:
        resident = sum(b for (s, e, b) in spans if s <= a < e)
        assert resident <= budget
    ctx.close()


def test_served_failures_are_isolated(L):
    ctx = L.Context(0)
    good = gg.batch_sbm(4, n_hi=3000, first=500)
    g = gg.from_edge_list(4, [(0, 1), (1, 2), (2, 3)])
    bad_col = np.array([1, 2, 0, 1, 3, 2], np.int32)             # unsorted row
    tickets = [ctx.submit(good[0].row_ptr, good[0].col, good[0].w),
               ctx.submit(g.row_ptr, bad_col, g.w),
               ctx.submit(good[1].row_ptr, good[1].col, good[1].w)]
    ctx.serve_budget(L.workspace_bytes(good[2].n, good[2].nnz) + L.workspace_bytes(good[3].n, good[3].nnz) +
                     L.workspace_bytes(good[0].n, good[0].nnz) + L.workspace_bytes(good[1].n, good[1].nnz))
    big = gg.random_small(50, 0.2, 3, seed=1)
    huge_n = 10_000_000                                           # footprint beyond the budget
    rp_big = np.zeros(huge_n + 1, np.int64)
    rp_big[1:] = 0
    tickets.append(ctx.submit(rp_big, np.zeros(0, np.int32), np.zeros(0, np.int32)))
    tickets.append(ctx.submit(good[2].row_ptr, good[2].col, good[2].w))
    tickets.append(ctx.submit(big.row_ptr, big.col, big.w))
    res = _drain(ctx, tickets)
    assert res[tickets[1]].status == L.LOUVAIN_EINVAL and res[tickets[1]].error
    assert res[tickets[3]].status == L.LOUVAIN_ENOMEM
    _check(good[0], res[tickets[0]], "good 0")
    _check(good[1], res[tickets[2]], "good 1")
    _check(good[2], res[tickets[4]], "good 2")
    _check(big, res[tickets[5]], "small")
    with pytest.raises(L.LouvainError):
        ctx.poll(tickets[0])          # retired
    ctx.close()


def test_served_c5_sizes_mixed_with_small(L):
    """Requests shaped like the served workload (Chung-Lu, 2e6..3.4e6 entries:
    the large-graph worker), one of them reweighted so that 2W >= 2^31 (the
    plain path), interleaved with small SBM requests (the small-graph
    worker).  Every result equals the oracle's; both batched workers and the
    plain worker hold requests at the same time; a request joins a worker
    whose batch is already running; and the heavy request does not hold back
    the large-graph worker."""
    import os
    oracle.set_threads(min(16, os.cpu_count() or 1))
    large = gg.served_chunglu(3, first=0, n_lo=60_000, n_hi=250_000)    # 3.4e6, 1.0e6, 3.1e6 entries
    large = [g for g in large if g.nnz > (1 << 20)] + gg.served_chunglu(1, first=5, n_lo=60_000, n_hi=250_000)
    heavy = gg.served_chunglu(1, first=6, n_lo=60_000, n_hi=250_000)[0]
    heavy = gg.Graph(heavy.n, heavy.row_ptr, heavy.col, (heavy.w.astype(np.int64) * 100).astype(np.int32),
                     heavy.planted, "served_6_x100")
    assert int(heavy.w.astype(np.int64).sum()) >= (1 << 31)
    assert all(g.nnz > (1 << 20) for g in large + [heavy])
    small = gg.batch_sbm(10, n_hi=20_000, first=700)
    assert all(g.nnz <= (1 << 20) for g in small)
    order = [("heavy", heavy), ("large", large[0])] + [("small", g) for g in small[:3]] + \
        [("large", large[1])] + [("small", g) for g in small[3:6]] + [("large", large[2])] + \
        [("small", g) for g in small[6:]]
    ctx = L.Context(0)
    tickets = []
    for k, (kind, g) in enumerate(order):
        tickets.append(ctx.submit(g.row_ptr, g.col, g.w))
        if k % 2 == 1:
            time.sleep(0.002)
    _say(f"submitted {len(tickets)} requests ({sum(g.nnz for _, g in order)} entries)")
    res = _drain(ctx, tickets, timeout_s=180.0)
    for k, ((kind, g), t) in enumerate(zip(order, tickets)):
        _check(g, res[t], f"request {k} ({kind} {g.name}, nnz {g.nnz})")
        assert res[t].t_submit_us <= res[t].t_admit_us <= res[t].t_done_us
    _say("every served result equals the oracle's")
    span = {t: (res[t].t_admit_us, res[t].t_done_us) for t in tickets}
    kinds = [kind for kind, _ in order]
    by = {kd: [t for t, k2 in zip(tickets, kinds) if k2 == kd] for kd in ("heavy", "large", "small")}

    def inside(a, b):   # request a admitted while request b was resident
        return span[b][0] < span[a][0] < span[b][1]

    # the large-graph worker admitted the next request while the heavy one ran
    assert inside(by["large"][0], by["heavy"][0]), "the heavy request blocked the large-graph worker"
    # the two batched workers held requests at the same time
    assert any(inside(s, lg) for s in by["small"] for lg in by["large"]), "workers never overlapped"
    # a request joined a worker whose batch was already running (a later
    # arrival admitted while an earlier request of the same worker was resident)
    joined = [(a, b) for kd in ("large", "small") for i, b in enumerate(by[kd]) for a in by[kd][i + 1:]
              if inside(a, b) and span[a][0] > span[b][0] + 500.0]
    assert joined, "no request joined a running batch"
    # the same graphs through the plain call
    for kind, g in (order[0], order[1]):
        G = ctx.graph_create(g.row_ptr, g.col, g.w)
        a = ctx.run(G)
        t = tickets[[x for x, _ in order].index(kind)]
        assert np.array_equal(a.labels, res[t].labels) and a.q_int == res[t].q_int
        G.destroy()
    ctx.close()
