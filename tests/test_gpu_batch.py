"""GPU parity of the batched call: every graph's outputs from one
louvain_run_batch call equal the oracle's for that graph alone (labels,
Q_int, per-level records, status) and the plain louvain_run's.
"""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import paper_1805_10904_amd as L
    return L


@pytest.fixture(scope="module")
def ctx(L):
    c = L.Context(0)
    yield c
    c.close()


def _levels(stats):
    return [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"]) for lv in stats["levels"]]


def _ref_levels(ref):
    return [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"]) for lv in ref.levels]


def check_batch(ctx, graphs, tag="", device=False, **kw):
    import torch
    dev = torch.device("cuda", 0)
    Gs = []
    for g in graphs:
        if device:
            Gs.append(ctx.graph_create(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                                       torch.from_numpy(g.w).to(dev)))
        else:
            Gs.append(ctx.graph_create(g.row_ptr, g.col, g.w))
    res = ctx.run_batch(Gs, **kw)
    okw = {k: v for k, v in kw.items() if k != "pass_batch"}   # a launch knob, not part of the method
    for k, (g, r) in enumerate(zip(graphs, res)):
        ref = oracle.louvain(g.row_ptr, g.col, g.w, **okw)
        labels = r.labels.cpu().numpy() if device else r.labels
        assert np.array_equal(labels, ref.labels), f"labels differ: {tag} graph {k} (n={g.n})"
        assert r.q_int == ref.q_int, f"Q_int differs: {tag} graph {k}"
        assert abs(r.q - ref.q) <= 1e-12 * max(abs(ref.q), 1e-3)
        assert _levels(r.stats) == _ref_levels(ref), f"level records differ: {tag} graph {k}"
        assert (r.status == 0) == (ref.status == 0), f"status differs: {tag} graph {k}"
    for G in Gs:
        G.destroy()
    return res


def mixed_graphs(count=40, seed=0):
    gs = []
    for s in range(count):
        n = 2 + (s * 13) % 150
        p = [0.05, 0.2, 0.5][s % 3]
        gs.append(gg.random_small(n, p, 1 + s % 7, seed=5000 + seed * 1000 + s,
                                  loop_prob=0.3 if s % 4 == 0 else 0.0, isolated=s % 3))
    return gs


def test_batch_small_mixed(ctx):
    _say("batch of 40 small random graphs")
    check_batch(ctx, mixed_graphs(), tag="mixed")


def test_batch_sizes_and_buckets(ctx):
    """Graphs at different depths and with every degree bucket in one batch."""
    from test_gpu_parity import hub_graph
    graphs = [gg.config("sbm1k"), hub_graph(), gg.config("chunglu_n20000")] + mixed_graphs(10, 1) + \
        [gg.config("rmat_s12")]
    _say("batch of sbm1k, hub, chunglu_n20000, rmat_s12 and small graphs")
    check_batch(ctx, graphs, tag="sizes")


def test_batch_many_tiny(ctx):
    """Hundreds of tiny graphs: workgroups span more graphs than their LDS
    per-graph sums hold (global atomics fallback)."""
    graphs = [gg.random_small(3 + s % 9, 0.6, 1 + s % 5, seed=9000 + s) for s in range(600)]
    _say("batch of 600 tiny graphs")
    check_batch(ctx, graphs, tag="tiny")


def test_batch_sbm_sample(ctx):
    graphs = gg.batch_sbm(48, n_hi=20_000)
    _say(f"batch of 48 SBM graphs, {sum(g.nnz for g in graphs)} entries")
    check_batch(ctx, graphs, tag="batch_sbm", device=True)


def test_batch_sbm_full_size_range():
    """The batched workload's own graphs across its whole size range: its 8
    largest (n near 100,000) and 24 more spread over the sizes, in one batch,
    each against the oracle."""
    import os
    sizes = gg.batch_sbm_sizes()
    order = np.argsort(sizes, kind="stable")
    picks = list(order[-8:]) + list(order[np.linspace(0, len(order) - 9, 24).astype(int)])
    graphs = [gg.batch_sbm(1, first=int(i))[0] for i in picks]
    assert max(g.n for g in graphs) > 90_000
    oracle.set_threads(min(16, os.cpu_count() or 1))
    import paper_1805_10904_amd as L
    c = L.Context(0)
    try:
        _say(f"batch of {len(graphs)} workload graphs, n {min(g.n for g in graphs)}..{max(g.n for g in graphs)}, "
             f"{sum(g.nnz for g in graphs)} entries")
        check_batch(c, graphs, tag="batch_sbm full range", device=True)
    finally:
        c.close()


def test_batch_caps_and_params(ctx):
    graphs = [gg.config("sbm1k")] + mixed_graphs(12, 2)
    for kw in (dict(max_levels=1), dict(max_levels=2), dict(max_sweeps=1), dict(max_sweeps=0),
               dict(theta_num=1, theta_den=100), dict(singlet_rule=False), dict(pass_batch=3)):
        _say(f"batch with {kw}")
        check_batch(ctx, graphs, tag=str(kw), **kw)


def test_batch_degenerate_and_heavy(ctx):
    from test_gpu_parity import heavy_graph
    graphs = [
        gg.from_edge_list(1, []),
        gg.from_edge_list(3, []),
        gg.from_edge_list(1, [(0, 0)], [5]),
        gg.from_edge_list(2, [(0, 1)]),
        heavy_graph(),                          # 2W >= 2^31: runs through the plain path
        gg.from_edge_list(5, [(0, 1), (1, 2)]),
        gg.random_small(30, 0.2, 4, seed=77),
    ]
    check_batch(ctx, graphs, tag="degenerate")
    # a graph without vertices
    G = ctx.graph_create(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    g2 = gg.random_small(20, 0.3, 3, seed=78)
    H = ctx.graph_create(g2.row_ptr, g2.col, g2.w)
    r = ctx.run_batch([G, H])
    assert r[0].labels.shape == (0,) and r[0].q_int == 0
    ref = oracle.louvain(g2.row_ptr, g2.col, g2.w)
    assert np.array_equal(r[1].labels, ref.labels)
    G.destroy()
    H.destroy()


def test_batch_equals_alone(ctx):
    """Batched outputs equal the plain call's, graph by graph."""
    graphs = gg.batch_sbm(16, n_hi=5000, first=100)
    Gs = [ctx.graph_create(g.row_ptr, g.col, g.w) for g in graphs]
    res = ctx.run_batch(Gs)
    for G, r in zip(Gs, res):
        a = ctx.run(G)
        assert np.array_equal(a.labels, r.labels) and a.q_int == r.q_int
        assert _levels(a.stats) == _levels(r.stats)
        assert a.stats["total_edges_swept"] == r.stats["total_edges_swept"]
    for G in Gs:
        G.destroy()


def test_autotune_batch_keeps_results(L, tmp_path):
    """The batched workload's autotuner (coordinate descent over every launch
    shape, timed on the batch itself) picks a setting under which every
    graph's result is unchanged, writes it to the tuning file, and the
    results still equal the oracle's."""
    graphs = gg.batch_sbm(40, n_hi=20_000, first=1200)
    path = str(tmp_path / "tune.txt")
    c = L.Context(0, tuning_path=path)
    Gs = [c.graph_create(g.row_ptr, g.col, g.w) for g in graphs]
    before = c.run_batch(Gs)
    best = c.autotune_batch(Gs)
    _say(f"batched autotune: {best}")
    assert best["ms"] > 0
    got = c.get_tuning()
    assert all(got[k] == best[k] for k in got)
    assert f"group_slots {best['group_slots']}" in open(path).read()
    after = c.run_batch(Gs)
    for k, (g, a, b) in enumerate(zip(graphs, before, after)):
        assert np.array_equal(a.labels, b.labels) and a.q_int == b.q_int, f"graph {k}"
    for k in (0, 17, 39):
        ref = oracle.louvain(graphs[k].row_ptr, graphs[k].col, graphs[k].w)
        assert np.array_equal(after[k].labels, ref.labels) and after[k].q_int == ref.q_int
    for G in Gs:
        G.destroy()
    c.close()
