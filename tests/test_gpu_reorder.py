"""GPU parity with the level-0 vertex order by row length (tuning reorder):
with the order forced on, whole runs, merged runs, dendrograms and resumed
runs equal the oracle's bit for bit on graphs of every kind (loops,
isolated vertices, hubs, 128-bit scores, compact and general levels); the
default (auto) order is covered at full size by the R-MAT scale-24 test."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from test_gpu_parity import heavy_graph, hub_graph, small_graphs

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
    c.set_tuning(reorder=1)
    yield c
    c.close()


def _levels(recs):
    return [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], int(lv["q_int"])) for lv in recs]


def check(ctx, g, **kw):
    ref = oracle.louvain(g.row_ptr, g.col, g.w, **kw)
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    r = ctx.run(G, **kw)
    assert np.array_equal(r.labels, ref.labels), f"labels differ on {g.name} {kw}"
    assert r.q_int == ref.q_int
    assert _levels(r.stats["levels"]) == _levels(ref.levels), f"level records differ on {g.name} {kw}"
    G.destroy()


def test_reorder_small_graphs(ctx):
    assert ctx.get_tuning()["reorder"] == 1
    for k, g in enumerate(small_graphs()):
        check(ctx, g)
        if k % 5 == 0:
            check(ctx, g, singlet_rule=False)
            check(ctx, g, merge=True)


@pytest.mark.parametrize("name", ["sbm1k", "chunglu_n65536", "rmat_s14", "rmat_s16", "hub", "heavy"])
def test_reorder_workloads(ctx, name):
    g = hub_graph() if name == "hub" else heavy_graph() if name == "heavy" else gg.config(name)
    _say(f"reordered run on {name} n={g.n} nnz={g.nnz}")
    check(ctx, g)
    check(ctx, g, merge=True)
    check(ctx, g, max_levels=1)


def test_reorder_dendrogram_and_resume(ctx):
    for g in (gg.config("sbm1k"), gg.config("rmat_s14"), gg.from_edge_list(5, [(0, 1)]),
              gg.random_small(40, 0.02, 3, seed=77, isolated=5)):
        ref = oracle.dendrogram(g.row_ptr, g.col, g.w)
        G = ctx.graph_create(g.row_ptr, g.col, g.w)
        res, D = ctx.run(G, dendrogram=True)
        assert np.array_equal(res.labels, ref.labels) and res.q_int == ref.q_int
        assert D.levels == len(ref.maps)
        for lvl, m in enumerate(ref.maps):
            assert np.array_equal(D.map(lvl), m), f"map {lvl} differs on {g.name}"
        last = D.graph()
        rp, col, w = last.export()
        assert np.array_equal(rp, ref.graphs[-1][0]) and np.array_equal(col, ref.graphs[-1][1])
        assert np.array_equal(w, ref.graphs[-1][2])
        if ref.maps:
            part, D1 = ctx.run(G, dendrogram=True, max_levels=1)
            G1 = D1.graph()
            rest = ctx.resume(G1, 1, part.labels)
            assert np.array_equal(rest.labels, ref.labels) and rest.q_int == ref.q_int
            G1.destroy()
            D1.destroy()
        last.destroy()
        D.destroy()
        G.destroy()


def test_reorder_level0_keeps_nothing(ctx):
    """A first phase that keeps no sweep (K2 without the singlet rule swaps
    and is rejected): the labels are the identity, and the dendrogram's
    graph is the given one, not the rebuilt one."""
    g = gg.from_edge_list(6, [(0, 1), (4, 5)], name="two_k2")
    ref = oracle.dendrogram(g.row_ptr, g.col, g.w, singlet_rule=False)
    assert ref.maps == [] and ref.levels[0]["sweeps_accepted"] == 0
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    res, D = ctx.run(G, dendrogram=True, singlet_rule=False)
    assert res.labels.tolist() == list(range(6)) and res.q_int == ref.q_int
    assert D.levels == 0
    last = D.graph()
    rp, col, w = last.export()
    assert np.array_equal(rp, g.row_ptr) and np.array_equal(col, g.col) and np.array_equal(w, g.w)
    last.destroy()
    D.destroy()
    G.destroy()


def test_reorder_on_off_auto_agree_full_chunglu1m(ctx):
    g = gg.config("chunglu1m")
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    try:
        got = {}
        for mode in (1, 2, 0):
            ctx.set_tuning(reorder=mode)
            got[mode] = ctx.run(G)
        for mode in (1, 0):
            assert np.array_equal(got[mode].labels, got[2].labels), f"reorder={mode} changed the labels"
            assert got[mode].q_int == got[2].q_int
            assert _levels(got[mode].stats["levels"]) == _levels(got[2].stats["levels"])
    finally:
        ctx.set_tuning(reorder=1)
        G.destroy()
