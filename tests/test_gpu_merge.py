"""GPU parity of the optional final merge of a phase (Section 5.1, end of
"Generating one level"): whole runs, dendrograms and resumed runs with
merge=True against the oracle, bit for bit (labels, Q_int, level records)."""
import sys

import numpy as np
import pytest

import graphgen as gg
import oracle
from test_gpu_parity import heavy_graph, hub_graph

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


def search_graphs():
    # random graphs on which the merge changes the run
    return [gg.random_small(4 + s % 6, 0.35, 1, seed=7000 + s) for s in (243, 467, 592, 717, 1444, 1665, 2200)]


def cases():
    out = search_graphs() + [gg.from_edge_list(4, [(0, 2), (0, 3), (1, 2), (1, 3)], name="c4")]
    out += [gg.config("sbm1k"), gg.config("chunglu_n65536"), gg.config("rmat_s14"), hub_graph(), heavy_graph()]
    for s in range(16):
        out.append(gg.random_small(3 + 9 * s, [0.08, 0.2, 0.5][s % 3], 1 + s % 7, seed=8800 + s,
                                   loop_prob=0.25 if s % 4 == 0 else 0.0, isolated=s % 3))
    return out


def _levels(recs):
    return [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], int(lv["q_int"])) for lv in recs]


def check_merge_run(ctx, g, singlet=True):
    ref = oracle.louvain(g.row_ptr, g.col, g.w, merge=True, singlet_rule=singlet)
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    r = ctx.run(G, merge=True, singlet_rule=singlet)
    assert np.array_equal(r.labels, ref.labels), f"labels differ on {g.name}"
    assert r.q_int == ref.q_int
    assert abs(r.q - ref.q) <= 1e-12 * max(abs(ref.q), 1e-3)
    assert _levels(r.stats["levels"]) == _levels(ref.levels), f"level records differ on {g.name}"
    assert (r.status == 0) == (ref.status == 0)
    G.destroy()


@pytest.mark.parametrize("g", cases(), ids=lambda g: f"{g.name}-n{g.n}")
def test_run_with_merge(ctx, g):
    _say(f"merge run on {g.name} n={g.n} nnz={g.nnz}")
    check_merge_run(ctx, g)


def test_merge_singlet_off_and_caps(ctx):
    for g in search_graphs() + [gg.config("sbm1k")]:
        check_merge_run(ctx, g, singlet=False)
    g = gg.config("chunglu_n65536")
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    for kw in (dict(max_levels=1), dict(max_levels=2), dict(max_sweeps=1), dict(theta_num=1, theta_den=100)):
        ref = oracle.louvain(g.row_ptr, g.col, g.w, merge=True, **kw)
        r = ctx.run(G, merge=True, **kw)
        assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int, f"differs under {kw}"
        assert _levels(r.stats["levels"]) == _levels(ref.levels)
    G.destroy()


def test_merge_full_chunglu1m(ctx):
    g = gg.config("chunglu1m")
    _say("merge run on chunglu1m")
    check_merge_run(ctx, g)


def test_merge_dendrogram_and_resume(ctx):
    for g in [gg.config("sbm1k"), gg.config("rmat_s14")] + search_graphs()[:3]:
        ref = oracle.dendrogram(g.row_ptr, g.col, g.w, merge=True)
        G = ctx.graph_create(g.row_ptr, g.col, g.w)
        res, D = ctx.run(G, dendrogram=True, merge=True)
        assert np.array_equal(res.labels, ref.labels) and res.q_int == ref.q_int
        assert D.levels == len(ref.maps)
        for lvl, m in enumerate(ref.maps):
            assert np.array_equal(D.map(lvl), m), f"map {lvl} differs on {g.name}"
        last = D.graph()
        rp, col, w = last.export()
        assert np.array_equal(rp, ref.graphs[-1][0]) and np.array_equal(col, ref.graphs[-1][1])
        assert np.array_equal(w, ref.graphs[-1][2])
        last.destroy()
        D.destroy()
        if len(ref.maps) >= 1:
            part, D1 = ctx.run(G, dendrogram=True, merge=True, max_levels=1)
            G1 = D1.graph()
            rest = ctx.resume(G1, 1, part.labels, merge=True)
            assert np.array_equal(rest.labels, ref.labels) and rest.q_int == ref.q_int
            G1.destroy()
            D1.destroy()
        G.destroy()


def test_merge_batched(ctx):
    """Batched calls with the merge: every graph's result equals the oracle's
    (graphs end their phases at different passes; a heavy graph runs alone)."""
    graphs = search_graphs() + [gg.from_edge_list(4, [(0, 2), (0, 3), (1, 2), (1, 3)], name="c4"),
                                gg.config("sbm1k"), gg.config("chunglu_n65536"), gg.config("rmat_s14"), hub_graph(),
                                heavy_graph()]
    graphs += [gg.random_small(3 + 7 * s, 0.3, 1 + s % 5, seed=9100 + s, isolated=s % 2) for s in range(12)]
    Gs = [ctx.graph_create(g.row_ptr, g.col, g.w) for g in graphs]
    for kw in (dict(), dict(singlet_rule=False), dict(max_levels=2)):
        res = ctx.run_batch(Gs, merge=True, **kw)
        for g, r in zip(graphs, res):
            ref = oracle.louvain(g.row_ptr, g.col, g.w, merge=True, **kw)
            assert np.array_equal(r.labels, ref.labels), f"batched labels differ on {g.name} {kw}"
            assert r.q_int == ref.q_int, f"batched Q differs on {g.name} {kw}"
            assert _levels(r.stats["levels"]) == _levels(ref.levels), f"batched records differ on {g.name} {kw}"
    for G in Gs:
        G.destroy()


def test_merge_served(ctx):
    import time
    graphs = search_graphs() + [gg.config("sbm1k"), gg.config("rmat_s14"), heavy_graph()]
    tickets = []
    for k, g in enumerate(graphs):
        tickets.append((g, ctx.submit(g.row_ptr, g.col, g.w, merge=(k % 2 == 0))))
    t_end = time.time() + 120
    for g, t in tickets:
        r = None
        while r is None:
            assert time.time() < t_end, "served requests did not finish in time"
            r = ctx.poll(t, wait_us=2000)
        k = [x[1] for x in tickets].index(t)
        ref = oracle.louvain(g.row_ptr, g.col, g.w, merge=(k % 2 == 0))
        assert np.array_equal(r.labels, ref.labels), f"served labels differ on {g.name}"
        assert r.q_int == ref.q_int
        assert _levels(r.levels) == _levels(ref.levels)


def test_merge_off_is_the_default(ctx):
    g = gg.config("rmat_s14")
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    ref = oracle.louvain(g.row_ptr, g.col, g.w)
    assert np.array_equal(ctx.run(G).labels, ref.labels)
    assert np.array_equal(ctx.run_batch([G])[0].labels, ref.labels)
    G.destroy()
