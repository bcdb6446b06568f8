"""GPU parity of the dendrogram export and of resuming a run from a level
state (louvain_run_dendro, louvain_dendro_*, louvain_resume) against the
oracle's level-by-level run: every map, the last level's graph, the labels
and Q_int bit for bit, and a resumed run equal to one whole run."""
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


def cases():
    out = [gg.config("sbm1k"), gg.config("chunglu_n65536"), gg.config("rmat_s14")]
    for s in range(8):
        out.append(gg.random_small(5 + 11 * s, [0.1, 0.3][s % 2], 1 + s, seed=4000 + s,
                                   loop_prob=0.2 if s % 3 == 0 else 0.0, isolated=s % 3))
    out.append(heavy_graph())
    out.append(gg.from_edge_list(6, []))   # TW = 0
    return out


def _export(G):
    rp, col, w = G.export()
    return rp, col, w


def check_dendro(ctx, g, **kw):
    _say(f"dendrogram of {g.name} n={g.n} nnz={g.nnz} {kw}")
    ref = oracle.dendrogram(g.row_ptr, g.col, g.w, **kw)
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    res, D = ctx.run(G, dendrogram=True, **kw)
    plain = ctx.run(G, **kw)
    assert np.array_equal(res.labels, ref.labels), "labels differ"
    assert np.array_equal(plain.labels, res.labels), "a dendrogram run changed the labels"
    assert res.q_int == ref.q_int == plain.q_int
    assert res.status == plain.status and (res.status == 0) == (ref.status == 0)
    got_lv = [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"])
              for lv in res.stats["levels"]]
    ref_lv = [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"]) for lv in ref.levels]
    assert got_lv == ref_lv, "level records differ"
    assert D.levels == len(ref.maps)
    assert D.n == [gr[0].shape[0] - 1 for gr in ref.graphs]
    for lvl, m in enumerate(ref.maps):
        assert np.array_equal(D.map(lvl), m), f"map {lvl} differs"
    last = D.graph()
    rp, col, w = _export(last)
    assert np.array_equal(rp, ref.graphs[-1][0]) and np.array_equal(col, ref.graphs[-1][1]) \
        and np.array_equal(w, ref.graphs[-1][2]), "last level's graph differs"
    assert last.info()[2] == G.info()[2]
    D.destroy()
    last.destroy()
    G.destroy()
    return ref


@pytest.mark.parametrize("g", cases(), ids=lambda g: f"{g.name}-n{g.n}")
def test_dendrogram(ctx, g):
    check_dendro(ctx, g)


@pytest.mark.parametrize("g", cases()[:4] + [hub_graph()], ids=lambda g: f"{g.name}-n{g.n}")
def test_resume_from_every_level(ctx, g):
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    full = ctx.run(G)
    nmaps = len([lv for lv in full.stats["levels"] if lv["sweeps_accepted"] > 0])
    for cap in sorted({64, max(1, nmaps)}):
        want = ctx.run(G, max_levels=cap)
        ref = oracle.louvain(g.row_ptr, g.col, g.w, max_levels=cap)
        assert np.array_equal(want.labels, ref.labels)
        for lvl in range(1, min(nmaps, cap) + 1):
            _say(f"{g.name}: resume after {lvl} levels, cap {cap}")
            part, D = ctx.run(G, max_levels=lvl, dendrogram=True)
            Gl = D.graph()
            rest = ctx.resume(Gl, lvl, part.labels, max_levels=cap)
            assert np.array_equal(rest.labels, want.labels), f"resume after {lvl} levels differs"
            assert rest.q_int == want.q_int
            assert (rest.status == 0) == (want.status == 0)
            Gl.destroy()
            D.destroy()
    G.destroy()


def test_dendrogram_cut_and_device_pointers(ctx, L):
    import torch
    g = gg.config("chunglu_n65536")
    ref = oracle.dendrogram(g.row_ptr, g.col, g.w, max_levels=2)
    dev = torch.device("cuda", 0)
    G = ctx.graph_create(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev),
                         torch.from_numpy(g.w).to(dev))
    res, D = ctx.run(G, max_levels=2, dendrogram=True)
    assert res.status == L.LOUVAIN_ELIMIT and ref.status == oracle.ORC_ELIMIT
    assert np.array_equal(res.labels.cpu().numpy(), ref.labels)
    assert D.levels == 2
    for lvl in range(2):
        m = D.map(lvl)
        assert m.is_cuda and np.array_equal(m.cpu().numpy(), ref.maps[lvl])
    last = D.graph()
    rp, col, w = last.export()
    assert np.array_equal(rp, ref.graphs[-1][0]) and np.array_equal(col, ref.graphs[-1][1])
    assert np.array_equal(w, ref.graphs[-1][2])
    # resume on the device: the rest of the run equals one whole run
    rest = ctx.resume(last, 2, res.labels)
    full = oracle.louvain(g.row_ptr, g.col, g.w)
    assert np.array_equal(rest.labels.cpu().numpy(), full.labels) and rest.q_int == full.q_int
    # nothing left to run: the labels so far, ELIMIT
    again = ctx.resume(last, 64, res.labels)
    assert again.status == L.LOUVAIN_ELIMIT and torch.equal(again.labels, res.labels)
    assert again.q_int == oracle.modularity(g.row_ptr, g.col, g.w, ref.labels)[0]
    last.destroy()
    D.destroy()
    G.destroy()


def test_dendrogram_errors(ctx, L):
    g = gg.config("sbm1k")
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    _, D = ctx.run(G, dendrogram=True)
    with pytest.raises(L.LouvainError):
        D.map(D.levels)
    with pytest.raises(L.LouvainError):
        D.map(-1)
    last = D.graph()
    with pytest.raises(L.LouvainError):
        D.graph()
    bad = np.full(g.n, last.info()[0], np.int32)   # one past the level graph's vertices
    with pytest.raises(L.LouvainError):
        ctx.resume(last, 1, bad)
    with pytest.raises(L.LouvainError):
        ctx.resume(last, -1, np.zeros(g.n, np.int32))
    last.destroy()
    D.destroy()
    G.destroy()
