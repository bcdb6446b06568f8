"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Integer results (labels, e_{i->C}, deg_C, renumber maps, contracted graphs,
Q_int, per-level sweep counts) must match bit for bit; the reported double Q
is checked to 1e-12 relative (both sides form it from the same integer).
Inputs are the seeded graphs of ``graphgen``; expected values come only from
``oracle``.
"""
import os
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


def small_graphs():
    gs = []
    for s in range(60):
        n = 2 + (s * 7) % 90
        p = [0.05, 0.15, 0.4, 0.9][s % 4]
        gs.append(gg.random_small(n, p, 1 + s % 9, seed=1000 + s, loop_prob=0.25 if s % 3 == 0 else 0.0,
                                  isolated=s % 4))
    return gs


def hub_graph(seed=7, leaves=15000, mid=5000, extra=20000, n=20000):
    """Two stars plus random edges: vertex 0 with 15,000 leaves (a row past
    every LDS kernel: the HBM hub path) and vertex 1 with 5,000 (the
    1,024-thread LDS kernel), so that every row kernel is used."""
    rng = np.random.default_rng(seed)
    u = np.concatenate([np.zeros(leaves, np.int64), np.ones(mid, np.int64), rng.integers(0, n, extra)])
    v = np.concatenate([np.arange(2, leaves + 2), rng.choice(np.arange(2, n), mid, replace=False),
                        rng.integers(0, n, extra)])
    keys = gg.canonical_keys(u, v)
    rp, col, w = gg.csr_from_canonical_keys(n, keys, seed, lambda h: gg.weights_uniform(h, 20))
    return gg.Graph(n, rp, col, w, None, "hub")


def heavy_graph(seed=3, n=300, p=0.05, scale=10**9):
    """Weights near 2^31 so TW exceeds the int64 score range (128-bit scores)."""
    g = gg.random_small(n, p, 2, seed=seed, loop_prob=0.1)
    w = (g.w.astype(np.int64) * scale).clip(1, 2**31 - 1).astype(np.int32)
    return gg.Graph(g.n, g.row_ptr, g.col, w, None, "heavy")


def check_local_move(ctx, g, labels, singlet=True, tag=""):
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    got_l, got_d, got_e = ctx.local_move(G, labels, singlet_rule=singlet)
    ref = oracle.local_move(g.row_ptr, g.col, g.w, labels, singlet_rule=singlet)
    assert np.array_equal(got_l, ref.labels), f"labels differ {tag}"
    assert np.array_equal(got_d, ref.deg), f"deg_C differ {tag}"
    assert np.array_equal(got_e, ref.e_own), f"e_own differ {tag}"
    G.destroy()


def check_run(ctx, g, tag="", **kw):
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    r = ctx.run(G, **kw)
    ref = oracle.louvain(g.row_ptr, g.col, g.w, **kw)
    assert np.array_equal(r.labels, ref.labels), f"final labels differ {tag}"
    assert r.q_int == ref.q_int, f"Q_int differs {tag}"
    assert abs(r.q - ref.q) <= 1e-12 * max(abs(ref.q), 1e-3)
    got = [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"])
           for lv in r.stats["levels"]]
    want = [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"])
            for lv in ref.levels]
    assert got == want, f"level records differ {tag}"
    assert (r.status == 0) == (ref.status == 0)
    G.destroy()
    return r


# --------------------------------------------------------------- one sweep --

def test_local_move_small_graphs(ctx):
    for k, g in enumerate(small_graphs()):
        for t, lab in enumerate([None, gg.random_labels(g.n, 2, k), gg.random_labels(g.n, max(1, g.n // 3), k + 1),
                                 np.zeros(g.n, np.int32)]):
            for singlet in (True, False):
                check_local_move(ctx, g, lab, singlet, tag=f"graph {k} labels {t} singlet {singlet}")


@pytest.mark.parametrize("name", ["sbm1k", "hub", "heavy", "chunglu_n20000"])
def test_local_move_buckets(ctx, name):
    _say(f"local_move parity on {name}")
    g = hub_graph() if name == "hub" else heavy_graph() if name == "heavy" else gg.config(name)
    check_local_move(ctx, g, None, tag=name)
    check_local_move(ctx, g, gg.random_labels(g.n, 5, 11), tag=name + " 5 communities")
    check_local_move(ctx, g, gg.random_labels(g.n, max(1, g.n // 20), 12), tag=name + " many communities")


def test_local_move_full_chunglu1m(ctx):
    """The benchmark workload at full size, one sweep from singletons and one
    from a seeded labelling with few large communities."""
    _say("local_move parity on chunglu1m")
    g = gg.config("chunglu1m")
    check_local_move(ctx, g, None, tag="chunglu1m singletons")
    check_local_move(ctx, g, gg.random_labels(g.n, 64, 5), tag="chunglu1m 64 communities")


# -------------------------------------------------------------- modularity --

def test_modularity(ctx):
    for k, g in enumerate(small_graphs()[::3] + [gg.config("sbm1k"), heavy_graph()]):
        G = ctx.graph_create(g.row_ptr, g.col, g.w)
        for lab in [np.arange(g.n, dtype=np.int32), gg.random_labels(g.n, 3, k), np.zeros(g.n, np.int32)]:
            qi, q = ctx.modularity(G, lab)
            ref_qi, ref_q = oracle.modularity(g.row_ptr, g.col, g.w, lab)
            assert qi == ref_qi
            assert abs(q - ref_q) <= 1e-12 * max(abs(ref_q), 1e-3)
        n, nnz, tw = G.info()
        assert (n, nnz) == (g.n, g.nnz) and tw == oracle.degrees(g.row_ptr, g.col, g.w)[1]
        G.destroy()


# ------------------------------------------------------------- aggregation --

@pytest.mark.parametrize("name", ["small", "sbm1k", "hub"])
def test_aggregate(ctx, name):
    graphs = small_graphs()[::5] if name == "small" else [gg.config("sbm1k") if name == "sbm1k" else hub_graph()]
    for k, g in enumerate(graphs):
        G = ctx.graph_create(g.row_ptr, g.col, g.w)
        for lab in [gg.random_labels(g.n, 3, k), gg.random_labels(g.n, max(1, g.n // 4), k + 7),
                    np.arange(g.n, dtype=np.int32)]:
            G2, ren = ctx.aggregate(G, lab)
            m, kk = oracle.renumber(lab)
            assert np.array_equal(ren, m[lab])
            rp, cl, w = oracle.contract(g.row_ptr, g.col, g.w, m[lab], kk)
            grp, gcl, gw = G2.export()
            assert np.array_equal(grp, rp) and np.array_equal(gcl, cl) and np.array_equal(gw, w)
            assert G2.info()[2] == G.info()[2]
            G2.destroy()
        G.destroy()


# ---------------------------------------------------------- the whole method --

def test_run_small_graphs(ctx):
    for k, g in enumerate(small_graphs()):
        check_run(ctx, g, tag=f"graph {k}")
        if k % 4 == 0:
            check_run(ctx, g, tag=f"graph {k} singlet off", singlet_rule=False)


@pytest.mark.parametrize("name", ["sbm1k", "hub", "heavy", "chunglu_n20000", "rmat_s14"])
def test_run(ctx, name):
    _say(f"run parity on {name}")
    g = hub_graph() if name == "hub" else heavy_graph() if name == "heavy" else gg.config(name)
    check_run(ctx, g, tag=name)


def test_run_caps(ctx):
    g = gg.config("sbm1k")
    for kw in (dict(max_levels=1), dict(max_sweeps=1), dict(max_sweeps=0), dict(theta_num=1, theta_den=100)):
        check_run(ctx, g, tag=str(kw), **kw)


def test_run_full_chunglu1m(ctx):
    """The benchmark workload, end to end at full size."""
    _say("run parity on chunglu1m")
    g = gg.config("chunglu1m")
    r = check_run(ctx, g, tag="chunglu1m")
    _say(f"chunglu1m: levels {len(r.stats['levels'])}, Q = {r.q:.6f}")
    # the packed classes software-pipelined over four tiles per workgroup
    ctx.set_tuning(group_tiles=4)
    try:
        check_run(ctx, g, tag="chunglu1m, group_tiles 4")
    finally:
        ctx.set_tuning()


def test_determinism_and_batching(ctx):
    g = gg.config("chunglu_n20000")
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    base = ctx.run(G)
    for batch in (1, 2, 3, 8):
        r = ctx.run(G, pass_batch=batch)
        assert np.array_equal(r.labels, base.labels) and r.q_int == base.q_int
    G.destroy()


def test_device_pointers(ctx):
    import torch
    g = gg.config("sbm1k")
    dev = torch.device("cuda", 0)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    G = ctx.graph_create(rp, cl, w)
    r = ctx.run(G)
    ref = oracle.louvain(g.row_ptr, g.col, g.w)
    assert r.labels.is_cuda and np.array_equal(r.labels.cpu().numpy(), ref.labels)
    lab = torch.from_numpy(gg.random_labels(g.n, 4, 2)).to(dev)
    out, deg, eown = ctx.local_move(G, lab)
    lm = oracle.local_move(g.row_ptr, g.col, g.w, lab.cpu().numpy())
    assert np.array_equal(out.cpu().numpy(), lm.labels) and np.array_equal(deg.cpu().numpy(), lm.deg)
    G.destroy()


def test_binding_checks_device_tensors(ctx, L):
    """Device arrays of the wrong dtype, length, layout or kind are refused
    by the binding (EINVAL) before the library reads them."""
    import torch
    g = gg.config("sbm1k")
    dev = torch.device("cuda", 0)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    cl = torch.from_numpy(g.col).to(dev)
    w = torch.from_numpy(g.w).to(dev)
    bad = [
        lambda: ctx.graph_create(rp.to(torch.int32), cl, w),                      # int32 row_ptr
        lambda: ctx.graph_create(rp, cl.cpu(), w),                                # mixed kinds
        lambda: ctx.graph_create(rp, torch.stack([cl, cl], 1)[:, 0], w),          # strided col
        lambda: ctx.graph_create(rp, cl, w[:-1]),                                 # short weights
    ]
    for k, f in enumerate(bad):
        with pytest.raises(L.LouvainError) as e:
            f()
        assert e.value.code == L.LOUVAIN_EINVAL, k
    G = ctx.graph_create(rp, cl, w)
    for labels in (torch.zeros(g.n - 1, dtype=torch.int32, device=dev),           # short
                   torch.zeros(g.n, dtype=torch.int64, device=dev),               # int64
                   np.zeros(g.n, np.int32)):                                      # host memory
        with pytest.raises(L.LouvainError) as e:
            ctx.modularity(G, labels)
        assert e.value.code == L.LOUVAIN_EINVAL
    with pytest.raises(L.LouvainError):
        ctx.run(G, labels_out=torch.empty(g.n, dtype=torch.int32))                # CPU tensor as device output
    r = ctx.run(G)   # the graph is unharmed
    assert np.array_equal(r.labels.cpu().numpy(), oracle.louvain(g.row_ptr, g.col, g.w).labels)
    G.destroy()


def test_int64_weights(ctx):
    g = heavy_graph(seed=9)
    w64 = g.w.astype(np.int64) * 4096      # beyond int32
    G = ctx.graph_create(g.row_ptr, g.col, w64)
    r = ctx.run(G)
    ref = oracle.louvain(g.row_ptr, g.col, w64)
    assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int
    G.destroy()


@pytest.mark.parametrize("scale", [1 << 26, 1 << 36])
def test_heavy_hubs(ctx, scale):
    """Hubs on the kernels for 2W >= 2^31: with weights near 2^30 the hub
    tables hold one word per slot (label and e fit 64 bits together); with
    weights near 2^40 (int64) they fall back to separate key and value
    arrays."""
    g = hub_graph(seed=11)
    w = g.w.astype(np.int64) * scale
    _say(f"hub graph with weights x {scale}")
    G = ctx.graph_create(g.row_ptr, g.col, w)
    r = ctx.run(G)
    ref = oracle.louvain(g.row_ptr, g.col, w)
    assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int
    lm = ctx.local_move(G, None)
    ref_lm = oracle.local_move(g.row_ptr, g.col, w, None)
    assert np.array_equal(lm[0], ref_lm.labels) and np.array_equal(lm[2], ref_lm.e_own)
    G.destroy()


@pytest.mark.parametrize("scale,kind", [(3676, "64-bit scores"), (8000, "128-bit scores")])
def test_general_score_width(scale, kind):
    """Levels with 2W above the 64-bit range of TW^2 score in 64 bits while
    TW times the level's largest delta stays below 2^62 (every product of a
    score is at most that), else in 128 bits.  The hub graph with weights x
    3676 has TW = 3.10e9 and TW max delta = 0.39 * 2^62; x 8000 puts it past
    2^62.  The level log (LOUVAIN_LOG, read once per process, so in a child
    process) names the width, and the results equal the oracle's."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
            "import numpy as np, oracle, paper_1805_10904_amd as L\n"
            "from test_gpu_parity import hub_graph\n"
            "g = hub_graph(seed=11); ctx = L.Context(0)\n"
            "w = g.w.astype(np.int64) * %d\n"
            "G = ctx.graph_create(g.row_ptr, g.col, w)\n"
            "r = ctx.run(G)\n"
            "ref = oracle.louvain(g.row_ptr, g.col, w)\n"
            "assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int\n"
            "lm = ctx.local_move(G, None)\n"
            "ref_lm = oracle.local_move(g.row_ptr, g.col, w, None)\n"
            "assert np.array_equal(lm[0], ref_lm.labels) and np.array_equal(lm[1], ref_lm.deg)\n"
            "assert np.array_equal(lm[2], ref_lm.e_own)\n"
            "print('OK', flush=True)\n") % (os.path.dirname(here), here, scale)
    _say(f"hub graph with weights x {scale} in a child process")
    env = dict(os.environ, LOUVAIN_LOG="1")
    p = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=240)
    assert p.returncode == 0 and "OK" in p.stdout, p.stderr[-2000:]
    lines = [ln for ln in p.stderr.splitlines() if ln.startswith("[louvain] level 0: ")]
    assert lines and all(kind in ln for ln in lines), lines


@pytest.mark.parametrize("shrink", [8, 64])
def test_hub_bucket_spills(shrink):
    """Hubs are summed in buckets (compact levels, and levels with 2W >=
    2^31 and published words); LOUVAIN_HUB_BUCKET_SHRINK (read once per
    process, so in a child process) makes the bucket regions and tables that
    many times smaller, so buckets overflow their region (pairs appended past
    it) and their table (more distinct labels than it may claim) and spill to
    the hub table.  The results equal the oracle's, with the hub graph's own
    weights (compact levels) and with weights x 2^26."""
    import os
    import subprocess
    here = os.path.dirname(os.path.abspath(__file__))
    code = ("import sys; sys.path.insert(0, %r); sys.path.insert(0, %r)\n"
            "import numpy as np, oracle, paper_1805_10904_amd as L\n"
            "from test_gpu_parity import hub_graph\n"
            "g = hub_graph(seed=11); ctx = L.Context(0)\n"
            "for w in (g.w, g.w.astype(np.int64) << 26):\n"
            "  G = ctx.graph_create(g.row_ptr, g.col, w)\n"
            "  r = ctx.run(G); ref = oracle.louvain(g.row_ptr, g.col, w)\n"
            "  assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int, 'run'\n"
            "  assert [lv['q_int'] for lv in r.stats['levels']] == [lv['q_int'] for lv in ref.levels], 'levels'\n"
            "  lm = ctx.local_move(G, None); rl = oracle.local_move(g.row_ptr, g.col, w, None)\n"
            "  assert np.array_equal(lm[0], rl.labels) and np.array_equal(lm[2], rl.e_own), 'local move'\n"
            "  lab = r.labels.astype(np.int32)\n"
            "  lm = ctx.local_move(G, lab); rl = oracle.local_move(g.row_ptr, g.col, w, lab)\n"
            "  assert np.array_equal(lm[0], rl.labels) and np.array_equal(lm[2], rl.e_own), 'from labels'\n"
            "  G.destroy()\n"
            "print('ok')\n") % (os.path.dirname(here), here)
    env = dict(os.environ, LOUVAIN_HUB_BUCKET_SHRINK=str(shrink))
    _say(f"hub graph, own weights and x 2^26, bucket shrink {shrink} (child process)")
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-3000:]
    assert p.stdout.strip().endswith("ok")


# -------------------------------------------------------------- edge cases --

def test_degenerate_graphs(ctx, L):
    cases = [
        gg.from_edge_list(1, []),
        gg.from_edge_list(3, []),
        gg.from_edge_list(1, [(0, 0)], [5]),
        gg.from_edge_list(2, [(0, 0), (1, 1)], [3, 4]),
        gg.from_edge_list(2, [(0, 1)]),
        gg.from_edge_list(5, [(0, 1), (1, 2)]),
    ]
    for k, g in enumerate(cases):
        check_run(ctx, g, tag=f"degenerate {k}")
        check_local_move(ctx, g, None, tag=f"degenerate {k}")
    # no vertices at all
    G = ctx.graph_create(np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
    r = ctx.run(G)
    assert r.labels.shape == (0,) and r.q_int == 0
    G.destroy()


def test_errors_leave_outputs_untouched(ctx, L):
    g = gg.from_edge_list(4, [(0, 1), (1, 2), (2, 3)])
    bad = [
        (g.row_ptr, np.array([1, 2, 0, 1, 3, 2], np.int32), g.w),             # unsorted row
        (g.row_ptr, np.array([1, 0, 2, 1, 9, 2], np.int32), g.w),             # column out of range
        (g.row_ptr, g.col, np.array([1, 1, 0, 1, 1, 1], np.int32)),           # weight 0
        (np.array([0, 1, 3, 2, 6], np.int64), g.col, g.w),                     # row_ptr not monotone
        (np.array([0, 1, 3, 5, 7], np.int64), g.col, g.w),                     # row_ptr[n] != nnz
    ]
    for rp, cl, w in bad:
        with pytest.raises(L.LouvainError) as ei:
            ctx.graph_create(rp, cl, w)
        assert ei.value.code == L.LOUVAIN_EINVAL
    asym = gg.from_edge_list(3, [(0, 1), (1, 2)])
    w = asym.w.copy()
    w[0] = 7
    ctx.graph_create(asym.row_ptr, asym.col, w).destroy()     # not checked by default
    with pytest.raises(L.LouvainError) as ei:
        ctx.graph_create(asym.row_ptr, asym.col, w, check_symmetry=True)
    assert ei.value.code == L.LOUVAIN_EINVAL
    import ctypes
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    out = np.full(4, -5, np.int32)
    bad_labels = np.array([0, 1, 2, 7], np.int32)
    rc = ctx.lib.louvain_local_move(ctx.h, G.h, bad_labels.ctypes.data_as(ctypes.c_void_p),
                                    out.ctypes.data_as(ctypes.c_void_p), None, None, 0)
    assert rc == L.LOUVAIN_EINVAL and np.all(out == -5)
    assert b"out of range" in ctx.lib.louvain_last_error(ctx.h)
    with pytest.raises(L.LouvainError):
        ctx.modularity(G, np.array([0, -1, 2, 3], np.int32))
    G.destroy()


# --------------------------------------------------------- launch shapes --

def test_launch_shapes_do_not_change_results(ctx):
    """Every row-length threshold and pass batching gives the oracle's result
    (rows move between the thread, LDS and HBM hub kernels)."""
    graphs = [gg.config("chunglu_n20000"), hub_graph(), gg.config("rmat_s14")]
    refs = [oracle.louvain(g.row_ptr, g.col, g.w) for g in graphs]
    Gs = [ctx.graph_create(g.row_ptr, g.col, g.w) for g in graphs]
    try:
        for shp in [(1, 341, 1, 4, 1, 0, 1, 1), (4, 1024, 2, 8, 2, 1, 2, 1), (8, 1365, 1, 2, 2, 0, 0, 1),
                    (2, 2730, 3, 4, 1, 1, 1, 4), (4, 10922, 2, 8, 1, 0, 2, 3), (3, 700, 1, 2, 1, 1, 1, 2),
                    (4, 5000, 2, 4, 2, 1, 0, 1), (4, 10922, 2, 4, 1, 1, 1, 8), (4, 2730, 2, 4, 1, 0, 2, 4)]:
            ctx.set_tuning(*shp)
            keys = ("small_max", "block_max", "pass_batch", "group_slots", "group_vertices", "overlap", "reorder",
                    "group_tiles")
            assert ctx.get_tuning() == dict(zip(keys, shp))
            for k, (G, ref) in enumerate(zip(Gs, refs)):
                r = ctx.run(G)
                assert np.array_equal(r.labels, ref.labels), f"labels differ, graph {k}, shapes {shp}"
                assert r.q_int == ref.q_int
            res = ctx.run_batch(Gs)
            for k, (r, ref) in enumerate(zip(res, refs)):
                assert np.array_equal(r.labels, ref.labels), f"batched labels differ, graph {k}, {shp}"
    finally:
        ctx.set_tuning()
        for G in Gs:
            G.destroy()


def test_autotune(ctx, L):
    g = gg.config("chunglu_n20000")
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    try:
        best = ctx.autotune(G)
        assert best["small_max"] in (4, 8) and best["block_max"] in (1365, 2730, 10922)
        assert best["pass_batch"] in (1, 2) and best["group_slots"] == 4 and best["ms"] > 0
        assert best["group_vertices"] in (1, 2) and best["overlap"] == 0 and best["reorder"] == 0
        assert best["group_tiles"] in (1, 4)
        assert ctx.get_tuning() == {k: best[k] for k in ("small_max", "block_max", "pass_batch", "group_slots",
                                                         "group_vertices", "overlap", "reorder", "group_tiles")}
        r = ctx.run(G)
        ref = oracle.louvain(g.row_ptr, g.col, g.w)
        assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int
        with pytest.raises(L.LouvainError):
            ctx.set_tuning(small_max=9)
        with pytest.raises(L.LouvainError):
            ctx.set_tuning(block_max=100)
        with pytest.raises(L.LouvainError):
            ctx.set_tuning(group_slots=6)
        with pytest.raises(L.LouvainError):
            ctx.set_tuning(group_vertices=3)
        with pytest.raises(L.LouvainError):
            ctx.set_tuning(overlap=2)
        with pytest.raises(L.LouvainError):
            ctx.set_tuning(reorder=3)
        with pytest.raises(L.LouvainError):
            ctx.set_tuning(group_tiles=9)
    finally:
        ctx.set_tuning()
        G.destroy()
