"""Full-size parity on the R-MAT scale-24 workload (n = 2^24, about 5.2e8
entries, hubs of about 4e5 entries, five levels of contraction).

The oracle needs about ten minutes on this graph, so its results are kept
as SHA-256 digests of whole output arrays plus the scalar results in
``golden/rmat24_expected.json``, written by ``golden/make_rmat24_expected.py``
from ``graphgen`` and ``oracle`` alone.  The GPU outputs are digested the
same way: equal digests mean bit-identical arrays.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _say(msg):
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()


def digest(a, dtype):
    if hasattr(a, "cpu"):
        a = a.cpu().numpy()
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a, dtype=dtype)).tobytes()).hexdigest()


@pytest.fixture(scope="module")
def exp():
    with open(os.path.join(HERE, "golden", "rmat24_expected.json")) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def graph(exp):
    _say("generating rmat24")
    g = gg.config("rmat24")
    _say(f"rmat24: n={g.n} nnz={g.nnz}")
    got = {"row_ptr": digest(g.row_ptr, np.int64), "col": digest(g.col, np.int32), "w": digest(g.w, np.int32)}
    assert got == exp["graph"], "the generator no longer produces the graph the expected values were computed on"
    return g


@pytest.fixture(scope="module")
def ctx_graph(graph):
    import torch
    import paper_1805_10904_amd as L
    dev = torch.device("cuda", 0)
    c = L.Context(0)
    G = c.graph_create(torch.from_numpy(graph.row_ptr).to(dev), torch.from_numpy(graph.col).to(dev),
                       torch.from_numpy(graph.w).to(dev))
    yield c, G
    G.destroy()
    c.close()


def _labels(desc, n):
    if desc == "singletons":
        return None
    assert desc.startswith("random_labels(n, ")
    k, seed = (int(x) for x in desc[len("random_labels(n, "):-1].split(","))
    return gg.random_labels(n, k, seed)


def test_rmat24_local_move(ctx_graph, graph, exp):
    ctx, G = ctx_graph
    for case in exp["local_move"]:
        _say(f"rmat24 local_move from {case['labels_in']}")
        lab, deg, eown = ctx.local_move(G, _labels(case["labels_in"], graph.n), device=False)
        assert digest(lab, np.int32) == case["labels"], f"labels differ ({case['labels_in']})"
        assert digest(deg, np.int64) == case["deg"], f"deg_C differ ({case['labels_in']})"
        assert digest(eown, np.int64) == case["e_own"], f"e_own differ ({case['labels_in']})"


def test_rmat24_aggregate(ctx_graph, graph, exp):
    ctx, G = ctx_graph
    want = exp["aggregate"]
    _say(f"rmat24 aggregate of {want['labels_in']}")
    G2, ren = ctx.aggregate(G, _labels(want["labels_in"], graph.n), device=False)
    assert G2.info()[0] == want["n_new"]
    assert digest(ren, np.int32) == want["renumbered"]
    rp, cl, w = G2.export()
    assert digest(rp, np.int64) == want["row_ptr"], "contracted row_ptr differs"
    assert digest(cl, np.int32) == want["col"], "contracted columns differ"
    assert digest(w, np.int64) == want["w"], "contracted weights differ"
    G2.destroy()


def test_rmat24_run(ctx_graph, exp):
    ctx, G = ctx_graph
    want = exp["run"]
    _say("rmat24 run")
    r = ctx.run(G, device=False)
    _say(f"rmat24: {len(r.stats['levels'])} levels, Q = {r.q:.6f}")
    assert digest(r.labels, np.int32) == want["labels"], "final labels differ"
    assert r.q_int == int(want["q_int"])
    assert abs(r.q - want["q"]) <= 1e-12 * max(abs(want["q"]), 1e-3)
    got = [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], lv["q_int"]) for lv in r.stats["levels"]]
    ref = [(lv["n"], lv["nnz"], lv["sweeps_executed"], lv["sweeps_accepted"], int(lv["q_int"])) for lv in want["levels"]]
    assert got == ref, "level records differ"
    assert (r.status == 0) == (want["status"] == 0)
