"""Host-side checks of the C ABI (no GPU needed): the library loads and
exports every function include/louvain.h declares, and the Python binding
covers exactly those."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "louvain.h")
PKG = os.path.join(ROOT, "paper_1805_10904_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(louvain_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("louvain_graph_create", "louvain_local_move", "louvain_aggregate", "louvain_run",
              "louvain_modularity"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_1805_10904_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        from paper_1805_10904_amd import build
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", _native.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (louvain_[a-z0-9_]+)\b", out))
    missing = [f for f in declared_functions() if f not in exported]
    assert not missing, f"declared but not exported: {missing}"
    # the binding's list matches the header
    assert sorted(_native.ABI_SYMBOLS) == declared_functions()
    # and ctypes resolves them
    assert sorted(_native.exported_symbols()) == declared_functions()


def test_product_path_never_touches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\boracle\b", text), f"{f} mentions the oracle"


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1805_10904_amd import _native
    with pytest.raises(RuntimeError, match="not built"):
        _native.load_library(str(tmp_path / "missing.so"))


def test_workspace_bytes_bounds_the_served_footprint():
    """The admission estimate grows with the graph and covers at least the
    bytes a level-0 graph occupies in the batch (resident CSR, two union
    copies, sort keys and values of the contraction)."""
    from paper_1805_10904_amd import workspace_bytes
    assert workspace_bytes(0, 0) > 0
    prev = 0
    for n, nnz in [(10, 20), (1000, 20000), (10**5, 2 * 10**6), (2 * 10**6, 6 * 10**7)]:
        b = workspace_bytes(n, nnz)
        assert b > prev
        prev = b
        floor = (8 * (n + 1) + 4 * nnz + 4 * nnz + 8 * n + 4 * n) + 2 * (16 * n + 12 * nnz) + 32 * nnz
        assert b >= floor
    assert workspace_bytes(-1, 5) == 0


def test_served_and_batched_calls_are_declared():
    names = declared_functions()
    for f in ("louvain_run_batch", "louvain_submit", "louvain_poll", "louvain_workspace_bytes",
              "louvain_serve_budget"):
        assert f in names


def test_recorded_traffic_lookup():
    """The bench's counter-based traffic lookup parses the committed summary
    and reports nothing for a kernel or workload it does not cover."""
    import bench
    got = bench.recorded_traffic("chunglu1m", "k_cpt_groups<4,1,int>")
    assert got is None or got > 0
    assert bench.recorded_traffic("chunglu1m", "no_such_kernel") is None
    assert bench.recorded_traffic("no_such_workload", "k_cpt_groups<4,1,int>") is None


def test_shard_csr_reassembles_the_graph():
    """The bench's one-GPU share: every shard's local rows map back to the
    graph's rows (columns ascending, ghosts renumbered after the local
    vertices), and the shards together hold every entry once."""
    import numpy as np

    import bench
    import graphgen as gg
    g = gg.config("chunglu_n20000")
    b = bench.shard_bounds(g.row_ptr, 8)
    assert b[0] == 0 and b[-1] == g.n and np.all(np.diff(b) > 0)
    total = 0
    for k in range(8):
        lo, hi = int(b[k]), int(b[k + 1])
        rp, col, w, ghosts, frac = bench.shard_csr(g.row_ptr, g.col, g.w, lo, hi)
        nl = hi - lo
        assert rp.shape[0] == nl + ghosts.shape[0] + 1 and rp[0] == 0 and np.all(np.diff(rp) >= 0)
        assert np.all(rp[nl:] == rp[nl])                      # ghost rows are empty
        assert np.all((ghosts < lo) | (ghosts >= hi)) and np.all(np.diff(ghosts) > 0)
        back = np.where(col < nl, col.astype(np.int64) + lo, ghosts[np.maximum(col.astype(np.int64) - nl, 0)])
        for v in range(lo, hi):
            seg = slice(rp[v - lo], rp[v - lo + 1])
            assert np.all(np.diff(col[seg]) > 0)
            order = np.argsort(back[seg])
            assert np.array_equal(back[seg][order], g.col[g.row_ptr[v]:g.row_ptr[v + 1]])
            assert np.array_equal(w[seg][order], g.w[g.row_ptr[v]:g.row_ptr[v + 1]])
        assert 0.0 <= frac <= 1.0
        total += int(rp[-1])
    assert total == g.nnz


def test_bench_refuses_more_than_one_gpu():
    """The benchmark measures one GPU; asked for more it says so and exits."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and r.stdout == ""
    assert "one GPU" in r.stderr
