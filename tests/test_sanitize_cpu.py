"""Sanitizer builds of host code (CPU only): the oracle under AddressSanitizer
and UndefinedBehaviorSanitizer through a small C driver, with its results
compared to the regular build's; and the library's device-region allocator
(paper_1805_10904_amd/csrc/arena.hpp, plain C++) exercised by random
allocation sequences under the same sanitizers."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import graphgen as gg
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="3")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "oracle_driver")
    subprocess.check_call(["gcc", "-std=c11", "-fopenmp", *SAN, "-o", exe,
                           os.path.join(ROOT, "oracle", "louvain_oracle.c"),
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c")])
    return exe


def _graphs():
    yield gg.config("sbm1k"), gg.random_labels(1000, 7, seed=1)
    for s in range(4):
        g = gg.random_small(40 + 10 * s, 0.15, 9, seed=100 + s, loop_prob=0.2)
        yield g, gg.random_labels(g.n, 5, seed=s)
    tri = gg.from_edge_list(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (2, 3)])
    yield tri, np.array([0, 0, 0, 3, 3, 3], np.int32)
    iso = gg.from_edge_list(5, [])
    yield iso, np.arange(5, dtype=np.int32)
    g = gg.config("chunglu_n20000")
    yield g, gg.random_labels(g.n, 64, seed=3)


def _expected(g, lab):
    out = []
    for threads in (1, 3):
        oracle.set_threads(threads)
        for merge in (False, True):
            r = oracle.louvain(g.row_ptr, g.col, g.w, merge=merge)
            out.append(r.labels.astype(np.int32).tobytes())
            out.append(oracle.i128_to_pair(r.q_int).astype(np.int64).tobytes())
        lm = oracle.local_move(g.row_ptr, g.col, g.w, lab)
        out += [lm.labels.astype(np.int32).tobytes(), lm.deg.astype(np.int64).tobytes(),
                lm.e_own.astype(np.int64).tobytes()]
        q = oracle.modularity(g.row_ptr, g.col, g.w, lab)[0]
        out.append(oracle.i128_to_pair(q).astype(np.int64).tobytes())
        m, k = oracle.renumber(lab)
        rp, cl, w = oracle.contract(g.row_ptr, g.col, g.w, m[lab], k)
        out += [np.array([k, cl.shape[0]], np.int64).tobytes(), rp.astype(np.int64).tobytes(),
                cl.astype(np.int32).tobytes(), w.astype(np.int64).tobytes()]
    oracle.set_threads(1)
    return b"".join(out)


def test_oracle_under_asan_ubsan(driver, tmp_path):
    for k, (g, lab) in enumerate(_graphs()):
        src = tmp_path / f"g{k}.bin"
        dst = tmp_path / f"o{k}.bin"
        with open(src, "wb") as f:
            f.write(np.array([g.n, g.nnz], np.int64).tobytes())
            f.write(g.row_ptr.astype(np.int64).tobytes())
            f.write(g.col.astype(np.int32).tobytes())
            f.write(g.w.astype(np.int64).tobytes())
            f.write(np.asarray(lab, np.int32).tobytes())
        r = subprocess.run([driver, str(src), str(dst)], env=ENV, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, f"graph {k} ({g.name}): sanitizer run failed\n{r.stderr[-4000:]}"
        assert dst.read_bytes() == _expected(g, lab), f"graph {k} ({g.name}): results differ from the regular build"


def test_arena_allocator_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "arena_driver")
    subprocess.check_call(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_1805_10904_amd", "csrc"),
                           "-o", exe, os.path.join(ROOT, "tests", "sanitize", "arena_driver.cpp")])
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "arena ok" in r.stdout
