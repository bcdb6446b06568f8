"""GPU tests of the context boundary: device memory from a caller-provided
region (a torch tensor), ENOMEM when it runs out with the context still
usable, the allocation fault-injection hook, concurrent use of a context
(EBUSY), the launch-shape file, and the served footprint estimate against
the real high-water mark of the region.
"""
import os
import sys
import threading

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


@pytest.fixture(autouse=True)
def _threads():
    oracle.set_threads(min(16, os.cpu_count() or 1))


def _check_run(g, r, tag=""):
    ref = oracle.louvain(g.row_ptr, g.col, g.w)
    labels = r.labels.cpu().numpy() if hasattr(r.labels, "cpu") else r.labels
    assert np.array_equal(labels, ref.labels), f"{tag}: labels differ"
    assert r.q_int == ref.q_int, f"{tag}: Q_int differs"


def test_chunglu1m_inside_a_torch_pool(L):
    """The full benchmark graph runs with every device buffer carved from one
    torch tensor; results equal the oracle's; nothing stays live afterwards."""
    import torch
    g = gg.config("chunglu1m")
    ctx = L.Context(0, pool_bytes=3 << 30)
    before = torch.cuda.memory_allocated(0)
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    r = ctx.run(G)
    m = ctx.memory()
    _say(f"chunglu1m in a 3 GiB pool: high water {m['pool_high_water'] / 2**20:.1f} MiB")
    assert 0 < m["pool_high_water"] <= m["pool_bytes"]
    # torch saw no new allocation: the library used the region only
    assert torch.cuda.memory_allocated(0) == before
    _check_run(g, r, "chunglu1m in a pool")
    G.destroy()
    assert ctx.memory()["live_bytes"] == 0
    ctx.close()


def test_exhausted_pool_gives_enomem_and_context_stays_usable(L):
    g_big = gg.config("chunglu_n65536")
    g_small = gg.config("sbm1k")
    csr_bytes = g_big.row_ptr.nbytes + g_big.col.nbytes + g_big.w.nbytes + 8 * g_big.n
    ctx = L.Context(0, pool_bytes=csr_bytes // 2)
    with pytest.raises(L.LouvainError) as e:
        ctx.graph_create(g_big.row_ptr, g_big.col, g_big.w)
    assert e.value.code == L.LOUVAIN_ENOMEM
    assert "pool" in str(e.value)
    assert ctx.memory()["live_bytes"] == 0
    G = ctx.graph_create(g_small.row_ptr, g_small.col, g_small.w)
    _check_run(g_small, ctx.run(G), "sbm1k after ENOMEM")
    G.destroy()
    ctx.close()
    # a region that holds the graph but not its run: the run fails, the graph stays usable
    for factor in (1.2, 1.5, 2.0, 3.0):
        ctx = L.Context(0, pool_bytes=int(csr_bytes * factor))
        try:
            G = ctx.graph_create(g_big.row_ptr, g_big.col, g_big.w)
        except L.LouvainError as e2:
            assert e2.code == L.LOUVAIN_ENOMEM
            ctx.close()
            continue
        try:
            ctx.run(G)
            G.destroy()
            ctx.close()
            continue
        except L.LouvainError as e3:
            assert e3.code == L.LOUVAIN_ENOMEM
        _say(f"pool of {factor} x the CSR: graph created, run ENOMEM")
        m = ctx.memory()
        n, nnz, tw = G.info()
        assert n == g_big.n and nnz == g_big.nnz
        q = ctx.modularity(G, np.arange(g_big.n, dtype=np.int32))
        assert q[0] == oracle.modularity(g_big.row_ptr, g_big.col, g_big.w, np.arange(g_big.n, dtype=np.int32))[0]
        G.destroy()
        assert ctx.memory()["live_bytes"] == 0 and m["pool_in_use"] <= m["pool_bytes"]
        ctx.close()
        break
    else:
        pytest.fail("no region size between the graph and its run was found")


def test_pool_argument_errors(L):
    import ctypes as C
    lib = L.load_library()
    h = C.c_void_p()
    host = (C.c_uint8 * 4096)()
    # host memory is not a device region; pointer and size must come together
    assert lib.louvain_ctx_create(0, None, C.cast(host, C.c_void_p), 4096, None, C.byref(h)) == L.LOUVAIN_EINVAL
    assert lib.louvain_ctx_create(0, None, None, 4096, None, C.byref(h)) == L.LOUVAIN_EINVAL
    assert lib.louvain_ctx_create(-1, None, None, 0, None, C.byref(h)) == L.LOUVAIN_EINVAL
    assert lib.louvain_ctx_create(0, None, None, 0, None, None) == L.LOUVAIN_EINVAL


def _fault_sweep(L, work, max_k=400):
    """Runs work(ctx) on a fresh context whose k-th allocation request fails,
    for k = 1, 2, ... until one run sees no injected failure.  Every failure
    must be ENOMEM, leave nothing live, and the same context must then run
    work correctly."""
    failures = 0
    for k in range(1, max_k):
        os.environ["LOUVAIN_FAULT_ALLOC_AT"] = str(k)
        try:
            ctx = L.Context(0)
        finally:
            del os.environ["LOUVAIN_FAULT_ALLOC_AT"]
        try:
            work(ctx)
        except L.LouvainError as e:
            assert e.code == L.LOUVAIN_ENOMEM, f"k={k}: {e}"
            assert "LOUVAIN_FAULT_ALLOC_AT" in str(e)
            failures += 1
            assert ctx.memory()["live_bytes"] == 0, f"k={k}: blocks leaked after the failure"
            work(ctx)            # the context still works, and gives the right results
            assert ctx.memory()["live_bytes"] == 0
            ctx.close()
            continue
        ctx.close()
        return failures
    pytest.fail("allocation requests never ran out")


def test_fault_injection_every_allocation_of_a_run(L):
    g = gg.config("chunglu_n20000")
    ref = oracle.louvain(g.row_ptr, g.col, g.w)

    def work(ctx):
        G = ctx.graph_create(g.row_ptr, g.col, g.w)
        try:
            r = ctx.run(G)
            assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int
        finally:
            G.destroy()

    k = _fault_sweep(L, work)
    _say(f"run: {k} allocation requests failed one at a time, each cleanly")
    assert k > 10


def test_fault_injection_batch_dendrogram_aggregate(L):
    graphs = gg.batch_sbm(5, n_hi=4000, first=900) + [gg.config("sbm1k")]
    refs = [oracle.louvain(g.row_ptr, g.col, g.w) for g in graphs]
    g0 = graphs[-1]
    lab = gg.random_labels(g0.n, 37, seed=5)
    ref_agg = oracle.contract(g0.row_ptr, g0.col, g0.w, *_renumbered(lab))

    def work(ctx):
        Gs = [ctx.graph_create(g.row_ptr, g.col, g.w) for g in graphs]
        try:
            out = ctx.run_batch(Gs)
            for r, ref in zip(out, refs):
                assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int
            r, d = ctx.run(Gs[-1], dendrogram=True)
            d.destroy()
            assert np.array_equal(r.labels, refs[-1].labels)
            A, _ = ctx.aggregate(Gs[-1], lab)
            try:
                rp, cl, w = A.export()
                assert np.array_equal(rp, ref_agg[0]) and np.array_equal(cl, ref_agg[1])
                assert np.array_equal(w, ref_agg[2])
            finally:
                A.destroy()
        finally:
            for G in Gs:
                G.destroy()

    k = _fault_sweep(L, work, max_k=600)
    _say(f"batch + dendrogram + aggregate: {k} injected failures, each clean")
    assert k > 10


def _renumbered(lab):
    uniq, inv = np.unique(lab, return_inverse=True)
    return inv.astype(np.int32), int(uniq.size)


def test_concurrent_use_of_a_context_is_refused(L):
    g = gg.config("chunglu_n65536")
    s = gg.config("sbm1k")
    ctx = L.Context(0)
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    S = ctx.graph_create(s.row_ptr, s.col, s.w)
    ident = np.arange(s.n, dtype=np.int32)
    q_ref = oracle.modularity(s.row_ptr, s.col, s.w, ident)[0]
    ref = oracle.louvain(g.row_ptr, g.col, g.w)
    stop = threading.Event()
    errors = []
    runner_busy = [0]

    def runner():
        # whichever thread enters second is refused: EBUSY here too is an outcome
        runs = 0
        while runs < 40 and not stop.is_set():
            try:
                r = ctx.run(G)
            except L.LouvainError as e:
                if e.code != L.LOUVAIN_EBUSY:
                    errors.append(repr(e))
                    return
                runner_busy[0] += 1
                continue
            except Exception as e:   # noqa: BLE001
                errors.append(repr(e))
                return
            runs += 1
            if not (np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int):
                errors.append("wrong result under contention")

    th = threading.Thread(target=runner)
    th.start()
    busy = ok = 0
    while th.is_alive() and busy < 50:
        try:
            q = ctx.modularity(S, ident)
            assert q[0] == q_ref
            ok += 1
        except L.LouvainError as e:
            assert e.code == L.LOUVAIN_EBUSY, str(e)
            busy += 1
    stop.set()
    th.join()
    _say(f"EBUSY {busy} times here, {runner_busy[0]} times in the other thread, {ok} calls between runs")
    assert not errors, errors
    assert busy + runner_busy[0] > 0
    # once the other thread is out, calls proceed again
    assert ctx.modularity(S, ident)[0] == q_ref
    G.destroy()
    S.destroy()
    ctx.close()


def test_tuning_file(L, tmp_path):
    g = gg.config("chunglu_n65536")
    path = str(tmp_path / "louvain_tuning.txt")
    ctx = L.Context(0, tuning_path=path)             # no file yet: defaults
    defaults = ctx.get_tuning()
    G = ctx.graph_create(g.row_ptr, g.col, g.w)
    best = ctx.autotune(G)
    G.destroy()
    ctx.close()
    text = open(path).read()
    assert "arch gfx950" in text and f"small_max {best['small_max']}" in text
    ctx2 = L.Context(0, tuning_path=path)            # read back
    got = ctx2.get_tuning()
    assert all(got[k] == best[k] for k in got), (got, best)
    ctx2.close()
    # written for another architecture: ignored
    other = str(tmp_path / "other.txt")
    with open(other, "w") as f:
        f.write("arch gfx000\nsmall_max 8\nblock_max 10922\n")
    ctx3 = L.Context(0, tuning_path=other)
    assert ctx3.get_tuning() == defaults
    ctx3.close()
    # malformed values or keys are refused
    arch = [ln for ln in text.splitlines() if ln.startswith("arch ")][0]
    for body in ("small_max 99\n", "unknown_key 1\n", "block_max\n"):
        bad = str(tmp_path / "bad.txt")
        with open(bad, "w") as f:
            f.write(arch + "\n" + body)
        with pytest.raises(L.LouvainError) as e:
            L.Context(0, tuning_path=bad)
        assert e.value.code == L.LOUVAIN_EINVAL


def test_served_footprint_estimate_bounds_the_real_high_water(L):
    """louvain_workspace_bytes, by which the request loop admits graphs, is
    at least the device memory a served graph really takes: each request
    runs alone on a fresh context whose region records its high-water mark."""
    graphs = [gg.config("sbm1k"), gg.batch_sbm(1, n_lo=50_000, n_hi=60_000, first=11)[0],
              gg.config("chunglu_n65536")] + gg.served_chunglu(2, first=0, n_lo=60_000, n_hi=250_000)
    for g in graphs:
        est = L.workspace_bytes(g.n, g.nnz)
        ctx = L.Context(0, pool_bytes=max(4 * est, 256 << 20))
        t = ctx.submit(g.row_ptr, g.col, g.w)
        r = ctx.poll(t, wait_us=-1)
        assert r.status == 0
        _check_run(g, r, g.name)
        high = ctx.memory()["pool_high_water"]
        _say(f"{g.name}: n {g.n} nnz {g.nnz}: high water {high / 2**20:.1f} MiB, estimate {est / 2**20:.1f} MiB "
             f"({high / est:.2f})")
        ctx.close()
        assert high <= est, f"{g.name}: footprint {high} above the estimate {est}"


def test_log_environment_variable(tmp_path):
    """LOUVAIN_LOG=1 prints one progress line per level on stderr (checked
    in a child process, since the switch is read once per process); the
    run's result is unchanged."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys; sys.path.insert(0, %r)\n"
            "import numpy as np, graphgen as gg, oracle, paper_1805_10904_amd as L\n"
            "g = gg.config('sbm1k'); ctx = L.Context(0); G = ctx.graph_create(g.row_ptr, g.col, g.w)\n"
            "r = ctx.run(G); ref = oracle.louvain(g.row_ptr, g.col, g.w)\n"
            "assert np.array_equal(r.labels, ref.labels) and r.q_int == ref.q_int\n"
            "print(len(r.stats['levels']))\n") % root
    env = dict(os.environ, LOUVAIN_LOG="1")
    p = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=240)
    assert p.returncode == 0, p.stderr[-3000:]
    levels = int(p.stdout.strip().splitlines()[-1])
    lines = [ln for ln in p.stderr.splitlines() if ln.startswith("[louvain] level ")]
    _say("\n".join(lines))
    assert len(lines) == levels and lines[0].startswith("[louvain] level 0: n 1000, nnz 14496")
