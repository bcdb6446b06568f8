"""GPU test of louvain_modularity_noalloc, the allocation-free variant of
louvain_modularity (its kernels work in the library's fixed device scratch
array): two calls in a row through the C ABI, the second on a smaller
graph, each equal to louvain_modularity's result and to the oracle's; no
device memory is taken from the context's region or cache; sizes beyond
the limit and labels out of range are refused."""
import ctypes as C
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


def _noalloc(L, ctx, G, labels, device):
    """One call of the entry point through the C ABI."""
    from paper_1805_10904_amd._native import louvain_i128, _ptr
    qi = louvain_i128()
    q = C.c_double()
    rc = ctx.lib.louvain_modularity_noalloc(ctx.h, G.h, _ptr(labels), C.byref(qi), C.byref(q),
                                            L.LOUVAIN_DEVICE_PTRS if device else 0)
    return rc, qi.value(), q.value


def test_noalloc_modularity_two_calls_second_smaller():
    import torch
    import paper_1805_10904_amd as L
    oracle.set_threads(min(16, os.cpu_count() or 1))
    dev = torch.device("cuda", 0)
    big = gg.config("chunglu_n65536")
    small = gg.config("sbm1k")
    lab_big = gg.random_labels(big.n, 300, seed=21)
    lab_small = gg.random_labels(small.n, 10, seed=22)
    for pool_bytes in (None, 512 << 20):
        ctx = L.Context(0, pool_bytes=pool_bytes)
        Gb = ctx.graph_create(big.row_ptr, big.col, big.w)
        Gs = ctx.graph_create(torch.from_numpy(small.row_ptr).to(dev), torch.from_numpy(small.col).to(dev),
                              torch.from_numpy(small.w).to(dev))
        before = ctx.memory()
        # first call: the larger graph, host labels
        rc, qi, q = _noalloc(L, ctx, Gb, np.ascontiguousarray(lab_big), device=False)
        assert rc == L.LOUVAIN_OK, ctx.lib.louvain_last_error(ctx.h)
        after_first = ctx.memory()
        ref_qi, ref_q = ctx.modularity(Gb, lab_big)
        assert qi == ref_qi == oracle.modularity(big.row_ptr, big.col, big.w, lab_big)[0]
        assert abs(q - ref_q) <= 1e-12 * max(abs(ref_q), 1e-3)
        # second call: a smaller graph, device labels
        lab_d = torch.from_numpy(lab_small).to(dev)
        torch.cuda.synchronize()
        mid = ctx.memory()
        rc, qi2, q2 = _noalloc(L, ctx, Gs, lab_d, device=True)
        assert rc == L.LOUVAIN_OK, ctx.lib.louvain_last_error(ctx.h)
        assert ctx.memory() == mid
        ref2 = ctx.modularity(Gs, lab_d)
        assert qi2 == ref2[0] == oracle.modularity(small.row_ptr, small.col, small.w, lab_small)[0]
        assert abs(q2 - ref2[1]) <= 1e-12 * max(abs(ref2[1]), 1e-3)
        # the entry point took nothing from the context's memory
        assert before == after_first, (before, after_first)
        # the binding's method is the same call
        assert ctx.modularity_noalloc(Gb, lab_big)[0] == ref_qi
        _say(f"pool {pool_bytes}: Q_int {qi} then {qi2}, memory unchanged")
        # errors: a label out of range, a graph beyond the limit
        bad = lab_small.copy()
        bad[5] = small.n
        rc, _, _ = _noalloc(L, ctx, Gs, np.ascontiguousarray(bad), device=False)
        assert rc == L.LOUVAIN_EINVAL
        assert b"out of range" in ctx.lib.louvain_last_error(ctx.h)
        n_over = 4194305
        Gh = ctx.graph_create(np.zeros(n_over + 1, np.int64), np.zeros(0, np.int32), np.zeros(0, np.int32))
        rc, _, _ = _noalloc(L, ctx, Gh, np.zeros(n_over, np.int32), device=False)
        assert rc == L.LOUVAIN_EINVAL
        assert b"limit" in ctx.lib.louvain_last_error(ctx.h)
        # and a valid call still works after the errors
        rc, qi3, _ = _noalloc(L, ctx, Gb, np.ascontiguousarray(lab_big), device=False)
        assert rc == L.LOUVAIN_OK and qi3 == ref_qi
        for G in (Gb, Gs, Gh):
            G.destroy()
        ctx.close()
