"""The Python binding checks every array before the C library sees it (no
GPU needed): wrong dtype, length, dimension, non-integer values, values
outside the dtype, and host memory where device pointers are expected all
raise LouvainError(EINVAL) without any library call."""
import numpy as np
import pytest

from paper_1805_10904_amd import _native as N


class _NoCalls:
    """Stands in for the loaded library: any call is a test failure."""

    def __getattr__(self, name):
        def f(*a, **k):
            raise AssertionError(f"the library was called ({name}) before the arguments were checked")
        return f


def _ctx():
    ctx = N.Context.__new__(N.Context)
    ctx.lib = _NoCalls()
    ctx.device = 0
    ctx.torch_device = None
    ctx.h = None
    ctx._inflight = {}
    return ctx


def _graph(ctx, n=4, nnz=6, dev=False):
    g = N.Graph.__new__(N.Graph)
    g.ctx, g.h, g.dev = ctx, 1, dev
    g.info = lambda: (n, nnz, 2 * nnz)
    g.destroy = lambda: None
    return g


RP = np.array([0, 1, 3, 5, 6], np.int64)
COL = np.array([1, 0, 2, 1, 3, 2], np.int32)
W = np.ones(6, np.int32)


def _einval(fn):
    with pytest.raises(N.LouvainError) as e:
        fn()
    assert e.value.code == N.LOUVAIN_EINVAL
    return str(e.value)


def test_graph_create_rejects_bad_csr_arrays():
    ctx = _ctx()
    _einval(lambda: ctx.graph_create(RP, COL[:5], W))                              # col and w disagree
    assert "w" in _einval(lambda: ctx.graph_create(RP, COL, W[:4]))                 # length
    assert "integers" in _einval(lambda: ctx.graph_create(RP, COL, W.astype(np.float32)))
    assert "range" in _einval(lambda: ctx.graph_create(RP, COL.astype(np.int64) + (1 << 32), W))
    assert "1-D" in _einval(lambda: ctx.graph_create(RP.reshape(1, -1), COL, W))
    _einval(lambda: ctx.graph_create(np.zeros(0, np.int64), COL[:0], W[:0]))       # no row_ptr[0]
    _einval(lambda: ctx.graph_create(None, COL, W))


def test_submit_rejects_bad_arrays_and_outputs():
    ctx = _ctx()
    _einval(lambda: ctx.submit(RP, COL, W[:3]))
    # an output of the wrong dtype, length or kind
    _einval(lambda: ctx.submit(RP, COL, W, labels_out=np.empty(4, np.int64)))
    _einval(lambda: ctx.submit(RP, COL, W, labels_out=np.empty(3, np.int32)))
    _einval(lambda: ctx.submit(RP, COL, W, labels_out=[0, 0, 0, 0]))
    ro = np.empty(4, np.int32)
    ro.flags.writeable = False
    _einval(lambda: ctx.submit(RP, COL, W, labels_out=ro))
    _einval(lambda: ctx.submit(RP, COL, W, labels_out=np.empty(8, np.int32)[::2]))


def test_labels_are_checked_per_call():
    ctx = _ctx()
    g = _graph(ctx)
    _einval(lambda: ctx.modularity(g, np.zeros(3, np.int32)))                      # short
    _einval(lambda: ctx.modularity(g, None))
    _einval(lambda: ctx.modularity(g, np.zeros(4, np.float64) + 0.5))              # not integers
    _einval(lambda: ctx.local_move(g, np.zeros(5, np.int32)))                      # long
    _einval(lambda: ctx.aggregate(g, np.zeros((2, 2), np.int32)))                   # 2-D
    _einval(lambda: ctx.resume(g, 1, None))
    _einval(lambda: ctx.run(g, labels_out=np.empty(4, np.int64)))


def test_host_memory_where_device_pointers_are_expected():
    """device=True makes every array a device pointer: a numpy array there
    would hand the library a host address as device memory."""
    ctx = _ctx()
    g = _graph(ctx, dev=False)
    msg = _einval(lambda: ctx.modularity(g, np.zeros(4, np.int32), device=True))
    assert "CUDA tensor" in msg
    _einval(lambda: ctx.local_move(g, np.zeros(4, np.int32), device=True))
    _einval(lambda: ctx.aggregate(g, np.zeros(4, np.int32), device=True))
    _einval(lambda: ctx.resume(g, 1, np.zeros(4, np.int32), device=True))


def test_batch_outputs_are_checked():
    ctx = _ctx()
    gs = [_graph(ctx, n=4), _graph(ctx, n=6)]
    _einval(lambda: ctx.run_batch(gs, labels_out=[np.empty(4, np.int32)]))          # one output for two graphs
    _einval(lambda: ctx.run_batch(gs, labels_out=[np.empty(4, np.int32), np.empty(5, np.int32)]))
    other = _ctx()
    _einval(lambda: ctx.run_batch([gs[0], _graph(other)]))                           # graph of another context


def test_valid_host_arguments_pass_the_checks():
    """Well-formed host arguments get through the checks (the stub library
    is reached, which here is the signal that checking is over)."""
    ctx = _ctx()
    with pytest.raises(AssertionError, match="library was called"):
        ctx.graph_create(RP.tolist(), COL.tolist(), W.tolist())
    with pytest.raises(AssertionError, match="library was called"):
        ctx.modularity(_graph(ctx), np.zeros(4, np.int64))   # int64 labels in range are converted
