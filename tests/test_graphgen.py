"""The seeded input generators: well-formed symmetric CSR, reproducible, and
the batched / served mixes drawn from the stated ranges."""
import math

import numpy as np

import graphgen as gg


def assert_wellformed(g):
    rp, col, w = g.row_ptr, g.col, g.w
    assert rp.dtype == np.int64 and col.dtype == np.int32 and w.dtype == np.int32
    assert rp[0] == 0 and rp[-1] == col.shape[0] and np.all(np.diff(rp) >= 0)
    assert np.all(w >= 1)
    if g.nnz:
        assert col.min() >= 0 and col.max() < g.n
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    for r in range(0, g.n, max(1, g.n // 50)):
        c = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(c) > 0)
    # symmetric with equal weights
    a = dict(zip(zip(rows.tolist(), col.tolist()), w.tolist()))
    for (u, v), x in list(a.items())[:5000]:
        assert a[(v, u)] == x


def test_batch_sbm_reproducible_and_in_range():
    gs = gg.batch_sbm(12, n_hi=5000)
    again = gg.batch_sbm(4, n_hi=5000, first=8)
    for a, b in zip(gs[8:], again):
        assert a.n == b.n and np.array_equal(a.col, b.col) and np.array_equal(a.w, b.w)
    for g in gs:
        assert 100 <= g.n <= 5000
        assert g.w.max() <= 10
        assert_wellformed(g)
        mean = g.nnz / g.n
        assert 1.0 < mean < 80.0


def test_batch_sbm_size_mix_is_log_uniform():
    # parameter draws only (cheap): the first draw of stream (seed, g) is the size
    logs = []
    for k in range(2000):
        rng = np.random.default_rng([1004, k])
        logs.append(rng.uniform(math.log(100), math.log(100_000)))
    logs = np.array(logs)
    # log-uniform: the log-size is uniform on [ln 100, ln 1e5]
    q = np.quantile(logs, [0.25, 0.5, 0.75])
    span = math.log(100_000) - math.log(100)
    assert np.allclose(q, math.log(100) + span * np.array([0.25, 0.5, 0.75]), atol=0.1 * span)
    g = gg.batch_sbm(1, first=3)[0]
    rng = np.random.default_rng([1004, 3])
    assert g.n == int(round(math.exp(rng.uniform(math.log(100), math.log(100_000)))))
    sizes = gg.batch_sbm_sizes(40)
    assert sizes[3] == g.n
    assert [x.n for x in gg.batch_sbm(6, n_hi=100_000, first=30)] == sizes[30:36].tolist()


def test_served_chunglu_small_requests():
    gs = gg.served_chunglu(3, n_lo=1000, n_hi=3000)
    for g in gs:
        assert 1000 <= g.n <= 3000
        assert g.w.max() <= 50
        assert_wellformed(g)
        assert 8.0 <= g.nnz / g.n <= 32.0 + 1e-9
