"""Seeded synthetic graph generators.

Inputs only: nothing in this package computes any part of the community
detection method (no degrees, communities, gains or modularity).  Both the
CPU oracle's tests and the GPU path's tests and benchmark draw their graphs
from here, so that the two sides see byte-identical inputs.

Every generator returns a symmetric CSR graph as a ``Graph`` tuple:

* ``row_ptr``: int64[n+1], ``col``: int32[nnz], ``w``: int32[nnz]
* columns strictly ascending inside every row (no multi-edges),
* an undirected edge {u, v} with u != v is stored in both rows with one
  weight, a self-loop (u, u) is stored once,
* weights are integers >= 1 (the method's problem statement asks for
  positive weights; an unweighted graph is given weight 1 everywhere).

Randomness: numpy's PCG64 stream seeded per config for the structure, and
SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) over the canonical pair key
(min(u,v) << 32 | max(u,v)) xor a per-config salt for the edge weights, so a
pair drawn several times always gets the same weight.
"""
from __future__ import annotations

import math
from typing import NamedTuple, Optional

import numpy as np

__all__ = [
    "Graph", "splitmix64", "csr_from_canonical_keys", "canonical_keys",
    "weights_uniform", "weights_geometric", "sbm_dense", "sbm_sparse",
    "chung_lu", "rmat", "random_small", "random_labels", "config", "batch_sbm", "served_chunglu",
    "CONFIG_NAMES",
]

_M32 = np.uint64(0xFFFFFFFF)


class Graph(NamedTuple):
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[nnz]
    w: np.ndarray        # int32[nnz]
    planted: Optional[np.ndarray] = None  # int32[n] planted block of each vertex, if any
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied element-wise to uint64 words."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def weights_uniform(h: np.ndarray, wmax: int) -> np.ndarray:
    """Integer weights uniform on {1..wmax} from 64-bit hashes."""
    top = h >> np.uint64(11)  # 53 random bits
    with np.errstate(over="ignore"):
        v = (top * np.uint64(wmax)) >> np.uint64(53)
    return (v + np.uint64(1)).astype(np.int32)


def weights_geometric(h: np.ndarray, p: float) -> np.ndarray:
    """Integer weights 1 + F where F ~ Geometric(p) counts failures before the
    first success (support {1, 2, ...}, mean 1/p).  Inverse-CDF sampling."""
    u = ((h >> np.uint64(11)).astype(np.float64) + 1.0) * (2.0 ** -53)  # (0, 1]
    f = np.floor(np.log(u) / math.log1p(-p))
    return np.minimum(1.0 + f, 2 ** 31 - 1).astype(np.int32)


def canonical_keys(u: np.ndarray, v: np.ndarray, keep_loops: bool = False) -> np.ndarray:
    """Sorted unique canonical pair keys (min << 32 | max) of the pairs (u, v)."""
    u = np.asarray(u, dtype=np.uint64)
    v = np.asarray(v, dtype=np.uint64)
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    if not keep_loops:
        m = lo != hi
        lo = lo[m]
        hi = hi[m]
    k = (lo << np.uint64(32)) | hi
    return np.unique(k)


def csr_from_canonical_keys(n: int, keys: np.ndarray, salt: int, weight_fn) -> tuple:
    """Symmetric CSR from sorted unique canonical keys.

    Each key min<<32|max becomes entries (min, max) and, if min != max,
    (max, min); weights are ``weight_fn(splitmix64(key ^ salt))``."""
    keys = np.asarray(keys, dtype=np.uint64)
    lo = keys >> np.uint64(32)
    hi = keys & _M32
    nl = lo != hi
    rev = (hi[nl] << np.uint64(32)) | lo[nl]
    del lo, hi, nl
    allk = np.concatenate([keys, rev])
    del rev
    allk.sort()
    return _csr_from_entry_keys(n, allk, salt, weight_fn)


def _csr_from_entry_keys(n: int, allk: np.ndarray, salt: int, weight_fn, pool=None) -> tuple:
    """CSR from the sorted unique entry keys row << 32 | col of a symmetric
    graph; the weight of an entry comes from its canonical pair key.  With a
    thread pool, the per-entry work is split into slices."""
    m = allk.size
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(m, np.int32)
    w = np.empty(m, np.int32)

    def part(lo_hi):
        a, b = lo_hi
        k = allk[a:b]
        r = k >> np.uint64(32)
        c = k & _M32
        col[a:b] = c.astype(np.int32)
        ck = (np.minimum(r, c) << np.uint64(32)) | np.maximum(r, c)
        w[a:b] = weight_fn(splitmix64(ck ^ np.uint64(salt)))

    step = max(1, 1 << 22)
    slices = [(a, min(m, a + step)) for a in range(0, m, step)]
    if pool is not None and len(slices) > 1:
        list(pool.map(part, slices))
    else:
        for sl in slices:
            part(sl)
    if m:
        # first entry of every row: rows are the high words of the sorted keys
        row_ptr[:] = np.searchsorted(allk, np.arange(n + 1, dtype=np.uint64) << np.uint64(32))
    return row_ptr, col, w


def sbm_dense(n: int, nblocks: int, p_in: float, p_out: float, wmax: int, seed: int,
              name: str = "sbm") -> Graph:
    """Planted-partition stochastic block model by one Bernoulli draw per vertex
    pair (for small n).  Blocks are equal; a seeded permutation of vertex IDs
    keeps blocks from lining up with ID ranges."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    bsize = n // nblocks
    block = np.minimum(perm // bsize, nblocks - 1).astype(np.int32)
    iu, ju = np.triu_indices(n, 1)
    same = block[iu] == block[ju]
    prob = np.where(same, p_in, p_out)
    hit = rng.random(iu.shape[0]) < prob
    keys = canonical_keys(iu[hit], ju[hit])
    rp, col, w = csr_from_canonical_keys(n, keys, seed, lambda h: weights_uniform(h, wmax))
    return Graph(n, rp, col, w, block, name)


def sbm_sparse(n: int, nblocks: int, mean_deg: float, mixing: float, wmax: int,
               rng: np.random.Generator, salt: int, name: str = "sbm") -> Graph:
    """Stochastic block model for larger n: each block pair gets a Poisson
    number of uniformly drawn vertex pairs (duplicates and loops dropped), with
    a fraction ``mixing`` of each vertex's expected degree leaving its block."""
    nblocks = max(1, min(nblocks, n // 2 if n >= 2 else 1))
    perm = rng.permutation(n)
    block = (perm * nblocks // n).astype(np.int64)
    order = np.argsort(block, kind="stable")
    sizes = np.bincount(block, minlength=nblocks)
    starts = np.concatenate([[0], np.cumsum(sizes)])
    m_total = n * mean_deg / 2.0
    m_in = m_total * (1.0 - mixing)
    m_out = m_total * mixing
    us, vs = [], []
    # intra-block pairs, expected count proportional to block pair count
    pair_in = sizes * (sizes - 1) / 2.0
    tot_in = pair_in.sum()
    if tot_in > 0:
        cnt = rng.poisson(m_in * pair_in / tot_in)
        bid = np.repeat(np.arange(nblocks), cnt)
        a = starts[bid] + (rng.random(bid.size) * sizes[bid]).astype(np.int64)
        b = starts[bid] + (rng.random(bid.size) * sizes[bid]).astype(np.int64)
        us.append(order[a])
        vs.append(order[b])
    # inter-block pairs: uniform vertex pairs, kept when blocks differ
    if nblocks > 1 and m_out > 0:
        k = rng.poisson(m_out * n * n / max(1.0, n * n - float((sizes.astype(np.float64) ** 2).sum())))
        a = rng.integers(0, n, size=k)
        b = rng.integers(0, n, size=k)
        keep = block[a] != block[b]
        us.append(a[keep])
        vs.append(b[keep])
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    keys = canonical_keys(u, v)
    rp, col, w = csr_from_canonical_keys(n, keys, salt, lambda h: weights_uniform(h, wmax))
    return Graph(n, rp, col, w, block.astype(np.int32), name)


def chung_lu(n: int, gamma: float, mean_deg: float, nblocks: int, mixing: float,
             seed: int, weight_fn, name: str = "chung_lu") -> Graph:
    """Chung-Lu power-law graph with planted blocks.

    Expected-degree sequence w_r proportional to (r+1)^(-1/(gamma-1)) for
    ranks r, scaled to the requested mean and assigned to vertices through a
    seeded permutation.  Endpoint pairs are drawn in batches: the first
    endpoint proportional to w over all vertices, the second with probability
    1-mixing proportional to w inside the first endpoint's block (blocks are
    contiguous ID ranges), else proportional to w globally.  Loops and
    repeated pairs are dropped, and batches continue until the graph holds
    round(n*mean_deg/2) distinct edges (a seeded subset of the last batch's
    surplus is discarded), so the realised mean degree is mean_deg."""
    rng = np.random.default_rng(seed)
    r = np.arange(n, dtype=np.float64)
    wr = (r + 1.0) ** (-1.0 / (gamma - 1.0))
    wr *= mean_deg * n / wr.sum()
    perm = rng.permutation(n)
    wv = wr[perm]
    cw = np.cumsum(wv)
    total = cw[-1]
    cw0 = np.concatenate([[0.0], cw])
    target_m = int(round(n * mean_deg / 2.0))
    target_m = min(target_m, n * (n - 1) // 2)
    bsize = max(1, n // nblocks)

    def draw(m):
        u = np.searchsorted(cw, rng.random(m) * total, side="right")
        u = np.minimum(u, n - 1)
        inblock = rng.random(m) < (1.0 - mixing)
        b = np.minimum(u // bsize, nblocks - 1)
        lo_idx = b * bsize
        hi_idx = np.where(b == nblocks - 1, n, (b + 1) * bsize)
        x = rng.random(m)
        tgt = np.where(inblock, cw0[lo_idx] + x * (cw0[hi_idx] - cw0[lo_idx]), x * total)
        v = np.searchsorted(cw, tgt, side="right")
        v = np.minimum(v, n - 1)
        v = np.where(inblock, np.clip(v, lo_idx, hi_idx - 1), v)
        return canonical_keys(u, v)

    keys = draw(target_m)
    for _ in range(64):
        if keys.size >= target_m:
            break
        deficit = target_m - keys.size
        extra = draw(int(deficit * 1.5) + 16)
        extra = extra[~np.isin(extra, keys, assume_unique=True)]
        if extra.size > deficit:
            extra = np.sort(rng.choice(extra, size=deficit, replace=False))
        keys = np.union1d(keys, extra)
    rp, col, w = csr_from_canonical_keys(n, keys, seed, weight_fn)
    planted = np.minimum(np.arange(n) // bsize, nblocks - 1).astype(np.int32)
    return Graph(n, rp, col, w, planted, name)


def rmat(scale: int, edge_factor: int, a: float, b: float, c: float, seed: int,
         weight_fn, name: str = "rmat", chunk: int = 1 << 22, threads: Optional[int] = None) -> Graph:
    """R-MAT graph (Chakrabarti, Zhan and Faloutsos, SDM 2004): each edge picks
    one adjacency-matrix quadrant per bit with probabilities (a, b, c, d), no
    noise.  Edges are drawn in chunks of ``chunk``, chunk i from its own
    PCG64 stream seeded (seed, i); vertex IDs go through a permutation seeded
    by ``seed``; the result is symmetrised, deduplicated and loop-free.  The
    chunks, the sort and the weights run on a thread pool (numpy releases
    the interpreter lock in them); the graph does not depend on ``threads``."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    n = 1 << scale
    m = edge_factor * n
    perm = np.random.default_rng(seed).permutation(n).astype(np.uint64)
    ab = a + b
    abc = a + b + c
    nchunks = (m + chunk - 1) // chunk
    nb = min(64, n)                                   # row ranges of the merge
    bounds = (np.arange(nb + 1, dtype=np.uint64) * np.uint64(n // nb)) << np.uint64(32)
    bounds[-1] = np.uint64(n) << np.uint64(32)

    def draw(i):
        k = min(chunk, m - i * chunk)
        rng = np.random.default_rng([seed, i])
        u = np.zeros(k, dtype=np.uint64)
        v = np.zeros(k, dtype=np.uint64)
        for bit in range(scale):
            r = rng.random(k)
            ubit = r >= ab
            vbit = ((r >= a) & (r < ab)) | (r >= abc)
            u |= ubit.astype(np.uint64) << np.uint64(bit)
            v |= vbit.astype(np.uint64) << np.uint64(bit)
        u = perm[u]
        v = perm[v]
        keep = u != v
        u = u[keep]
        v = v[keep]
        ent = np.concatenate([(u << np.uint64(32)) | v, (v << np.uint64(32)) | u])
        ent.sort()
        cut = np.searchsorted(ent, bounds)
        return [ent[cut[j]:cut[j + 1]] for j in range(nb)]

    def merge(j):
        x = np.concatenate([p[j] for p in parts])
        x.sort()
        if x.size:
            x = x[np.concatenate(([True], x[1:] != x[:-1]))]
        return x

    workers = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(workers) as pool:
        parts = list(pool.map(draw, range(nchunks)))
        merged = list(pool.map(merge, range(nb)))
        del parts
        allk = np.concatenate(merged)
        del merged
        rp, col, w = _csr_from_entry_keys(n, allk, seed, weight_fn, pool)
    return Graph(n, rp, col, w, None, name)


def random_small(n: int, p: float, wmax: int, seed: int, loop_prob: float = 0.0,
                 isolated: int = 0, name: str = "random") -> Graph:
    """Small Erdos-Renyi style graph for tests: each pair an edge with
    probability p, each vertex a self-loop with probability loop_prob, and the
    last ``isolated`` vertices left without edges."""
    rng = np.random.default_rng(seed)
    m = max(0, n - isolated)
    us, vs = [], []
    if m >= 2:
        iu, ju = np.triu_indices(m, 1)
        hit = rng.random(iu.shape[0]) < p
        us.append(iu[hit])
        vs.append(ju[hit])
    if loop_prob > 0 and m > 0:
        li = np.nonzero(rng.random(m) < loop_prob)[0]
        us.append(li)
        vs.append(li)
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    keys = canonical_keys(u, v, keep_loops=True)
    salt = seed * 0x9E37 + 17
    rp, col, w = csr_from_canonical_keys(n, keys, salt, lambda h: weights_uniform(h, wmax))
    return Graph(n, rp, col, w, None, name)


def from_edge_list(n: int, edges, weights=None, name: str = "edges") -> Graph:
    """Symmetric CSR from an explicit undirected edge list [(u, v), ...] with
    explicit weights (default 1).  Used for hand-written test graphs."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    wt = np.ones(len(e), np.int64) if weights is None else np.asarray(weights, np.int64)
    ent = {}
    for (u, v), x in zip(e.tolist(), wt.tolist()):
        key = (min(u, v), max(u, v))
        if key in ent:
            raise ValueError(f"repeated edge {key}")
        ent[key] = x
    rows = [[] for _ in range(n)]
    for (u, v), x in ent.items():
        rows[u].append((v, x))
        if u != v:
            rows[v].append((u, x))
    rp = np.zeros(n + 1, np.int64)
    cols, ws = [], []
    for i in range(n):
        r = sorted(rows[i])
        rp[i + 1] = rp[i] + len(r)
        cols += [c for c, _ in r]
        ws += [x for _, x in r]
    return Graph(n, rp, np.asarray(cols, np.int32), np.asarray(ws, np.int32), None, name)


def random_labels(n: int, k: int, seed: int) -> np.ndarray:
    """A seeded labelling with values in [0, n): k distinct community labels
    picked among vertex IDs (labels of a partition are vertex IDs)."""
    rng = np.random.default_rng(seed)
    k = max(1, min(k, n))
    pool = rng.choice(n, size=k, replace=False)
    return pool[rng.integers(0, k, size=n)].astype(np.int32)


# --- the benchmark workloads -------------------------------------------------

CONFIG_NAMES = ("sbm1k", "chunglu1m", "rmat24")


def _log_uniform(rng: np.random.Generator, lo: float, hi: float) -> float:
    return float(math.exp(rng.uniform(math.log(lo), math.log(hi))))


def batch_sbm(count: int = 4096, seed: int = 1004, n_lo: int = 100, n_hi: int = 100_000, first: int = 0) -> list:
    """Many independent SBM graphs of uneven sizes (the batched workload).

    Graph g draws from its own stream (seed, g): n log-uniform in
    [n_lo, n_hi], block count log-uniform in [2, 200] (at most n / 2), mean
    degree log-uniform in [4, 64], mixing 0.3, weights uniform 1..10.
    ``first`` skips the first graphs (graph g is the same in every call)."""
    out = []
    for g in range(first, first + count):
        rng = np.random.default_rng([seed, g])
        n = int(round(_log_uniform(rng, n_lo, n_hi)))
        k = int(round(_log_uniform(rng, 2, 200)))
        k = max(1, min(k, n // 2))
        d = _log_uniform(rng, 4, 64)
        out.append(sbm_sparse(n, k, d, 0.3, 10, rng, (seed << 32) ^ g, f"batch_sbm_{g}"))
    return out


def batch_sbm_sizes(count: int = 4096, seed: int = 1004, n_lo: int = 100, n_hi: int = 100_000) -> np.ndarray:
    """Vertex counts of ``batch_sbm``'s graphs 0..count-1 without building
    them (the first draw of each graph's stream)."""
    return np.array([int(round(_log_uniform(np.random.default_rng([seed, g]), n_lo, n_hi)))
                     for g in range(count)], dtype=np.int64)


def served_chunglu(count: int, seed: int = 1005, first: int = 0, n_lo: int = 1000,
                   n_hi: int = 2_000_000) -> list:
    """Requests of the served workload: Chung-Lu graphs with exponent uniform
    in [2.1, 2.5], n log-uniform in [n_lo, n_hi], mean degree uniform in
    [8, 32], planted blocks of about 4,096 vertices with mixing 0.3 and
    weights uniform 1..50.  Request g draws its parameters from stream
    (seed, g) and its structure from seed (seed << 32) | g."""
    out = []
    for g in range(first, first + count):
        rng = np.random.default_rng([seed, g])
        gamma = float(rng.uniform(2.1, 2.5))
        n = int(round(_log_uniform(rng, n_lo, n_hi)))
        d = float(rng.uniform(8.0, 32.0))
        out.append(chung_lu(n, gamma, d, max(1, n // 4096), 0.3, (seed << 32) | g,
                            lambda h: weights_uniform(h, 50), f"served_{g}"))
    return out


def config(name: str) -> Graph:
    """The synthetic workloads standing in for the paper's test graphs.

    * ``sbm1k``: planted-partition SBM, 1,000 vertices in 10 equal blocks,
      p_in 0.1, p_out 0.005, weights uniform 1..10, seed 1001.
    * ``chunglu1m``: Chung-Lu, n = 2^20, exponent 2.1, mean degree 16,
      256 planted blocks with mixing 0.3, weights 1 + Geometric(0.3)
      failures, seed 1002 (shaped like a co-occurrence landscape).
    * ``rmat24``: R-MAT scale 24, edge factor 16, (0.57, 0.19, 0.19, 0.05),
      weights uniform 1..100, seed 1003 (web / social graph shape).
    """
    if name == "sbm1k":
        return sbm_dense(1000, 10, 0.1, 0.005, 10, 1001, name)
    if name == "chunglu1m":
        return chung_lu(1 << 20, 2.1, 16.0, 256, 0.3, 1002,
                        lambda h: weights_geometric(h, 0.3), name)
    if name == "rmat24":
        return rmat(24, 16, 0.57, 0.19, 0.19, 1003, lambda h: weights_uniform(h, 100), name)
    if name.startswith("chunglu_n"):  # chunglu_n<N>: the chunglu1m recipe at another size
        n = int(name[len("chunglu_n"):])
        return chung_lu(n, 2.1, 16.0, max(1, n // 4096), 0.3, 1002,
                        lambda h: weights_geometric(h, 0.3), name)
    if name.startswith("rmat_s"):  # rmat_s<scale>: the rmat24 recipe at another scale
        s = int(name[len("rmat_s"):])
        return rmat(s, 16, 0.57, 0.19, 0.19, 1003, lambda h: weights_uniform(h, 100), name)
    raise KeyError(name)
