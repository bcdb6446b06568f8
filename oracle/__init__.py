"""CPU oracle of synchronous parallel Louvain -- TEST INFRASTRUCTURE ONLY.

Python access to ``louvain_oracle.c``, a plain C implementation (single
threaded, with an OpenMP variant over vertices that gives the same
results) written from the paper (R. Forster, "Parallel Louvain
Community Detection Optimized for GPUs", arXiv 1805.10904; Section 2
eqs. 1-5, Section 3.1 heuristics, Alg. 1 and Alg. 2, and the renumbering
and graph-rebuilding processes of Section 5.1).  Only ``tests/``, the
``smoke()`` check and the benchmark's CPU-baseline leg may use this
package; the GPU library shares no code with it.

Inputs are numpy arrays: symmetric CSR ``row_ptr`` (int64[n+1]), ``col``
(int32[nnz]) and integer weights (any integer dtype, widened to int64 here).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import NamedTuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "louvain_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liblouvain_oracle.so")
# a test may point the package at another build of the oracle (mutation tests)
_LIB = os.environ.get("LOUVAIN_ORACLE_LIB", _LIB_DEFAULT)

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_ELIMIT = 0, -1, -2, -6


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/liblouvain_oracle.so``."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if _LIB == _LIB_DEFAULT and (not os.path.exists(_LIB)
                                     or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        lib = C.CDLL(_LIB)
        p = C.c_void_p
        i64 = C.c_int64
        lib.orc_degrees.argtypes = [i64, p, p, p, p]
        lib.orc_modularity.argtypes = [i64, p, p, p, p, p, p]
        lib.orc_accept.argtypes = [p, p, i64, i64]
        lib.orc_local_move.argtypes = [i64, p, p, p, p, C.c_int, p, p, p]
        lib.orc_renumber.argtypes = [i64, p, p]
        lib.orc_renumber.restype = i64
        lib.orc_contract.argtypes = [i64, p, p, p, p, i64, p, p, p]
        lib.orc_contract.restype = i64
        lib.orc_louvain.argtypes = [i64, p, p, p, i64, i64, C.c_int32, C.c_int32, C.c_int, C.c_int,
                                    p, p, p, p, p]
        lib.orc_merge.argtypes = [i64, p, p, p, p, C.c_int, p]
        lib.orc_set_threads.argtypes = [C.c_int]
        lib.orc_get_threads.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _csr(row_ptr, col, w):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    wt = np.ascontiguousarray(w, dtype=np.int64)
    n = rp.shape[0] - 1
    if n < 0 or cl.shape[0] != rp[-1] or wt.shape[0] != cl.shape[0]:
        raise ValueError("inconsistent CSR")
    return n, rp, cl, wt


def i128_from_pair(q: np.ndarray) -> int:
    """Python int from the (low, high) int64 words of a 128-bit integer."""
    lo = int(q[0]) & ((1 << 64) - 1)
    hi = int(q[1])
    return (hi << 64) | lo


def i128_to_pair(v: int) -> np.ndarray:
    u = v & ((1 << 128) - 1)
    lo = u & ((1 << 64) - 1)
    hi = u >> 64
    to_s = lambda x: x - (1 << 64) if x >= (1 << 63) else x
    return np.array([to_s(lo), to_s(hi)], dtype=np.int64)


def set_threads(threads: int) -> None:
    """Threads of the OpenMP variant (the sweep's vertex loop and the inner
    weight of eq. 3); 1 = the plain single-threaded oracle.  Results do not
    depend on it."""
    _load().orc_set_threads(int(threads))


def get_threads() -> int:
    return int(_load().orc_get_threads())


def degrees(row_ptr, col, w):
    """(delta int64[n], TW) -- weighted degrees and their sum 2W (Section 2)."""
    n, rp, cl, wt = _csr(row_ptr, col, w)
    d = np.zeros(max(n, 1), np.int64)
    tw = C.c_int64(0)
    _load().orc_degrees(n, _ptr(rp), _ptr(wt), _ptr(d), C.byref(tw))
    return d[:n], tw.value


def modularity(row_ptr, col, w, labels):
    """(Q_int, Q): eq. 3 as the exact integer TW^2 * Q, and Q in float64."""
    n, rp, cl, wt = _csr(row_ptr, col, w)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    q2 = np.zeros(2, np.int64)
    q = C.c_double(0)
    rc = _load().orc_modularity(n, _ptr(rp), _ptr(cl), _ptr(wt), _ptr(lab), _ptr(q2), C.byref(q))
    if rc != ORC_OK:
        raise ValueError(f"orc_modularity failed ({rc})")
    return i128_from_pair(q2), q.value


def accept(q_new: int, q_prev: int, theta_num: int = 1, theta_den: int = 1_000_000) -> bool:
    """The sweep acceptance test: theta_den*(q_new-q_prev) > theta_num*|q_prev|."""
    a = i128_to_pair(q_new)
    b = i128_to_pair(q_prev)
    return bool(_load().orc_accept(_ptr(a), _ptr(b), theta_num, theta_den))


class LocalMove(NamedTuple):
    labels: np.ndarray   # int32[n] decisions of the sweep
    deg: np.ndarray      # int64[n] deg_C of the new labelling, indexed by label
    e_own: np.ndarray    # int64[n] e_{i->labels_in[i]} including i's loop


def local_move(row_ptr, col, w, labels_in=None, singlet_rule: bool = True) -> LocalMove:
    """One synchronous sweep of Alg. 1 from ``labels_in`` (None = singletons)."""
    n, rp, cl, wt = _csr(row_ptr, col, w)
    nn = max(n, 1)
    lin = None if labels_in is None else np.ascontiguousarray(labels_in, dtype=np.int32)
    out = np.zeros(nn, np.int32)
    deg = np.zeros(nn, np.int64)
    eown = np.zeros(nn, np.int64)
    rc = _load().orc_local_move(n, _ptr(rp), _ptr(cl), _ptr(wt),
                                None if lin is None else _ptr(lin), int(bool(singlet_rule)),
                                _ptr(out), _ptr(deg), _ptr(eown))
    if rc != ORC_OK:
        raise ValueError(f"orc_local_move failed ({rc})")
    return LocalMove(out[:n], deg[:n], eown[:n])


def renumber(labels):
    """(map int32[n] indexed by label (-1 where absent), n_communities)."""
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    n = lab.shape[0]
    m = np.zeros(max(n, 1), np.int32)
    k = _load().orc_renumber(n, _ptr(lab), _ptr(m))
    return m[:n], int(k)


def contract(row_ptr, col, w, new_labels, n_new: int):
    """Graph rebuilding: (row_ptr', col', w' int64) of the contracted graph
    whose vertex a is the set {i : new_labels[i] == a}."""
    n, rp, cl, wt = _csr(row_ptr, col, w)
    nl = np.ascontiguousarray(new_labels, dtype=np.int32)
    nnz = cl.shape[0]
    rp2 = np.zeros(n_new + 1, np.int64)
    cl2 = np.zeros(max(nnz, 1), np.int32)
    wt2 = np.zeros(max(nnz, 1), np.int64)
    m = _load().orc_contract(n, _ptr(rp), _ptr(cl), _ptr(wt), _ptr(nl), n_new,
                             _ptr(rp2), _ptr(cl2), _ptr(wt2))
    if m < 0:
        raise MemoryError("orc_contract")
    return rp2, cl2[:m].copy(), wt2[:m].copy()


class _LevelStats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("sweeps_executed", C.c_int32),
                ("sweeps_accepted", C.c_int32), ("q_int", C.c_int64 * 2)]


class RunResult(NamedTuple):
    labels: np.ndarray     # int32[n] final dense community IDs
    q_int: int             # TW^2 * Q of the final partition
    q: float
    levels: list           # per-level dicts: n, nnz, sweeps_executed, sweeps_accepted, q_int
    status: int            # ORC_OK or ORC_ELIMIT


def merge(row_ptr, col, w, labels, singlet_rule: bool = True) -> np.ndarray:
    """The final merge of a phase alone (Section 5.1): vertices alone in
    their community whose neighbours all carry one label join it when that
    beats staying (as a sweep decides, singlet rule included)."""
    n, rp, cl, wt = _csr(row_ptr, col, w)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.zeros(max(n, 1), np.int32)
    rc = _load().orc_merge(n, _ptr(rp), _ptr(cl), _ptr(wt), _ptr(lab), int(bool(singlet_rule)), _ptr(out))
    if rc != ORC_OK:
        raise ValueError(f"orc_merge failed ({rc})")
    return out[:n]


def louvain(row_ptr, col, w, theta_num: int = 1, theta_den: int = 1_000_000,
            max_sweeps: int = 1000, max_levels: int = 64, singlet_rule: bool = True,
            merge: bool = False) -> RunResult:
    """The whole method (Alg. 2 over Alg. 1 phases), single-threaded; merge:
    apply the final merge after every phase that kept a sweep."""
    n, rp, cl, wt = _csr(row_ptr, col, w)
    lab = np.zeros(max(n, 1), np.int32)
    q2 = np.zeros(2, np.int64)
    q = C.c_double(0)
    stats = (_LevelStats * max(1, max_levels))()
    levels = C.c_int32(0)
    rc = _load().orc_louvain(n, _ptr(rp), _ptr(cl), _ptr(wt), theta_num, theta_den,
                             max_sweeps, max_levels, int(bool(singlet_rule)), int(bool(merge)), _ptr(lab),
                             _ptr(q2), C.byref(q), C.cast(stats, C.c_void_p), C.byref(levels))
    if rc not in (ORC_OK, ORC_ELIMIT):
        raise RuntimeError(f"orc_louvain failed ({rc})")
    lv = [dict(n=s.n, nnz=s.nnz, sweeps_executed=s.sweeps_executed,
               sweeps_accepted=s.sweeps_accepted, q_int=i128_from_pair(np.array(s.q_int[:])))
          for s in stats[:levels.value]]
    return RunResult(lab[:n], i128_from_pair(q2), q.value, lv, rc)


class Dendro(NamedTuple):
    maps: list         # map l (int32[n_l]): vertex of level l's graph -> vertex of level l+1's
    graphs: list       # (row_ptr, col, w int64) of levels 0 .. len(maps)
    labels: np.ndarray # int32[n] composition of the maps
    q_int: int         # Q_int of labels on the input graph
    levels: list       # per-phase records, as louvain()'s
    status: int        # ORC_OK or ORC_ELIMIT


def dendrogram(row_ptr, col, w, theta_num: int = 1, theta_den: int = 1_000_000,
               max_sweeps: int = 1000, max_levels: int = 64, singlet_rule: bool = True,
               merge: bool = False) -> Dendro:
    """Alg. 2 taken level by level, keeping every level of the dendrogram:
    a phase (Alg. 1 from singletons on the level's graph) and its
    renumbering give the level's map; the graph rebuilt from that map is the
    next level's graph.  The last graph is the one a further phase would run
    on: the graph of the phase that kept no sweep, or the contraction by the
    last map when max_levels cuts the run short."""
    n, rp, cl, wt = _csr(row_ptr, col, w)
    graphs = [(rp, cl, wt)]
    maps, levels = [], []
    lab = np.arange(n, dtype=np.int32)
    status = ORC_OK
    _, tw = degrees(rp, cl, wt)
    q_int = modularity(rp, cl, wt, lab)[0] if tw > 0 else 0
    while tw > 0 and len(levels) < max_levels:
        g = graphs[-1]
        # one phase and its renumbering: louvain() cut after one level
        r = louvain(*g, theta_num=theta_num, theta_den=theta_den, max_sweeps=max_sweeps, max_levels=1,
                    singlet_rule=singlet_rule, merge=merge)
        rec = r.levels[0]
        levels.append(rec)
        if rec["sweeps_accepted"] >= max_sweeps:
            status = ORC_ELIMIT
        q_int = rec["q_int"]
        if rec["sweeps_accepted"] == 0:
            break
        m = r.labels
        k = int(m.max()) + 1 if m.shape[0] else 0
        maps.append(m)
        lab = m[lab]
        graphs.append(contract(*g, m, k))
        if len(levels) >= max_levels:
            status = ORC_ELIMIT
    return Dendro(maps, graphs, lab, q_int, levels, status)
