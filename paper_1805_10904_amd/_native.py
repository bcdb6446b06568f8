"""ctypes binding of the C ABI in include/louvain.h (marshalling only)."""
from __future__ import annotations

import ctypes as C
import os
from typing import NamedTuple, Optional

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblouvain_hip.so")

LOUVAIN_OK = 0
LOUVAIN_EINVAL = -1
LOUVAIN_ENOMEM = -2
LOUVAIN_EDEVICE = -3
LOUVAIN_EAGAIN = -4
LOUVAIN_EBUSY = -5
LOUVAIN_ELIMIT = -6
LOUVAIN_EOVERFLOW = -7

LOUVAIN_DEVICE_PTRS = 0x1
LOUVAIN_CHECK_SYMMETRY = 0x2
LOUVAIN_NO_SINGLET = 0x4
LOUVAIN_WEIGHTS_I64 = 0x8

# Every symbol the header declares (checked by the CPU test-suite).
ABI_SYMBOLS = (
    "louvain_ctx_create", "louvain_ctx_destroy", "louvain_last_error", "louvain_memory_stats",
    "louvain_memory_reset_peak",
    "louvain_graph_create", "louvain_graph_destroy", "louvain_graph_info", "louvain_graph_export",
    "louvain_local_move", "louvain_modularity", "louvain_modularity_noalloc", "louvain_aggregate", "louvain_run", "louvain_run_batch",
    "louvain_workspace_bytes", "louvain_serve_budget", "louvain_submit", "louvain_poll",
    "louvain_set_tuning", "louvain_get_tuning", "louvain_autotune", "louvain_autotune_batch",
    "louvain_run_dendro", "louvain_dendro_info", "louvain_dendro_map", "louvain_dendro_graph",
    "louvain_dendro_destroy", "louvain_resume",
)


class louvain_i128(C.Structure):
    _fields_ = [("lo", C.c_uint64), ("hi", C.c_int64)]

    def value(self) -> int:
        return (int(self.hi) << 64) | int(self.lo)


class louvain_memory(C.Structure):
    _fields_ = [("pool_bytes", C.c_uint64), ("pool_in_use", C.c_uint64), ("pool_high_water", C.c_uint64),
                ("live_bytes", C.c_uint64), ("cached_bytes", C.c_uint64)]


class louvain_params(C.Structure):
    _fields_ = [("theta_num", C.c_int64), ("theta_den", C.c_int64), ("max_sweeps", C.c_int32),
                ("max_levels", C.c_int32), ("singlet_rule", C.c_int32), ("pass_batch", C.c_int32),
                ("merge", C.c_int32), ("reserved", C.c_int32)]


class louvain_level_stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz", C.c_int64), ("sweeps_executed", C.c_int32),
                ("sweeps_accepted", C.c_int32), ("gpu_passes", C.c_int32), ("reserved", C.c_int32),
                ("q_int", louvain_i128), ("ms_sweep", C.c_double), ("ms_contract", C.c_double)]


class louvain_kernel_stats(C.Structure):
    _fields_ = [("name", C.c_char * 40), ("launches", C.c_int64), ("ms", C.c_double),
                ("alg_bytes", C.c_double)]


class louvain_request_result(C.Structure):
    _fields_ = [("status", C.c_int32), ("levels", C.c_int32), ("n", C.c_int64), ("nnz", C.c_int64),
                ("total_edges_swept", C.c_int64), ("q_int", louvain_i128), ("q", C.c_double),
                ("t_submit_us", C.c_double), ("t_admit_us", C.c_double), ("t_done_us", C.c_double),
                ("level", louvain_level_stats * 64), ("error", C.c_char * 128)]


class louvain_tuning(C.Structure):
    _fields_ = [("small_max", C.c_int32), ("block_max", C.c_int32), ("pass_batch", C.c_int32),
                ("group_slots", C.c_int32), ("group_vertices", C.c_int32), ("overlap", C.c_int32),
                ("reorder", C.c_int32), ("group_tiles", C.c_int32), ("ms", C.c_double)]


class louvain_run_stats(C.Structure):
    _fields_ = [("timing", C.c_int32), ("levels", C.c_int32), ("status", C.c_int32),
                ("n_kernels", C.c_int32), ("total_edges_swept", C.c_int64), ("ms_total", C.c_double),
                ("level", louvain_level_stats * 64), ("kernels", louvain_kernel_stats * 64),
                ("timing_only", C.c_char * 40)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run paper_1805_10904_amd/build.py or __graft_entry__.build())")
    # torch ships its own HIP runtime under the same soname; load it first so
    # that the library and torch share one runtime (device memory, streams).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    p, i64, u32, i32 = C.c_void_p, C.c_int64, C.c_uint32, C.c_int
    lib.louvain_ctx_create.argtypes = [i32, p, p, C.c_size_t, C.c_char_p, C.POINTER(p)]
    lib.louvain_memory_stats.argtypes = [p, C.POINTER(louvain_memory)]
    lib.louvain_memory_reset_peak.argtypes = [p]
    lib.louvain_ctx_destroy.argtypes = [p]
    lib.louvain_last_error.argtypes = [p]
    lib.louvain_last_error.restype = C.c_char_p
    lib.louvain_graph_create.argtypes = [p, i64, i64, p, p, p, u32, C.POINTER(p)]
    lib.louvain_graph_destroy.argtypes = [p]
    lib.louvain_graph_info.argtypes = [p, p, p, p]
    lib.louvain_graph_export.argtypes = [p, p, p, p, u32]
    lib.louvain_local_move.argtypes = [p, p, p, p, p, p, u32]
    lib.louvain_modularity.argtypes = [p, p, p, C.POINTER(louvain_i128), p, u32]
    lib.louvain_modularity_noalloc.argtypes = [p, p, p, C.POINTER(louvain_i128), p, u32]
    lib.louvain_aggregate.argtypes = [p, p, p, p, C.POINTER(p), u32]
    lib.louvain_run.argtypes = [p, p, C.POINTER(louvain_params), p, C.POINTER(louvain_i128), p,
                                C.POINTER(louvain_run_stats), u32]
    lib.louvain_run_batch.argtypes = [p, i64, p, C.POINTER(louvain_params), p, p, p, p, p, u32]
    lib.louvain_set_tuning.argtypes = [p, C.POINTER(louvain_tuning)]
    lib.louvain_get_tuning.argtypes = [p, C.POINTER(louvain_tuning)]
    lib.louvain_autotune.argtypes = [p, p, C.POINTER(louvain_params), C.POINTER(louvain_tuning)]
    lib.louvain_autotune_batch.argtypes = [p, i64, p, C.POINTER(louvain_params), C.POINTER(louvain_tuning)]
    lib.louvain_workspace_bytes.argtypes = [i64, i64]
    lib.louvain_workspace_bytes.restype = C.c_size_t
    lib.louvain_serve_budget.argtypes = [p, C.c_size_t]
    lib.louvain_submit.argtypes = [p, i64, i64, p, p, p, C.POINTER(louvain_params), p, u32, C.POINTER(C.c_uint64)]
    lib.louvain_poll.argtypes = [p, C.c_uint64, C.c_int32, C.POINTER(louvain_request_result)]
    lib.louvain_run_dendro.argtypes = [p, p, C.POINTER(louvain_params), p, C.POINTER(louvain_i128), p,
                                       C.POINTER(louvain_run_stats), C.POINTER(p), u32]
    lib.louvain_dendro_info.argtypes = [p, p, p]
    lib.louvain_dendro_map.argtypes = [p, i32, p, u32]
    lib.louvain_dendro_graph.argtypes = [p, C.POINTER(p)]
    lib.louvain_dendro_destroy.argtypes = [p]
    lib.louvain_resume.argtypes = [p, p, C.POINTER(louvain_params), i32, i64, p, p, C.POINTER(louvain_i128), p,
                                   C.POINTER(louvain_run_stats), u32]
    for f in ABI_SYMBOLS:
        if f not in ("louvain_last_error", "louvain_workspace_bytes"):
            getattr(lib, f).restype = C.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def exported_symbols(path: str = LIB_PATH):
    """Names of the ABI functions the library exports (via the dynamic loader)."""
    lib = C.CDLL(path)
    return [f for f in ABI_SYMBOLS if hasattr(lib, f)]


class LouvainError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"louvain error {code}: {msg}")
        self.code = code


# ------------------------------------------------------------- marshalling --

_NP_OF = {"int32": np.int32, "int64": np.int64}


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x):
    if x is None:
        return None
    if _is_torch(x):
        return C.c_void_p(x.data_ptr())
    return x.ctypes.data_as(C.c_void_p)


def _bad(msg: str):
    raise LouvainError(LOUVAIN_EINVAL, msg)


def _is_dev(x) -> bool:
    return _is_torch(x) and x.is_cuda


def _arg(x, name: str, dtype: str, length: Optional[int], dev: bool, device: int, output: bool = False):
    """Check one array argument before it reaches the library and return the
    object whose memory the library is given.

    dev=True: x must be a 1-D contiguous torch CUDA tensor on `device` of
    dtype `dtype` with `length` elements.  dev=False: host memory; inputs
    are coerced to a contiguous numpy array of `dtype` (integer values only,
    none outside the dtype's range), outputs must already be a writable
    contiguous numpy array of that dtype.  Anything else raises
    LouvainError(EINVAL) without calling the library."""
    if dev:
        import torch
        if not _is_dev(x):
            _bad(f"{name}: expected a torch CUDA tensor (device pointers), got {type(x).__name__}")
        if x.device.index != device:
            _bad(f"{name}: tensor on cuda:{x.device.index}, the context is on device {device}")
        if x.dtype != getattr(torch, dtype):
            _bad(f"{name}: dtype {x.dtype}, expected torch.{dtype}")
        if x.dim() != 1 or not x.is_contiguous():
            _bad(f"{name}: expected a contiguous 1-D tensor")
        if length is not None and x.numel() != length:
            _bad(f"{name}: {x.numel()} elements, expected {length}")
        return x
    if _is_dev(x):
        _bad(f"{name}: a CUDA tensor where host arrays are expected (all arrays of a call are of one kind)")
    if _is_torch(x):
        x = x.numpy()
    want = np.dtype(_NP_OF[dtype])
    if output:
        if not isinstance(x, np.ndarray) or x.dtype != want or x.ndim != 1 or not x.flags.c_contiguous \
                or not x.flags.writeable:
            _bad(f"{name}: expected a writable contiguous 1-D numpy array of {dtype}")
    else:
        a = np.asarray(x)
        if a.size and a.dtype.kind not in "iu":
            _bad(f"{name}: expected integers, got dtype {a.dtype}")
        if a.ndim != 1:
            _bad(f"{name}: expected a 1-D array")
        if a.dtype != want and a.size:
            info = np.iinfo(want)
            if int(a.min()) < info.min or int(a.max()) > info.max:
                _bad(f"{name}: values outside the range of {dtype}")
        x = np.ascontiguousarray(a, dtype=want)
    if length is not None and x.shape[0] != length:
        _bad(f"{name}: {x.shape[0]} elements, expected {length}")
    return x


def _weights_wide(w) -> bool:
    """int64 weights are passed as they are (LOUVAIN_WEIGHTS_I64); anything
    else as int32."""
    if _is_torch(w):
        return str(w.dtype) == "torch.int64"
    return np.asarray(w).dtype == np.int64


def _empty_like_kind(ref_is_dev, n, dtype_np, device=None):
    if ref_is_dev:
        import torch
        tdt = {np.int32: torch.int32, np.int64: torch.int64}[dtype_np]
        return torch.empty(max(n, 0), dtype=tdt, device=device)
    return np.empty(max(n, 0), dtype=dtype_np)


class RunResult(NamedTuple):
    labels: object       # int32[n] final dense community IDs (numpy or torch)
    q_int: int           # TW^2 * Q, exact
    q: float
    status: int          # LOUVAIN_OK or LOUVAIN_ELIMIT
    stats: dict


class ServeResult(NamedTuple):
    labels: object       # int32[n] final dense community IDs (numpy or torch)
    q_int: int
    q: float
    status: int          # LOUVAIN_OK, LOUVAIN_ELIMIT or the request's error
    levels: list         # per-level records
    total_edges_swept: int
    t_submit_us: float   # library steady clock
    t_admit_us: float
    t_done_us: float
    error: str


def workspace_bytes(n: int, nnz: int) -> int:
    """Device bytes the request loop budgets for a graph of n vertices and nnz entries."""
    return int(load_library().louvain_workspace_bytes(n, nnz))


class Graph:
    """A device-resident graph handle (louvain_graph)."""

    def __init__(self, ctx: "Context", handle: C.c_void_p, device_kind: bool):
        self.ctx = ctx
        self.h = handle
        self.dev = device_kind

    def info(self):
        n, m, tw = C.c_int64(), C.c_int64(), C.c_int64()
        self.ctx._check(self.ctx.lib.louvain_graph_info(self.h, C.byref(n), C.byref(m), C.byref(tw)))
        return n.value, m.value, tw.value

    def export(self, device: bool = False):
        n, m, _ = self.info()
        rp = _empty_like_kind(device, n + 1, np.int64, self.ctx.torch_device)
        col = _empty_like_kind(device, m, np.int32, self.ctx.torch_device)
        w = _empty_like_kind(device, m, np.int64, self.ctx.torch_device)
        self.ctx._check(self.ctx.lib.louvain_graph_export(
            self.h, _ptr(rp), _ptr(col), _ptr(w), LOUVAIN_DEVICE_PTRS if device else 0))
        return rp, col, w

    def destroy(self):
        if self.h:
            self.ctx.lib.louvain_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Dendrogram:
    """A run's dendrogram (louvain_dendro): the map of every level and the
    graph a further phase would run on."""

    def __init__(self, ctx: "Context", handle: C.c_void_p, device_kind: bool):
        self.ctx = ctx
        self.h = handle
        self.dev = device_kind
        levels = C.c_int32()
        sizes = (C.c_int64 * 65)()
        ctx._check(ctx.lib.louvain_dendro_info(self.h, C.byref(levels), sizes))
        self.levels = levels.value
        self.n = [sizes[i] for i in range(self.levels + 1)]

    def map(self, level: int, device: Optional[bool] = None):
        """Map `level`: int32[n[level]], vertex -> vertex of the next level's graph."""
        dev = self.dev if device is None else device
        out = _empty_like_kind(dev, self.n[level] if 0 <= level < self.levels else 0, np.int32,
                               self.ctx.torch_device)
        self.ctx._check(self.ctx.lib.louvain_dendro_map(self.h, level, _ptr(out), LOUVAIN_DEVICE_PTRS if dev else 0))
        return out

    def graph(self) -> "Graph":
        """The last level's graph (once; the caller owns it)."""
        h = C.c_void_p()
        self.ctx._check(self.ctx.lib.louvain_dendro_graph(self.h, C.byref(h)))
        return Graph(self.ctx, h, self.dev)

    def destroy(self):
        if self.h:
            self.ctx.lib.louvain_dendro_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Context:
    """A louvain_ctx on one HIP device, enqueuing on the given stream handle
    (default: torch's current stream on that device when torch has a GPU,
    else the null stream).

    pool_bytes: when given, a torch uint8 tensor of that many bytes is
    allocated on the device and handed to the library, which then takes
    every device buffer from it (LOUVAIN_ENOMEM when it runs out) and
    allocates no device memory itself; the tensor lives as long as the
    context.  tuning_path: a file of launch shapes, read when it exists and
    rewritten by autotune()."""

    def __init__(self, device: int = 0, stream: Optional[int] = None, pool_bytes: Optional[int] = None,
                 tuning_path: Optional[str] = None):
        self.lib = load_library()
        self.device = device
        self.torch_device = None
        self.pool = None
        try:
            import torch
            self.torch_device = torch.device("cuda", device)
            if stream is None and torch.cuda.is_available():
                stream = torch.cuda.current_stream(self.torch_device).cuda_stream
        except ImportError:
            pass
        pool_ptr = None
        if pool_bytes is not None:
            if int(pool_bytes) <= 0:
                _bad("pool_bytes must be positive")
            import torch
            self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8, device=self.torch_device)
            torch.cuda.synchronize(self.torch_device)
            pool_ptr = self.pool.data_ptr()
        h = C.c_void_p()
        path = tuning_path.encode() if tuning_path else None
        rc = self.lib.louvain_ctx_create(device, C.c_void_p(stream or 0), C.c_void_p(pool_ptr),
                                         int(pool_bytes or 0), path, C.byref(h))
        if rc != LOUVAIN_OK:
            raise LouvainError(rc, "louvain_ctx_create failed")
        self.h = h
        self._inflight = {}

    def memory(self) -> dict:
        """Device-memory accounting (louvain_memory_stats)."""
        m = louvain_memory()
        self._check(self.lib.louvain_memory_stats(self.h, C.byref(m)))
        return {k: int(getattr(m, k)) for k, _ in m._fields_}

    def reset_peak(self):
        self._check(self.lib.louvain_memory_reset_peak(self.h))

    def _check(self, rc: int, ok=(LOUVAIN_OK,)):
        if rc not in ok:
            msg = self.lib.louvain_last_error(self.h)
            raise LouvainError(rc, msg.decode() if msg else "")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self._check(self.lib.louvain_ctx_destroy(self.h))
            self.h = None
        # self.pool stays referenced: graphs made on the context (which keep
        # the context object alive) may still hold blocks of it

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ---------------------------------------------------------------

    def _csr(self, row_ptr, col, w):
        """Checked CSR arguments: (dev, n, nnz, wide, row_ptr, col, w)."""
        dev = _is_dev(row_ptr)
        if row_ptr is None or col is None or w is None:
            _bad("row_ptr, col and w must be given")
        n = int(row_ptr.shape[0]) - 1 if hasattr(row_ptr, "shape") else len(row_ptr) - 1
        if n < 0:
            _bad("row_ptr needs at least one element")
        nnz = int(col.shape[0]) if hasattr(col, "shape") else len(col)
        wide = _weights_wide(w)
        row_ptr = _arg(row_ptr, "row_ptr", "int64", n + 1, dev, self.device)
        col = _arg(col, "col", "int32", nnz, dev, self.device)
        w = _arg(w, "w", "int64" if wide else "int32", nnz, dev, self.device)
        return dev, n, nnz, wide, row_ptr, col, w

    def graph_create(self, row_ptr, col, w, check_symmetry: bool = False) -> Graph:
        """Copy a symmetric CSR graph (numpy arrays or torch CUDA tensors, all
        of one kind) into the library."""
        dev, n, nnz, wide, row_ptr, col, w = self._csr(row_ptr, col, w)
        flags = (LOUVAIN_DEVICE_PTRS if dev else 0) | (LOUVAIN_CHECK_SYMMETRY if check_symmetry else 0) \
            | (LOUVAIN_WEIGHTS_I64 if wide else 0)
        h = C.c_void_p()
        self._check(self.lib.louvain_graph_create(self.h, n, nnz, _ptr(row_ptr), _ptr(col),
                                                  _ptr(w), flags, C.byref(h)))
        return Graph(self, h, dev)

    def set_tuning(self, small_max: int = 4, block_max: int = 2730, pass_batch: int = 2, group_slots: int = 4,
                   group_vertices: int = 1, overlap: int = 0, reorder: int = 0, group_tiles: int = 1):
        """Launch shapes of compact levels and the level-0 vertex order
        (0 auto, 1 by row length, 2 as given); results do not depend on them."""
        t = louvain_tuning(small_max, block_max, pass_batch, group_slots, group_vertices, overlap, reorder,
                           group_tiles, 0.0)
        self._check(self.lib.louvain_set_tuning(self.h, C.byref(t)))

    def get_tuning(self) -> dict:
        t = louvain_tuning()
        self._check(self.lib.louvain_get_tuning(self.h, C.byref(t)))
        return dict(small_max=t.small_max, block_max=t.block_max, pass_batch=t.pass_batch,
                    group_slots=t.group_slots, group_vertices=t.group_vertices, overlap=t.overlap,
                    reorder=t.reorder, group_tiles=t.group_tiles)

    def autotune(self, g: "Graph", theta_num: int = 1, theta_den: int = 1_000_000, max_sweeps: int = 1000,
                 max_levels: int = 64, singlet_rule: bool = True) -> dict:
        """Time whole runs of g under the candidate launch shapes; the fastest becomes the context's."""
        prm = louvain_params(theta_num, theta_den, max_sweeps, max_levels, 1 if singlet_rule else 0, 0)
        t = louvain_tuning()
        self._check(self.lib.louvain_autotune(self.h, g.h, C.byref(prm), C.byref(t)))
        return dict(small_max=t.small_max, block_max=t.block_max, pass_batch=t.pass_batch,
                    group_slots=t.group_slots, group_vertices=t.group_vertices, overlap=t.overlap,
                    reorder=t.reorder, group_tiles=t.group_tiles, ms=t.ms)

    def autotune_batch(self, graphs, theta_num: int = 1, theta_den: int = 1_000_000, max_sweeps: int = 1000,
                       max_levels: int = 64, singlet_rule: bool = True) -> dict:
        """Tune the launch shapes on a batched call over these graphs (coordinate
        descent over every shape field); the pick becomes the context's."""
        prm = louvain_params(theta_num, theta_den, max_sweeps, max_levels, 1 if singlet_rule else 0, 0)
        hs = (C.c_void_p * len(graphs))(*[g.h for g in graphs])
        t = louvain_tuning()
        self._check(self.lib.louvain_autotune_batch(self.h, len(graphs), hs, C.byref(prm), C.byref(t)))
        return dict(small_max=t.small_max, block_max=t.block_max, pass_batch=t.pass_batch,
                    group_slots=t.group_slots, group_vertices=t.group_vertices, overlap=t.overlap,
                    reorder=t.reorder, group_tiles=t.group_tiles, ms=t.ms)

    def serve_budget(self, nbytes: int):
        """Device-memory budget of the request loop (0: 80% of free memory at start)."""
        self._check(self.lib.louvain_serve_budget(self.h, int(nbytes)))

    def submit(self, row_ptr, col, w, theta_num: int = 1, theta_den: int = 1_000_000, max_sweeps: int = 1000,
               max_levels: int = 64, singlet_rule: bool = True, pass_batch: int = 0, labels_out=None,
               merge: bool = False,
               check_symmetry: bool = False) -> int:
        """Queue one graph for the request loop; returns a ticket for poll().

        The arrays are kept referenced until the result is polled.  Device
        (torch) inputs must be complete on their streams before the call."""
        dev, n, nnz, wide, row_ptr, col, w = self._csr(row_ptr, col, w)
        if labels_out is None:
            out = _empty_like_kind(dev, n, np.int32, self.torch_device)
        else:
            out = _arg(labels_out, "labels_out", "int32", n, dev, self.device, output=True)
        flags = (LOUVAIN_DEVICE_PTRS if dev else 0) | (LOUVAIN_CHECK_SYMMETRY if check_symmetry else 0) \
            | (LOUVAIN_WEIGHTS_I64 if wide else 0)
        prm = louvain_params(theta_num, theta_den, max_sweeps, max_levels, 1 if singlet_rule else 0, pass_batch,
                             1 if merge else 0)
        t = C.c_uint64()
        rc = self.lib.louvain_submit(self.h, n, nnz, _ptr(row_ptr), _ptr(col), _ptr(w), C.byref(prm), _ptr(out),
                                     flags, C.byref(t))
        if rc != LOUVAIN_OK:
            raise LouvainError(rc, "submit rejected the request")
        self._inflight[t.value] = (row_ptr, col, w, out)
        return t.value

    def poll(self, ticket: int, wait_us: int = 0) -> Optional["ServeResult"]:
        """None while pending; the ServeResult once done (the ticket is then retired).
        A failed request is returned with its status and error text."""
        res = louvain_request_result()
        rc = self.lib.louvain_poll(self.h, ticket, int(wait_us), C.byref(res))
        if rc == LOUVAIN_EAGAIN:
            return None
        if rc == LOUVAIN_EINVAL and ticket not in self._inflight:
            raise LouvainError(rc, f"unknown ticket {ticket}")
        keep = self._inflight.pop(ticket)
        levels = [dict(n=lv.n, nnz=lv.nnz, sweeps_executed=lv.sweeps_executed, sweeps_accepted=lv.sweeps_accepted,
                       gpu_passes=lv.gpu_passes, q_int=lv.q_int.value()) for lv in res.level[:res.levels]]
        return ServeResult(keep[3], res.q_int.value(), res.q, rc, levels, res.total_edges_swept,
                           res.t_submit_us, res.t_admit_us, res.t_done_us, res.error.decode(errors="replace"))

    def _labels(self, labels, dev, n, name="labels"):
        if labels is None:
            return None
        return _arg(labels, name, "int32", n, dev, self.device)

    def local_move(self, g: Graph, labels=None, singlet_rule: bool = True, device: Optional[bool] = None):
        """One synchronous sweep: (labels_out, deg_C of labels_out, e_own)."""
        dev = g.dev if device is None else device
        n, _, _ = g.info()
        lab = self._labels(labels, dev, n)
        out = _empty_like_kind(dev, n, np.int32, self.torch_device)
        deg = _empty_like_kind(dev, n, np.int64, self.torch_device)
        eown = _empty_like_kind(dev, n, np.int64, self.torch_device)
        flags = (LOUVAIN_DEVICE_PTRS if dev else 0) | (0 if singlet_rule else LOUVAIN_NO_SINGLET)
        self._check(self.lib.louvain_local_move(self.h, g.h, _ptr(lab), _ptr(out), _ptr(deg), _ptr(eown), flags))
        return out, deg, eown

    def modularity(self, g: Graph, labels, device: Optional[bool] = None):
        """(Q_int, Q) of a labelling (eq. 3)."""
        dev = g.dev if device is None else device
        n, _, _ = g.info()
        if labels is None:
            _bad("labels must be given")
        lab = self._labels(labels, dev, n)
        qi = louvain_i128()
        q = C.c_double()
        self._check(self.lib.louvain_modularity(self.h, g.h, _ptr(lab), C.byref(qi), C.byref(q),
                                                LOUVAIN_DEVICE_PTRS if dev else 0))
        return qi.value(), q.value

    def modularity_noalloc(self, g: Graph, labels, device: Optional[bool] = None):
        """(Q_int, Q) as modularity(), computed in the library's fixed device
        scratch array without any device allocation (graphs of at most
        LOUVAIN_NOALLOC_MAX_N vertices)."""
        dev = g.dev if device is None else device
        n, _, _ = g.info()
        if labels is None:
            _bad("labels must be given")
        lab = self._labels(labels, dev, n)
        qi = louvain_i128()
        q = C.c_double()
        self._check(self.lib.louvain_modularity_noalloc(self.h, g.h, _ptr(lab), C.byref(qi), C.byref(q),
                                                        LOUVAIN_DEVICE_PTRS if dev else 0))
        return qi.value(), q.value

    def aggregate(self, g: Graph, labels, device: Optional[bool] = None):
        """(contracted Graph, renumbered community of every vertex)."""
        dev = g.dev if device is None else device
        n, _, _ = g.info()
        if labels is None:
            _bad("labels must be given")
        lab = self._labels(labels, dev, n)
        ren = _empty_like_kind(dev, n, np.int32, self.torch_device)
        h = C.c_void_p()
        self._check(self.lib.louvain_aggregate(self.h, g.h, _ptr(lab), _ptr(ren), C.byref(h),
                                               LOUVAIN_DEVICE_PTRS if dev else 0))
        return Graph(self, h, dev), ren

    @staticmethod
    def _timing_stats(timing) -> louvain_run_stats:
        st = louvain_run_stats()
        if isinstance(timing, str):
            st.timing = 2
            st.timing_only = timing.encode()[:39]
        else:
            st.timing = 1 if timing else 0
        return st

    def run(self, g: Graph, theta_num: int = 1, theta_den: int = 1_000_000, max_sweeps: int = 1000,
            max_levels: int = 64, singlet_rule: bool = True, pass_batch: int = 0, timing=False,
            device: Optional[bool] = None, labels_out=None, dendrogram: bool = False, merge: bool = False):
        """The whole method (Alg. 2 over Alg. 1 phases).

        timing: False, True (device time of every launch, from HIP events
        filled by the dispatches) or a kernel name as it appears in
        stats["kernels"] (only its launches are timed).
        dendrogram: also keep the per-level maps and the last level's graph;
        returns (RunResult, Dendrogram) then.
        merge: apply the final merge after every phase that kept a sweep."""
        dev = g.dev if device is None else device
        n, _, _ = g.info()
        if labels_out is None:
            out = _empty_like_kind(dev, n, np.int32, self.torch_device)
        else:
            out = _arg(labels_out, "labels_out", "int32", n, dev, self.device, output=True)
        prm = louvain_params(theta_num, theta_den, max_sweeps, max_levels, 1 if singlet_rule else 0, pass_batch,
                             1 if merge else 0)
        qi = louvain_i128()
        q = C.c_double()
        st = self._timing_stats(timing)
        flags = LOUVAIN_DEVICE_PTRS if dev else 0
        if dendrogram:
            h = C.c_void_p()
            rc = self._check(self.lib.louvain_run_dendro(self.h, g.h, C.byref(prm), _ptr(out), C.byref(qi),
                                                         C.byref(q), C.byref(st), C.byref(h), flags),
                             ok=(LOUVAIN_OK, LOUVAIN_ELIMIT))
            return RunResult(out, qi.value(), q.value, rc, stats_dict(st)), Dendrogram(self, h, dev)
        rc = self._check(self.lib.louvain_run(self.h, g.h, C.byref(prm), _ptr(out), C.byref(qi), C.byref(q),
                                              C.byref(st), flags),
                         ok=(LOUVAIN_OK, LOUVAIN_ELIMIT))
        return RunResult(out, qi.value(), q.value, rc, stats_dict(st))

    def resume(self, g_level: Graph, levels_done: int, labels_so_far, theta_num: int = 1,
               theta_den: int = 1_000_000, max_sweeps: int = 1000, max_levels: int = 64, singlet_rule: bool = True,
               pass_batch: int = 0, timing=False, device: Optional[bool] = None, merge: bool = False) -> RunResult:
        """Continue a run from the graph of level `levels_done` and the labels
        so far (one per original vertex); the result equals one run's."""
        dev = g_level.dev if device is None else device
        if labels_so_far is None:
            _bad("labels_so_far must be given")
        lab = self._labels(labels_so_far, dev, None, "labels_so_far")
        n0 = int(lab.shape[0])
        out = _empty_like_kind(dev, n0, np.int32, self.torch_device)
        prm = louvain_params(theta_num, theta_den, max_sweeps, max_levels, 1 if singlet_rule else 0, pass_batch,
                             1 if merge else 0)
        qi = louvain_i128()
        q = C.c_double()
        st = self._timing_stats(timing)
        rc = self._check(self.lib.louvain_resume(self.h, g_level.h, C.byref(prm), levels_done, n0, _ptr(lab),
                                                 _ptr(out), C.byref(qi), C.byref(q), C.byref(st),
                                                 LOUVAIN_DEVICE_PTRS if dev else 0),
                         ok=(LOUVAIN_OK, LOUVAIN_ELIMIT))
        return RunResult(out, qi.value(), q.value, rc, stats_dict(st))


    def run_batch(self, graphs, theta_num: int = 1, theta_den: int = 1_000_000, max_sweeps: int = 1000,
                  max_levels: int = 64, singlet_rule: bool = True, pass_batch: int = 0, timing: bool = False,
                  stats: bool = True, device: Optional[bool] = None, labels_out=None, merge: bool = False):
        """The whole method on many graphs in one call (one RunResult per graph).

        stats=False skips the per-graph statistics records (about 9 KB each).
        With timing=True the first result's stats hold the call's kernel table.
        """
        k = len(graphs)
        if k == 0:
            return []
        dev = graphs[0].dev if device is None else device
        outs = []
        if labels_out is not None and len(labels_out) != k:
            _bad(f"labels_out has {len(labels_out)} arrays for {k} graphs")
        for i, g in enumerate(graphs):
            if not isinstance(g, Graph) or g.ctx is not self or not g.h:
                _bad(f"graphs[{i}] is not a live graph of this context")
            n, _, _ = g.info()
            if labels_out is not None:
                outs.append(_arg(labels_out[i], f"labels_out[{i}]", "int32", n, dev, self.device, output=True))
            else:
                outs.append(_empty_like_kind(dev, n, np.int32, self.torch_device))
        prm = louvain_params(theta_num, theta_den, max_sweeps, max_levels, 1 if singlet_rule else 0, pass_batch,
                             1 if merge else 0)
        handles = (C.c_void_p * k)(*[g.h for g in graphs])
        ptrs = (C.c_void_p * k)(*[_ptr(o) for o in outs])
        qi = (louvain_i128 * k)()
        q = (C.c_double * k)()
        status = (C.c_int32 * k)()
        st = None
        if stats or timing:
            st = (louvain_run_stats * k)()
            st[0].timing = 1 if timing else 0
        self._check(self.lib.louvain_run_batch(self.h, k, handles, C.byref(prm), ptrs, qi, q, status,
                                               st, LOUVAIN_DEVICE_PTRS if dev else 0),
                    ok=(LOUVAIN_OK, LOUVAIN_ELIMIT))
        return [RunResult(outs[i], qi[i].value(), q[i], status[i], stats_dict(st[i]) if st is not None else None)
                for i in range(k)]


def stats_dict(st: louvain_run_stats) -> dict:
    levels = []
    for k in range(st.levels):
        lv = st.level[k]
        levels.append(dict(n=lv.n, nnz=lv.nnz, sweeps_executed=lv.sweeps_executed,
                           sweeps_accepted=lv.sweeps_accepted, gpu_passes=lv.gpu_passes,
                           q_int=lv.q_int.value(), ms_sweep=lv.ms_sweep, ms_contract=lv.ms_contract))
    kernels = {}
    for k in range(st.n_kernels):
        kk = st.kernels[k]
        kernels[kk.name.decode()] = dict(launches=kk.launches, ms=kk.ms, alg_bytes=kk.alg_bytes)
    return dict(levels=levels, kernels=kernels, total_edges_swept=st.total_edges_swept,
                ms_total=st.ms_total, status=st.status)
