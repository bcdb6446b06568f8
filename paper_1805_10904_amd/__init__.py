"""MI355X (gfx950) synchronous parallel Louvain -- Python binding.

A thin ctypes layer over ``liblouvain_hip.so`` (the C ABI declared in
``include/louvain.h``): argument marshalling only, every step of the method
runs in the library's HIP kernels.  There is no CPU fallback: importing
works without a GPU, but every call needs the built library and a device.

Arrays may be numpy arrays (host pointers) or torch CUDA tensors (device
pointers); outputs come back in the same kind as the inputs.
"""
from __future__ import annotations

from ._native import (  # noqa: F401
    LOUVAIN_DEVICE_PTRS, LOUVAIN_CHECK_SYMMETRY, LOUVAIN_NO_SINGLET, LOUVAIN_WEIGHTS_I64,
    LOUVAIN_OK, LOUVAIN_EINVAL, LOUVAIN_ENOMEM, LOUVAIN_EDEVICE, LOUVAIN_EAGAIN, LOUVAIN_EBUSY, LOUVAIN_ELIMIT, LOUVAIN_EOVERFLOW,
    LIB_PATH, LouvainError, Context, Graph, Dendrogram, RunResult, ServeResult, load_library, exported_symbols,
    workspace_bytes,
)
