"""citron -- exact k-clique counting on AMD Instinct MI355X (gfx950).

A thin ctypes binding of ``libcitron.so`` (C ABI in ``include/citron.h``).
Every step of the computation runs in the library's HIP kernels; this module
only marshals arguments.  PyTorch supplies device memory and streams.  There
is no CPU fallback: if the library is missing or no GPU is present, calls
raise.

    import paper_2112_10913_amd as citron
    g = citron.Graph.from_csr(row_ptr, col)   # numpy int32 or torch int32 tensors
    g.order()                                  # degree-ordered DAG (Section IV)
    g.count(5)                                 # number of 5-cliques (int)
    citron.count_batch([g, g], [4, 5])         # one persistent launch
"""
from __future__ import annotations

from ._lib import (CitronError, Graph, Server, Tuning, batch_progress, count_batch, device_info,
                   lib_path, load_library, order_noalloc, STATUS_NAMES, NSTATS, STAT_NAMES, KMAX)

__all__ = ["CitronError", "Graph", "Server", "Tuning", "batch_progress", "count_batch", "device_info",
           "lib_path", "load_library", "order_noalloc", "STATUS_NAMES", "NSTATS", "STAT_NAMES",
           "KMAX"]
