"""ctypes binding of libcitron.so.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, fields

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libcitron.so")

OK, EINVAL, ENOMEM, EOVERFLOW, EDEVICE, ESTATE, EBUSY = range(7)
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "ENOMEM", 3: "EOVERFLOW", 4: "EDEVICE",
                5: "ESTATE", 6: "EBUSY"}
DEVICE_PTRS = 1
KMAX = 32
NSTATS = 32
STAT_NAMES = ["vertices", "rows", "entries", "word_ops", "pushes", "dag_bytes", "heavy_steps",
              "compactions", "compact_rows", "light_iters", "light_active", "light_units",
              "flushes", "heavy_leaf_cand", "light_pops", "wave_busy", "wave_first", "wave_last",
              "waves", "arc_lds", "need3_lanes",
              "donations", "wave_busy_max", "item_max", "resident_now", "resident_max",
              "cyc_total", "cyc_light", "cyc_copy", "cyc_need3", "need3_nodes", "need3_min_ops"]

_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_lib = None


class CitronError(RuntimeError):
    """A libcitron call failed; ``status`` is the citron_status code."""

    def __init__(self, status: int, message: str, value: int | None = None):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
        self.value = value


class _Tuning(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("wg_waves", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("light_rows", ctypes.c_int32),
                ("flush_rows", ctypes.c_int32), ("build_blocks_per_cu", ctypes.c_int32),
                ("split_pct", ctypes.c_int32), ("arc_lds_max", ctypes.c_int32)]


@dataclass
class Tuning:
    """Speed-only knobs of the count kernel (0 = library default)."""

    wg_waves: int = 0
    blocks_per_cu: int = 0
    light_rows: int = 0
    flush_rows: int = 0
    build_blocks_per_cu: int = 0
    split_pct: int = 0
    arc_lds_max: int = 0

    def _c(self) -> _Tuning:
        t = _Tuning()
        t.size = ctypes.sizeof(_Tuning)
        for f in fields(self):
            setattr(t, f.name, int(getattr(self, f.name)))
        return t

    @staticmethod
    def _from_c(t: _Tuning) -> "Tuning":
        return Tuning(**{f.name: int(getattr(t, f.name)) for f in fields(Tuning)})


class _Result(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("graph_id", ctypes.c_int32), ("k", ctypes.c_int32),
                ("count", ctypes.c_uint64), ("status", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64)]


def lib_path() -> str:
    return _LIB_PATH


def load_library():
    """Load libcitron.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with "
                          "`python -m paper_2112_10913_amd.build` (hipcc, gfx950)")
    # libcitron.so needs libamdhip64.so.7, and torch ships a copy of that
    # runtime of its own: loading torch first binds the library to torch's
    # copy, so that one HIP runtime serves both (torch's device pointers and
    # streams are then valid in the library).
    _torch()
    lib = ctypes.CDLL(_LIB_PATH)
    vp = ctypes.c_void_p
    lib.citron_load_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp, ctypes.c_uint32, vp,
                                    ctypes.POINTER(vp)]
    lib.citron_load_csr.restype = ctypes.c_int32
    lib.citron_order.argtypes = [vp]
    lib.citron_order.restype = ctypes.c_int32
    lib.citron_order_core.argtypes = [vp]
    lib.citron_order_core.restype = ctypes.c_int32
    lib.citron_get_order_key.argtypes = [vp, _i32p, _i32p]
    lib.citron_get_order_key.restype = ctypes.c_int32
    lib.citron_count.argtypes = [vp, ctypes.c_int32, _i32p]
    lib.citron_count.restype = ctypes.c_uint64
    lib.citron_batch_progress.argtypes = [_i32p, _i32p]
    lib.citron_batch_progress.restype = ctypes.c_int32
    lib.citron_list_arcs.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, vp, vp, ctypes.c_int64,
                                     ctypes.POINTER(ctypes.c_int64)]
    lib.citron_list_arcs.restype = ctypes.c_int32
    lib.citron_count_vertex_rooted.argtypes = [vp, ctypes.c_int32, _i32p]
    lib.citron_count_vertex_rooted.restype = ctypes.c_uint64
    lib.citron_count_per_arc.argtypes = [vp, ctypes.c_int32, vp, _i32p]
    lib.citron_count_per_arc.restype = ctypes.c_uint64
    lib.citron_count_part.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _i32p]
    lib.citron_count_part.restype = ctypes.c_uint64
    lib.citron_count_arcs.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, vp, _i32p]
    lib.citron_count_arcs.restype = ctypes.c_uint64
    lib.citron_count_batch.argtypes = [ctypes.POINTER(vp), _i32p, ctypes.c_int32, _u64p, _i32p,
                                       ctypes.POINTER(_Tuning)]
    lib.citron_count_batch.restype = ctypes.c_int32
    lib.citron_get_dag.argtypes = [vp, _i32p, _i32p]
    lib.citron_get_dag.restype = ctypes.c_int32
    lib.citron_graph_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      _i32p, ctypes.POINTER(ctypes.c_int64)]
    lib.citron_graph_info.restype = ctypes.c_int32
    lib.citron_set_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    lib.citron_set_tuning.restype = ctypes.c_int32
    lib.citron_get_tuning.argtypes = [vp, ctypes.POINTER(_Tuning)]
    lib.citron_get_tuning.restype = ctypes.c_int32
    lib.citron_work_stats.argtypes = [vp, ctypes.c_int32, _u64p]
    lib.citron_work_stats.restype = ctypes.c_int32
    lib.citron_free.argtypes = [vp]
    lib.citron_free.restype = None
    lib.citron_last_error.argtypes = []
    lib.citron_last_error.restype = ctypes.c_char_p
    lib.citron_device_info.argtypes = [_i32p, _i32p, ctypes.c_char_p]
    lib.citron_device_info.restype = ctypes.c_int32
    lib.citron_server_create.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_Tuning)]
    lib.citron_server_create.restype = vp
    lib.citron_server_add_graph.argtypes = [vp, vp, _i32p]
    lib.citron_server_add_graph.restype = ctypes.c_int32
    lib.citron_server_submit.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]
    lib.citron_server_submit.restype = ctypes.c_int32
    lib.citron_server_poll.argtypes = [vp, ctypes.POINTER(_Result), ctypes.c_int32]
    lib.citron_server_poll.restype = ctypes.c_int32
    lib.citron_server_pending.argtypes = [vp]
    lib.citron_server_pending.restype = ctypes.c_int32
    lib.citron_server_destroy.argtypes = [vp]
    lib.citron_server_destroy.restype = None
    lib.citron_order_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int64, vp, vp, vp, vp, _i32p, vp]
    lib.citron_order_noalloc.restype = ctypes.c_int32
    lib.citron_test_seed_accumulator.argtypes = [vp, ctypes.c_uint64]
    lib.citron_test_seed_accumulator.restype = ctypes.c_int32
    _lib = lib
    return lib


def _err(status: int, value: int | None = None) -> CitronError:
    msg = load_library().citron_last_error()
    return CitronError(status, msg.decode(errors="replace") if msg else "", value)


def _torch():
    import torch
    return torch


def _current_stream():
    torch = _torch()
    if torch.cuda.is_available():
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(None)


def device_info() -> dict:
    lib = load_library()
    cus = ctypes.c_int32(0)
    lds = ctypes.c_int32(0)
    name = ctypes.create_string_buffer(64)
    st = lib.citron_device_info(ctypes.byref(cus), ctypes.byref(lds), name)
    if st:
        raise _err(st)
    return {"cus": cus.value, "lds_bytes": lds.value, "arch": name.value.decode()}


class Graph:
    """A graph resident in device memory (handle over citron_graph)."""

    def __init__(self, handle, n: int, m: int, stream):
        self._h = ctypes.c_void_p(handle)
        self.n = n
        self.m = m
        self._stream = stream

    @classmethod
    def from_csr(cls, row_ptr, col, stream=None) -> "Graph":
        """Load an undirected CSR (int32; numpy arrays or torch tensors).

        CUDA/HIP tensors are read in place (CITRON_DEVICE_PTRS); host arrays
        are copied by the library.  ``stream`` is a torch stream (default:
        torch's current stream)."""
        lib = load_library()
        flags = 0
        keep = []
        if hasattr(row_ptr, "is_cuda") and row_ptr.is_cuda:
            torch = _torch()
            rp = row_ptr.to(torch.int32).contiguous()
            cl = col.to(torch.int32).contiguous()
            if not cl.is_cuda:
                raise ValueError("row_ptr and col must both be device tensors or both host arrays")
            keep = [rp, cl]
            n = rp.numel() - 1
            nnz = cl.numel()
            prp, pcl = rp.data_ptr(), (cl.data_ptr() if nnz else None)
            flags = DEVICE_PTRS
        else:
            if hasattr(row_ptr, "numpy"):
                row_ptr = row_ptr.numpy()
                col = col.numpy()
            rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
            cl = np.ascontiguousarray(col, dtype=np.int32)
            keep = [rp, cl]
            n = rp.shape[0] - 1
            nnz = cl.shape[0]
            prp = rp.ctypes.data
            pcl = cl.ctypes.data if nnz else None
        if n < 0:
            raise ValueError("row_ptr must have n+1 >= 1 entries")
        s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _current_stream()
        out = ctypes.c_void_p()
        st = lib.citron_load_csr(n, nnz, prp, pcl, flags, s, ctypes.byref(out))
        del keep
        if st:
            raise _err(st)
        return cls(out.value, n, nnz // 2, s)

    def _handle(self):
        if self._h is None or not self._h.value:
            raise CitronError(EINVAL, "graph has been freed")
        return self._h

    def order(self, ordering: str = "degree") -> "Graph":
        """The ordering phase: "degree" (Section IV, the default) or "core"
        (the level-synchronous form of Algorithm 1's core ordering)."""
        lib = load_library()
        if ordering == "degree":
            st = lib.citron_order(self._handle())
        elif ordering == "core":
            st = lib.citron_order_core(self._handle())
        else:
            raise ValueError("ordering must be 'degree' or 'core'")
        if st:
            raise _err(st)
        return self

    def order_key(self) -> tuple[np.ndarray, int]:
        """(per-vertex order key, number of peeling rounds): the degree under
        the degree ordering, the peeling round under the core ordering."""
        key = np.zeros(max(self.n, 1), np.int32)
        rounds = ctypes.c_int32(0)
        st = load_library().citron_get_order_key(self._handle(), key.ctypes.data_as(_i32p),
                                                 ctypes.byref(rounds))
        if st:
            raise _err(st)
        return key[:self.n], rounds.value

    def count_checked(self, k: int) -> tuple[int, bool]:
        """(count mod 2^64, overflowed)."""
        st = ctypes.c_int32(0)
        v = load_library().citron_count(self._handle(), int(k), ctypes.byref(st))
        if st.value not in (OK, EOVERFLOW):
            raise _err(st.value)
        return int(v), st.value == EOVERFLOW

    def count(self, k: int) -> int:
        """Exact number of k-cliques; raises CitronError on overflow."""
        v, ovf = self.count_checked(k)
        if ovf:
            raise CitronError(EOVERFLOW, "count is >= 2^64", v)
        return v

    def list_arcs(self, k: int, arcs=None):
        """k-cliques of the listed arcs (default: every arc): (cliques as an
        int32 tensor of shape (total, k) on the device, offsets as an int64
        tensor of n_arcs + 1 entries: the cliques of arc i are rows
        offsets[i]..offsets[i+1]).  Two calls: the first sizes the output."""
        torch = _torch()
        lib = load_library()
        if arcs is None:
            arcs = torch.arange(self.m, dtype=torch.int32, device="cuda")
        elif not (hasattr(arcs, "is_cuda") and arcs.is_cuda):
            arcs = torch.as_tensor(np.ascontiguousarray(arcs, dtype=np.int32)).cuda()
        arcs = arcs.to(torch.int32).contiguous()
        n = arcs.numel()
        offsets = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
        total = ctypes.c_int64(0)
        pa = arcs.data_ptr() if n else None
        st = lib.citron_list_arcs(self._handle(), int(k), pa, n, offsets.data_ptr(), None, 0,
                                  ctypes.byref(total))
        if st not in (OK, ENOMEM):
            raise _err(st)
        out = torch.empty((max(total.value, 1), k), dtype=torch.int32, device="cuda")
        if total.value > 0:
            st = lib.citron_list_arcs(self._handle(), int(k), pa, n, offsets.data_ptr(), out.data_ptr(),
                                      total.value, ctypes.byref(total))
            if st:
                raise _err(st)
        return out[:total.value], offsets

    def count_vertex_rooted(self, k: int) -> int:
        """The same count with the vertex-rooted unit (one work item per
        vertex, no split): the ablation of the edge-rooted unit."""
        st = ctypes.c_int32(0)
        v = load_library().citron_count_vertex_rooted(self._handle(), int(k), ctypes.byref(st))
        if st.value == EOVERFLOW:
            raise CitronError(EOVERFLOW, "count is >= 2^64", int(v))
        if st.value != OK:
            raise _err(st.value)
        return int(v)

    def count_per_arc(self, k: int):
        """(total, per-arc counts as a uint64 numpy array in DAG arc order)."""
        torch = _torch()
        buf = torch.empty(max(self.m, 1), dtype=torch.int64, device="cuda")
        st = ctypes.c_int32(0)
        v = load_library().citron_count_per_arc(self._handle(), int(k), buf.data_ptr(), ctypes.byref(st))
        if st.value not in (OK, EOVERFLOW):
            raise _err(st.value)
        arr = buf[:self.m].cpu().numpy().view(np.uint64)
        return int(v), arr

    def count_part(self, k: int, part: int, nparts: int) -> tuple[int, bool]:
        """(share, overflow) of the count: work items part (mod nparts)."""
        st = ctypes.c_int32(0)
        v = load_library().citron_count_part(self._handle(), int(k), int(part), int(nparts), ctypes.byref(st))
        if st.value not in (OK, EOVERFLOW):
            raise _err(st.value)
        return int(v), st.value == EOVERFLOW

    def count_arcs(self, k: int, arcs) -> np.ndarray:
        """Edge-rooted k-clique counts of the listed DAG arcs (uint64 array)."""
        torch = _torch()
        a = torch.as_tensor(np.ascontiguousarray(arcs, dtype=np.int32)).cuda()
        n = int(a.numel())
        out = torch.empty(max(n, 1), dtype=torch.int64, device="cuda")   # every entry is written
        # the arc list is copied on torch's current stream; the library works
        # on the graph's stream, which need not be the same one
        torch.cuda.current_stream().synchronize()
        st = ctypes.c_int32(0)
        load_library().citron_count_arcs(self._handle(), int(k), a.data_ptr(), n, out.data_ptr(),
                                         ctypes.byref(st))
        if st.value not in (OK, EOVERFLOW):
            raise _err(st.value)
        return out[:n].cpu().numpy().view(np.uint64)

    def dag(self) -> tuple[np.ndarray, np.ndarray]:
        dptr = np.zeros(self.n + 1, np.int32)
        dcol = np.zeros(max(self.m, 1), np.int32)
        st = load_library().citron_get_dag(self._handle(), dptr.ctypes.data_as(_i32p),
                                           dcol.ctypes.data_as(_i32p))
        if st:
            raise _err(st)
        return dptr, dcol[:self.m]

    def info(self) -> dict:
        n = ctypes.c_int64()
        m = ctypes.c_int64()
        mx = ctypes.c_int32()
        db = ctypes.c_int64()
        st = load_library().citron_graph_info(self._handle(), ctypes.byref(n), ctypes.byref(m),
                                              ctypes.byref(mx), ctypes.byref(db))
        if st:
            raise _err(st)
        return {"n": n.value, "m": m.value, "max_outdeg": mx.value, "device_bytes": db.value}

    def set_tuning(self, tuning: Tuning | None = None, **kw) -> None:
        if tuning is None and kw:
            tuning = Tuning(**kw)
        ct = tuning._c() if tuning is not None else None
        st = load_library().citron_set_tuning(self._handle(), ctypes.byref(ct) if ct is not None else None)
        if st:
            raise _err(st)

    def get_tuning(self) -> Tuning:
        t = _Tuning()
        st = load_library().citron_get_tuning(self._handle(), ctypes.byref(t))
        if st:
            raise _err(st)
        return Tuning._from_c(t)

    def work_stats(self, k: int) -> dict:
        arr = np.zeros(NSTATS, np.uint64)
        st = load_library().citron_work_stats(self._handle(), int(k), arr.ctypes.data_as(_u64p))
        if st:
            raise _err(st)
        return {name: int(v) for name, v in zip(STAT_NAMES, arr)}

    def seed_accumulator(self, base: int) -> None:
        """Test hook: the next count starts its accumulator at ``base``."""
        st = load_library().citron_test_seed_accumulator(self._handle(), int(base))
        if st:
            raise _err(st)

    def free(self) -> None:
        if self._h is not None and self._h.value:
            load_library().citron_free(self._h)
        self._h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def order_noalloc(row_ptr, col, dag_ptr, dag_col, stream=None) -> int:
    """citron_order_noalloc: the degree-ordered DAG of a device CSR written
    into the device tensors dag_ptr (int32[n+1]) and dag_col (int32[m]),
    with no device allocation; returns the largest out-degree."""
    lib = load_library()
    torch = _torch()
    for t in (row_ptr, col, dag_ptr, dag_col):
        if not (t.is_cuda and t.dtype == torch.int32 and t.is_contiguous()):
            raise ValueError("order_noalloc takes contiguous int32 device tensors")
    n = row_ptr.numel() - 1
    nnz = col.numel()
    if dag_ptr.numel() < n + 1 or dag_col.numel() < nnz // 2:
        raise ValueError("dag_ptr needs n+1 entries and dag_col nnz/2")
    s = ctypes.c_void_p(stream.cuda_stream) if stream is not None else _current_stream()
    mx = ctypes.c_int32(-1)
    st = lib.citron_order_noalloc(n, nnz, row_ptr.data_ptr(), col.data_ptr() if nnz else None,
                                  dag_ptr.data_ptr(), dag_col.data_ptr() if nnz else None,
                                  ctypes.byref(mx), s)
    if st:
        raise _err(st)
    return mx.value


def batch_progress() -> tuple[int, int]:
    """(items claimed, items total) of the batch launch running now, from
    another thread; (0, 0) when none runs."""
    a = ctypes.c_int32(0)
    b = ctypes.c_int32(0)
    st = load_library().citron_batch_progress(ctypes.byref(a), ctypes.byref(b))
    if st:
        raise _err(st)
    return a.value, b.value


def count_batch(graphs, ks, tuning: Tuning | None = None, return_status: bool = False):
    """Counts for the queries (graphs[i], ks[i]) from one persistent launch."""
    lib = load_library()
    nq = len(ks)
    if len(graphs) != nq:
        raise ValueError("graphs and ks differ in length")
    hs = (ctypes.c_void_p * max(nq, 1))(*[g._handle().value for g in graphs])
    karr = np.ascontiguousarray(ks, dtype=np.int32)
    counts = np.zeros(max(nq, 1), np.uint64)
    sts = np.zeros(max(nq, 1), np.int32)
    ct = tuning._c() if tuning is not None else None
    st = lib.citron_count_batch(hs, karr.ctypes.data_as(_i32p), nq, counts.ctypes.data_as(_u64p),
                                sts.ctypes.data_as(_i32p), ctypes.byref(ct) if ct is not None else None)
    if st and not return_status:
        raise _err(st)
    out = [int(c) for c in counts[:nq]]
    if return_status:
        return out, [int(s) for s in sts[:nq]]
    return out


class Server:
    """Continuous-batching request server over resident graphs."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, max_slots: int = 64,
                 tuning: Tuning | None = None):
        lib = load_library()
        ct = tuning._c() if tuning is not None else None
        h = lib.citron_server_create(int(hbm_budget_bytes), int(max_slots),
                                     ctypes.byref(ct) if ct is not None else None)
        if not h:
            raise _err(EINVAL)
        self._h = ctypes.c_void_p(h)
        self._graphs = []

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_int32()
        st = load_library().citron_server_add_graph(self._h, g._handle(), ctypes.byref(gid))
        if st:
            raise _err(st)
        self._graphs.append(g)
        return gid.value

    def submit(self, graph_id: int, k: int, tag: int = 0) -> None:
        st = load_library().citron_server_submit(self._h, int(graph_id), int(k), int(tag))
        if st:
            raise _err(st)

    def poll(self, max_results: int = 1024) -> list[dict]:
        buf = (_Result * max_results)()
        got = load_library().citron_server_poll(self._h, buf, max_results)
        out = []
        for i in range(got):
            r = buf[i]
            out.append({"tag": r.tag, "graph_id": r.graph_id, "k": r.k, "count": r.count,
                        "status": r.status, "t_submit_ns": r.t_submit_ns,
                        "t_admit_ns": r.t_admit_ns, "t_done_ns": r.t_done_ns})
        return out

    def pending(self) -> int:
        return int(load_library().citron_server_pending(self._h))

    def close(self) -> None:
        if self._h is not None and self._h.value:
            load_library().citron_server_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
