"""Python access to the reference k-clique counter (``citron_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this module; the product package never imports it.

``build()`` compiles the C source with gcc into ``liboracle.so`` next to it.
All functions take int32 CSR arrays (numpy) and return Python ints.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "citron_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = ctypes.POINTER(ctypes.c_int32)
_u64p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C11, -O2)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ctypes.CDLL(_LIB)
        lib.oracle_check_csr.argtypes = [ctypes.c_int32, _i32p, _i32p]
        lib.oracle_orient.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p, _i32p]
        lib.oracle_count_dag.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, _u64p, _i32p, _u64p]
        lib.oracle_count_dag_from.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_int32, ctypes.c_uint64, _u64p, _i32p, _u64p]
        lib.oracle_count.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32,
                                     ctypes.c_int32, _u64p, _i32p, _u64p]
        lib.oracle_count_arcs.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32,
                                          _i32p, _i32p, ctypes.c_int64, _u64p, _i32p]
        lib.oracle_arc_stats.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32,
                                         _u64p, _u64p]
        lib.oracle_core_rank.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p]
        lib.oracle_orient_rank.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p]
        lib.oracle_peel_rounds.argtypes = [ctypes.c_int32, _i32p, _i32p, _i32p]
        lib.oracle_list_arcs.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32,
                                         _i32p, _i32p, ctypes.c_int64, _u64p, _i32p,
                                         ctypes.c_uint64, _u64p]
        lib.oracle_list_dag.argtypes = [ctypes.c_int32, _i32p, _i32p, ctypes.c_int32,
                                        ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                        _i32p, ctypes.c_uint64, _u64p]
        _lib = lib
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _check(st):
    if st != 0:
        raise RuntimeError(f"oracle call failed with status {st}")


def check_csr(n, row_ptr, col) -> bool:
    rp, prp = _i32(row_ptr)
    c, pc = _i32(col if len(col) else np.zeros(1, np.int32))
    return _load().oracle_check_csr(n, prp, pc) == 0


def orient(n, row_ptr, col):
    """Degree-ordered DAG: (dag_ptr int32[n+1], dag_col int32[m])."""
    rp, prp = _i32(row_ptr)
    c, pc = _i32(col if len(col) else np.zeros(1, np.int32))
    m = int(rp[n]) // 2
    dptr = np.zeros(n + 1, np.int32)
    dcol = np.zeros(max(m, 1), np.int32)
    _check(_load().oracle_orient(n, prp, pc, dptr.ctypes.data_as(_i32p),
                                 dcol.ctypes.data_as(_i32p)))
    return dptr, dcol[:m]


def count_dag(n, dptr, dcol, k, first=0, last=None, step=1, prune=True,
              visits=False, base=0):
    """k-cliques rooted at vertices first, first+step, ... < last, added to
    ``base`` (mod 2^64; the flag tells whether base + count >= 2^64)."""
    last = n if last is None else last
    a, pa = _i32(dptr)
    b, pb = _i32(dcol if len(dcol) else np.zeros(1, np.int32))
    cnt = ctypes.c_uint64(0)
    ovf = ctypes.c_int32(0)
    vis = np.zeros(k + 1, np.uint64) if visits else None
    _check(_load().oracle_count_dag_from(n, pa, pb, k, first, last, step, int(prune), int(base),
                                         ctypes.byref(cnt), ctypes.byref(ovf),
                                         vis.ctypes.data_as(_u64p) if visits else None))
    if visits:
        return int(cnt.value), bool(ovf.value), [int(x) for x in vis]
    return int(cnt.value), bool(ovf.value)


def count(g, k, prune=True, visits=False):
    """(count mod 2^64, overflow flag[, visits]) for a graphgen.CSR."""
    rp, prp = _i32(g.row_ptr)
    c, pc = _i32(g.col if g.nnz else np.zeros(1, np.int32))
    cnt = ctypes.c_uint64(0)
    ovf = ctypes.c_int32(0)
    vis = np.zeros(k + 1, np.uint64) if visits else None
    _check(_load().oracle_count(g.n, prp, pc, k, int(prune), ctypes.byref(cnt),
                                ctypes.byref(ovf),
                                vis.ctypes.data_as(_u64p) if visits else None))
    if visits:
        return int(cnt.value), bool(ovf.value), [int(x) for x in vis]
    return int(cnt.value), bool(ovf.value)


def count_arcs(n, dptr, dcol, k, arc_u, arc_v):
    """Per-arc k-clique counts of the edge-rooted unit (uint64 array)."""
    a, pa = _i32(dptr)
    b, pb = _i32(dcol if len(dcol) else np.zeros(1, np.int32))
    au, pau = _i32(arc_u)
    av, pav = _i32(arc_v)
    out = np.zeros(max(len(au), 1), np.uint64)
    ovf = ctypes.c_int32(0)
    _check(_load().oracle_count_arcs(n, pa, pb, k, pau, pav, len(au),
                                     out.ctypes.data_as(_u64p), ctypes.byref(ovf)))
    return out[:len(au)], bool(ovf.value)


STAT_NAMES = ["arcs", "sum_duv", "sum_s", "sum_dw", "max_s", "arcs_kept",
              "kept_sum_duv", "kept_sum_s", "kept_sum_dw", "max_outdeg"]


def arc_stats(n, dptr, dcol, k):
    """Work statistics of the edge-rooted unit (dict) and the s histogram."""
    a, pa = _i32(dptr)
    b, pb = _i32(dcol if len(dcol) else np.zeros(1, np.int32))
    st = np.zeros(10, np.uint64)
    hist = np.zeros(33, np.uint64)
    _check(_load().oracle_arc_stats(n, pa, pb, k, st.ctypes.data_as(_u64p),
                                    hist.ctypes.data_as(_u64p)))
    return {name: int(v) for name, v in zip(STAT_NAMES, st)}, [int(x) for x in hist]


def list_dag(n, dptr, dcol, k, first=0, last=None, step=1, cap=None):
    """k-cliques rooted at vertices first, first+step, ... < last, as an
    int32 array of shape (found, k), each row in increasing degree order;
    returns (array, total).  At most ``cap`` rows are kept (default: all,
    sized by a first pass that only counts them)."""
    last = n if last is None else last
    lib = _load()
    a, pa = _i32(dptr)
    b, pb = _i32(dcol if len(dcol) else np.zeros(1, np.int32))
    total = ctypes.c_uint64(0)
    if cap is None:
        _check(lib.oracle_list_dag(n, pa, pb, k, first, last, step, None, 0, ctypes.byref(total)))
        cap = int(total.value)
    out = np.zeros((max(cap, 1), k), np.int32)
    _check(lib.oracle_list_dag(n, pa, pb, k, first, last, step, out.ctypes.data_as(_i32p), cap,
                               ctypes.byref(total)))
    got = min(cap, int(total.value))
    return out[:got], int(total.value)


def list_cliques(g, k):
    """All k-cliques of graph g (rows in increasing degree order)."""
    dptr, dcol = orient(g.n, g.row_ptr, g.col)
    return list_dag(g.n, dptr, dcol, k)[0]


def core_rank(n, row_ptr, col):
    """Removal position of each vertex in the core ordering (Algorithm 1)."""
    a, pa = _i32(row_ptr)
    b, pb = _i32(col if len(col) else np.zeros(1, np.int32))
    rank = np.zeros(max(n, 1), np.int32)
    _check(_load().oracle_core_rank(n, pa, pb, rank.ctypes.data_as(_i32p)))
    return rank[:n]


def orient_rank(n, row_ptr, col, rank):
    """(dag_ptr, dag_col) with u -> v iff rank[u] < rank[v]."""
    a, pa = _i32(row_ptr)
    b, pb = _i32(col if len(col) else np.zeros(1, np.int32))
    r, pr = _i32(rank if len(rank) else np.zeros(1, np.int32))
    m = int(a[n]) // 2
    dptr = np.zeros(n + 1, np.int32)
    dcol = np.zeros(max(m, 1), np.int32)
    _check(_load().oracle_orient_rank(n, pa, pb, pr, dptr.ctypes.data_as(_i32p), dcol.ctypes.data_as(_i32p)))
    return dptr, dcol[:m]


def peel_rounds(n, row_ptr, col):
    """Round in which each vertex leaves the level-synchronous peeling
    (the parallel form of the core ordering)."""
    a, pa = _i32(row_ptr)
    b, pb = _i32(col if len(col) else np.zeros(1, np.int32))
    rnd = np.zeros(max(n, 1), np.int32)
    _check(_load().oracle_peel_rounds(n, pa, pb, rnd.ctypes.data_as(_i32p)))
    return rnd[:n]


def peel_rank(n, row_ptr, col):
    """Total order of the peeling: position of each vertex when sorted by
    (round, id)."""
    rnd = peel_rounds(n, row_ptr, col)
    order = np.lexsort((np.arange(n), rnd))
    rank = np.empty(n, np.int32)
    rank[order] = np.arange(n, dtype=np.int32)
    return rank


def orient_peel(g):
    """The DAG of the level-synchronous peeling of graph g."""
    return orient_rank(g.n, g.row_ptr, g.col, peel_rank(g.n, g.row_ptr, g.col))


def orient_core(g):
    """The core-ordered DAG of graph g."""
    return orient_rank(g.n, g.row_ptr, g.col, core_rank(g.n, g.row_ptr, g.col))


def list_arcs(n, dptr, dcol, k, arc_u, arc_v):
    """Edge-rooted listing: (cliques as an int32 array (total, k), per-arc
    clique counts as uint64); the cliques of arc i come before those of arc
    i+1, each starting with the arc's two vertices."""
    lib = _load()
    a, pa = _i32(dptr)
    b, pb = _i32(dcol if len(dcol) else np.zeros(1, np.int32))
    u, pu = _i32(arc_u if len(arc_u) else np.zeros(1, np.int32))
    v, pv = _i32(arc_v if len(arc_v) else np.zeros(1, np.int32))
    na = len(arc_u)
    per_arc = np.zeros(max(na, 1), np.uint64)
    total = ctypes.c_uint64(0)
    _check(lib.oracle_list_arcs(n, pa, pb, k, pu, pv, na, per_arc.ctypes.data_as(_u64p), None, 0,
                                ctypes.byref(total)))
    cap = int(total.value)
    out = np.zeros((max(cap, 1), k), np.int32)
    _check(lib.oracle_list_arcs(n, pa, pb, k, pu, pv, na, per_arc.ctypes.data_as(_u64p),
                                out.ctypes.data_as(_i32p), cap, ctypes.byref(total)))
    return out[:cap], per_arc[:na]
