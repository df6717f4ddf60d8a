"""All-core timing wrapper of the reference counter -- TEST INFRASTRUCTURE ONLY.

Used by the benchmark's CPU-baseline leg and by the tests; the product
package never imports it.

The whole count is a sum over root vertices (Section III, Algorithm 2: each
clique is counted once, from its lowest vertex in the ordering), so the roots
can be dealt out cyclically, as the paper's OpenMP loop over vertices does:
residue class r of a stride S holds the roots r, r + S, r + 2S, ...  Each
class is counted by the unmodified single-threaded oracle in a worker
process; the class results are summed as exact Python integers, so the
total and its overflow flag equal those of one single-threaded run.

A checkpoint file (JSON, one entry per finished class) lets a long count
resume where it stopped: classes already in the file are not counted again.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import time

import numpy as np

from . import count_dag

_DAG = {}


def _class(args):
    k, r, stride = args
    n, dptr, dcol = _DAG["n"], _DAG["dptr"], _DAG["dcol"]
    t = time.perf_counter()
    c, ovf = count_dag(n, dptr, dcol, k, r, n, stride)
    return r, c, ovf, time.perf_counter() - t


def _load_checkpoint(path, key):
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    if data.get("key") != key:
        return {}
    return {int(r): tuple(v) for r, v in data.get("classes", {}).items()}


def _save_checkpoint(path, key, done):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"key": key, "classes": {str(r): list(v) for r, v in sorted(done.items())}}, f)
    os.replace(tmp, path)


def count_classes(n, dptr, dcol, k, stride, classes=None, workers=None, checkpoint=None, graph_key=""):
    """Count the k-cliques rooted at the residue classes `classes` (default:
    all of 0..stride-1) of `stride`, on `workers` processes (default: every
    host core, at most 16).  Returns a dict: count (mod 2^64), overflow,
    classes counted, per-class seconds, wall seconds, workers.

    With `checkpoint`, finished classes are recorded in that JSON file (keyed
    by graph_key, k and stride) and skipped when the call is repeated."""
    classes = list(range(stride)) if classes is None else [int(r) for r in classes]
    workers = workers or min(16, os.cpu_count() or 1)
    key = f"{graph_key}|k={k}|stride={stride}"
    done = _load_checkpoint(checkpoint, key)
    todo = [r for r in classes if r not in done]
    t0 = time.perf_counter()
    if todo:
        _DAG.update(n=int(n), dptr=np.ascontiguousarray(dptr, np.int32),
                    dcol=np.ascontiguousarray(dcol, np.int32))
        ctx = mp.get_context("fork")
        with ctx.Pool(min(workers, len(todo))) as pool:
            for r, c, ovf, dt in pool.imap_unordered(_class, [(k, r, stride) for r in todo]):
                done[r] = (int(c), bool(ovf), float(dt))
                if checkpoint:
                    _save_checkpoint(checkpoint, key, done)
        _DAG.clear()
    wall = time.perf_counter() - t0
    total = sum(done[r][0] for r in classes)
    ovf = any(done[r][1] for r in classes) or total >= 2**64
    return {"count": total % 2**64, "overflow": bool(ovf), "classes": len(classes),
            "class_seconds": [done[r][2] for r in classes], "wall_s": wall,
            "workers": min(workers, max(len(todo), 1))}
