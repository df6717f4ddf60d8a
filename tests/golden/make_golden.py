"""Write the stored expected values of the large parity cases.

Calls only ``oracle/`` (and the input generators).  Whole-graph counts are
split over worker processes by vertex residue class (each worker runs the
unmodified single-threaded oracle on vertices r, r+P, r+2P, ...); the sum of
the parts is the count because the recursion is a sum over root vertices.
Per-arc values are the edge-rooted counts of a seeded sample of arcs.

    python tests/golden/make_golden.py rmat14          # counts k = 3..6
    python tests/golden/make_golden.py rmat14 --ks 7 8 # ~3 min on 8 processes
    python tests/golden/make_golden.py rmat20 --ks 3 4 --arcs 5 6 7 8
    python tests/golden/make_golden.py rmat20 --ks 5       # whole count, ~18 min on 8 processes
    python tests/golden/make_golden.py chunglu22 --ks 3 4 --arcs 5 6 7
    python tests/golden/make_golden.py chunglu22 --ks 5    # whole count, ~13 min on 8 processes
    python tests/golden/make_golden.py rmat20 --ks --work-model 5 6 7 8   # ~2 min

The work model of a k (``--work-model``) is the oracle's per-arc statistics
over the arcs that survive pruning (|C_uv| >= k - 2): the sums of
d->(u) + d->(v), of |C_uv| and of the out-degrees of the candidates, from
which the per-query algorithmic bytes of the merge-based construction are
formed.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

_G = {}


def _init(name, cache=None):
    if cache and os.path.exists(cache):
        # the graph the parent generated (generating it once per worker
        # would multiply the generator's time and memory)
        z = np.load(cache)
        g = gg.CSR(int(z["row_ptr"].shape[0] - 1), z["row_ptr"], z["col"], name)
    else:
        g = gg.config_graph(name)
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    _G.update(g=g, dptr=dptr, dcol=dcol)


def _part(args):
    k, r, P = args
    g = _G["g"]
    c, ovf = oracle.count_dag(g.n, _G["dptr"], _G["dcol"], k, r, g.n, P)
    return c, ovf


def _arc(args):
    k, u, v = args
    g = _G["g"]
    t = time.time()
    c, ovf = oracle.count_arcs(g.n, _G["dptr"], _G["dcol"], k, np.array([u]), np.array([v]))
    return int(c[0]), bool(ovf), time.time() - t


def _work_model(k):
    g = _G["g"]
    st, _ = oracle.arc_stats(g.n, _G["dptr"], _G["dcol"], k)
    return st


def sample_arcs(dptr, dcol, n_uniform, n_heavy, seed, heavy_outdeg=64):
    """Seeded uniform arcs plus arcs leaving vertices of out-degree > 64."""
    rng = np.random.default_rng(seed)
    m = int(dptr[-1])
    src = np.repeat(np.arange(len(dptr) - 1), np.diff(dptr))
    idx = set(rng.choice(m, size=min(n_uniform, m), replace=False).tolist())
    heavy = np.nonzero(np.diff(dptr)[src] > heavy_outdeg)[0]
    if heavy.size:
        idx |= set(rng.choice(heavy, size=min(n_heavy, heavy.size), replace=False).tolist())
    idx = np.array(sorted(idx), dtype=np.int64)
    return idx, src[idx], dcol[idx]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("name")
    ap.add_argument("--ks", type=int, nargs="*", default=[3, 4, 5, 6])
    ap.add_argument("--arcs", type=int, nargs="*", default=[])
    ap.add_argument("--n-uniform", type=int, default=192)
    ap.add_argument("--n-heavy", type=int, default=64)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--work-model", type=int, nargs="*", default=[])
    args = ap.parse_args()
    out_path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{args.name}.json")
    data = {}
    if os.path.exists(out_path):
        with open(out_path) as f:
            data = json.load(f)
    g0 = gg.config_graph(args.name)
    cache = os.path.join("/tmp", f"golden_{args.name}_{os.getpid()}.npz")
    np.savez(cache, row_ptr=g0.row_ptr, col=g0.col)
    del g0
    _init(args.name, cache)
    g = _G["g"]
    data.update(graph=args.name, config=gg.CONFIGS[args.name], n=g.n, m=g.m, sha256=g.sha256(),
                max_outdeg=int(np.diff(_G["dptr"]).max(initial=0)),
                generator="graphgen (numpy PCG64), numpy " + np.__version__)
    counts = data.setdefault("counts", {})
    if args.work_model:
        wm = data.setdefault("work_model", {})
        with Pool(min(args.procs, len(args.work_model)), initializer=_init, initargs=(args.name, cache)) as pool:
            res = pool.map(_work_model, args.work_model)
        for k, st in zip(args.work_model, res):
            wm[str(k)] = st
            print(f"work model k={k}: {st}", flush=True)
        with open(out_path, "w") as f:
            json.dump(data, f, indent=1)
    P = args.procs
    with Pool(P, initializer=_init, initargs=(args.name, cache)) as pool:
        for k in args.ks:
            t = time.time()
            parts = pool.map(_part, [(k, r, P) for r in range(P)])
            total = sum(c for c, _ in parts)
            ovf = any(o for _, o in parts) or total >= 2**64
            counts[str(k)] = {"count": total % 2**64, "overflow": bool(ovf)}
            print(f"k={k} count={total} ({time.time() - t:.1f} s on {P} processes)", flush=True)
            with open(out_path, "w") as f:
                json.dump(data, f, indent=1)
        if args.arcs:
            idx, us, vs = sample_arcs(_G["dptr"], _G["dcol"], args.n_uniform, args.n_heavy, seed=2112)
            arcs = data.setdefault("arcs", {})
            arcs["index"] = [int(i) for i in idx]
            arcs["u"] = [int(u) for u in us]
            arcs["v"] = [int(v) for v in vs]
            for k in args.arcs:
                t = time.time()
                res = pool.map(_arc, [(k, int(u), int(v)) for u, v in zip(us, vs)], chunksize=1)
                arcs[str(k)] = [c for c, _, _ in res]
                print(f"arcs k={k}: {len(res)} arcs, max {max(r[2] for r in res):.1f} s, "
                      f"total {time.time() - t:.1f} s", flush=True)
                with open(out_path, "w") as f:
                    json.dump(data, f, indent=1)
    os.remove(cache)


if __name__ == "__main__":
    main()
