"""Write the stored expected values of the batched-form parity test.

Calls only ``oracle/`` (and the input generators).  The batch is the mixed
suite of 512 graphs (seeds 4000 + i: half R-MAT of scale 8..16 with edge
factor 8..32, half Erdos-Renyi with n in 1k..50k and mean degree 10..40,
shuffled).  The oracle counts k = 3..8 for a subset that spans both
families and the small and middle R-MAT scales: the first `--er` Erdos-Renyi
graphs and the first `--rmat` R-MAT graphs of scale <= `--max-scale`, in the
suite's order.  Larger members are checked against plain counts.

    python tests/golden/make_batch_golden.py        # ~2 min on 8 processes
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from multiprocessing import get_context

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

KS = (3, 4, 5, 6, 7, 8)


def _counts(job):
    i, seed0 = job
    g = gg.batch_suite_member(i, seed0)
    out = {}
    for k in KS:
        c, ovf = oracle.count(g, k)
        out[str(k)] = {"count": c, "overflow": bool(ovf)}
    return g.name, g.sha256(), out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--seed0", type=int, default=4000)
    ap.add_argument("--er", type=int, default=24)
    ap.add_argument("--rmat", type=int, default=24)
    ap.add_argument("--max-scale", type=int, default=11)
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    t = time.time()
    order = gg.batch_suite_order(args.count, args.seed0)
    members = gg.batch_suite_specs(args.count, args.seed0)
    pick = []
    n_er = n_rm = 0
    for pos, i in enumerate(order):
        kind, size = members[i]
        if kind == "er" and n_er < args.er:
            pick.append((pos, i))
            n_er += 1
        elif kind == "rmat" and size <= args.max_scale and n_rm < args.rmat:
            pick.append((pos, i))
            n_rm += 1
    with get_context("spawn").Pool(args.procs) as pool:
        res = pool.map(_counts, [(i, args.seed0) for _, i in pick], chunksize=1)
    data = {"suite": {"count": args.count, "seed0": args.seed0}, "ks": list(KS),
            "generator": "graphgen.batch_suite (numpy PCG64)", "members": []}
    for (pos, i), (name, sha, counts) in zip(pick, res):
        data["members"].append({"position": pos, "name": name, "sha256": sha, "counts": counts})
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch512.json")
    with open(path, "w") as f:
        json.dump(data, f, indent=1)
    print(f"{len(pick)} members in {time.time() - t:.1f} s -> {path}")


if __name__ == "__main__":
    main()
