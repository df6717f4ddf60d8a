#!/usr/bin/env python3
"""Benchmark of the k-clique counting path on one MI355X.

Workload (default): R-MAT scale 20 (2^20 vertices), edge factor 16,
a/b/c/d = 0.57/0.19/0.19/0.05, seed 20, symmetrised and cleaned; int32 CSR;
k = 5, 6, 7 each counted separately (k = 8 with --ks 8: it runs for tens of
minutes, beyond a default run).  The CSR is resident in device memory before
the timed region.

One step = load the CSR into a fresh graph handle (device-to-device copy +
validation), order it (Section IV), build the subgraph rows and count
k-cliques for every k.  The reported value is edges/s: (number of k values x
m) / step time, with m the number of undirected edges.  Per-k count times
come from HIP events on the stream the kernels run on.

Time budget: warm-up and timed steps stop once another step would end past
--budget-s seconds after the process started (default 500 s, so that a
run asked for many steps of a workload whose steps take tens of seconds
still ends within a ten-minute limit); at least one step is always timed.
The line reports the steps actually run and the ones asked for.

Roofline of the dominant kernel (the count kernel): algorithmic int32 VALU
lane-ops per launch (4 per 64-bit AND+popcount, one per j-clique for
j = 3..k-1) over the mean launch time, against 256 CUs x 64 lanes x 2.4 GHz.
Per k, the line also gives the HBM figure of the paper's merge-based
subgraph construction: the algorithmic bytes of every arc that survives
pruning over the count time, against 8 TB/s.

The CPU baseline is the oracle on the host's cores (one process per core, at
most 16, roots dealt by residue class) on a sample of the roots, for the
smallest k of the step, run before the GPU is touched.

Prints ONE JSON line.  Only N=1 is supported: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

T_PROCESS_START = time.monotonic()
ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

WORKLOADS = {
    "rmat14": "R-MAT scale 14, edge factor 16, a/b/c/d 0.57/0.19/0.19/0.05, seed 14",
    "rmat20": "R-MAT scale 20, edge factor 16, a/b/c/d 0.57/0.19/0.19/0.05, seed 20",
    "chunglu22": "Chung-Lu, 2^22 vertices, degree exponent 2.1, mean degree 25, max weight 2e4, "
                 "plus 2,000 planted cliques of size 10..40 (seeds 22, 2201)",
}
PEAK_HBM_GBS = 8000.0
# int32 VALU lane-ops per second: 256 CUs x 64 lanes x 2.4 GHz
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
# one row-word AND + popcount-accumulate on 64-bit words = 4 int32 lane-ops
OPS_PER_WORD = 4


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(g, k, budget_s=20.0, workers=None):
    """The oracle as it stands on the host's cores (one process per core, at
    most 16), each counting the roots of one residue class of a stride S
    (roots v = r mod S, ids randomly permuted by the generator), for the
    smallest k of the step: at larger k the oracle's time per root is
    spread over many orders of magnitude (a hub vertex alone runs for
    minutes), so no bounded sample estimates it.  The whole-graph time at
    that core count is estimated as (sum of the class times) x (S /
    classes) / cores.  S is chosen from a one-class probe so that the run
    takes about budget_s seconds."""
    import oracle
    from oracle import parallel as opar
    workers = workers or min(16, os.cpu_count() or 1)
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    # probe on one core, growing the sample until it takes a tenth of the
    # budget (a few roots alone say little: their times are very uneven)
    probe_stride = 1 << 16
    while True:
        t = time.perf_counter()
        oracle.count_dag(g.n, dptr, dcol, k, 0, g.n, probe_stride)
        t_probe = max(time.perf_counter() - t, 1e-6)
        if t_probe >= budget_s / 10 or probe_stride <= 64:
            break
        probe_stride //= 4
    # class time at stride S ~ t_probe * probe_stride / S, one class per worker
    stride = int(min(probe_stride, max(workers, t_probe * probe_stride / budget_s)))
    res = opar.count_classes(g.n, dptr, dcol, k, stride, classes=range(workers), workers=workers)
    cpu = sum(res["class_seconds"])
    est = cpu * (stride / workers) / workers
    return {"value": g.m / est, "unit": "edges/s", "cores": workers, "kind": "oracle",
            "k": k, "est_full_graph_s": est, "stride": stride, "cpu_s": cpu, "wall_s": res["wall_s"],
            "sample": f"k = {k} only; roots v = r mod {stride} for r = 0..{workers - 1} "
                      f"({workers} of {stride} residue classes, ids randomly permuted), one process per "
                      f"class on {workers} host cores, {res['wall_s']:.1f} s wall, {cpu:.1f} s of CPU; "
                      f"whole-graph time at {workers} cores estimated as the class CPU time "
                      f"x {stride} / {workers} / {workers} = {est:.1f} s"}


def kernel_digest(path):
    """sha256 of a kernel source with its // comments and blank lines
    removed: the code the counters were taken on, not its commentary."""
    import hashlib
    lines = []
    for line in open(path).read().splitlines():
        code = line.split("//", 1)[0].strip()
        if code:
            lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()


def traffic_per_launch(ks):
    """HBM bytes per count-kernel launch from the committed rocprofv3 counter
    summary, if it was taken on the same kernel source and the same k set;
    else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "count_kernel_rmat20_hbm.md")
    src = os.path.join(ROOT, "paper_2112_10913_amd", "csrc", "kernels_count.hip")
    try:
        text = open(path).read()
        digest = kernel_digest(src)
    except OSError:
        return None
    rec = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            key, val = line[2:].split(": ", 1)
            rec[key.strip()] = val.strip().strip("`")
    if rec.get("kernel code sha256") != digest or rec.get("ks") != " ".join(map(str, ks)):
        return None
    try:
        return float(rec["HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def load_golden(name):
    """The stored oracle values of a configuration graph (tests/golden), or
    None.  Written by tests/golden/make_golden.py, which calls only the
    oracle."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    try:
        with open(path) as f:
            return json.load(f)
    except OSError:
        return None


def alg_bytes(gold, k):
    """Algorithmic HBM bytes of one k-clique count under the paper's
    merge-based subgraph construction (Algorithm 5 per arc, no reuse): for
    every arc u -> v that survives pruning (|C_uv| >= k - 2), the two
    out-lists 4 (d(u) + d(v)), the candidates' out-lists 4 sum_{w in C_uv}
    d(w), and the compact output 8 (|C_uv| + 1).  From the oracle's stored
    per-arc statistics; None when they are not stored for this k."""
    if not gold:
        return None
    st = gold.get("work_model", {}).get(str(k))
    if not st:
        return None
    return float(4 * st["kept_sum_duv"] + 4 * st["kept_sum_dw"] + 8 * (st["kept_sum_s"] + st["arcs_kept"]))


def batch_with_progress(citron, gs, ks, every_s=20.0):
    """count_batch(gs, ks) on a worker thread; this thread reports the
    launch's progress (work items claimed, read from the device) while it
    runs.  Returns (counts, seconds)."""
    import threading
    out = {}

    def work():
        t = time.perf_counter()
        try:
            out["counts"] = citron.count_batch(gs, ks)
        except Exception as e:          # re-raised below
            out["error"] = e
        out["s"] = time.perf_counter() - t

    th = threading.Thread(target=work)
    th.start()
    last = -1
    while th.is_alive():
        th.join(timeout=every_s)
        if th.is_alive():
            taken, total = citron.batch_progress()
            if total and taken != last:
                log(f"    batch launch: {taken} of {total} work items claimed")
                last = taken
    if "error" in out:
        raise out["error"]
    return out["counts"], out["s"]


def batch_class(name, n, k):
    """Query class of the batched suite: family, size band and k."""
    if name.startswith("rmat"):
        sc = int(name[4:].split("_")[0])
        band = "small" if sc <= 12 else ("mid" if sc <= 14 else "large")
        return f"rmat-{band}-k{k}"
    band = "small" if n <= 10000 else ("mid" if n <= 30000 else "large")
    return f"er-{band}-k{k}"


def run_batch(args, citron, gg, torch, graphs):
    """Batched form: a mixed suite of graphs, every graph queried at every k
    of --batch-ks, in one persistent launch (captured into a HIP graph on the
    first call, replayed later) against the same queries as sequential plain
    counts; the ratio overall and per query class (family, size band, k),
    each class's queries also run as a batch of their own.  Counts are
    checked against the plain counts and against the oracle's stored counts
    of the suite's pinned members (tests/golden/batch512.json)."""
    t_start = time.perf_counter()
    hs = []
    for i, x in enumerate(graphs):
        h = citron.Graph.from_csr(x.row_ptr, x.col).order()
        h.count(3)                       # subgraph rows built: resident graphs
        hs.append(h)
        if i % 64 == 63:
            log(f"  loaded {i + 1} graphs")
    torch.cuda.synchronize()
    bks = args.batch_ks
    qs = [(i, k) for i in range(len(hs)) for k in bks]
    gs = [hs[i] for i, _ in qs]
    ks = [k for _, k in qs]
    cls = [batch_class(graphs[i].name, graphs[i].n, k) for i, k in qs]
    log(f"{len(ks)} queries; sequential plain counts")
    plain, t_q = [], []
    t = time.perf_counter()
    for j, (h, k) in enumerate(zip(gs, ks)):
        t1 = time.perf_counter()
        plain.append(h.count(k))
        t_q.append(time.perf_counter() - t1)
        if j % 256 == 255:
            log(f"  {j + 1} plain counts, {time.perf_counter() - t:.1f} s")
    t_seq = time.perf_counter() - t
    log(f"  sequential {t_seq:.2f} s; batched launch")
    got, t_first = batch_with_progress(citron, gs, ks)    # captured, then run
    log(f"  batched (capture + run) {t_first:.2f} s")
    if got != plain:
        raise SystemExit("batched counts differ from plain counts")
    t_replay = None
    if time.perf_counter() - t_start + t_first < args.budget_s:
        got, t_replay = batch_with_progress(citron, gs, ks)
        log(f"  batched replay {t_replay:.2f} s")
        if got != plain:
            raise SystemExit("batched replay differs from plain counts")
    # the oracle's stored counts of the pinned members
    gold = load_golden("batch512")
    pinned = 0
    if gold and len(graphs) == gold["suite"]["count"]:
        pos = {m["position"]: m for m in gold["members"]}
        for (i, k), c in zip(qs, got):
            if i in pos and str(k) in pos[i]["counts"]:
                if c != pos[i]["counts"][str(k)]["count"]:
                    raise SystemExit(f"batched count differs from the oracle: {graphs[i].name} k={k}")
                pinned += 1
    # per class: the class's sequential time and its own batched launch
    by = {}
    for j, c in enumerate(cls):
        by.setdefault(c, []).append(j)
    per_class = []
    for c in sorted(by, key=lambda c: sum(t_q[j] for j in by[c])):
        js = by[c]
        seq = sum(t_q[j] for j in js)
        rec = {"class": c, "queries": len(js), "sequential_s": seq}
        if time.perf_counter() - t_start + 2 * seq < args.budget_s:
            sub_g, sub_k = [gs[j] for j in js], [ks[j] for j in js]
            batch_with_progress(citron, sub_g, sub_k)       # capture
            sub, rec["batched_s"] = batch_with_progress(citron, sub_g, sub_k)
            rec["speedup"] = seq / rec["batched_s"]
            if sub != [plain[j] for j in js]:
                raise SystemExit(f"class {c}: batched counts differ from plain counts")
        per_class.append(rec)
        log(f"  {rec}")
    t_b = t_replay if t_replay is not None else t_first
    line = {
        "metric": "k-clique count time & edges/s per (graph,k); batched/served vs plain; p99 lat",
        "form": "batched", "value": len(ks) / t_b, "unit": "queries/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": t_b * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"batch of {len(graphs)} graphs (R-MAT scale 8..16, edge factor 8..32; "
                               f"Erdos-Renyi n 1k..50k, mean degree 10..40; seeds 4000+i), "
                               f"k = {bks}", "queries": len(ks),
                   "edges_total": int(sum(x.m for x in graphs))},
        "sequential_plain_s": t_seq, "batched_first_call_s": t_first, "batched_replay_s": t_replay,
        "speedup_vs_sequential": t_seq / t_b, "counts_equal_plain": True,
        "counts_equal_oracle_pinned": pinned, "per_class": per_class,
    }
    print(json.dumps(line), flush=True)


def run_list(args, citron, gg, torch):
    """Listing form: every k-clique of the workload graph, listed arc by arc
    (citron_list_arcs over all arcs: per-arc counts, their scan, the
    listing launch), for each k of --ks; output-bound, 4k bytes per clique.
    The number listed is checked against the oracle's stored count."""
    g = gg.config_graph(args.workload)
    gold = load_golden(args.workload)
    h = citron.Graph.from_csr(g.row_ptr, g.col).order()
    h.count(3)
    arcs = torch.arange(g.m, dtype=torch.int32, device="cuda")
    per_k = {}
    for k in args.ks:
        got, offs = h.list_arcs(k, arcs)                  # sizes the buffers (allocator warm)
        n_cl = int(got.shape[0])
        del got, offs
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        got, offs = h.list_arcs(k, arcs)
        b.record()
        b.synchronize()
        ms = a.elapsed_time(b)
        rec = {"cliques": n_cl, "ms": ms, "cliques_per_s": n_cl / (ms / 1e3),
               "output_GBps": 4 * k * n_cl / (ms / 1e3) / 1e9}
        if gold and str(k) in gold.get("counts", {}):
            rec["equals_oracle_count"] = n_cl == gold["counts"][str(k)]["count"]
        per_k[str(k)] = rec
        log(f"  k={k}: {rec}")
        del got, offs
        torch.cuda.empty_cache()
    tot_cl = sum(r["cliques"] for r in per_k.values())
    tot_s = sum(r["ms"] for r in per_k.values()) / 1e3
    line = {
        "metric": "k-clique count time & edges/s per (graph,k); batched/served vs plain; p99 lat",
        "form": "listing", "value": tot_cl / tot_s, "unit": "cliques/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": tot_s * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "i32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: " + WORKLOADS.get(args.workload, args.workload),
                   "n": g.n, "m": g.m, "ks": args.ks, "arcs": "all"},
        "per_k": per_k,
        "roofline": {"bound": "hbm", "unit": "GB/s", "peak": PEAK_HBM_GBS,
                     "achieved": sum(4 * int(k) * r["cliques"] for k, r in per_k.items()) / tot_s / 1e9,
                     "note": "bytes of clique output written over the listing time (per-arc counts, scan "
                             "and listing launch)"},
    }
    line["roofline"]["frac"] = line["roofline"]["achieved"] / PEAK_HBM_GBS
    print(json.dumps(line), flush=True)


def latency_breakdown(req, results, classes):
    """Arrival-to-completion latency per (graph class, k): request i of
    ``req`` is (graph index, k), results carry its index as their tag, and
    classes[graph index] names the graph's class (e.g. its R-MAT scale)."""
    groups = {}
    for r in results:
        gi, k = req[r["tag"]]
        groups.setdefault((classes[gi], k), []).append((r["t_done_ns"] - r["t_submit_ns"]) / 1e6)
    return [{"graph": c, "k": k, "n": len(v), "p50_ms": float(np.percentile(v, 50)),
             "p99_ms": float(np.percentile(v, 99))} for (c, k), v in sorted(groups.items())]


def run_serve(args, citron, gg, torch):
    """Served form: resident graphs, Poisson arrivals of (graph, k) requests,
    continuous batching; latency percentiles and counts/s, against the same
    arrival trace served first-come-first-served by plain counts."""
    t = time.perf_counter()
    big = gg.config_graph("chunglu22") if args.serve_big else gg.rmat(17, 16, seed=17)
    graphs = gg.serve_suite(count=args.serve_graphs, seed0=5000, scale_min=12,
                            scale_max=args.serve_scale_max, big=big)
    log(f"generated {len(graphs)} graphs in {time.perf_counter() - t:.1f} s")
    classes = [x.name.split("_")[0] for x in graphs[:-1]] + ["chunglu22" if args.serve_big else "rmat17"]
    hs = []
    for x in graphs:
        h = citron.Graph.from_csr(x.row_ptr, x.col).order()
        h.count(3)
        hs.append(h)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5999)
    nreq = args.serve_requests
    kmin, kmax = args.serve_k
    req = [(int(rng.integers(len(hs))), int(rng.integers(kmin, kmax + 1))) for _ in range(nreq)]
    # plain counts (the reference values and the per-request service times)
    log("plain counts of every distinct request")
    plain, svc = {}, {}
    for j, (gi, k) in enumerate(sorted(set(req))):
        if j % 50 == 0:
            log(f"  {j} distinct requests counted")
        t = time.perf_counter()
        plain[(gi, k)] = hs[gi].count(k)
        svc[(gi, k)] = time.perf_counter() - t
    srv = citron.Server(hbm_budget_bytes=8 << 30, max_slots=64)
    ids = [srv.add_graph(h) for h in hs]

    def serve(arrivals):
        done = []
        t0 = time.perf_counter()
        i = 0
        shown = 0
        while len(done) < len(arrivals):
            now = time.perf_counter() - t0
            while i < len(arrivals) and arrivals[i] <= now:
                gi, k = req[i]
                srv.submit(ids[gi], k, i)
                i += 1
            done += srv.poll()
            if len(done) >= shown + 100:
                shown = len(done) - len(done) % 100
                log(f"    {len(done)} of {len(arrivals)} served, {time.perf_counter() - t0:.1f} s")
            time.sleep(0.0002)
        return done, time.perf_counter() - t0

    # saturated throughput: every request at time 0
    res, span = serve([0.0] * nreq)
    sat = nreq / span
    for r in res:
        if r["status"] != 0 or r["count"] != plain[req[r["tag"]]]:
            raise SystemExit(f"served result differs from plain: {r}")
    log(f"saturated: {sat:.1f} requests/s")
    points = []
    for frac in args.serve_load:
        lam = frac * sat
        arr = np.cumsum(rng.exponential(1.0 / lam, nreq)).tolist()
        res, span = serve(arr)
        lat = []
        for r in res:
            gi, k = req[r["tag"]]
            if r["status"] != 0 or r["count"] != plain[(gi, k)]:
                raise SystemExit(f"served result differs from plain: {r}")
            lat.append((r["t_done_ns"] - r["t_submit_ns"]) / 1e6)
        # FIFO plain service of the same trace (one request at a time)
        clock, fifo = 0.0, []
        for j, a in enumerate(arr):
            clock = max(clock, a) + svc[req[j]]
            fifo.append((clock - a) * 1e3)
        p = {"load": frac, "lambda_rps": lam, "served_rps": nreq / span,
             "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
             "fifo_plain_p50_ms": float(np.percentile(fifo, 50)),
             "fifo_plain_p99_ms": float(np.percentile(fifo, 99)),
             "fifo_plain_rps": nreq / clock,
             "by_graph_k": latency_breakdown(req, res, classes)}
        log(f"  load {frac}: {p}")
        points.append(p)
    srv.close()
    line = {
        "metric": "k-clique count time & edges/s per (graph,k); batched/served vs plain; p99 lat",
        "form": "served", "value": sat, "unit": "requests/s (saturated)", "n_gpus": 1,
        "steps": len(points), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{len(graphs)} resident graphs (R-MAT scale 12..{args.serve_scale_max}, "
                               f"edge factor 16, seeds 5000+i, plus "
                               f"{'the Chung-Lu 2^22 graph' if args.serve_big else 'R-MAT scale 17'}), "
                               f"Poisson arrivals, k uniform in {kmin}..{kmax}",
                   "requests_per_point": nreq},
        "fifo_plain_saturated_rps": nreq / sum(svc[r] for r in req),
        "points": points, "counts_equal": True,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="rmat20")
    ap.add_argument("--ks", type=int, nargs="+", default=[5, 6, 7])
    ap.add_argument("--order", choices=["degree", "core"], default="degree",
                    help="ordering phase: the degree ordering (Section IV, default) or the core "
                         "ordering (level-synchronous peeling)")
    ap.add_argument("--unit", choices=["edge", "vertex"], default="edge",
                    help="unit of work of the count: arcs with heavy ones split (default) or whole "
                         "vertices (the paper's unit; an ablation)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget-s", type=float, default=20.0,
                    help="seconds of host wall time the CPU baseline aims for")
    ap.add_argument("--budget-s", type=float, default=500.0,
                    help="warm-up and timed steps stop when another step would end later than "
                         "this many seconds after the process started (at least one step is timed)")
    ap.add_argument("--part-range", type=int, nargs=2, default=None,
                    help="with --parts: run only shares LO..HI-1 (a long count split over "
                         "several runs; the line then reports those shares)")
    ap.add_argument("--parts", type=int, default=1,
                    help="run each count as this many strided shares of its work items "
                         "(one launch each, progress after each); for counts of many minutes")
    ap.add_argument("--stats", action="store_true",
                    help="also run instrumented launches and report the kernel's work counters")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--form", choices=["plain", "batch", "serve", "list"], default="plain",
                    help="plain (default): the workload above; batch / serve: the batched and "
                         "served forms against sequential plain counts")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--batch-ks", type=int, nargs="+", default=[3, 4, 5, 6, 7, 8],
                    help="the k values every graph of the batched suite is queried at")
    ap.add_argument("--serve-graphs", type=int, default=64)
    ap.add_argument("--serve-requests", type=int, default=600)
    ap.add_argument("--serve-scale-max", type=int, default=16)
    ap.add_argument("--serve-k", type=int, nargs=2, default=[3, 8],
                    help="served requests draw k uniformly from this range")
    ap.add_argument("--serve-big", action="store_true",
                    help="the last served graph is the Chung-Lu 2^22 graph (else R-MAT scale 17)")
    ap.add_argument("--serve-load", type=float, nargs="+", default=[0.5, 0.9])
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}))
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus 1)", file=sys.stderr)
        sys.exit(2)

    import graphgen as gg
    pre = None
    if args.form == "batch":
        # generated before the GPU is touched (worker processes)
        t = time.perf_counter()
        pre = gg.batch_suite(count=args.batch_graphs, seed0=4000, workers=16)
        log(f"generated {len(pre)} graphs, m = {sum(x.m for x in pre)} in "
            f"{time.perf_counter() - t:.1f} s")

    if args.form in ("batch", "serve", "list"):
        import torch
        import paper_2112_10913_amd as citron

        torch.cuda.set_device(0)
        # load the device code objects once (not a step: a tiny graph)
        tiny = gg.rmat(8, 8, seed=1)
        citron.Graph.from_csr(tiny.row_ptr, tiny.col).order().count(4)
        torch.cuda.synchronize()
        if args.form == "batch":
            return run_batch(args, citron, gg, torch, pre)
        if args.form == "list":
            return run_list(args, citron, gg, torch)
        return run_serve(args, citron, gg, torch)
    t = time.perf_counter()
    g = gg.config_graph(args.workload)
    log(f"generated {args.workload}: n={g.n} m={g.m} in {time.perf_counter() - t:.1f} s")
    gold = load_golden(args.workload)
    cpu = None
    if not args.no_cpu_baseline and not args.parts > 1:
        # before the GPU is touched: worker processes fork from a process
        # without device state, and the host is otherwise idle
        log("cpu baseline (oracle, all host cores, sampled roots)")
        t = time.perf_counter()
        cpu = cpu_baseline(g, min(args.ks), budget_s=args.cpu_budget_s)
        log(f"  {cpu['value']:.4g} edges/s on {cpu['cores']} cores ({time.perf_counter() - t:.1f} s)")

    import torch
    import paper_2112_10913_amd as citron

    torch.cuda.set_device(0)
    # load the device code objects once (not a step: a tiny graph)
    tiny = gg.rmat(8, 8, seed=1)
    citron.Graph.from_csr(tiny.row_ptr, tiny.col).order().count(4)
    torch.cuda.synchronize()
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    torch.cuda.synchronize()

    shares = {}

    def step():
        ev = {}
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        h = citron.Graph.from_csr(rp, col)
        h.order(args.order)
        e1.record()
        ev["order"] = (e0, e1)
        counts = {}
        for k in args.ks:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            if args.parts > 1:
                # the count as strided shares of its work items, one launch
                # each (progress after each share; the shares add up)
                tot, ovf = 0, False
                lo, hi = args.part_range if args.part_range else (0, args.parts)
                for p in range(lo, hi):
                    pa = torch.cuda.Event(enable_timing=True)
                    pb = torch.cuda.Event(enable_timing=True)
                    pa.record()
                    v, o = h.count_part(k, p, args.parts)
                    pb.record()
                    pb.synchronize()
                    shares.setdefault(k, []).append({"part": p, "value": v, "overflow": o,
                                                     "ms": pa.elapsed_time(pb)})
                    tot += v
                    ovf |= o
                    log(f"    k={k} share {p + 1}/{args.parts}: {v} in {pa.elapsed_time(pb):.1f} ms")
                counts[k] = (tot % 2**64, ovf or tot >= 2**64)
            elif args.unit == "vertex":
                counts[k] = (h.count_vertex_rooted(k), False)
            else:
                counts[k] = h.count_checked(k)
            b.record()
            ev[k] = (a, b)
            b.synchronize()
            log(f"  k={k} count={counts[k][0]} overflow={counts[k][1]} "
                f"{a.elapsed_time(b):.1f} ms")
        return h, counts, ev

    def elapsed():
        return time.monotonic() - T_PROCESS_START

    warm_done, t_step = 0, None
    for i in range(args.warmup):
        # after the first warm-up step (code paths and allocations warmed),
        # further ones run only while the budget still holds every step asked for
        if t_step is not None and elapsed() + (args.warmup - i + args.steps) * t_step > args.budget_s:
            log(f"warm-up stops after {warm_done} of {args.warmup} steps (time budget)")
            break
        log(f"warmup step {i + 1}/{args.warmup}")
        t = time.perf_counter()
        h, _, _ = step()
        torch.cuda.synchronize()
        t_step = time.perf_counter() - t
        h.free()
        warm_done += 1
    torch.cuda.synchronize()
    per_k_ms = {k: [] for k in args.ks}
    order_ms = []
    results = None
    h = None
    steps_done = 0
    t0 = time.perf_counter()
    for i in range(args.steps):
        if steps_done > 0 and elapsed() + (time.perf_counter() - t0) / steps_done > args.budget_s:
            log(f"timed steps stop after {steps_done} of {args.steps} (time budget)")
            break
        log(f"timed step {i + 1}/{args.steps}")
        if h is not None:
            h.free()
        h, counts, ev = step()
        torch.cuda.synchronize()
        order_ms.append(ev["order"][0].elapsed_time(ev["order"][1]))
        for k in args.ks:
            per_k_ms[k].append(ev[k][0].elapsed_time(ev[k][1]))
        results = counts
        steps_done += 1
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall * 1e3 / steps_done
    info = h.info()
    m = g.m
    value = len(args.ks) * m / (ms_per_step / 1e3)

    per_k = {}
    for k in args.ks:
        t_ms = float(np.mean(per_k_ms[k]))
        per_k[str(k)] = {"count": results[k][0], "overflow": results[k][1],
                         "t_count_ms_mean": t_ms, "t_count_ms_median": float(np.median(per_k_ms[k])),
                         "edges_per_s": m / (t_ms / 1e3),
                         # the first count of a step also builds the graph's
                         # subgraph rows and schedule (once per graph)
                         "includes_subgraph_build": k == args.ks[0]}
        if gold and str(k) in gold.get("counts", {}):
            per_k[str(k)]["equals_oracle"] = (results[k][0] == gold["counts"][str(k)]["count"])

    # Algorithmic work of a count (Section III, Algorithm 2 with the
    # degrees-only last level): one 64-bit AND (+ popcount on the last
    # level) per j-clique for j = 3 .. k-1, i.e. sum_{j=3}^{k-1} c_j word
    # operations, each 4 int32 VALU lane-ops.  c_j are exact counts of
    # smaller k, taken from this run or counted outside the timed region.
    # (a partial run of shares does its share of the work)
    frac_run = 1.0
    if args.parts > 1 and args.part_range:
        frac_run = (args.part_range[1] - args.part_range[0]) / args.parts
    cj = {k: results[k][0] for k in args.ks} if frac_run == 1.0 else {}
    for j in range(3, max(args.ks)):
        if j not in cj:
            cj[j] = h.count(j)
    tot_ops, tot_ms = 0, 0.0
    for k in args.ks:
        words = int(sum(cj[j] for j in range(3, k)) * frac_run)
        t_s = per_k[str(k)]["t_count_ms_mean"] / 1e3
        per_k[str(k)]["alg_word_ops"] = words
        per_k[str(k)]["valu"] = {"achieved_Tops": OPS_PER_WORD * words / t_s / 1e12,
                                 "frac": OPS_PER_WORD * words / t_s / 1e12 / PEAK_VALU_TOPS}
        # (the stored work model is that of the degree-ordered DAG)
        hb = alg_bytes(gold, k) if args.order == "degree" else None
        if hb is not None:
            hb *= frac_run
            per_k[str(k)]["hbm"] = {"alg_bytes": hb, "achieved_GBps": hb / t_s / 1e9,
                                    "frac": hb / t_s / 1e9 / PEAK_HBM_GBS}
        tot_ops += OPS_PER_WORD * words
        tot_ms += per_k[str(k)]["t_count_ms_mean"]
    achieved = tot_ops / (tot_ms / 1e3) / 1e12
    roofline = {"bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "Top/s",
                "frac": achieved / PEAK_VALU_TOPS, "traffic": traffic_per_launch(args.ks),
                "kernel": "count_kernel",
                "algorithmic_unit": "int32 VALU lane-ops: 4 per 64-bit AND+popcount, one per j-clique, "
                                    "j = 3..k-1",
                "launch_ms_mean": tot_ms / len(args.ks),
                "hbm_model": "per k: bytes of the merge-based subgraph construction over every arc with "
                             "|C_uv| >= k-2, 4(d(u)+d(v)) + 4 sum_{w in C_uv} d(w) + 8(|C_uv|+1), "
                             "over the count time, against 8 TB/s (per_k[k].hbm)"}
    if args.stats:
        # instrumented launches (not timed): the kernel's own word operations
        for k in args.ks:
            log(f"  work counters k={k}")
            per_k[str(k)]["work"] = h.work_stats(k)

    line = {
        "metric": "k-clique count time & edges/s per (graph,k); batched/served vs plain; p99 lat",
        "value": value, "unit": "edges/s", "n_gpus": 1, "steps": steps_done, "warmup": warm_done,
        "steps_requested": args.steps, "warmup_requested": args.warmup, "budget_s": args.budget_s,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: " + WORKLOADS.get(args.workload, args.workload),
                   "n": g.n, "m": m, "ks": args.ks, "max_outdeg": info["max_outdeg"],
                   "device_bytes": info["device_bytes"],
                   "ordering": args.order, "unit": args.unit, "parallelism": "single GPU"},
        "t_order_ms_mean": float(np.mean(order_ms)),
        "per_k": per_k,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if shares:
        line["shares"] = {str(k): v for k, v in shares.items()}
        if args.part_range:
            # only some shares ran: the counts above are partial sums
            line["partial"] = {"nparts": args.parts, "range": args.part_range}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
