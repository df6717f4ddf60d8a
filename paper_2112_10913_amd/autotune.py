"""Autotuner of the count launch for a query set.

The count kernel's speed-only knobs -- workgroup size (``wg_waves``),
resident workgroups per CU (``blocks_per_cu``), the light-engine queue
threshold (``flush_rows``), the subgraph representation switch
(``arc_lds_max``: the largest node copied to LDS) and the split factor of
heavy arcs and light vertices (``split_pct``, a scale of the default
parts; it is part of each graph's schedule, so it is set on the graphs) --
are swept over a query set with the batched entry point (one persistent
launch per trial, replayed from its captured HIP graph).  Every trial must return the same counts as the first one: the
knobs never change results, so a difference is a bug and raises.  The
fastest setting (median over repetitions) is returned and cached per device
and query-set signature in a JSON file.

    import paper_2112_10913_amd as citron
    from paper_2112_10913_amd.autotune import autotune
    best, report = autotune(graphs, ks)     # also sets best.split_pct on the graphs
    citron.count_batch(graphs, ks, tuning=best)
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import time

from ._lib import CitronError, Tuning, count_batch, device_info

DEFAULT_SPACE = {
    "wg_waves": [1, 2, 4, 8],
    "blocks_per_cu": [1, 2, 4, 8],
    "flush_rows": [64, 128],
    "arc_lds_max": [128, 192, 256],
    "split_pct": [50, 100, 200],
}
# waves per CU worth trying: registers allow 16 count waves (k <= 8: 128
# VGPRs, 4 per SIMD), LDS 16 with LDS copies up to 192 candidates
MAX_WAVES_PER_CU = 16


def default_cache_path() -> str:
    base = os.environ.get("XDG_CACHE_HOME", os.path.join(os.path.expanduser("~"), ".cache"))
    return os.path.join(base, "citron", "autotune.json")


def signature(graphs, ks) -> str:
    """Identity of a query set: sizes of its graphs and its k values."""
    h = hashlib.sha256()
    for g, k in zip(graphs, ks):
        h.update(f"{g.n},{g.m},{int(k)};".encode())
    return h.hexdigest()[:32]


def candidates(space=None):
    space = dict(DEFAULT_SPACE, **(space or {}))
    out = []
    for wg, bpc, fr, am, sp in itertools.product(space["wg_waves"], space["blocks_per_cu"], space["flush_rows"],
                                                 space["arc_lds_max"], space["split_pct"]):
        if wg * bpc > MAX_WAVES_PER_CU:
            continue
        out.append(Tuning(wg_waves=wg, blocks_per_cu=bpc, flush_rows=fr, arc_lds_max=am, split_pct=sp))
    return out


def _set_split(graphs, pct):
    """Give every graph of the query set the split scale pct (its schedule)."""
    seen = set()
    for g in graphs:
        if id(g) in seen:
            continue
        seen.add(id(g))
        t = g.get_tuning()
        if t.split_pct != pct:
            t.split_pct = pct
            g.set_tuning(t)


def _time(graphs, ks, t, reps):
    _set_split(graphs, t.split_pct or 100)
    count_batch(graphs, ks, tuning=t)          # capture (first call) and warm
    times = []
    counts = None
    for _ in range(reps):
        t0 = time.perf_counter()
        counts = count_batch(graphs, ks, tuning=t)
        times.append(time.perf_counter() - t0)
    times.sort()
    return times[len(times) // 2], counts


def autotune(graphs, ks, space=None, reps: int = 3, cache_path: str | None = None,
             use_cache: bool = True, log=None, tunings=None):
    """Fastest count-launch tuning for the queries (graphs[i], ks[i]).

    The trials are ``tunings`` if given, else the product of ``space``
    (a dict of lists over DEFAULT_SPACE's keys).  Returns (Tuning, report);
    report lists every trial with its median time in seconds (None when the
    launch was refused, e.g. LDS too small for that shape)."""
    dev = device_info()
    key = signature(graphs, ks)
    path = cache_path or default_cache_path()
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                hit = json.load(f).get(dev["arch"], {}).get(key)
            if hit:
                best = Tuning(**hit["tuning"])
                _set_split(graphs, best.split_pct or 100)
                return best, {"cached": True, "best_s": hit["seconds"]}
        except (OSError, ValueError, TypeError):
            pass
    trials = []
    ref = None
    best = None
    for t in (tunings if tunings is not None else candidates(space)):
        try:
            sec, counts = _time(graphs, ks, t, reps)
        except CitronError as e:
            trials.append({"tuning": t.__dict__, "seconds": None, "error": str(e)})
            continue
        if ref is None:
            ref = counts
        elif counts != ref:
            raise RuntimeError(f"tuning {t} changed a count: the kernel is wrong")
        trials.append({"tuning": t.__dict__, "seconds": sec})
        if log:
            log(f"autotune {t.wg_waves}x{t.blocks_per_cu} flush {t.flush_rows} lds<={t.arc_lds_max} "
                f"split {t.split_pct}%: {sec * 1e3:.2f} ms")
        if best is None or sec < best[1]:
            best = (t, sec)
    if best is None:
        raise RuntimeError("no tuning candidate could be launched")
    _set_split(graphs, best[0].split_pct or 100)
    report = {"cached": False, "best_s": best[1], "trials": trials, "signature": key}
    if use_cache:
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            data = {}
            if os.path.exists(path):
                with open(path) as f:
                    data = json.load(f)
            data.setdefault(dev["arch"], {})[key] = {"tuning": best[0].__dict__, "seconds": best[1]}
            with open(path, "w") as f:
                json.dump(data, f, indent=1)
        except (OSError, ValueError):
            pass
    return best[0], report
