"""Batched form: replays of the captured launch and the autotuner; the mixed
512-graph suite checked against the oracle's stored counts on a subset of
its members and against plain counts for the rest.  Every count must be
exact."""
import json
import os
import time

import numpy as np
import pytest

import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def queries(citron_gpu):
    graphs = gg.batch_suite(count=12, seed0=4000, scale_max=11)
    hs = [citron_gpu.Graph.from_csr(g.row_ptr, g.col).order() for g in graphs]
    gs, ks = [], []
    for h in hs:
        for k in range(3, 9):
            gs.append(h)
            ks.append(k)
    plain = [h.count(k) for h, k in zip(gs, ks)]
    return gs, ks, plain


def test_replays_with_eager_work_between(citron_gpu, queries):
    gs, ks, plain = queries
    for i in range(4):          # the first call captures, the rest replay
        assert citron_gpu.count_batch(gs, ks) == plain, i
        assert gs[i].count(ks[i]) == plain[i]       # eager work between replays


def test_query_subsets_and_order(citron_gpu, queries):
    gs, ks, plain = queries
    rng = np.random.default_rng(3)
    perm = rng.permutation(len(ks))[:40]
    got = citron_gpu.count_batch([gs[i] for i in perm], [ks[i] for i in perm])
    assert got == [plain[i] for i in perm]


def test_autotune_keeps_counts(citron_gpu, queries, tmp_path):
    from paper_2112_10913_amd.autotune import autotune
    gs, ks, plain = queries
    space = {"wg_waves": [2, 4], "blocks_per_cu": [1, 2], "flush_rows": [64, 128], "arc_lds_max": [128, 256],
             "split_pct": [50, 200]}
    cache = str(tmp_path / "tune.json")
    best, report = autotune(gs, ks, space=space, reps=1, cache_path=cache)
    assert not report["cached"] and len(report["trials"]) == 32
    assert citron_gpu.count_batch(gs, ks, tuning=best) == plain
    again, rep2 = autotune(gs, ks, space=space, reps=1, cache_path=cache)
    assert rep2["cached"] and again == best


def test_mixed_suite_of_512_graphs_against_the_oracle(citron_gpu, progress):
    """The batched configuration: 512 graphs (R-MAT scale 8..16 with edge
    factor 8..32, Erdos-Renyi with n 1k..50k and mean degree 10..40), every
    graph at k = 3..7 and at k = 8 except the R-MAT graphs of scale 15 and 16
    (their k = 8 counts take 345 s of the suite's 384 s as plain counts), in
    one count_batch call.  The oracle's stored counts
    (tests/golden/batch512.json, k = 3..8) pin a subset that spans both
    families; the other queries must equal plain counts."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "batch512.json")) as f:
        gold = json.load(f)
    graphs = gg.batch_suite(count=gold["suite"]["count"], seed0=gold["suite"]["seed0"], workers=8)
    progress(f"  generated {len(graphs)} graphs")
    hs = [citron_gpu.Graph.from_csr(g.row_ptr, g.col).order() for g in graphs]
    progress("  loaded and ordered")
    gs, ks, where = [], [], []
    for i, (g, h) in enumerate(zip(graphs, hs)):
        big = g.name.startswith(("rmat15", "rmat16"))
        for k in range(3, 9):
            if k == 8 and big:
                continue
            gs.append(h)
            ks.append(k)
            where.append((i, k))
    t = time.perf_counter()
    got = citron_gpu.count_batch(gs, ks)
    progress(f"  batch of {len(ks)} queries: {time.perf_counter() - t:.1f} s")
    pos = {m["position"]: m for m in gold["members"]}
    checked = set()
    for (i, k), c in zip(where, got):
        if i in pos:
            assert graphs[i].sha256() == pos[i]["sha256"]
            assert c == pos[i]["counts"][str(k)]["count"], (graphs[i].name, k)
            checked.add(i)
    assert checked == set(pos)
    kinds = {graphs[i].name[:2] for i in checked}
    assert kinds == {"rm", "er"}
    t = time.perf_counter()
    plain = []
    for j, (h, k) in enumerate(zip(gs, ks)):
        plain.append(h.count(k))
        if j % 500 == 499:
            progress(f"  {j + 1} plain counts, {time.perf_counter() - t:.1f} s")
    assert got == plain


def test_progress_of_a_running_batch(citron_gpu):
    """citron_batch_progress from another thread while a batch runs: the
    items claimed grow, never exceed the total, and read (0, 0) after."""
    import threading
    g = gg.rmat(15, 28, seed=4456)
    h = citron_gpu.Graph.from_csr(g.row_ptr, g.col).order()
    want = h.count(7)
    out = {}
    th = threading.Thread(target=lambda: out.setdefault("c", citron_gpu.count_batch([h, h], [7, 6])))
    th.start()
    seen = []
    while th.is_alive():
        taken, total = citron_gpu.batch_progress()
        if total:
            assert 0 <= taken <= total
            seen.append(taken)
        time.sleep(0.005)
    th.join()
    assert out["c"][0] == want
    assert seen and seen[-1] >= seen[0]
    assert citron_gpu.batch_progress() == (0, 0)
