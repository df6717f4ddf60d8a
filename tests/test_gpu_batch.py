"""Batched form: replays of the captured launch and the autotuner.  Every
count must equal the plain count exactly."""
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
