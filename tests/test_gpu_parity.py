"""GPU parity: libcitron (HIP, gfx950) against the reference counter.

Integer results must agree bit for bit: DAGs byte for byte, counts exactly.
Large graphs compare against stored values written by
tests/golden/make_golden.py (which calls only oracle/), or against sampled
per-arc counts that the oracle computes one arc at a time.
"""
import json
import math
import os
import sys
import time

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def load(citron, g):
    return citron.Graph.from_csr(g.row_ptr, g.col).order()


def ocount(g, k):
    c, ovf = oracle.count(g, k)
    assert not ovf
    return c


# ------------------------------------------------------------------ DAG

@pytest.mark.parametrize("name", ["fig1", "rmat12", "er", "rmat14"])
def test_dag_matches_oracle(citron_gpu, name):
    g = {"fig1": gg.fig1_example, "rmat12": lambda: gg.rmat(12, 16, seed=5),
         "er": lambda: gg.erdos_renyi(5000, 20, seed=6),
         "rmat14": lambda: gg.config_graph("rmat14")}[name]()
    say("dag", name, g.n, g.m)
    h = load(citron_gpu, g)
    dptr, dcol = h.dag()
    optr, ocol = oracle.orient(g.n, g.row_ptr, g.col)
    assert np.array_equal(dptr, optr)
    assert np.array_equal(dcol, ocol)
    assert h.info()["max_outdeg"] == int(np.diff(optr).max(initial=0))


# ------------------------------------------------------------ small graphs

def test_fig1_counts(citron_gpu):
    with open(os.path.join(GOLDEN, "fig1.json")) as f:
        fig = json.load(f)
    h = load(citron_gpu, gg.fig1_example())
    for k, want in fig["clique_counts"].items():
        assert h.count(int(k)) == want


def _esym(parts, k):
    from itertools import combinations
    return sum(math.prod(c) for c in combinations(parts, k))


def test_closed_forms(citron_gpu):
    """Expected values are the closed forms themselves (complete graphs,
    Turan graphs, bipartite graphs, wheels, disjoint cliques, Kneser and
    Paley graphs, empty)."""
    cases = [
        (gg.complete(30), lambda k: math.comb(30, k), 8),
        (gg.complete(64), lambda k: math.comb(64, k), 6),
        (gg.complete(65), lambda k: math.comb(65, k), 6),     # two-word rows
        (gg.complete(130), lambda k: math.comb(130, k), 5),   # three-word rows
        (gg.complete(600), lambda k: math.comb(600, k), 4),   # rows staged in device memory
        (gg.turan(40, 7), lambda k: _esym([6, 6, 6, 6, 6, 5, 5], k), 8),
        (gg.complete_bipartite(20, 30), lambda k: [0, 50, 600][k] if k < 3 else 0, 8),
        (gg.hypercube(7), lambda k: [0, 128, 448][k] if k < 3 else 0, 8),
        (gg.wheel(50), lambda k: [0, 51, 100, 50][k] if k < 4 else 0, 8),
        (gg.disjoint_cliques([3, 10, 66, 129, 1]),
         lambda k: sum(math.comb(s, k) for s in [3, 10, 66, 129, 1]), 5),
        # Kneser K(11,3): k pairwise disjoint 3-subsets of 11 elements
        (gg.kneser(11, 3), lambda k: [1, 165, 4620, 15400][k] if k < 4 else 0, 7),
        # Paley(101): strongly regular, q(q-1)/4 edges, q(q-1)(q-5)/48 triangles
        (gg.paley(101), lambda k: [1, 101, 2525, 20200][k], 3),
        (gg.empty(5), lambda k: 5 if k == 1 else 0, 8),
        (gg.empty(0), lambda k: 0, 8),
    ]
    for g, want, kmax in cases:
        say("closed form", g.name)
        h = load(citron_gpu, g)
        for k in range(1, kmax + 1):
            assert h.count(k) == want(k), (g.name, k)


def test_large_k_stack_modes(citron_gpu):
    """k above 8 keeps the search stacks in LDS (k <= 12) or in device
    memory (k >= 13): closed forms and the oracle at those k, plain and
    per-arc launches."""
    cases = [
        (gg.complete(32), lambda k: math.comb(32, k), range(9, 21)),
        (gg.complete(66), lambda k: math.comb(66, k), range(9, 11)),   # two-word rows
        (gg.turan(36, 12), lambda k: _esym([3] * 12, k), range(9, 14)),
    ]
    for g, want, ks in cases:
        h = load(citron_gpu, g)
        for k in ks:
            say("large k", g.name, k)
            assert h.count(k) == want(k), (g.name, k)
            total, per_arc = h.count_per_arc(k)
            assert total == want(k) and int(per_arc.sum(dtype=np.uint64)) == total, (g.name, k)
    g = gg.erdos_renyi(120, 0.6 * 119, seed=12)
    h = load(citron_gpu, g)
    for k in range(9, 15):
        say("large k ER", k)
        assert h.count(k) == ocount(g, k), k


def test_random_fuzz(citron_gpu):
    rng = np.random.default_rng(2112)
    for i in range(40):
        n = int(rng.integers(2, 300))
        p = float(rng.uniform(0.02, 0.6 if n <= 100 else 0.25))
        iu, ju = np.triu_indices(n, 1)
        keep = rng.random(iu.size) < p
        g = gg.csr_from_edges(n, iu[keep], ju[keep], perm_seed=i)
        h = load(citron_gpu, g)
        for k in range(3, 8):
            assert h.count(k) == ocount(g, k), (i, n, p, k)


def test_dense_random_graphs(citron_gpu):
    # out-degrees of several hundred: multi-word rows, some staged in device memory
    for n, p, seed in [(600, 0.5, 1), (1200, 0.3, 2), (300, 0.8, 3)]:
        g = gg.erdos_renyi(n, p * (n - 1), seed=seed)
        h = load(citron_gpu, g)
        say("dense", n, p, h.info())
        for k in (3, 4):
            assert h.count(k) == ocount(g, k), (n, p, k)


def test_heavy_vertices_and_ragged_batches(citron_gpu):
    g = gg.chung_lu(n=20000, mean_degree=30, w_max=3000, planted=50, clique_min=20,
                    clique_max=70, seed=40, clique_seed=50)
    h = load(citron_gpu, g)
    say("chung-lu", g.n, g.m, h.info())
    for k in (3, 4, 5):
        assert h.count(k) == ocount(g, k), k


# --------------------------------------------------------- named workloads

def _golden(name):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        return json.load(f)


def test_rmat14_counts(citron_gpu):
    gold = _golden("rmat14")
    g = gg.config_graph("rmat14")
    assert g.sha256() == gold["sha256"]
    h = load(citron_gpu, g)
    for k, rec in gold["counts"].items():
        say("rmat14 k", k)
        assert h.count(int(k)) == rec["count"]


def test_rmat14_per_arc(citron_gpu):
    gold = _golden("rmat14")
    g = gg.config_graph("rmat14")
    h = load(citron_gpu, g)
    idx = np.array(gold["arcs"]["index"])
    for k in range(3, 9):
        if str(k) not in gold["arcs"]:
            continue
        total, per_arc = h.count_per_arc(k)
        assert int(per_arc.sum(dtype=np.uint64)) == total
        assert [int(x) for x in per_arc[idx]] == gold["arcs"][str(k)], k
        if str(k) in gold["counts"]:
            assert total == gold["counts"][str(k)]["count"]


def test_count_arcs_matches_per_arc(citron_gpu):
    """List mode (citron_count_arcs) against the full per-arc count, on a
    shuffled list with repeats; errors for bad indices."""
    g = gg.config_graph("rmat14")
    h = load(citron_gpu, g)
    m = h.m
    rng = np.random.default_rng(77)
    arcs = np.concatenate([rng.permutation(m), rng.integers(0, m, 500)]).astype(np.int32)
    for k in range(2, 9):
        total, per_arc = h.count_per_arc(k)
        got = h.count_arcs(k, arcs)
        say("count_arcs k", k, int(got.sum(dtype=np.uint64)))
        assert np.array_equal(got, per_arc[arcs]), k
    assert h.count_arcs(5, np.zeros(0, np.int32)).size == 0
    for bad in ([m], [-1], [0, m + 5]):
        with pytest.raises(citron_gpu.CitronError):
            h.count_arcs(5, np.array(bad, np.int32))


def test_outdegree_one_arcs_read_zero(citron_gpu):
    """Arcs whose source has out-degree 1 close no triangle and are not
    built; their sizes and rows must read as zero even in reused device
    memory (a freed graph's rows are handed out again)."""
    big = load(citron_gpu, gg.config_graph("rmat14"))
    big.count(5)
    big.free()
    # a path, a star, a triangle and a K5: many out-degree-1 sources
    n = 400
    k5 = [(360 + a, 360 + b) for a in range(5) for b in range(a + 1, 5)]
    src = list(range(0, 199)) + [200] * 150 + [350, 351, 352, 350] + [a for a, _ in k5]
    dst = list(range(1, 200)) + list(range(201, 351)) + [351, 352, 350, 353] + [b for _, b in k5]
    g = gg.csr_from_edges(n, np.array(src), np.array(dst), perm_seed=None, name="paths")
    h = load(citron_gpu, g)
    dptr, dcol = h.dag()
    us = np.repeat(np.arange(g.n), np.diff(dptr)).astype(np.int32)
    for k in (3, 4, 5):
        want, ovf = oracle.count_arcs(g.n, dptr, dcol, k, us, dcol)
        assert not ovf
        total, per_arc = h.count_per_arc(k)
        bad = np.flatnonzero(per_arc != want)
        assert bad.size == 0, (k, h.info(), bad[:8], per_arc[bad[:8]], want[bad[:8]], us[bad[:8]], dcol[bad[:8]])
        assert np.array_equal(h.count_arcs(k, np.arange(h.m, dtype=np.int32)), want), k


def test_count_parts_add_up(citron_gpu):
    """Strided shares of the work items add up to the count."""
    gold = _golden("rmat14")
    g = gg.config_graph("rmat14")
    h = load(citron_gpu, g)
    for k in range(2, 9):
        want = h.count(k)
        for nparts in (1, 3, 7):
            shares = [h.count_part(k, p, nparts)[0] for p in range(nparts)]
            assert sum(shares) % 2**64 == want, (k, nparts)
        if str(k) in gold["counts"]:
            assert want == gold["counts"][str(k)]["count"]
    for bad in ((0, 0), (3, 3), (-1, 2)):
        with pytest.raises(citron_gpu.CitronError):
            h.count_part(5, *bad)


def test_count_parts_across_handles(citron_gpu):
    """Shares counted by separately loaded handles of one graph add up to the
    count: the schedule (ties in degree and in |C_uv| included) is fixed by
    the graph, not by the order in which threads of one build ran."""
    graphs = ((gg.config_graph("rmat14"), (5, 7)),
              (gg.chung_lu(n=1 << 14, w_max=2000.0, planted=40, clique_max=24, seed=7, clique_seed=8), (6,)))
    for g, ks in graphs:
        for k in ks:
            want = load(citron_gpu, g).count(k)
            nparts = 5
            shares = [load(citron_gpu, g).count_part(k, p, nparts)[0] for p in range(nparts)]
            assert sum(shares) % 2**64 == want, (g.name, k)


_RMAT20 = {}


def _rmat20(citron):
    if "h" not in _RMAT20:
        gold = _golden("rmat20")
        g = gg.config_graph("rmat20")
        assert g.sha256() == gold["sha256"]
        _RMAT20.update(g=g, gold=gold, h=load(citron, g))
    return _RMAT20["g"], _RMAT20["gold"], _RMAT20["h"]


def test_rmat20_counts(citron_gpu):
    """Full-size R-MAT scale 20: whole-graph counts against the oracle's."""
    g, gold, h = _rmat20(citron_gpu)
    assert h.info()["max_outdeg"] == gold["max_outdeg"]
    for k, rec in gold["counts"].items():
        say("rmat20 k", k)
        assert h.count(int(k)) == rec["count"]


def test_rmat20_per_arc_full_launch(citron_gpu, progress):
    """Full-size per-arc counts (the whole-graph launch) at the sampled arcs."""
    g, gold, h = _rmat20(citron_gpu)
    idx = np.array(gold["arcs"]["index"])
    dptr, dcol = h.dag()
    src = np.repeat(np.arange(g.n), np.diff(dptr))
    assert list(src[idx]) == gold["arcs"]["u"] and list(dcol[idx]) == gold["arcs"]["v"]
    for k in (5, 6, 7):
        progress(f"  rmat20 per-arc launch k={k}")
        total, per_arc = h.count_per_arc(k)
        assert int(per_arc.sum(dtype=np.uint64)) % 2**64 == total
        assert [int(x) for x in per_arc[idx]] == gold["arcs"][str(k)], k
        # the launch the benchmark times (no per-arc output) gives the same
        # whole count as the per-arc launch checked above
        progress(f"  rmat20 whole-count launch k={k}")
        assert h.count(k) == total, k


@pytest.mark.parametrize("k", [5, 6, 7, 8])
def test_rmat20_sampled_arcs(citron_gpu, k):
    """Full-size sampled arcs through the list-mode launch, up to k = 8."""
    g, gold, h = _rmat20(citron_gpu)
    idx = np.array(gold["arcs"]["index"], dtype=np.int32)
    want = gold["arcs"][str(k)]
    step = 32
    for lo in range(0, len(idx), step):
        t = time.perf_counter()
        got = h.count_arcs(k, idx[lo:lo + step])
        say(f"rmat20 count_arcs k={k} arcs {lo}..{lo + step - 1}: {time.perf_counter() - t:.2f} s")
        assert [int(x) for x in got] == want[lo:lo + step], (k, lo)


_CL22 = {}


def _chunglu22(citron):
    if "h" not in _CL22:
        gold = _golden("chunglu22")
        g = gg.config_graph("chunglu22")
        assert g.sha256() == gold["sha256"]
        _CL22.update(g=g, gold=gold, h=load(citron, g))
    return _CL22["g"], _CL22["gold"], _CL22["h"]


def test_chunglu22_counts(citron_gpu):
    """Full-size Chung-Lu graph (2^22 vertices, 2,000 planted cliques):
    whole-graph counts against the oracle's."""
    g, gold, h = _chunglu22(citron_gpu)
    assert h.info()["max_outdeg"] == gold["max_outdeg"]
    for k, rec in gold["counts"].items():
        say("chunglu22 k", k)
        assert h.count(int(k)) == rec["count"]


def test_chunglu22_per_arc_full_launch(citron_gpu, progress):
    g, gold, h = _chunglu22(citron_gpu)
    idx = np.array(gold["arcs"]["index"])
    for k in (5, 6, 7):
        progress(f"  chunglu22 per-arc launch k={k}")
        total, per_arc = h.count_per_arc(k)
        assert int(per_arc.sum(dtype=np.uint64)) % 2**64 == total
        assert [int(x) for x in per_arc[idx]] == gold["arcs"][str(k)], k
        assert h.count(k) == total, k


@pytest.mark.parametrize("k", [5, 6, 7, 8, 9])
def test_chunglu22_sampled_arcs(citron_gpu, k):
    g, gold, h = _chunglu22(citron_gpu)
    if str(k) not in gold["arcs"]:
        pytest.skip(f"no stored per-arc values for k = {k}")
    idx = np.array(gold["arcs"]["index"], dtype=np.int32)
    want = gold["arcs"][str(k)]
    step = 32
    for lo in range(0, len(idx), step):
        t = time.perf_counter()
        got = h.count_arcs(k, idx[lo:lo + step])
        say(f"chunglu22 count_arcs k={k} arcs {lo}..{lo + step - 1}: {time.perf_counter() - t:.2f} s")
        assert [int(x) for x in got] == want[lo:lo + step], (k, lo)


# -------------------------------------------------------------- invariants

def test_tuning_invariance(citron_gpu):
    gold = _golden("rmat14")
    g = gg.config_graph("rmat14")
    want = {k: gold["counts"][str(k)]["count"] for k in (3, 4, 5, 6)}
    idx = np.array(gold["arcs"]["index"])
    deep = {}
    for tu in [dict(wg_waves=1, blocks_per_cu=1, light_rows=64, flush_rows=64, build_blocks_per_cu=1),
               dict(wg_waves=8, blocks_per_cu=1, light_rows=1024, flush_rows=256, build_blocks_per_cu=16),
               dict(wg_waves=2, blocks_per_cu=8, light_rows=128, flush_rows=100, build_blocks_per_cu=2),
               dict(split_pct=25, arc_lds_max=64), dict(split_pct=400, arc_lds_max=128),
               dict(split_pct=250, arc_lds_max=192)]:
        h = citron_gpu.Graph.from_csr(g.row_ptr, g.col)
        h.set_tuning(citron_gpu.Tuning(**tu))   # before the first count: shapes the build too
        h.order()
        for k, w in want.items():
            assert h.count(k) == w, (tu, k)
        for k in (7, 8):    # split factors matter most here
            total, per_arc = h.count_per_arc(k)
            assert [int(x) for x in per_arc[idx]] == gold["arcs"][str(k)], (tu, k)
            deep.setdefault(k, set()).add(total)
    assert all(len(v) == 1 for v in deep.values()), deep


def test_relabel_invariance_gpu(citron_gpu):
    g = gg.rmat(13, 16, seed=9)
    base = {k: load(citron_gpu, g).count(k) for k in (3, 5, 6)}
    p = np.random.default_rng(1).permutation(g.n)
    h = load(citron_gpu, gg.relabel(g, p))
    for k, v in base.items():
        assert h.count(k) == v


def test_repeat_determinism(citron_gpu):
    g = gg.config_graph("rmat14")
    h = load(citron_gpu, g)
    vals = [h.count(6) for _ in range(3)]
    assert len(set(vals)) == 1


def test_batch_equals_plain(citron_gpu):
    graphs = [gg.rmat(s, ef, seed=100 + s) for s, ef in [(8, 8), (10, 32), (12, 16), (9, 20)]]
    graphs += [gg.erdos_renyi(3000, 25, seed=7), gg.fig1_example()]
    hs = [load(citron_gpu, g) for g in graphs]
    gs, ks = [], []
    for h in hs:
        for k in range(1, 9):
            gs.append(h)
            ks.append(k)
    plain = [h.count(k) for h, k in zip(gs, ks)]
    for _ in range(3):  # first call captures, later calls replay
        assert citron_gpu.count_batch(gs, ks) == plain
    tu = citron_gpu.Tuning(wg_waves=2, blocks_per_cu=3, flush_rows=128)
    assert citron_gpu.count_batch(gs, ks, tuning=tu) == plain


# ------------------------------------------------------------ error paths

def test_overflow_flag_forced(citron_gpu):
    g = gg.complete(20)
    h = load(citron_gpu, g)
    want = math.comb(20, 5)
    h.seed_accumulator(2**64 - 10)
    v, ovf = h.count_checked(5)
    assert ovf and v == (2**64 - 10 + want) % 2**64
    v, ovf = h.count_checked(5)          # the seed applies to one call only
    assert not ovf and v == want
    h.seed_accumulator(2**64 - want)     # exactly 2^64 carries
    v, ovf = h.count_checked(5)
    assert ovf and v == 0
    with pytest.raises(citron_gpu.CitronError):
        h.seed_accumulator(2**64 - 1)
        h.count(5)


def _expect_einval(citron, n, rp, col):
    with pytest.raises(citron.CitronError) as ei:
        citron.Graph.from_csr(np.asarray(rp, np.int32), np.asarray(col, np.int32))
    assert ei.value.status == 1


def test_invalid_csr_rejected(citron_gpu):
    c = citron_gpu
    _expect_einval(c, 3, [0, 1, 2, 3], [1, 0])           # row_ptr[n] != nnz
    _expect_einval(c, 2, [0, 1, 1], [1])                 # odd nnz
    _expect_einval(c, 3, [0, 2, 1, 4], [1, 2, 0, 0])     # decreasing row_ptr
    _expect_einval(c, 3, [0, 1, 2, 2], [5, 0])           # out-of-range id
    _expect_einval(c, 2, [0, 1, 2], [0, 1])              # self-loops
    _expect_einval(c, 3, [0, 2, 3, 4], [2, 1, 0, 0])     # unsorted row
    _expect_einval(c, 3, [0, 2, 3, 4], [1, 1, 0, 0])     # duplicate entry
    _expect_einval(c, 3, [0, 1, 1, 2], [1, 0])           # asymmetric: 0-1 and 2-0 one-sided
    _expect_einval(c, 3, [1, 1, 2, 2], [1, 0])           # row_ptr[0] != 0


def test_state_and_k_errors(citron_gpu):
    c = citron_gpu
    g = gg.complete(5)
    h = c.Graph.from_csr(g.row_ptr, g.col)
    with pytest.raises(c.CitronError) as ei:
        h.count(3)
    assert ei.value.status == 5                        # ESTATE before order
    h.order()
    h.order()                                          # idempotent
    for k in (0, -1, 33):
        with pytest.raises(c.CitronError) as ei:
            h.count(k)
        assert ei.value.status == 1
    assert h.count(1) == 5 and h.count(2) == 10 and h.count(5) == 1 and h.count(6) == 0
    assert h.count(32) == 0


def test_device_pointer_input(citron_gpu):
    import torch
    g = gg.rmat(11, 16, seed=3)
    rp = torch.from_numpy(g.row_ptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    h = citron_gpu.Graph.from_csr(rp, col).order()
    assert h.count(4) == ocount(g, 4)


def test_outdegree_limits(citron_gpu, progress):
    """Between the configs' largest out-degree (666) and the 4096 limit the
    rows span up to 64 words (one per lane): closed forms on K_1500 (24-word
    rows) up to k = 4 and K_4097 (out-degree 4096, 64-word rows) at k = 3,
    both units; an out-degree of 4097 is refused with EINVAL."""
    g = gg.complete(1500)
    h = load(citron_gpu, g)
    assert h.info()["max_outdeg"] == 1499
    for k in (3, 4):
        progress(f"  K_1500 k={k}")
        assert h.count(k) == math.comb(1500, k), k
        assert h.count_vertex_rooted(k) == math.comb(1500, k), k
    h.free()
    g = gg.complete(4097)
    h = load(citron_gpu, g)
    assert h.info()["max_outdeg"] == 4096
    progress("  K_4097 k=3")
    assert h.count(3) == math.comb(4097, 3)
    h.free()
    g = gg.complete(4098)
    h = load(citron_gpu, g)
    assert h.info()["max_outdeg"] == 4097
    with pytest.raises(citron_gpu.CitronError) as e:
        h.count(3)
    assert e.value.status == 1
    assert h.count(2) == g.m                 # trivial values need no rows
    h.free()
