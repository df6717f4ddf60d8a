"""The vertex-rooted unit (Algorithm 2 per vertex, no split): counts against
closed forms, the Figure 1 values, the oracle on random and dense graphs and
the stored oracle counts of the configuration graphs; the same counts as the
edge-rooted launch."""
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _load(citron, g):
    return citron.Graph.from_csr(g.row_ptr, g.col).order()


def _esym(parts, k):
    from itertools import combinations
    return sum(math.prod(c) for c in combinations(parts, k))


def test_fig1_and_closed_forms(citron_gpu):
    with open(os.path.join(GOLDEN, "fig1.json")) as f:
        fig = json.load(f)
    h = _load(citron_gpu, gg.fig1_example())
    for k, want in fig["clique_counts"].items():
        assert h.count_vertex_rooted(int(k)) == want, k
    cases = [
        (gg.complete(30), lambda k: math.comb(30, k), range(1, 9)),
        (gg.complete(65), lambda k: math.comb(65, k), range(3, 7)),     # a two-word root
        (gg.complete(130), lambda k: math.comb(130, k), range(3, 6)),   # three words, LDS copy
        (gg.complete(300), lambda k: math.comb(300, k), range(3, 5)),   # rows walked in device memory
        (gg.turan(40, 7), lambda k: _esym([6, 6, 6, 6, 6, 5, 5], k), range(3, 9)),
        (gg.complete_bipartite(20, 30), lambda k: 0, range(3, 9)),
        (gg.wheel(50), lambda k: [0, 51, 100, 50][k] if k < 4 else 0, range(3, 9)),
        (gg.disjoint_cliques([3, 10, 66, 129, 1]),
         lambda k: sum(math.comb(s, k) for s in [3, 10, 66, 129, 1]), range(3, 6)),
        (gg.empty(5), lambda k: 0, range(3, 6)),
    ]
    for g, want, ks in cases:
        h = _load(citron_gpu, g)
        for k in ks:
            assert h.count_vertex_rooted(k) == want(k), (g.name, k)


def test_deep_k_stack_modes(citron_gpu):
    # a root unit has one more level than an arc unit: k = 8 already takes
    # the LDS stacks, k >= 12 the device-memory stacks
    for g, want, ks in [(gg.complete(32), lambda k: math.comb(32, k), range(7, 19)),
                        (gg.complete(66), lambda k: math.comb(66, k), range(7, 10)),
                        (gg.turan(36, 12), lambda k: _esym([3] * 12, k), range(7, 14))]:
        h = _load(citron_gpu, g)
        for k in ks:
            assert h.count_vertex_rooted(k) == want(k), (g.name, k)


def test_random_and_dense_graphs_against_the_oracle(citron_gpu):
    rng = np.random.default_rng(77)
    for i in range(20):
        n = int(rng.integers(2, 250))
        p = float(rng.uniform(0.02, 0.5 if n <= 100 else 0.2))
        iu, ju = np.triu_indices(n, 1)
        keep = rng.random(iu.size) < p
        g = gg.csr_from_edges(n, iu[keep], ju[keep], perm_seed=i)
        h = _load(citron_gpu, g)
        for k in range(3, 8):
            assert h.count_vertex_rooted(k) == oracle.count(g, k)[0], (i, n, p, k)
    for n, p, seed in [(600, 0.5, 1), (300, 0.8, 3)]:
        g = gg.erdos_renyi(n, p * (n - 1), seed=seed)
        h = _load(citron_gpu, g)
        for k in (3, 4):
            assert h.count_vertex_rooted(k) == oracle.count(g, k)[0], (n, p, k)


def test_rmat14_and_rmat20_against_stored_counts(citron_gpu, progress):
    for name, ks in (("rmat14", range(3, 9)), ("rmat20", range(3, 6))):
        with open(os.path.join(GOLDEN, f"{name}.json")) as f:
            gold = json.load(f)
        g = gg.config_graph(name)
        assert g.sha256() == gold["sha256"]
        h = _load(citron_gpu, g)
        for k in ks:
            progress(f"  vertex-rooted {name} k={k}")
            assert h.count_vertex_rooted(k) == gold["counts"][str(k)]["count"], (name, k)
        h.free()
