"""Core ordering on the GPU (level-synchronous peeling, the parallel form of
Algorithm 1): the peeling rounds, the DAG byte for byte and the largest
out-degree against the oracle's peeling; counts on the core DAG against the
oracle's counts (any acyclic orientation counts each clique once)."""
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _csr(n, rows):
    rp = np.zeros(n + 1, np.int32)
    for u in range(n):
        rp[u + 1] = rp[u] + len(rows[u])
    return gg.CSR(n, rp, np.array([v for u in range(n) for v in rows[u]], np.int32), "hand")


def _check_dag(citron, g):
    h = citron.Graph.from_csr(g.row_ptr, g.col).order("core")
    key, rounds = h.order_key()
    want_rounds = oracle.peel_rounds(g.n, g.row_ptr, g.col)
    assert np.array_equal(key, want_rounds), g.name
    assert rounds == (int(want_rounds.max()) + 1 if g.n else 0)
    dptr, dcol = h.dag()
    optr, ocol = oracle.orient_peel(g)
    assert np.array_equal(dptr, optr) and np.array_equal(dcol, ocol), g.name
    assert h.info()["max_outdeg"] == int(np.diff(optr).max(initial=0))
    return h


@pytest.mark.parametrize("name", ["fig1", "path5", "cycle_pendant", "rmat12", "er", "rmat14", "k30",
                                  "hypercube6", "grid", "cliques", "empty"])
def test_core_dag_matches_oracle(citron_gpu, name):
    g = {"fig1": gg.fig1_example, "path5": lambda: _csr(5, [[1], [0, 2], [1, 3], [2, 4], [3]]),
         "cycle_pendant": lambda: _csr(5, [[1, 3], [0, 2], [1, 3, 4], [0, 2], [2]]),
         "rmat12": lambda: gg.rmat(12, 16, seed=12), "er": lambda: gg.erdos_renyi(3000, 25, seed=3),
         "rmat14": lambda: gg.rmat(14, 16, seed=14), "k30": lambda: gg.complete(30),
         "hypercube6": lambda: gg.hypercube(6), "grid": lambda: gg.grid(17, 9),
         "cliques": lambda: gg.disjoint_cliques([3, 7, 12, 5]), "empty": lambda: gg.empty(5)}[name]()
    h = _check_dag(citron_gpu, g)
    for k in range(3, 7):
        want = math.comb(30, k) if name == "k30" else oracle.count(g, k)[0]
        assert h.count(k) == want, (name, k)


def test_core_ordering_reaches_the_degeneracy(citron_gpu):
    # the largest out-degree equals Algorithm 1's (the degeneracy)
    for seed in range(6):
        g = gg.rmat(10, 8 + 4 * seed, seed=600 + seed)
        h = _check_dag(citron_gpu, g)
        core_mx = int(np.diff(oracle.orient_core(g)[0]).max())
        assert h.info()["max_outdeg"] == core_mx


def test_orderings_do_not_mix(citron_gpu):
    g = gg.rmat(9, 8, seed=9)
    h = citron_gpu.Graph.from_csr(g.row_ptr, g.col).order()
    with pytest.raises(citron_gpu.CitronError) as e:
        h.order("core")
    assert e.value.status == 5
    h.order("degree")                      # the same ordering again: a no-op
    h2 = citron_gpu.Graph.from_csr(g.row_ptr, g.col).order("core")
    assert h2.count(5) == h.count(5)
    key, rounds = h.order_key()
    assert np.array_equal(key, np.diff(g.row_ptr)) and rounds == 0


@pytest.mark.parametrize("name", ["rmat20", "chunglu22"])
def test_core_ordering_full_size(citron_gpu, name, progress):
    with open(os.path.join(GOLDEN, f"{name}.json")) as f:
        gold = json.load(f)
    g = gg.config_graph(name)
    assert g.sha256() == gold["sha256"]
    progress(f"  {name}: core ordering on the device")
    h = _check_dag(citron_gpu, g)
    progress(f"  {name}: max out-degree {h.info()['max_outdeg']} (degree ordering {gold['max_outdeg']})")
    assert h.info()["max_outdeg"] <= gold["max_outdeg"]
    for k, rec in gold["counts"].items():
        assert h.count(int(k)) == rec["count"], (name, k)
