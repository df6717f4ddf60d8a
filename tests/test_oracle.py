"""Pins of the reference counter (oracle/) against facts fixed by the paper
and by mathematics, never against the oracle itself:

* the worked example of Fig. 1 (DAG, induced subgraph, counts, per arc);
* brute-force subset enumeration on random small graphs (definition);
* closed forms: complete, Turan, bipartite, grid, hypercube, wheel,
  disjoint cliques, Paley (strongly regular), Kneser, empty graphs;
* triangles = trace(A^3)/6 computed by scipy sparse matrix products;
* invariance of every count under vertex relabelling;
* per-size visit counts equal to the counts at smaller k;
* counts rooted at vertex classes and ranges adding up to the brute-force
  count (how the stored whole counts of the large graphs were split);
* DAG invariants of the degree ordering (Section IV);
* listing: the listed cliques equal brute-force enumeration as a set;
* core ordering (Algorithm 1): maximum out-degree equals the brute-force
  degeneracy and closed forms; counts on its DAG equal brute force.
"""
import json
import math
import os
from itertools import combinations

import numpy as np
import pytest
import scipy.sparse as sp

import graphgen as gg
import oracle
from tests._brute import brute_count, brute_rooted

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ocount(g, k, prune=True):
    c, ovf = oracle.count(g, k, prune=prune)
    assert not ovf
    return c


# ------------------------------------------------------------------ Fig. 1

@pytest.fixture(scope="module")
def fig1():
    with open(os.path.join(GOLDEN, "fig1.json")) as f:
        return json.load(f)


def test_fig1_graph_and_degrees(fig1):
    g = gg.fig1_example()
    assert g.n == fig1["n"] and g.m == len(fig1["edges"])
    assert list(g.degrees()) == fig1["degrees"]


def test_fig1_dag(fig1):
    g = gg.fig1_example()
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    for u in range(g.n):
        assert list(dcol[dptr[u]:dptr[u + 1]]) == fig1["dag_out_lists"][str(u)], u


def test_fig1_subgraph_of_vertex0(fig1):
    g = gg.fig1_example()
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    nu = list(dcol[dptr[0]:dptr[1]])
    assert nu == fig1["subgraph_induced_by_0"]["vertices"]
    arcs = []
    for w in nu:
        for x in dcol[dptr[w]:dptr[w + 1]]:
            if x in nu:
                arcs.append([w, int(x)])
    assert sorted(arcs) == sorted(fig1["subgraph_induced_by_0"]["arcs"])


def test_fig1_counts(fig1):
    g = gg.fig1_example()
    for k, want in fig1["clique_counts"].items():
        assert ocount(g, int(k)) == want
        assert ocount(g, int(k), prune=False) == want


def test_fig1_per_arc(fig1):
    g = gg.fig1_example()
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    src = np.repeat(np.arange(g.n), np.diff(dptr))
    for k, key in ((3, "per_arc_k3"), (4, "per_arc_k4")):
        got, _ = oracle.count_arcs(g.n, dptr, dcol, k, src, dcol)
        table = {f"{u},{v}": int(c) for u, v, c in zip(src, dcol, got)}
        for arc, want in fig1[key].items():
            assert table[arc] == want, (k, arc)
        assert sum(table.values()) == fig1["clique_counts"][str(k)]


# ------------------------------------------------------------- brute force

def _random_graphs(count, nmin, nmax, seed):
    rng = np.random.default_rng(seed)
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        p = float(rng.uniform(0.2, 0.9))
        iu, ju = np.triu_indices(n, 1)
        keep = rng.random(iu.size) < p
        yield gg.csr_from_edges(n, iu[keep], ju[keep], perm_seed=int(rng.integers(1 << 30)))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_random(seed):
    for g in _random_graphs(8, 1, 13, seed):
        for k in range(1, 9):
            assert ocount(g, k) == brute_count(g, k), (g.n, g.m, k)


def test_brute_force_unpruned_and_rooted():
    for g in _random_graphs(6, 5, 11, 7):
        dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
        deg = g.degrees()

        def less(a, b):
            return deg[a] < deg[b] or (deg[a] == deg[b] and a < b)

        src = np.repeat(np.arange(g.n), np.diff(dptr))
        for k in range(2, 7):
            assert ocount(g, k, prune=False) == brute_count(g, k)
            got, _ = oracle.count_arcs(g.n, dptr, dcol, k, src, dcol)
            for u, v, c in zip(src, dcol, got):
                assert int(c) == brute_rooted(g, k, int(u), int(v), less)


def test_root_classes_and_ranges_add_up():
    # the stored whole counts of the large graphs are sums of the counts
    # rooted at vertex residue classes (one worker process per class); a
    # clique is rooted at its lowest vertex, so the classes partition them
    for g in _random_graphs(4, 9, 14, 21):
        dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
        for k in range(3, 7):
            want = brute_count(g, k)
            for P in (1, 2, 3, 5):
                parts = [oracle.count_dag(g.n, dptr, dcol, k, r, g.n, P)[0] for r in range(P)]
                assert sum(parts) == want, (k, P)
            h = g.n // 3
            ranges = [oracle.count_dag(g.n, dptr, dcol, k, a, b)[0] for a, b in ((0, h), (h, g.n))]
            assert sum(ranges) == want, k


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", [1, 2, 5, 9, 13, 20])
def test_complete(n):
    g = gg.complete(n)
    for k in range(1, min(n + 2, 12)):
        assert ocount(g, k) == math.comb(n, k)


def _elementary_symmetric(parts, k):
    return sum(math.prod(c) for c in combinations(parts, k))


@pytest.mark.parametrize("n,r", [(10, 3), (12, 4), (15, 5), (9, 2), (17, 6)])
def test_turan(n, r):
    g = gg.turan(n, r)
    parts = [n // r + (1 if i < n % r else 0) for i in range(r)]
    for k in range(2, r + 3):
        assert ocount(g, k) == _elementary_symmetric(parts, k)


def test_turan_quoted_values():
    # T(10,3) with parts (4,3,3) and T(12,4) with parts (3,3,3,3)
    assert [ocount(gg.turan(10, 3), k) for k in (2, 3, 4)] == [33, 36, 0]
    assert [ocount(gg.turan(12, 4), k) for k in (2, 3, 4)] == [54, 108, 81]


@pytest.mark.parametrize("g", [gg.complete_bipartite(5, 7), gg.grid(6, 5), gg.hypercube(5),
                               gg.complete_bipartite(1, 9)])
def test_bipartite_has_no_triangles(g):
    assert ocount(g, 2) == g.m
    for k in range(3, 7):
        assert ocount(g, k) == 0


@pytest.mark.parametrize("rim", [4, 5, 8, 13])
def test_wheel(rim):
    g = gg.wheel(rim)
    assert ocount(g, 3) == rim
    assert ocount(g, 4) == 0


def test_wheel_rim3_is_k4():
    assert [ocount(gg.wheel(3), k) for k in (3, 4, 5)] == [4, 1, 0]


def test_disjoint_cliques():
    sizes = [3, 7, 12, 5, 20, 1]
    g = gg.disjoint_cliques(sizes)
    for k in range(1, 10):
        assert ocount(g, k) == sum(math.comb(s, k) for s in sizes)


@pytest.mark.parametrize("q", [5, 13, 17, 29, 37, 101])
def test_paley_triangles(q):
    # Paley graphs are strongly regular with degree (q-1)/2 and (q-5)/4 common
    # neighbours per edge: m = q(q-1)/4 and q(q-1)(q-5)/48 triangles
    g = gg.paley(q)
    assert ocount(g, 2) == q * (q - 1) // 4
    assert ocount(g, 3) == q * (q - 1) * (q - 5) // 48


def test_paley17_has_no_k4():
    # the Paley graph on 17 vertices shows R(4,4) > 17: no 4-clique (and,
    # being self-complementary, no independent 4-set)
    g = gg.paley(17)
    assert ocount(g, 3) == 68 and ocount(g, 4) == 0


def _kneser_cliques(n, r, k):
    # a k-clique is an unordered choice of k pairwise disjoint r-subsets
    if r * k > n:
        return 0
    return math.factorial(n) // (math.factorial(r) ** k * math.factorial(k) * math.factorial(n - r * k))


@pytest.mark.parametrize("n,r", [(5, 2), (7, 2), (8, 2), (10, 2), (9, 3), (11, 3)])
def test_kneser(n, r):
    g = gg.kneser(n, r)
    assert g.n == math.comb(n, r)
    for k in range(1, n // r + 2):
        assert ocount(g, k) == _kneser_cliques(n, r, k), k


def test_petersen():
    g = gg.kneser(5, 2)
    assert (g.n, g.m) == (10, 15)
    assert [ocount(g, k) for k in (3, 4)] == [0, 0]


def test_empty():
    g = gg.empty(10)
    assert ocount(g, 1) == 10
    for k in range(2, 6):
        assert ocount(g, k) == 0
    g0 = gg.empty(0)
    assert ocount(g0, 1) == 0 and ocount(g0, 3) == 0


# ------------------------------------------------------- library routine pin

def _trace_triangles(g):
    a = sp.csr_matrix((np.ones(g.nnz, dtype=np.int64), g.col, g.row_ptr), shape=(g.n, g.n))
    return int((a @ a).multiply(a).sum()) // 6


@pytest.mark.parametrize("g", [gg.rmat(10, 16, seed=3), gg.erdos_renyi(2000, 30, seed=4),
                               gg.chung_lu(n=1 << 13, mean_degree=20, w_max=800, planted=20,
                                           seed=5, clique_seed=6)])
def test_triangles_equal_trace(g):
    assert ocount(g, 3) == _trace_triangles(g)


def test_triangles_rmat14_trace():
    g = gg.config_graph("rmat14")
    assert ocount(g, 3) == _trace_triangles(g)


# --------------------------------------------------------------- invariants

def test_relabel_invariance():
    g = gg.rmat(9, 16, seed=11)
    rng = np.random.default_rng(0)
    perms = [rng.permutation(g.n), np.arange(g.n)[::-1].copy()]
    for k in range(3, 7):
        base = ocount(g, k)
        for p in perms:
            assert ocount(gg.relabel(g, p), k) == base


def test_visits_are_smaller_counts():
    g = gg.rmat(9, 16, seed=12)
    k = 6
    c, ovf, vis = oracle.count(g, k, prune=False, visits=True)
    for j in range(1, k + 1):
        assert vis[j] == ocount(g, j), j
    assert vis[k] == c


def test_pruning_preserves_counts():
    g = gg.erdos_renyi(300, 25, seed=13)
    for k in range(3, 8):
        assert ocount(g, k, prune=True) == ocount(g, k, prune=False)


def test_dag_invariants():
    for g in (gg.rmat(11, 16, seed=14), gg.erdos_renyi(1000, 12, seed=15), gg.fig1_example()):
        dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
        deg = g.degrees()
        assert dptr[-1] == g.m
        src = np.repeat(np.arange(g.n), np.diff(dptr))
        # every edge once, in one direction, following omega
        assert np.all((deg[src] < deg[dcol]) | ((deg[src] == deg[dcol]) & (src < dcol)))
        s, d = g.edges()
        und = set(zip(s.tolist(), d.tolist()))
        arcs = set((min(a, b), max(a, b)) for a, b in zip(src.tolist(), dcol.tolist()))
        assert arcs == und and len(arcs) == g.m
        # rows ascending
        for u in range(g.n):
            row = dcol[dptr[u]:dptr[u + 1]]
            assert np.all(np.diff(row) > 0)
        # out-degree bound of the degree ordering: d->(u) <= floor(sqrt(2m))
        assert np.diff(dptr).max(initial=0) <= math.isqrt(2 * g.m)


def test_check_csr_rejects_defects():
    g = gg.fig1_example()
    assert oracle.check_csr(g.n, g.row_ptr, g.col)
    bad = g.col.copy()
    bad[0], bad[1] = bad[1], bad[0]          # unsorted row
    assert not oracle.check_csr(g.n, g.row_ptr, bad)
    bad = g.col.copy()
    bad[0] = 0                               # self-loop at vertex 0
    assert not oracle.check_csr(g.n, g.row_ptr, bad)


def _csr(n, rows):
    rp = np.zeros(n + 1, np.int32)
    for u in range(n):
        rp[u + 1] = rp[u] + len(rows[u])
    col = np.array([v for u in range(n) for v in rows[u]], np.int32)
    return rp, col


def test_check_csr_rejects_every_kind_of_defect():
    # a path 0-1-2 plus the edge 2-3: valid as given
    good = [[1], [0, 2], [1, 3], [2]]
    rp, col = _csr(4, good)
    assert oracle.check_csr(4, rp, col)
    # asymmetric: 3 lists 2, but 2 does not list 3
    rp, col = _csr(4, [[1], [0, 2], [1], [2]])
    assert not oracle.check_csr(4, rp, col)
    # column id out of range, above n - 1 and negative
    rp, col = _csr(4, [[1], [0, 2], [1, 4], [2]])
    assert not oracle.check_csr(4, rp, col)
    rp, col = _csr(4, [[-1, 1], [0, 2], [1, 3], [2]])
    assert not oracle.check_csr(4, rp, col)
    # duplicate entry (a multi-edge listed twice in both rows)
    rp, col = _csr(4, [[1, 1], [0, 0, 2], [1, 3], [2]])
    assert not oracle.check_csr(4, rp, col)
    # row_ptr not starting at 0, and decreasing
    rp, col = _csr(4, good)
    bad = rp.copy()
    bad[0] = 1
    assert not oracle.check_csr(4, bad, col)
    bad = rp.copy()
    bad[2], bad[3] = bad[3], bad[2]
    assert not oracle.check_csr(4, bad, col)
    # the empty graph and isolated vertices are valid
    rp, col = _csr(3, [[], [], []])
    assert oracle.check_csr(3, rp, col)


# ----------------------------------------------------------- counter width

def test_overflow_flag_set_exactly_at_2_to_64():
    """The counter width is not stated in the paper; the reading taken is
    uint64 with a flag raised iff the exact total is >= 2^64.  K_20 has
    C(20,5) = 15504 5-cliques: a start of 2^64 - 15504 must wrap to exactly
    0 with the flag set, one less must end at 2^64 - 1 with the flag clear."""
    g = gg.complete(20)
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    c5 = math.comb(20, 5)
    assert oracle.count_dag(g.n, dptr, dcol, 5) == (c5, False)
    assert oracle.count_dag(g.n, dptr, dcol, 5, base=2**64 - c5) == (0, True)
    assert oracle.count_dag(g.n, dptr, dcol, 5, base=2**64 - c5 - 1) == (2**64 - 1, False)
    # far beyond: the value is the total mod 2^64
    assert oracle.count_dag(g.n, dptr, dcol, 5, base=2**64 - 1) == (c5 - 1, True)
    # the flag does not depend on how the roots are split: both halves from
    # the same near-full base, summed, reach the same verdict
    h = g.n // 2
    a = oracle.count_dag(g.n, dptr, dcol, 5, 0, h, base=2**64 - c5)
    b = oracle.count_dag(g.n, dptr, dcol, 5, h, g.n)
    assert (a[0] + b[0]) % 2**64 == 0 and not a[1] and a[0] + b[0] == 2**64


# ------------------------------------------------------- a planted mistake

def test_a_planted_mistake_is_caught():
    """A counter that forgets the tie-break of the ordering counts some
    cliques twice or never; the closed form on a regular graph catches it."""
    g = gg.complete(6)                       # all degrees equal: only ids decide
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    # the wrong DAG keeps both directions of every tie
    wrong_ptr = g.row_ptr.copy()
    wrong_col = g.col.copy()
    c_right, _ = oracle.count_dag(g.n, dptr, dcol, 3)
    c_wrong, _ = oracle.count_dag(g.n, wrong_ptr, wrong_col, 3)
    assert c_right == math.comb(6, 3)
    assert c_wrong != math.comb(6, 3)


def _arc_stats_by_definition(g, k):
    """Per-arc work statistics from the undirected adjacency, by the
    definitions: orientation by (degree, id), C_uv = N->(u) & N->(v)."""
    adj = [set(g.col[g.row_ptr[u]:g.row_ptr[u + 1]].tolist()) for u in range(g.n)]
    deg = [len(a) for a in adj]
    out = [{v for v in adj[u] if (deg[u], u) < (deg[v], v)} for u in range(g.n)]
    st = dict(arcs=0, sum_duv=0, sum_s=0, sum_dw=0, max_s=0, arcs_kept=0, kept_sum_duv=0,
              kept_sum_s=0, kept_sum_dw=0, max_outdeg=max((len(o) for o in out), default=0))
    hist = [0] * 33
    for u in range(g.n):
        for v in out[u]:
            c = out[u] & out[v]
            s = len(c)
            duv = len(out[u]) + len(out[v])
            dw = sum(len(out[w]) for w in c)
            st["arcs"] += 1
            st["sum_duv"] += duv
            st["sum_s"] += s
            st["sum_dw"] += dw
            st["max_s"] = max(st["max_s"], s)
            if s >= k - 2:
                st["arcs_kept"] += 1
                st["kept_sum_duv"] += duv
                st["kept_sum_s"] += s
                st["kept_sum_dw"] += dw
            hist[s.bit_length()] += 1
    return st, hist


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_arc_stats_match_definitions(seed):
    """Work statistics against a set-based restatement of Section III-B's
    candidate sets; sum_s is the triangle count (trace(A^3)/6)."""
    g = gg.rmat(9, 12, seed=600 + seed)
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    for k in (3, 5, 7):
        st, hist = oracle.arc_stats(g.n, dptr, dcol, k)
        want, want_hist = _arc_stats_by_definition(g, k)
        assert st == want, k
        assert hist == want_hist
    a = sp.csr_matrix((np.ones(g.nnz), g.col, g.row_ptr), shape=(g.n, g.n))
    assert st["sum_s"] == round((a @ a @ a).diagonal().sum() / 6)
    assert st["arcs"] == g.m


# ------------------------------------------------------------- listing

def _brute_cliques(g, k):
    from tests._brute import adjacency
    a = adjacency(g)
    return {sub for sub in combinations(range(g.n), k) if all(a[x, y] for x, y in combinations(sub, 2))}


def _as_sets(rows):
    return [tuple(sorted(int(x) for x in r)) for r in rows]


@pytest.mark.parametrize("seed", [4, 5])
def test_listing_is_the_set_of_cliques(seed):
    for g in _random_graphs(6, 3, 13, seed):
        deg = g.degrees()
        for k in range(1, 8):
            rows = oracle.list_cliques(g, k)
            got = _as_sets(rows)
            assert len(got) == len(set(got)), "a clique listed twice"
            assert set(got) == _brute_cliques(g, k), (g.n, k)
            for r in rows:      # each in increasing degree order (ties by id)
                assert all((deg[x], x) < (deg[y], y) for x, y in zip(r[:-1], r[1:]))


def test_listing_fig1_and_complete():
    g = gg.fig1_example()
    assert _as_sets(oracle.list_cliques(g, 4)) == [(0, 1, 3, 4)]
    assert oracle.list_cliques(g, 5).shape == (0, 5)
    assert sorted(_as_sets(oracle.list_cliques(gg.complete(9), 4))) == list(combinations(range(9), 4))


def test_listing_roots_and_cap():
    g = gg.rmat(8, 16, seed=7)
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    whole, total = oracle.list_dag(g.n, dptr, dcol, 4)
    assert total == len(whole) == ocount(g, 4)
    parts = [oracle.list_dag(g.n, dptr, dcol, 4, r, g.n, 3)[0] for r in range(3)]
    assert sorted(_as_sets(np.concatenate(parts))) == sorted(_as_sets(whole))
    head, t2 = oracle.list_dag(g.n, dptr, dcol, 4, cap=10)
    assert t2 == total and np.array_equal(head, whole[:10])


# ------------------------------------------------------- core ordering

def _brute_degeneracy(g):
    # the largest minimum degree over all induced subgraphs (definition)
    from tests._brute import adjacency
    a = adjacency(g)
    best = 0
    for mask in range(1, 1 << g.n):
        vs = [v for v in range(g.n) if mask >> v & 1]
        best = max(best, min(int(a[v, vs].sum()) for v in vs))
    return best


def _core_outdeg(g):
    dptr, dcol = oracle.orient_core(g)
    return int(np.diff(dptr).max(initial=0)), dptr, dcol


@pytest.mark.parametrize("seed", [8, 9])
def test_core_ordering_reaches_the_degeneracy(seed):
    for g in _random_graphs(5, 2, 12, seed):
        mx, dptr, dcol = _core_outdeg(g)
        assert mx == _brute_degeneracy(g), g.n
        assert int(dptr[-1]) == g.m
        for k in range(1, 7):     # any acyclic orientation counts every clique once
            assert oracle.count_dag(g.n, dptr, dcol, k)[0] == brute_count(g, k), k


@pytest.mark.parametrize("g,degeneracy", [
    (gg.complete(12), 11), (gg.complete_bipartite(4, 9), 4), (gg.grid(5, 7), 2),
    (gg.hypercube(5), 5), (gg.wheel(9), 3), (gg.paley(29), 14), (gg.turan(12, 4), 9),
    (gg.empty(6), 0)])
def test_core_ordering_closed_forms(g, degeneracy):
    # complete K_n: n-1; K_a,b: min(a,b); grids: 2; d-regular graphs: d;
    # wheels: 3; Turan T(12,4) is 9-regular
    mx, dptr, dcol = _core_outdeg(g)
    assert mx == degeneracy
    rank = oracle.core_rank(g.n, g.row_ptr, g.col)
    assert sorted(rank.tolist()) == list(range(g.n))


def test_core_rank_tie_break_by_hand():
    """Algorithm 1 on a 4-cycle 0-1-2-3-0 with a pendant vertex 4 at 2,
    derived by hand (rank = removal position; among vertices of smallest
    current degree the smallest id goes first):
      degrees 0:2 1:2 2:3 3:2 4:1 -> remove 4 (degree 1); 2 drops to 2
      all of 0..3 now have degree 2 -> remove 0 (smallest id); 1, 3 drop to 1
      1 and 3 have degree 1 -> remove 1; 2 drops to 1
      2 and 3 have degree 1 -> remove 2; 3 drops to 0
      remove 3.
    Ties by the largest id would remove 3 second, and ties by the first
    vertex met in a degree bucket differ again, so the rank pins the rule."""
    rp, col = _csr(5, [[1, 3], [0, 2], [1, 3, 4], [0, 2], [2]])
    rank = oracle.core_rank(5, rp, col)
    assert rank.tolist() == [1, 2, 3, 4, 0]
    dptr, dcol = oracle.orient_rank(5, rp, col, rank)
    outs = [dcol[dptr[u]:dptr[u + 1]].tolist() for u in range(5)]
    assert outs == [[1, 3], [2], [3], [], [2]]
    # K_4 minus an edge (0-3 missing): degrees 0:2 1:3 2:3 3:2; remove 0
    # (tie with 3, smaller id); 1, 2 drop to 2; now 1, 2, 3 all at 2 ->
    # remove 1; 2, 3 drop to 1 -> remove 2; then 3.
    rp, col = _csr(4, [[1, 2], [0, 2, 3], [0, 1, 3], [1, 2]])
    assert oracle.core_rank(4, rp, col).tolist() == [0, 1, 2, 3]


def test_peeling_rounds_by_hand():
    """Level-synchronous peeling, derived by hand.
    4-cycle 0-1-2-3-0 with a pendant 4 at 2: degrees 2,2,3,2,1; t = 1:
    round 0 removes {4} (2 drops to 2); no vertex is left at degree <= 1, so
    t rises to 2 and round 1 removes {0, 1, 2, 3} together.
    Path 0-1-2-3-4: degrees 1,2,2,2,1; t = 1: round 0 removes {0, 4}, 1 and
    3 drop to 1; round 1 removes {1, 3}, 2 drops to 0; round 2 removes {2}.
    (Algorithm 1 would remove the path's vertices in id order 0..4.)"""
    rp, col = _csr(5, [[1, 3], [0, 2], [1, 3, 4], [0, 2], [2]])
    assert oracle.peel_rounds(5, rp, col).tolist() == [1, 1, 1, 1, 0]
    assert oracle.peel_rank(5, rp, col).tolist() == [1, 2, 3, 4, 0]
    rp, col = _csr(5, [[1], [0, 2], [1, 3], [2, 4], [3]])
    assert oracle.peel_rounds(5, rp, col).tolist() == [0, 1, 2, 1, 0]
    assert oracle.core_rank(5, rp, col).tolist() == [0, 1, 2, 3, 4]
    dptr, dcol = oracle.orient_rank(5, rp, col, oracle.peel_rank(5, rp, col))
    assert [dcol[dptr[u]:dptr[u + 1]].tolist() for u in range(5)] == [[1], [2], [], [2], [3]]


@pytest.mark.parametrize("seed", [10, 11])
def test_peeling_reaches_the_degeneracy(seed):
    for g in _random_graphs(5, 2, 12, seed):
        dptr, dcol = oracle.orient_peel(g)
        assert int(np.diff(dptr).max(initial=0)) == _brute_degeneracy(g), g.n
        assert int(dptr[-1]) == g.m
        for k in range(1, 7):
            assert oracle.count_dag(g.n, dptr, dcol, k)[0] == brute_count(g, k), k


@pytest.mark.parametrize("g,degeneracy", [
    (gg.complete(12), 11), (gg.complete_bipartite(4, 9), 4), (gg.grid(5, 7), 2),
    (gg.hypercube(5), 5), (gg.wheel(9), 3), (gg.paley(29), 14), (gg.turan(12, 4), 9),
    (gg.empty(6), 0)])
def test_peeling_closed_forms(g, degeneracy):
    dptr, dcol = oracle.orient_peel(g)
    assert int(np.diff(dptr).max(initial=0)) == degeneracy
    # a regular graph leaves in one round: the order is then by id
    if len(set(np.diff(g.row_ptr).tolist())) == 1 and g.n:
        assert set(oracle.peel_rounds(g.n, g.row_ptr, g.col).tolist()) == {0}


def test_peeling_matches_algorithm_1_maximum_outdegree():
    g = gg.rmat(12, 16, seed=5)
    core_mx = int(np.diff(oracle.orient_core(g)[0]).max())
    dptr, dcol = oracle.orient_peel(g)
    assert int(np.diff(dptr).max()) == core_mx
    assert oracle.count_dag(g.n, dptr, dcol, 5)[0] == ocount(g, 5)


def test_core_ordering_never_exceeds_the_degree_ordering():
    g = gg.rmat(12, 16, seed=5)
    core_mx, dptr, dcol = _core_outdeg(g)
    deg_mx = int(np.diff(oracle.orient(g.n, g.row_ptr, g.col)[0]).max())
    assert core_mx <= deg_mx
    assert oracle.count_dag(g.n, dptr, dcol, 5)[0] == ocount(g, 5)


def test_edge_rooted_listing():
    for g in _random_graphs(5, 4, 12, 31):
        dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
        deg = g.degrees()
        src = np.repeat(np.arange(g.n), np.diff(dptr)).astype(np.int32)
        for k in range(2, 7):
            rows, per_arc = oracle.list_arcs(g.n, dptr, dcol, k, src, dcol)
            got = _as_sets(rows)
            assert len(got) == len(set(got)) and set(got) == _brute_cliques(g, k), (g.n, k)
            counts, _ = oracle.count_arcs(g.n, dptr, dcol, k, src, dcol)
            assert per_arc.tolist() == [int(c) for c in counts]
            starts = np.concatenate([[0], np.cumsum(per_arc.astype(np.int64))])
            for i, (u, v) in enumerate(zip(src, dcol)):
                for r in rows[starts[i]:starts[i + 1]]:
                    assert (r[0], r[1]) == (u, v)
                    assert all((deg[x], x) < (deg[y], y) for x, y in zip(r[:-1], r[1:]))


# ------------------------------------------------- all-core timing wrapper

def test_parallel_wrapper_equals_one_thread(tmp_path):
    from oracle import parallel as opar
    g = gg.rmat(10, 16, seed=12)
    dptr, dcol = oracle.orient(g.n, g.row_ptr, g.col)
    for k in (3, 5):
        want = oracle.count_dag(g.n, dptr, dcol, k)
        res = opar.count_classes(g.n, dptr, dcol, k, stride=7, workers=3)
        assert (res["count"], res["overflow"]) == want
        # a run stopped after some classes resumes from its checkpoint
        ck = str(tmp_path / f"ck{k}.json")
        part = opar.count_classes(g.n, dptr, dcol, k, stride=7, classes=[0, 3, 5], workers=2,
                                  checkpoint=ck, graph_key=g.sha256())
        assert part["classes"] == 3
        res = opar.count_classes(g.n, dptr, dcol, k, stride=7, workers=2, checkpoint=ck,
                                 graph_key=g.sha256())
        assert (res["count"], res["overflow"]) == want
        # a checkpoint of another graph or k is not reused
        other = opar.count_classes(g.n, dptr, dcol, k + 1, stride=7, workers=2, checkpoint=ck,
                                   graph_key=g.sha256())
        assert other["count"] == oracle.count_dag(g.n, dptr, dcol, k + 1)[0]
