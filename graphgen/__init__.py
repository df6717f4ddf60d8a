"""Seeded synthetic graph generators shared by the tests, the benchmark and the
reference counter.

This module only produces inputs: simple undirected graphs as int32 CSR
(symmetric, rows sorted ascending, no duplicates, no self-loops), the input
form of the degree-ordering phase (Section IV).  It holds none of the
counting method's arithmetic: no orientation, no intersection, no counting.

Generators (all deterministic given their seed, numpy PCG64 streams):

* ``rmat``        -- recursive-matrix graph, quadrant probabilities a/b/c/d.
* ``chung_lu``    -- power-law expected-degree graph, optional planted cliques.
* ``erdos_renyi`` -- G(n, p) by geometric skipping (Batagelj & Brandes 2005).
* small families  -- complete, Turan, complete bipartite, wheel, grid,
  hypercube, disjoint cliques, the worked example of Fig. 1 of the paper.

Every generated graph is passed through :func:`csr_from_edges`, which
applies a seeded random relabelling (when asked), symmetrises, drops
self-loops and duplicate edges, and sorts rows.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

from itertools import combinations

import numpy as np

__all__ = [
    "CSR", "csr_from_edges", "rmat", "chung_lu", "erdos_renyi",
    "complete", "turan", "complete_bipartite", "wheel", "grid", "hypercube",
    "disjoint_cliques", "empty", "fig1_example", "relabel", "config_graph",
    "CONFIGS", "batch_suite", "serve_suite",
]


@dataclass
class CSR:
    """Undirected simple graph: ``row_ptr`` int32[n+1], ``col`` int32[2m]."""

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()

    def edges(self) -> tuple[np.ndarray, np.ndarray]:
        """Undirected edges (u < v) as two int64 arrays."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        dst = self.col.astype(np.int64)
        keep = src < dst
        return src[keep], dst[keep]


def csr_from_edges(n: int, src, dst, perm_seed: int | None = None,
                   name: str = "") -> CSR:
    """Clean an edge list into a simple undirected CSR.

    Drops self-loops, merges duplicates (either direction), symmetrises and
    sorts every row ascending.  With ``perm_seed`` the vertex ids are first
    renamed by a seeded random permutation, so that id order carries no
    degree information.
    """
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    if src.shape != dst.shape:
        raise ValueError("src and dst differ in length")
    if n < 0 or n >= 2**31:
        raise ValueError("n out of int32 range")
    if src.size and (src.min() < 0 or dst.min() < 0 or src.max() >= n or dst.max() >= n):
        raise ValueError("vertex id out of range")
    if perm_seed is not None:
        perm = np.random.Generator(np.random.PCG64(perm_seed)).permutation(n)
        src = perm[src]
        dst = perm[dst]
    keep = src != dst
    src, dst = src[keep], dst[keep]
    lo = np.minimum(src, dst)
    hi = np.maximum(src, dst)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key % n
    # both directions, sorted by (source, destination) as one int64 key
    both = np.concatenate([key, hi * n + lo])
    both.sort(kind="stable")
    both_src = both // n
    both_dst = both - both_src * n
    if both_dst.size >= 2**31:
        raise ValueError("too many edges for int32 CSR")
    counts = np.bincount(both_src, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), both_dst.astype(np.int32), name)


def relabel(g: CSR, perm: np.ndarray, name: str | None = None) -> CSR:
    """The same graph with vertex ``v`` renamed ``perm[v]``."""
    s, d = g.edges()
    perm = np.asarray(perm, dtype=np.int64)
    return csr_from_edges(g.n, perm[s], perm[d], name=name or g.name + "/relabel")


# ---------------------------------------------------------------- families

def rmat(scale: int, edge_factor: int, a=0.57, b=0.19, c=0.19, d=0.05,
         seed: int = 0, permute: bool = True) -> CSR:
    """R-MAT graph on 2**scale vertices from edge_factor * 2**scale samples.

    Each sample descends ``scale`` levels; at each level one uniform draw
    picks the quadrant (0,0) w.p. a, (0,1) w.p. b, (1,0) w.p. c, (1,1) w.p. d
    and sets the matching source and destination bits.  No noise is added.
    """
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("quadrant probabilities must sum to 1")
    n = 1 << scale
    m = edge_factor * n
    rng = np.random.Generator(np.random.PCG64(seed))
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    for level in range(scale):
        r = rng.random(m)
        sbit = r >= a + b
        dbit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
        bit = np.int64(1) << np.int64(level)
        src |= np.where(sbit, bit, 0)
        dst |= np.where(dbit, bit, 0)
    del r, sbit, dbit
    g = csr_from_edges(n, src, dst, perm_seed=(seed + 1) * 7919 if permute else None,
                       name=f"rmat-s{scale}-ef{edge_factor}-seed{seed}")
    g.meta.update(kind="rmat", scale=scale, edge_factor=edge_factor,
                  abcd=[a, b, c, d], seed=seed)
    return g


def _chung_lu_weights(n: int, gamma: float, mean: float, w_max: float) -> np.ndarray:
    """w_i = w_max * (i0 / (i + i0))**(1/(gamma-1)), i0 solved for the mean."""
    expo = 1.0 / (gamma - 1.0)
    idx = np.arange(n, dtype=np.float64)

    def mean_for(i0):
        return float(np.mean(w_max * (i0 / (idx + i0)) ** expo))

    lo, hi = 1e-6, float(n)
    for _ in range(64):        # the bracket is down to adjacent doubles by then
        mid = np.sqrt(lo * hi)
        if mean_for(mid) < mean:
            lo = mid
        else:
            hi = mid
    i0 = np.sqrt(lo * hi)
    return w_max * (i0 / (idx + i0)) ** expo


def chung_lu(n: int = 1 << 22, gamma: float = 2.1, mean_degree: float = 25.0,
             w_max: float = 2.0e4, planted: int = 2000, clique_min: int = 10,
             clique_max: int = 40, seed: int = 22, clique_seed: int = 2201,
             permute: bool = True) -> CSR:
    """Chung-Lu power-law graph with planted cliques.

    ``n * mean_degree / 2`` edge samples draw both endpoints independently
    with probability proportional to the weights (inverse-CDF sampling), so
    pair (i, j) appears with probability 1 - exp(-w_i w_j / S), S = sum w.
    Then ``planted`` cliques with sizes uniform in [clique_min, clique_max]
    are added on vertex sets drawn uniformly without replacement.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w = _chung_lu_weights(n, gamma, mean_degree, w_max)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    samples = int(round(n * mean_degree / 2))
    parts_s, parts_d = [], []
    chunk = 1 << 24
    done = 0
    while done < samples:
        # inverse-CDF lookups of sorted uniforms (fast), then the second
        # endpoints put in random order: the pairs are then independent
        # draws, as with unsorted uniforms
        k = min(chunk, samples - done)
        s = np.searchsorted(cdf, np.sort(rng.random(k)), side="right")
        d = np.searchsorted(cdf, np.sort(rng.random(k)), side="right")[rng.permutation(k)]
        parts_s.append(np.minimum(s, n - 1))
        parts_d.append(np.minimum(d, n - 1))
        done += k
    crng = np.random.Generator(np.random.PCG64(clique_seed))
    for _ in range(planted):
        size = int(crng.integers(clique_min, clique_max + 1))
        verts = crng.choice(n, size=size, replace=False).astype(np.int64)
        iu, ju = np.triu_indices(size, 1)
        parts_s.append(verts[iu])
        parts_d.append(verts[ju])
    src = np.concatenate(parts_s)
    dst = np.concatenate(parts_d)
    g = csr_from_edges(n, src, dst, perm_seed=(seed + 1) * 7919 if permute else None,
                       name=f"chunglu-n{n}-g{gamma}-d{mean_degree}-p{planted}-seed{seed}")
    g.meta.update(kind="chung_lu", n=n, gamma=gamma, mean_degree=mean_degree,
                  w_max=w_max, planted=planted, seed=seed, clique_seed=clique_seed)
    return g


def erdos_renyi(n: int, mean_degree: float, seed: int = 0) -> CSR:
    """G(n, p) with p = mean_degree / (n - 1), by geometric skipping.

    The n(n-1)/2 vertex pairs are walked in a fixed linear order; the gap to
    the next present pair is geometric with parameter p (Batagelj & Brandes,
    "Efficient generation of large random networks", 2005).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if n < 2:
        return csr_from_edges(n, [], [], name=f"er-n{n}")
    p = min(1.0, mean_degree / (n - 1))
    total = n * (n - 1) // 2
    if p >= 1.0:
        idx = np.arange(total, dtype=np.int64)
    else:
        parts = []
        pos = np.int64(-1)
        while True:
            k = int(total * p * 1.05) + 1024
            gaps = rng.geometric(p, size=k).astype(np.int64)
            idx = pos + np.cumsum(gaps)
            if idx[-1] >= total:
                parts.append(idx[idx < total])
                break
            parts.append(idx)
            pos = idx[-1]
        idx = np.concatenate(parts)
    # linear index L -> pair (i, j), i > j, L = i(i-1)/2 + j
    i = np.floor((1.0 + np.sqrt(1.0 + 8.0 * idx.astype(np.float64))) / 2.0).astype(np.int64)
    i = np.where(i * (i - 1) // 2 > idx, i - 1, i)
    i = np.where((i + 1) * i // 2 <= idx, i + 1, i)
    j = idx - i * (i - 1) // 2
    g = csr_from_edges(n, i, j, name=f"er-n{n}-d{mean_degree}-seed{seed}")
    g.meta.update(kind="erdos_renyi", n=n, mean_degree=mean_degree, seed=seed)
    return g


def complete(n: int) -> CSR:
    iu, ju = np.triu_indices(n, 1)
    return csr_from_edges(n, iu, ju, name=f"K{n}")


def turan(n: int, r: int) -> CSR:
    """Complete r-partite graph with parts as equal as possible."""
    part = np.arange(n) % r
    iu, ju = np.triu_indices(n, 1)
    keep = part[iu] != part[ju]
    return csr_from_edges(n, iu[keep], ju[keep], name=f"T({n},{r})")


def complete_bipartite(a: int, b: int) -> CSR:
    u = np.repeat(np.arange(a), b)
    v = np.tile(np.arange(a, a + b), a)
    return csr_from_edges(a + b, u, v, name=f"K{a},{b}")


def wheel(rim: int) -> CSR:
    """Hub 0 joined to a cycle on vertices 1..rim."""
    rimv = np.arange(1, rim + 1)
    nxt = np.roll(rimv, -1)
    s = np.concatenate([np.zeros(rim, np.int64), rimv])
    d = np.concatenate([rimv, nxt])
    return csr_from_edges(rim + 1, s, d, name=f"W{rim}")


def grid(rows: int, cols: int) -> CSR:
    idx = np.arange(rows * cols).reshape(rows, cols)
    s = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    d = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return csr_from_edges(rows * cols, s, d, name=f"grid{rows}x{cols}")


def hypercube(dim: int) -> CSR:
    n = 1 << dim
    v = np.arange(n)
    s = np.concatenate([v for _ in range(dim)])
    d = np.concatenate([v ^ (1 << b) for b in range(dim)])
    return csr_from_edges(n, s, d, name=f"Q{dim}")


def disjoint_cliques(sizes) -> CSR:
    s_all, d_all = [], []
    off = 0
    for sz in sizes:
        iu, ju = np.triu_indices(sz, 1)
        s_all.append(iu + off)
        d_all.append(ju + off)
        off += sz
    s = np.concatenate(s_all) if s_all else np.zeros(0, np.int64)
    d = np.concatenate(d_all) if d_all else np.zeros(0, np.int64)
    return csr_from_edges(off, s, d, name="cliques" + "+".join(map(str, sizes)))


def paley(q: int) -> CSR:
    """Paley graph of a prime q = 1 mod 4: x ~ y iff x - y is a nonzero square mod q."""
    if q < 5 or q % 4 != 1 or any(q % p == 0 for p in range(2, int(q ** 0.5) + 1)):
        raise ValueError("q must be a prime congruent to 1 mod 4")
    squares = np.zeros(q, bool)
    squares[(np.arange(1, q) ** 2) % q] = True
    iu, ju = np.triu_indices(q, 1)
    keep = squares[(ju - iu) % q]
    return csr_from_edges(q, iu[keep], ju[keep], name=f"Paley{q}")


def kneser(n: int, r: int) -> CSR:
    """Kneser graph K(n, r): the r-subsets of {0..n-1}, adjacent iff disjoint."""
    subsets = list(combinations(range(n), r))
    masks = np.array([sum(1 << e for e in s) for s in subsets], dtype=np.int64)
    iu, ju = np.triu_indices(len(subsets), 1)
    keep = (masks[iu] & masks[ju]) == 0
    return csr_from_edges(len(subsets), iu[keep], ju[keep], name=f"Kneser({n},{r})")


def empty(n: int) -> CSR:
    return csr_from_edges(n, [], [], name=f"empty{n}")


def fig1_example() -> CSR:
    """The 7-vertex, 11-edge undirected graph drawn in Fig. 1 of the paper."""
    e = [(0, 1), (0, 3), (0, 4), (1, 3), (1, 4), (1, 2), (2, 5),
         (3, 4), (4, 6), (4, 5), (5, 6)]
    s, d = zip(*e)
    return csr_from_edges(7, s, d, name="fig1")


# ------------------------------------------------------ named workloads

CONFIGS = {
    # R-MAT scale 14, edge factor 16, seed 14 -- small parity workload (k=4)
    "rmat14": dict(kind="rmat", scale=14, edge_factor=16, seed=14),
    # R-MAT scale 20, edge factor 16, seed 20 -- benchmark workload (k=5..8)
    "rmat20": dict(kind="rmat", scale=20, edge_factor=16, seed=20),
    # Chung-Lu 2**22 vertices, exponent 2.1, mean degree 25, 2000 planted cliques
    "chunglu22": dict(kind="chung_lu", n=1 << 22, seed=22, clique_seed=2201),
}


def config_graph(name: str) -> CSR:
    cfg = dict(CONFIGS[name])
    kind = cfg.pop("kind")
    if kind == "rmat":
        return rmat(**cfg)
    if kind == "chung_lu":
        return chung_lu(**cfg)
    raise KeyError(name)


def _batch_member(args):
    i, seed0, scale_max = args
    rng = np.random.default_rng(seed0 + i)
    if i % 2 == 0:
        scale = int(rng.integers(8, scale_max + 1))
        ef = int(rng.integers(8, 33))
        g = rmat(scale, ef, seed=seed0 + i)
        g.name = f"rmat{scale}_ef{ef}_s{seed0 + i}"
    else:
        n = int(rng.integers(1000, 50001))
        deg = float(rng.uniform(10.0, 40.0))
        g = erdos_renyi(n, deg, seed=seed0 + i)
        g.name = f"er{n}_d{deg:.1f}_s{seed0 + i}"
    return g


def batch_suite_member(i: int, seed0: int = 4000, scale_max: int = 16) -> CSR:
    """Graph i of the mixed batch (before the shuffle of batch_suite)."""
    return _batch_member((i, seed0, scale_max))


def batch_suite_specs(count: int = 512, seed0: int = 4000, scale_max: int = 16) -> list:
    """(kind, size) of every member without generating it: ("rmat", scale)
    or ("er", n), indexed like batch_suite_member."""
    out = []
    for i in range(count):
        rng = np.random.default_rng(seed0 + i)
        if i % 2 == 0:
            out.append(("rmat", int(rng.integers(8, scale_max + 1))))
        else:
            out.append(("er", int(rng.integers(1000, 50001))))
    return out


def batch_suite_order(count: int = 512, seed0: int = 4000) -> list:
    """Member index at each position of batch_suite's shuffled list."""
    return [int(j) for j in np.random.default_rng(seed0).permutation(count)]


def batch_suite(count: int = 512, seed0: int = 4000, scale_max: int = 16, workers: int = 1) -> list:
    """Mixed batch of graphs: half R-MAT (scale U{8..scale_max}, edge factor
    U{8..32}), half Erdos-Renyi (n U[1000, 50000], mean degree U[10, 40]),
    graph i drawn from seed seed0 + i and the list shuffled by seed0.  The
    result does not depend on ``workers`` (generator processes)."""
    jobs = [(i, seed0, scale_max) for i in range(count)]
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(workers) as pool:
            out = pool.map(_batch_member, jobs, chunksize=4)
    else:
        out = [_batch_member(j) for j in jobs]
    return [out[j] for j in batch_suite_order(count, seed0)]


def serve_suite(count: int = 64, seed0: int = 5000, scale_min: int = 12, scale_max: int = 20,
                big=None) -> list:
    """Resident graphs of the served form: count - 1 R-MAT graphs (scale
    U{scale_min..scale_max}, edge factor 16, seed seed0 + i) plus ``big`` (by
    default the Chung-Lu configuration graph)."""
    out = []
    for i in range(count - 1):
        rng = np.random.default_rng(seed0 + i)
        scale = int(rng.integers(scale_min, scale_max + 1))
        g = rmat(scale, 16, seed=seed0 + i)
        g.name = f"rmat{scale}_s{seed0 + i}"
        out.append(g)
    out.append(big if big is not None else config_graph("chunglu22"))
    return out
