"""Brute-force k-clique counting by subset enumeration (the definition of a
clique, Section II), for graphs with a handful of vertices.  No ordering and
no recursion: every k-subset is tested pair by pair."""
from itertools import combinations

import numpy as np


def adjacency(g):
    a = np.zeros((g.n, g.n), dtype=bool)
    for u in range(g.n):
        a[u, g.col[g.row_ptr[u]:g.row_ptr[u + 1]]] = True
    return a


def brute_count(g, k):
    a = adjacency(g)
    if k == 1:
        return g.n
    total = 0
    for sub in combinations(range(g.n), k):
        if all(a[x, y] for x, y in combinations(sub, 2)):
            total += 1
    return total


def brute_rooted(g, k, u, v, omega_less):
    """k-cliques whose two lowest vertices under omega are u and v."""
    a = adjacency(g)
    others = [w for w in range(g.n) if w not in (u, v) and a[u, w] and a[v, w]
              and omega_less(u, w) and omega_less(v, w)]
    total = 0
    for sub in combinations(others, k - 2):
        if all(a[x, y] for x, y in combinations(sub, 2)):
            total += 1
    return total
