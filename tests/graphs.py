"""Small closed-form graphs and independent reference routines for the tests.

Nothing here is the oracle: these are brute-force or library routes used to
pin it (pure-Python BFS, scipy's connected_components) plus explicit small
graph families whose component structure is known in closed form.
"""
from __future__ import annotations

import itertools

import numpy as np
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components

import graphgen


def bfs_labels(n: int, pairs) -> list[int]:
    """Brute force: BFS from each unvisited vertex in increasing id order and
    label its component with the start vertex (= the component minimum)."""
    adj = [[] for _ in range(n)]
    for u, v in pairs:
        adj[u].append(v)
        adj[v].append(u)
    lab = [-1] * n
    for s in range(n):
        if lab[s] >= 0:
            continue
        lab[s] = s
        frontier = [s]
        while frontier:
            nxt = []
            for x in frontier:
                for y in adj[x]:
                    if lab[y] < 0:
                        lab[y] = s
                        nxt.append(y)
            frontier = nxt
    return lab


def scipy_min_labels(n: int, offsets, nbrs) -> np.ndarray:
    """scipy's connected components, canonicalised to the minimum id."""
    if n == 0:
        return np.zeros(0, np.uint32)
    off = np.asarray(offsets, dtype=np.int64)
    nb = np.asarray(nbrs, dtype=np.int64)
    A = csr_matrix((np.ones(len(nb), np.int8), nb, off), shape=(n, n))
    k, comp = connected_components(A, directed=False)
    mins = np.full(k, n, np.int64)
    np.minimum.at(mins, comp, np.arange(n, dtype=np.int64))
    return mins[comp].astype(np.uint32)


def scipy_min_labels_pairs(n: int, src, dst) -> np.ndarray:
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    A = csr_matrix((np.ones(len(src), np.int8), (src, dst)), shape=(n, n))
    k, comp = connected_components(A, directed=False)
    mins = np.full(k, n, np.int64)
    np.minimum.at(mins, comp, np.arange(n, dtype=np.int64))
    return mins[comp].astype(np.uint32)


def all_graphs(n: int):
    """Every simple undirected graph on n labelled vertices (as pair lists)."""
    slots = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(slots)):
        yield [slots[i] for i in range(len(slots)) if mask >> i & 1]


def relabel(n: int, pairs, seed: int):
    """Apply a seeded random permutation of the vertex ids."""
    perm = np.random.default_rng(seed).permutation(n)
    return [(int(perm[u]), int(perm[v])) for u, v in pairs], perm


# ------------------------------------------------------------ closed forms
def path(n):
    return [(i, i + 1) for i in range(n - 1)]


def cycle(n):
    return path(n) + ([(n - 1, 0)] if n > 2 else [])


def star(n, center):
    return [(center, v) for v in range(n) if v != center]


def clique(n):
    return list(itertools.combinations(range(n), 2))


def matching(n):
    return [(2 * i, 2 * i + 1) for i in range(n // 2)]


def disjoint_cliques(sizes):
    pairs, base = [], 0
    for s in sizes:
        pairs += [(base + a, base + b) for a, b in itertools.combinations(range(s), 2)]
        base += s
    return pairs, base


def csr(n, pairs, name=""):
    return graphgen.from_pairs(n, pairs, name)


def first_k_edges(G: graphgen.CSR, k: int):
    """Explicit edge list of the first k entries of every row."""
    deg = G.degrees()
    take = np.minimum(deg, k)
    src = np.repeat(np.arange(G.n, dtype=np.int64), take)
    starts = np.repeat(G.offsets[:-1].astype(np.int64), take)
    within = np.arange(len(src)) - np.repeat(np.cumsum(take) - take, take)
    dst = G.nbrs[starts + within].astype(np.int64)
    return src, dst
