"""Pins for the CPU oracle: brute force, a library routine, closed forms and
invariants -- nothing here re-calls the oracle to check itself."""
from __future__ import annotations

from collections import Counter

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs as tg

# Published SplitMix64 outputs for state 1234567 (Vigna's reference splitmix64.c).
SPLITMIX_1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423,
                    4593380528125082431, 16408922859458223821]


def test_splitmix64_published_vectors():
    assert [oracle.splitmix64(1234567, i) for i in range(5)] == SPLITMIX_1234567
    assert graphgen.splitmix64_sequence(1234567, 5) == SPLITMIX_1234567


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5])
def test_exhaustive_tiny_graphs_against_bfs(n):
    for pairs in tg.all_graphs(n):
        want = tg.bfs_labels(n, pairs)
        G = tg.csr(n, pairs)
        assert oracle.cc(n, G.offsets, G.nbrs).tolist() == want, pairs
        src = [u for u, _ in pairs]
        dst = [v for _, v in pairs]
        assert oracle.cc_coo(n, src, dst).tolist() == want, pairs


@pytest.mark.parametrize("seed", range(6))
def test_random_graphs_against_bfs_and_scipy(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 2000))
    m = int(rng.integers(0, 3 * n))
    pairs = [(int(a), int(b)) for a, b in rng.integers(0, n, size=(m, 2))]
    G = tg.csr(n, pairs)
    got = oracle.cc(n, G.offsets, G.nbrs)
    assert got.tolist() == tg.bfs_labels(n, pairs)
    assert np.array_equal(got, tg.scipy_min_labels(n, G.offsets, G.nbrs))


@pytest.mark.parametrize("maker", ["er", "rmat", "grid2d", "grid3d"])
def test_generated_families_against_scipy(maker):
    G = {"er": lambda: graphgen.er(20000, 30000, 3),
         "rmat": lambda: graphgen.rmat(14, 8, 3),
         "grid2d": lambda: graphgen.grid2d(150, 130, 0.5, 3),
         "grid3d": lambda: graphgen.grid3d(30, 20, 25, 0.3, 3)}[maker]()
    got = oracle.cc(G.n, G.offsets, G.nbrs)
    want = tg.scipy_min_labels(G.n, G.offsets, G.nbrs)
    assert np.array_equal(got, want)
    # COO route over the same entries
    src, dst = G.coo()
    assert np.array_equal(oracle.cc_coo(G.n, src, dst), want)


def _labels(n, pairs):
    G = tg.csr(n, pairs)
    return oracle.cc(n, G.offsets, G.nbrs)


def test_closed_forms():
    n = 97
    assert _labels(n, []).tolist() == list(range(n))                      # no edges
    for seed in range(3):                                                  # relabelled path / cycle
        pairs, _ = tg.relabel(n, tg.path(n), seed)
        assert _labels(n, pairs).tolist() == [0] * n
        pairs, _ = tg.relabel(n, tg.cycle(n), seed + 10)
        assert _labels(n, pairs).tolist() == [0] * n
    assert _labels(n, tg.star(n, 50)).tolist() == [0] * n
    assert _labels(40, tg.clique(40)).tolist() == [0] * 40
    lab = _labels(100, tg.matching(100))
    assert lab[1::2].tolist() == list(range(0, 100, 2)) and lab[0::2].tolist() == list(range(0, 100, 2))
    sizes = [3, 1, 5, 2, 7]
    pairs, tot = tg.disjoint_cliques(sizes)
    want = np.repeat(np.cumsum([0] + sizes[:-1]), sizes)
    assert _labels(tot, pairs).tolist() == want.tolist()
    full = graphgen.grid2d(64, 48, 1.0, 1)
    assert oracle.cc(full.n, full.offsets, full.nbrs).tolist() == [0] * full.n
    empty = graphgen.grid2d(64, 48, 0.0, 1)
    assert empty.m == 0
    assert oracle.cc(empty.n, empty.offsets, empty.nbrs).tolist() == list(range(empty.n))
    assert oracle.cc(0, np.zeros(1, np.uint64), np.zeros(0, np.uint32)).tolist() == []


def test_invariants_rmat():
    G = graphgen.rmat(15, 16, 5)
    lab = oracle.cc(G.n, G.offsets, G.nbrs).astype(np.int64)
    src, dst = G.coo()
    assert np.all(lab[src.astype(np.int64)] == lab[dst.astype(np.int64)])
    assert np.all(lab <= np.arange(G.n))
    assert np.all(lab[lab] == lab)
    scipy_lab = tg.scipy_min_labels(G.n, G.offsets, G.nbrs)
    assert len(np.unique(lab)) == len(np.unique(scipy_lab))


@pytest.mark.parametrize("maker", ["tiny", "er", "rmat", "grid"])
def test_spanning_forest_invariants(maker):
    G = {"tiny": lambda: tg.csr(9, [(0, 1), (1, 2), (2, 0), (5, 6), (7, 8), (8, 7)]),
         "er": lambda: graphgen.er(5000, 6000, 2),
         "rmat": lambda: graphgen.rmat(13, 8, 2),
         "grid": lambda: graphgen.grid2d(70, 60, 0.55, 2)}[maker]()
    fu, fv = oracle.spanning_forest(G.n, G.offsets, G.nbrs)
    lab = tg.scipy_min_labels(G.n, G.offsets, G.nbrs)
    info = oracle.check_forest(G.n, G.offsets, G.nbrs, fu, fv, lab)
    assert info["edges"] == G.n - len(np.unique(lab))
    # min-linking fills exactly the slots of the non-minimum vertices
    assert np.array_equal(fu != oracle.EMPTY, lab != np.arange(G.n, dtype=np.uint32))


def test_forest_checker_rejects_planted_mistakes():
    G = graphgen.grid2d(20, 20, 1.0, 1)
    fu, fv = oracle.spanning_forest(G.n, G.offsets, G.nbrs)
    oracle.check_forest(G.n, G.offsets, G.nbrs, fu, fv)
    used = np.nonzero(fu != oracle.EMPTY)[0]
    bad = fu.copy(), fv.copy()
    bad[1][used[3]] = (bad[0][used[3]] + 2) % G.n            # not a lattice edge
    with pytest.raises(AssertionError):
        oracle.check_forest(G.n, G.offsets, G.nbrs, *bad)
    bad = fu.copy(), fv.copy()
    bad[0][used[5]] = bad[1][used[5]] = oracle.EMPTY         # one edge missing
    with pytest.raises(AssertionError):
        oracle.check_forest(G.n, G.offsets, G.nbrs, *bad)
    bad = fu.copy(), fv.copy()                                # duplicate edge -> cycle
    bad[0][used[7]], bad[1][used[7]] = bad[0][used[8]], bad[1][used[8]]
    with pytest.raises(AssertionError):
        oracle.check_forest(G.n, G.offsets, G.nbrs, *bad)


def test_incremental_batches_against_scipy_prefix():
    n = 3000
    src, dst = graphgen.er_edges(n, 4000, 11)
    uf = oracle.UnionFind(n)
    bounds = [0, 1, 17, 400, 401, 1500, 2600, len(src)]
    for i in range(len(bounds) - 1):
        lo, hi = bounds[i], bounds[i + 1]
        uf.insert(src[lo:hi], dst[lo:hi])
        want = tg.scipy_min_labels_pairs(n, src[:hi], dst[:hi])
        a, b = graphgen.uniform_pairs(n, 2000, 11, i)
        assert np.array_equal(uf.query(a, b), (want[a] == want[b]).astype(np.uint8))
        assert np.array_equal(uf.labels(), want)


def test_sampled_partitions_against_scipy():
    for G in (graphgen.rmat(14, 8, 4), graphgen.er(8000, 12000, 4), graphgen.grid2d(60, 50, 0.6, 4)):
        for k in (1, 2, 3):
            lab, e = oracle.sample_kout(G.n, G.offsets, G.nbrs, k)
            s, d = tg.first_k_edges(G, k)
            assert e == len(s)
            assert np.array_equal(lab, tg.scipy_min_labels_pairs(G.n, s, d))
        # HB: step-1 edges (v, first neighbour) where that neighbour is smaller,
        # step-2 first-N edges of the vertices that stayed roots
        N = 4
        lab, e = oracle.sample_hb(G.n, G.offsets, G.nbrs, N)
        deg = G.degrees()
        first = np.where(deg > 0, G.nbrs[np.minimum(G.offsets[:-1], max(G.m - 1, 0)).astype(np.int64)], 0)
        v = np.arange(G.n)
        step1 = (deg > 0) & (first < v)
        s1, d1 = v[step1], first[step1]
        s2, d2 = tg.first_k_edges(G, N)
        keep = ~step1[s2]
        s = np.concatenate([s1, s2[keep]])
        d = np.concatenate([d1, d2[keep]])
        assert np.array_equal(lab, tg.scipy_min_labels_pairs(G.n, s, d))
        assert e == int((deg > 0).sum() + keep.sum())
        # BFS: the component of the largest-degree vertex (smallest id on ties)
        lab, src_v = oracle.sample_bfs(G.n, G.offsets, G.nbrs)
        assert src_v == int(np.argmax(deg))
        full = tg.scipy_min_labels(G.n, G.offsets, G.nbrs)
        want = np.where(full == full[src_v], full, np.arange(G.n, dtype=np.uint32))
        assert np.array_equal(lab, want)


def _splitmix_py(state0, i):
    M = (1 << 64) - 1
    z = (state0 + (i + 1) * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_lmax_definition():
    # constant labels: the only label
    assert oracle.lmax(np.full(1000, 42, np.uint32), 1024, 3) == 42
    assert oracle.lmax(np.array([7], np.uint32), 1024, 3) == 7
    # overwhelming majority
    lab = np.full(100000, 5, np.uint32)
    lab[::100] = 9
    assert oracle.lmax(lab, 1024, 9) == 5
    # independent route: sample with a Python SplitMix64 (pinned by the
    # published vectors above), then mode with smallest label on ties
    assert [_splitmix_py(1234567, i) for i in range(5)] == SPLITMIX_1234567
    rng = np.random.default_rng(0)
    for trial in range(20):
        n = int(rng.integers(1, 5000))
        lab = rng.integers(0, max(1, n // 50), size=n).astype(np.uint32)
        s = int(rng.integers(1, 300))
        seed = int(rng.integers(0, 2**63))
        picks = [int(lab[((_splitmix_py(seed, j) >> 32) * n) >> 32]) for j in range(s)]
        cnt = Counter(picks)
        top = max(cnt.values())
        assert oracle.lmax(lab, s, seed) == min(k for k, c in cnt.items() if c == top)


def _clique_pairs(ids):
    return [(ids[i], ids[j]) for i in range(len(ids)) for j in range(i + 1, len(ids))]


def test_active_set_closed_forms():
    """Vertex gathering (Finish phase of the static algorithm): the active set
    is the vertices with degree > 0 whose label is not L_max, and the finish
    reads their whole rows.  Pinned by closed forms on graphs whose answer
    follows from their shape, with vertex ids shuffled so no block is
    contiguous."""
    # disjoint cliques K50, K3, K7, a star with 9 leaves, a path of 6 vertices,
    # and 5 isolated vertices
    sizes = {"k50": 50, "k3": 3, "k7": 7, "star": 10, "path": 6, "iso": 5}
    n = sum(sizes.values())
    perm = np.random.default_rng(7).permutation(n).astype(np.uint32)
    blocks, at = {}, 0
    for name, sz in sizes.items():
        blocks[name] = [int(x) for x in perm[at:at + sz]]
        at += sz
    pairs = (_clique_pairs(blocks["k50"]) + _clique_pairs(blocks["k3"])
             + _clique_pairs(blocks["k7"])
             + [(blocks["star"][0], x) for x in blocks["star"][1:]]
             + list(zip(blocks["path"][:-1], blocks["path"][1:])))
    G = graphgen.from_pairs(n, pairs)
    # labels: the component minimum of each block (the final labels)
    lab = np.arange(n, dtype=np.uint32)
    for ids in blocks.values():
        if ids is blocks["iso"]:
            continue
        lab[ids] = min(ids)
    big = min(blocks["k50"])
    # L_max = the K50 label: active = K3 + K7 + star + path; rows: a clique
    # K_s contributes s(s-1) entries, the star 2*9, the path 2*5
    assert oracle.active_count(n, G.offsets, lab, big) == 3 + 7 + 10 + 6
    assert oracle.active_edges(n, G.offsets, lab, big) == 3 * 2 + 7 * 6 + 18 + 10
    # L_max = the star's label: its 10 vertices drop out instead
    s0 = min(blocks["star"])
    assert oracle.active_count(n, G.offsets, lab, s0) == 50 + 3 + 7 + 6
    assert oracle.active_edges(n, G.offsets, lab, s0) == 50 * 49 + 3 * 2 + 7 * 6 + 10
    # a label that occurs nowhere: every vertex with an edge is active and the
    # finish reads every entry (isolated vertices never count)
    none = 0xFFFFFFFF
    assert oracle.active_count(n, G.offsets, lab, none) == n - 5
    assert oracle.active_edges(n, G.offsets, lab, none) == 2 * len(pairs)
    # an isolated vertex's own label as L_max removes nothing
    iso = blocks["iso"][0]
    assert oracle.active_count(n, G.offsets, lab, iso) == n - 5
    assert oracle.active_edges(n, G.offsets, lab, iso) == 2 * len(pairs)
    # sampled labels that split a component (the K7 cut 4 | 3, the path
    # 2 | 4): only the vertices labelled L_max drop out, whatever their
    # component; L_max = the label of the K7's 4-part
    k7 = blocks["k7"]
    lab2 = lab.copy()
    lab2[k7[4:]] = k7[4]
    lab2[blocks["path"][2:]] = blocks["path"][2]
    four = int(lab2[k7[0]])
    assert oracle.active_count(n, G.offsets, lab2, four) == n - 5 - 4
    assert oracle.active_edges(n, G.offsets, lab2, four) == 2 * len(pairs) - 4 * 6


def test_active_set_star_and_path():
    # a star K_{1,r} labelled 0 except the centre: L_max = 0 leaves only the
    # centre active, with its r entries
    for r in (1, 2, 17):
        G = graphgen.from_pairs(r + 1, [(0, x) for x in range(1, r + 1)])
        lab = np.zeros(r + 1, np.uint32)
        lab[0] = 1
        assert oracle.active_count(r + 1, G.offsets, lab, 0) == 1
        assert oracle.active_edges(r + 1, G.offsets, lab, 0) == r
        # the leaves: r vertices of degree 1
        assert oracle.active_count(r + 1, G.offsets, lab, 1) == r
        assert oracle.active_edges(r + 1, G.offsets, lab, 1) == r
    # a path 0-1-...-(L-1) with labels alternating 0/1: L_max = 1 keeps the
    # even positions: ceil(L/2) vertices, ends have degree 1
    for L in (2, 3, 10, 11):
        G = graphgen.from_pairs(L, [(i, i + 1) for i in range(L - 1)])
        lab = (np.arange(L) % 2).astype(np.uint32)
        evens = (L + 1) // 2
        ends_even = 1 + (1 if (L - 1) % 2 == 0 else 0)
        assert oracle.active_count(L, G.offsets, lab, 1) == evens
        assert oracle.active_edges(L, G.offsets, lab, 1) == 2 * evens - ends_even
