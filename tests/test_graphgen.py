"""Generator sanity: determinism, layout, and closed-form statistics."""
from __future__ import annotations

import math

import numpy as np

import graphgen


def _csr_ok(G):
    off = G.offsets.astype(np.int64)
    assert off[0] == 0 and np.all(np.diff(off) >= 0) and off[-1] == len(G.nbrs)
    if G.m:
        assert int(G.nbrs.max()) < G.n
        # rows sorted
        row_start = np.zeros(G.m, bool)
        row_start[off[:-1][np.diff(off) > 0]] = True
        d = np.diff(G.nbrs.astype(np.int64))
        assert np.all((d >= 0) | row_start[1:])
    # symmetric: multiset of (u,v) equals multiset of (v,u)
    src, dst = G.coo()
    a = np.sort(src.astype(np.uint64) << np.uint64(32) | dst.astype(np.uint64))
    b = np.sort(dst.astype(np.uint64) << np.uint64(32) | src.astype(np.uint64))
    assert np.array_equal(a, b)


def test_determinism_and_layout():
    for mk in (lambda: graphgen.er(3000, 9000, 5), lambda: graphgen.rmat(12, 16, 5),
               lambda: graphgen.grid2d(40, 33, 0.7, 5), lambda: graphgen.grid3d(9, 8, 7, 0.6, 5)):
        A, B = mk(), mk()
        assert np.array_equal(A.offsets, B.offsets) and np.array_equal(A.nbrs, B.nbrs)
        _csr_ok(A)


def test_er_counts():
    n, m = 100000, 1000000
    s, d = graphgen.er_edges(n, m, 1)
    assert np.all(s != d)
    # expected self-loops m/n = 10; keep count within a generous band
    assert m - 60 < len(s) <= m
    G = graphgen.csr_from_edges(n, s, d)
    assert G.m == 2 * len(s)


def test_rmat_isolated_fraction_closed_form():
    S, ef = 16, 16
    a, b, c = 0.57, 0.19, 0.19
    d = 1 - a - b - c
    M = ef << S
    G = graphgen.rmat(S, ef, 7)
    iso = int((G.degrees() == 0).sum())
    expect = 0.0
    for j in range(S + 1):
        pu = (a + b) ** (S - j) * (c + d) ** j
        pv = (a + c) ** (S - j) * (b + d) ** j
        puv = a ** (S - j) * d ** j
        expect += math.comb(S, j) * (1 - pu - pv + 2 * puv) ** M
    assert abs(iso - expect) < 6 * math.sqrt(expect) + 10, (iso, expect)


def test_rmat_scramble_is_a_bijection():
    A = graphgen.rmat(13, 8, 3, scramble=False)
    B = graphgen.rmat(13, 8, 3, scramble=True)
    assert A.m == B.m
    assert np.array_equal(np.sort(A.degrees()), np.sort(B.degrees()))
    # without the scramble the hub is vertex 0 (all-zero bits is the likeliest id)
    assert int(np.argmax(A.degrees())) == 0


def test_rmat_non_power_of_two():
    n = 3000
    G = graphgen.rmat(12, 10, 9, n=n)
    assert G.n == n and G.m > 0 and int(G.nbrs.max()) < n
    _csr_ok(G)


def test_grid_counts():
    W, H = 200, 150
    full = graphgen.grid2d(W, H, 1.0, 1)
    assert full.m == 2 * ((W - 1) * H + W * (H - 1))
    p = 0.7
    L = (W - 1) * H + W * (H - 1)
    G = graphgen.grid2d(W, H, p, 1)
    k = G.m // 2
    assert abs(k - p * L) < 6 * math.sqrt(L * p * (1 - p))
    X = Y = Z = 20
    full3 = graphgen.grid3d(X, Y, Z, 1.0, 1)
    assert full3.m == 2 * 3 * (X - 1) * Y * Z
    # every grid edge joins lattice neighbours
    src, dst = G.coo()
    diff = np.abs(src.astype(np.int64) - dst.astype(np.int64))
    assert np.all((diff == 1) | (diff == W))


def test_uniform_pairs_and_shuffle():
    a, b = graphgen.uniform_pairs(1000, 50000, 3, 0)
    assert a.max() < 1000 and b.max() < 1000
    assert abs(a.mean() - 499.5) < 10
    s, d = graphgen.er_edges(500, 2000, 2)
    s2, d2 = s.copy(), d.copy()
    graphgen.shuffle_edges(s2, d2, 4)
    key = lambda x, y: np.sort(x.astype(np.uint64) << np.uint64(32) | y.astype(np.uint64))
    assert np.array_equal(key(s, d), key(s2, d2)) and not np.array_equal(s, s2)


def test_batched_specs_ranges():
    specs = graphgen.batched_specs(2000, 1)
    ns = np.array([s[1] for s in specs])
    efs = np.array([s[2] for s in specs])
    assert ns.min() >= 1000 and ns.max() <= 1000000
    assert efs.min() >= 8 and efs.max() <= 32
    kinds = [s[0] for s in specs]
    assert 800 < kinds.count("rmat") < 1200
    # log-uniform: median near 10^4.5
    assert 10 ** 4.3 < np.median(ns) < 10 ** 4.7


def test_barabasi_albert_stream():
    n, k = 50000, 10
    s, d = graphgen.ba_edges(n, k, 3)
    s2, d2 = graphgen.ba_edges(n, k, 3)
    assert np.array_equal(s, s2) and np.array_equal(d, d2)
    # arrival order, k slots per vertex, every kept edge points to an earlier vertex
    assert np.all(np.diff(s.astype(np.int64)) >= 0)
    assert np.all(d < s)
    assert np.bincount(s, minlength=n).max() <= k
    # self-loops (dropped): slot e copies itself with probability 1/(2e+1),
    # about ln(2nk)/2 ~ 7 in total; allow generous slack
    assert n * k - len(s) < 60
    # preferential attachment: heavy tail (max degree far above the mean 2k)
    deg = np.bincount(np.concatenate([s, d]), minlength=n)
    assert deg.max() > 40 * 2 * k
    assert abs(deg.mean() - 2 * k * len(s) / (n * k)) < 1e-9
    # vertex 0 arrives first: its k slots can only point at itself
    assert 0 not in set(s.tolist())


def test_mixed_stream_composition():
    src, dst = graphgen.rmat_edges(12, 5000, 4)
    for ratio in (1.0, 4.0, 0.5):
        kind, a, b = graphgen.mixed_stream(src, dst, 1 << 12, ratio, 9)
        q = int(round(len(src) / ratio))
        assert len(kind) == len(src) + q and int(kind.sum()) == q
        ins = kind == 0
        got = sorted(zip(a[ins].tolist(), b[ins].tolist()))
        assert got == sorted(zip(src.tolist(), dst.tolist()))
        assert a.max() < (1 << 12) and b.max() < (1 << 12)
