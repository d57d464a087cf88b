"""GPU parity of BFS sampling on graphs built to drive the bottom-up kernel's
less common paths: rows whose first frontier neighbour lies deep in the row
(the part of the row spread over the wave, several 64-entry steps, the skip
past rows whose parent is known), rows with no frontier neighbour at all,
and a vertex count that is not a multiple of 4 or 32.

Besides the oracle's labels and source, the BFS forest is checked against a
level-synchronous BFS computed here: every parent lies one level up, and a
vertex found by a bottom-up level takes the first neighbour of its row that
lies in the frontier (the choice a sequential scan of the row makes)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _levels(n, off, nb, src):
    """Plain level-synchronous BFS (numpy): level of every vertex, -1 if unreached."""
    lev = np.full(n, -1, np.int64)
    lev[src] = 0
    front = np.array([src], np.int64)
    d = 0
    while len(front):
        d += 1
        starts, ends = off[front], off[front + 1]
        idx = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)]) if len(front) else []
        cand = np.unique(nb[np.asarray(idx, np.int64)].astype(np.int64))
        cand = cand[lev[cand] < 0]
        lev[cand] = d
        front = cand
    return lev


def _deep_rows_graph(seed: int):
    """Hub 0 -> A (2000 vertices) -> B (3000 vertices).  Rows are sorted by
    neighbour id and the private leaves take the smallest ids, so B vertex
    j's row holds its pad_j leaves first and then 30 A neighbours, with pad_j
    cycling through 0..3, 63..66, 127..130 and 150..200.  A further 500
    vertices (C) are joined to B and to leaves only, so their rows hold no
    level-1 vertex.  A few isolated vertices make n % 32 == 5."""
    rng = np.random.default_rng(seed)
    nA, nB, nC = 2000, 3000, 500
    pads = [0, 1, 2, 3, 63, 64, 65, 66, 127, 128, 129, 130] + list(range(150, 201, 10))
    padB = [pads[j % len(pads)] for j in range(nB)]
    padC = [int(x) for x in rng.integers(70, 140, size=nC)]
    leaves = sum(padB) + sum(padC)
    A = np.arange(1 + leaves, 1 + leaves + nA)
    B = np.arange(A[-1] + 1, A[-1] + 1 + nB)
    C = np.arange(B[-1] + 1, B[-1] + 1 + nC)
    n = int(C[-1]) + 1 + 5
    n += (5 - n % 32) % 32
    pairs = [(0, int(a)) for a in A]
    leaf = 1
    for b, p in zip(B, padB):
        pairs += [(int(b), leaf + i) for i in range(p)]
        leaf += p
        pairs += [(int(b), int(a)) for a in rng.choice(A, 30, replace=False)]
    for c, p in zip(C, padC):
        pairs += [(int(c), leaf + i) for i in range(p)]
        leaf += p
        pairs += [(int(c), int(b)) for b in rng.choice(B, 3, replace=False)]
    return graphgen.from_pairs(n, pairs, f"deep_rows_s{seed}")


@pytest.mark.parametrize("seed", [1, 2])
def test_bfs_bottom_up_deep_rows(gpu_available, seed):
    import torch
    from paper_2008_11839_amd import gconn as G
    Cg = _deep_rows_graph(seed)
    n = Cg.n
    off = Cg.offsets.astype(np.int64)
    nb = Cg.nbrs.astype(np.int64)
    deg = np.diff(off)
    assert n % 4 != 0 and n % 32 == 5
    want = oracle.cc(n, Cg.offsets, Cg.nbrs)
    b_lab, src = oracle.sample_bfs(n, Cg.offsets, Cg.nbrs)
    assert src == 0
    lev = _levels(n, off, nb, src)
    # the construction sends level 2 bottom-up: the direction rule switches
    # when 14 x (row entries of the frontier) exceeds the unexplored entries
    level1 = np.nonzero(lev == 1)[0]
    m_f = int(deg[level1].sum())
    m_u = int(off[-1]) - int(deg[src]) - m_f
    assert 14 * m_f > m_u

    dg = G.csr(Cg.offsets, Cg.nbrs, n)
    say(f"[bfs-deep] seed={seed} n={n} m={Cg.m}")
    lab, st = G.cc(dg, options=G.Options(sample="bfs"), stats=True)
    torch.cuda.synchronize()
    assert st["bfs_source"] == src
    assert np.array_equal(G.to_u32(lab), want)

    fu, fv, lab2 = G.spanning_forest(dg, want_labels=True, options=G.Options(sample="bfs"))
    torch.cuda.synchronize()
    fu, fv = G.to_u32(fu).astype(np.int64), G.to_u32(fv).astype(np.int64)
    assert np.array_equal(G.to_u32(lab2), want)
    oracle.check_forest(n, Cg.offsets, Cg.nbrs, fu.astype(np.uint32), fv.astype(np.uint32), want)
    reached = np.nonzero(lev > 0)[0]
    assert np.array_equal(fv[reached], reached)
    assert np.array_equal(lev[fu[reached]], lev[reached] - 1)
    # level 2 was bottom-up: each vertex there took the first level-1 entry of its row
    for v in np.nonzero(lev == 2)[0]:
        row = nb[off[v]:off[v + 1]]
        first = row[np.argmax(lev[row] == 1)]
        assert fu[v] == first, (v, fu[v], first)


def test_bfs_long_diameter_mesh(gpu_available):
    """A mesh whose BFS runs over a thousand levels: after the first batch of
    levels the frontier stays far below the switch point, so batches enqueue
    only the top-down kernels with grids sized to the frontier.  Labels,
    source and forest are checked as above (every parent one level up)."""
    import torch
    from paper_2008_11839_amd import gconn as G
    Cg = graphgen.grid2d(1024, 256, 0.9, 3)
    n = Cg.n
    off = Cg.offsets.astype(np.int64)
    nb = Cg.nbrs.astype(np.int64)
    want = oracle.cc(n, Cg.offsets, Cg.nbrs)
    _, src = oracle.sample_bfs(n, Cg.offsets, Cg.nbrs)
    lev = _levels(n, off, nb, src)
    assert lev.max() > 800  # many batches of eight levels
    dg = G.csr(Cg.offsets, Cg.nbrs, n)
    say(f"[bfs-mesh] n={n} m={Cg.m} levels={int(lev.max())}")
    lab, st = G.cc(dg, options=G.Options(sample="bfs"), stats=True)
    torch.cuda.synchronize()
    assert st["bfs_source"] == src
    assert st["rounds"] == int(lev.max()) + 1  # one per non-empty frontier, the source's included
    assert np.array_equal(G.to_u32(lab), want)
    fu, fv, lab2 = G.spanning_forest(dg, want_labels=True, options=G.Options(sample="bfs"))
    torch.cuda.synchronize()
    fu, fv = G.to_u32(fu).astype(np.int64), G.to_u32(fv).astype(np.int64)
    assert np.array_equal(G.to_u32(lab2), want)
    oracle.check_forest(n, Cg.offsets, Cg.nbrs, fu.astype(np.uint32), fv.astype(np.uint32), want)
    reached = np.nonzero(lev > 0)[0]
    assert np.array_equal(lev[fu[reached]], lev[reached] - 1)


def test_bfs_source_and_minimum_past_the_first_pass(gpu_available):
    """More vertices than one grid-stride pass of the source-selection kernel
    covers (its grid stops at 8,192 workgroups, 8,388,608 vertices with
    256-thread workgroups of four vertices per lane), with the two
    largest-degree vertices tied at degree 100 and both beyond that first
    pass: the source is the smaller id of the two.  The source's component
    also holds vertex 5, so its minimum comes from another workgroup's slot
    than the source's, and every other vertex keeps its own id or joins the
    second hub's or the third hub's (degree 99) component."""
    import torch
    from paper_2008_11839_amd import gconn as G
    n = 9_000_005
    hub_a, hub_b, hub_c = 8_500_000, 8_999_990, 3
    pairs = [(hub_a, 8_400_000 + i) for i in range(100)]
    pairs += [(hub_b, 8_800_000 + i) for i in range(100)]
    pairs += [(hub_c, 100 + i) for i in range(99)]
    pairs += [(8_400_050, 5)]
    Cg = graphgen.from_pairs(n, pairs, "two_tied_hubs")
    want = oracle.cc(n, Cg.offsets, Cg.nbrs)
    _, src = oracle.sample_bfs(n, Cg.offsets, Cg.nbrs)
    assert src == hub_a and want[hub_a] == 5 and want[hub_b] == 8_800_000
    dg = G.csr(Cg.offsets, Cg.nbrs, n)
    say(f"[bfs-tied-hubs] n={n} m={Cg.m}")
    lab, st = G.cc(dg, options=G.Options(sample="bfs"), stats=True)
    torch.cuda.synchronize()
    assert st["bfs_source"] == src
    assert st["rounds"] == 3  # frontiers {hub}, its leaves, {5}
    assert np.array_equal(G.to_u32(lab), want)
