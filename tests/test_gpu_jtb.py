"""GPU parity for Union-JTB (randomized linking by rank, 64-bit (rank, parent)
words, FindSimple / FindTwoTrySplit) through the C ABI against the CPU oracle.

Labels are canonical (component minima) and compared element by element.  The
roots of a JTB forest are not minima, so the spanning forest is checked by its
invariants, and L_max by what it must satisfy: the k-out partition is the same
whatever the union rule, so the tree JTB picks must be a most frequent tree of
the oracle's k-out labels over the same sampled vertices."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs as tg
from tests.test_gpu_static import _graphs

pytestmark = pytest.mark.gpu

FINDS = ("naive", "two_try_split")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cases(gpu_available):
    from paper_2008_11839_amd import gconn as G
    out = {}
    for name, C in _graphs().items():
        want = oracle.cc(C.n, C.offsets, C.nbrs)
        out[name] = (C, G.csr(C.offsets, C.nbrs, C.n), want)
    return out


def _labels(G, dg, **kw):
    import torch
    lab = G.cc(dg, options=G.Options(link="jtb", **kw))
    torch.cuda.synchronize()
    return G.to_u32(lab)


def _sampled_vertices(n, samples=1024, seed=1):
    return np.array([((oracle.splitmix64(seed, j) >> 32) * n) >> 32 for j in range(samples)],
                    np.int64)


def test_jtb_labels(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        for sample in ("none", "kout"):
            say(f"[jtb] graph={name} n={C.n} m={C.m} sample={sample}")
            for find in FINDS:
                got = _labels(G, dg, sample=sample, find=find)
                assert np.array_equal(got, want), (name, sample, find)
        for seed in (2, 3):  # other tie-breaking keys
            assert np.array_equal(_labels(G, dg, sample="kout", find="two_try_split", seed=seed),
                                  want), (name, seed)


def test_jtb_random_kout_larger_k_and_blocks(cases):
    from paper_2008_11839_amd import gconn as G
    for name in ("rmat14", "er_dense", "hub_segments", "grid3d"):
        C, dg, want = cases[name]
        say(f"[jtb-k] graph={name}")
        for k, rnd in ((1, False), (3, False), (3, True), (5, True)):
            got = _labels(G, dg, sample="kout", find="two_try_split", k=k, kout_random=rnd)
            assert np.array_equal(got, want), (name, k, rnd)
        for block in (64, 512, 1024):
            got = _labels(G, dg, sample="kout", find="naive", block=block)
            assert np.array_equal(got, want), (name, block)


def test_jtb_stats(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        c = int((want == np.arange(C.n, dtype=np.uint32)).sum())
        say(f"[jtb-stats] graph={name}")
        for find in FINDS:
            lab, st = G.cc(dg, options=G.Options(link="jtb", find=find, sample="none"), stats=True)
            assert np.array_equal(G.to_u32(lab), want)
            assert st["hooks"] == C.n - c, (name, find)
            if C.m == 0:
                continue
            s_lab, e = oracle.sample_kout(C.n, C.offsets, C.nbrs, 2)
            lab, st = G.cc(dg, options=G.Options(link="jtb", find=find, sample="kout"), stats=True)
            assert np.array_equal(G.to_u32(lab), want)
            assert st["hooks"] == C.n - c, (name, find)
            assert st["sampled_edges"] == e
            vs = _sampled_vertices(C.n)
            picked = s_lab[vs]
            _, counts = np.unique(picked, return_counts=True)
            tree = s_lab[st["lmax"]]
            assert int((picked == tree).sum()) == counts.max(), (name, find)
            assert st["active_vertices"] == oracle.active_count(C.n, C.offsets, s_lab, tree)
            assert st["finish_edges"] == oracle.active_edges(C.n, C.offsets, s_lab, tree)


def test_jtb_spanning_forest(cases):
    import torch
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        say(f"[jtb-sf] graph={name}")
        for sample in ("none", "kout"):
            for find in FINDS:
                for with_labels in (True, False):
                    fu, fv, lab = G.spanning_forest(
                        dg, want_labels=with_labels,
                        options=G.Options(link="jtb", sample=sample, find=find))
                    torch.cuda.synchronize()
                    oracle.check_forest(C.n, C.offsets, C.nbrs, G.to_u32(fu), G.to_u32(fv), want)
                    if with_labels:
                        assert np.array_equal(G.to_u32(lab), want), (name, sample, find)


def test_jtb_coo_and_uint64_offsets(cases):
    import torch
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        src, dst = C.coo()
        half = src < dst
        for s_, d_ in ((src, dst), (src[half], dst[half])):
            g = G.coo(s_, d_, C.n)
            say(f"[jtb-coo] graph={name} m={g.m}")
            for find in FINDS:
                lab = G.cc(g, options=G.Options(link="jtb", find=find))
                torch.cuda.synchronize()
                assert np.array_equal(G.to_u32(lab), want), (name, find)
    for name in ("rmat14", "grid2d", "hub_segments"):
        C, _, want = cases[name]
        dg = G.csr(C.offsets, C.nbrs, C.n, offsets64=True)
        for sample in ("none", "kout"):
            assert np.array_equal(_labels(G, dg, sample=sample, find="two_try_split"), want)


def test_jtb_repeated_runs_under_contention(cases):
    from paper_2008_11839_amd import gconn as G
    for name in ("star_center_max", "star_center_0", "clique", "hub_segments", "path_desc"):
        C, dg, want = cases[name]
        say(f"[jtb-repeat] graph={name}")
        for rep in range(30):
            find = FINDS[rep % 2]
            got = _labels(G, dg, sample="none" if rep % 3 else "kout", find=find, seed=rep + 1)
            assert np.array_equal(got, want), (name, rep)


def test_jtb_incremental_batches():
    import torch
    from paper_2008_11839_amd import gconn as G
    n = 20000
    src, dst = graphgen.rmat_edges(15, 60000, 21, n=n)
    graphgen.shuffle_edges(src, dst, 21)
    bounds = [0, 1, 10, 1000, 1001, 7000, 20000, 45000, len(src)]
    for find in FINDS:
        say(f"[jtb-inc] find={find}")
        inc = G.Incremental(n, options=G.Options(sample="none", link="jtb", find=find))
        uf = oracle.UnionFind(n)
        for i in range(len(bounds) - 1):
            lo, hi = bounds[i], bounds[i + 1]
            inc.insert(torch.from_numpy(src[lo:hi].view(np.int32)).cuda(),
                       torch.from_numpy(dst[lo:hi].view(np.int32)).cuda())
            uf.insert(src[lo:hi], dst[lo:hi])
            a, b = graphgen.uniform_pairs(n, 5000, 21, i)
            a = np.concatenate([a, src[lo:hi][:500]])
            b = np.concatenate([b, dst[lo:hi][:500]])
            out = inc.query(torch.from_numpy(a.view(np.int32)).cuda(),
                            torch.from_numpy(b.view(np.int32)).cuda())
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), uf.query(a, b)), (find, i)
            assert np.array_equal(G.to_u32(inc.labels()), uf.labels()), (find, i)
        inc.close()


def test_jtb_incremental_initial_graph_and_mixed():
    import torch
    from paper_2008_11839_amd import gconn as G
    C = graphgen.rmat(13, 8, 6)
    n_max = C.n + 500
    extra_s, extra_d = graphgen.er_edges(n_max, 3000, 6)
    for sample in ("none", "kout"):
        say(f"[jtb-inc-initial] sample={sample}")
        inc = G.Incremental(n_max, initial=G.csr(C.offsets, C.nbrs, C.n),
                            options=G.Options(sample=sample, link="jtb", find="two_try_split"))
        uf = oracle.UnionFind(n_max)
        s0, d0 = C.coo()
        uf.insert(s0, d0)
        assert np.array_equal(G.to_u32(inc.labels()), uf.labels())
        # a mixed batch: its inserts first, then its queries
        rng = np.random.default_rng(7)
        kind = (rng.random(len(extra_s)) < 0.5).astype(np.uint8)
        qa, qb = graphgen.uniform_pairs(n_max, len(extra_s), 7, 0)
        a = np.where(kind == 0, extra_s, qa).astype(np.uint32)
        b = np.where(kind == 0, extra_d, qb).astype(np.uint32)
        out = inc.mixed(torch.from_numpy(kind).cuda(), torch.from_numpy(a.view(np.int32)).cuda(),
                        torch.from_numpy(b.view(np.int32)).cuda())
        uf.insert(a[kind == 0], b[kind == 0])
        want = np.zeros(len(a), np.uint8)
        want[kind == 1] = uf.query(a[kind == 1], b[kind == 1])
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), want), sample
        assert np.array_equal(G.to_u32(inc.labels()), uf.labels()), sample
        inc.close()


def test_jtb_captured_replays(cases):
    import torch
    from paper_2008_11839_amd import gconn as G
    for name in ("rmat14", "grid2d", "star_center_max"):
        C, dg, want = cases[name]
        for sample in ("none", "kout"):
            say(f"[jtb-capture] graph={name} sample={sample}")
            o = G.Options(link="jtb", find="two_try_split", sample=sample)
            lab = torch.empty(C.n, dtype=torch.int32, device="cuda")
            ex = G.capture_cc(dg, lab, options=o)
            for rep in range(3):
                lab.fill_(-1)
                ex.launch()
                torch.cuda.synchronize()
                assert np.array_equal(G.to_u32(lab), want), (name, sample, rep)
            ex.close()


def test_jtb_option_errors():
    from paper_2008_11839_amd import gconn as G
    assert G.LINK["jtb"] == 10 and G.FIND["two_try_split"] == 4
    C = tg.csr(64, tg.path(64))
    with pytest.raises(G.GconnError) as e:
        G.cc(G.csr(C.offsets, C.nbrs, C.n), options=G.Options(link="jtb", find="split"))
    assert e.value.status == -7
