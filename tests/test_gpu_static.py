"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Labels are compared element by element (bit-exact); spanning forests, where
several answers are correct, are checked for validity plus the exact
slot-occupancy set; sampling intermediates (L_max, active set, sampled edge
count) are compared with the oracle's values for the same seeded sample."""
from __future__ import annotations

import itertools
import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs as tg

pytestmark = pytest.mark.gpu

UF_RULES = ([("async", f, "split_one") for f in ("naive", "split", "halve", "compress")]
            + [("hooks", f, "split_one") for f in ("naive", "split", "halve", "compress")]
            + [("early", f, "split_one") for f in ("naive", "split", "halve", "compress")]
            + [("rem_cas", f, s) for f in ("naive", "split", "halve")
               for s in ("split_one", "halve_one", "splice_atomic")]
            + [("ecl", "halve", "split_one"), ("afforest", "naive", "split_one")]
            + [("rem_lock", f, s) for f, s in (("naive", "split_one"), ("split", "split_one"),
                                              ("halve", "halve_one"), ("split", "splice_atomic"))])
SAMPLERS = ["none", "kout", "hb", "bfs"]
LT_VARIANTS = ["CUSA", "CRSA", "PUSA", "PRSA", "PUS", "PRS", "EUSA", "EUS",
               "CUFA", "CRFA", "PUFA", "PRFA", "PUF", "PRF", "EUFA", "EUF"]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _graphs():
    out = {}
    n = 300
    out["no_edges"] = tg.csr(50, [])
    out["single_vertex"] = tg.csr(1, [])
    out["path_desc"] = tg.csr(n, [(n - 1 - i, n - 2 - i) for i in range(n - 1)])
    out["path_shuffled"] = tg.csr(n, tg.relabel(n, tg.path(n), 3)[0])
    out["cycle"] = tg.csr(n, tg.relabel(n, tg.cycle(n), 4)[0])
    out["star_center_max"] = tg.csr(2000, tg.star(2000, 1999))
    out["star_center_0"] = tg.csr(2000, tg.star(2000, 0))
    out["clique"] = tg.csr(60, tg.clique(60))
    out["matching"] = tg.csr(400, tg.matching(400))
    dc, tot = tg.disjoint_cliques([5, 1, 40, 2, 3, 70, 1, 9])
    out["disjoint_cliques"] = tg.csr(tot, dc)
    out["loops_and_duplicates"] = tg.csr(8, [(0, 0), (1, 2), (2, 1), (1, 2), (3, 3), (4, 7),
                                             (7, 4), (5, 5), (6, 4)])
    out["er"] = graphgen.er(3000, 9000, 7)
    out["er_dense"] = graphgen.er(2000, 40000, 8)
    out["rmat12"] = graphgen.rmat(12, 16, 3)
    out["rmat14"] = graphgen.rmat(14, 8, 5)
    out["rmat13_plain_ids"] = graphgen.rmat(13, 16, 2, scramble=False)
    out["grid2d"] = graphgen.grid2d(120, 90, 0.6, 4)
    out["grid3d"] = graphgen.grid3d(16, 15, 14, 0.45, 4)
    # a hub whose row spans several 1024-edge segments, plus sparse noise
    s, d = graphgen.er_edges(6000, 3000, 9)
    hub = [(5999, v) for v in range(0, 5999, 2)]
    pairs = list(zip(s.tolist(), d.tolist())) + hub
    out["hub_segments"] = tg.csr(6000, pairs)
    return out


@pytest.fixture(scope="module")
def cases(gpu_available):
    import torch  # noqa: F401
    from paper_2008_11839_amd import gconn as G
    out = {}
    for name, C in _graphs().items():
        want = oracle.cc(C.n, C.offsets, C.nbrs)
        out[name] = (C, G.csr(C.offsets, C.nbrs, C.n), want)
    return out


def _labels(G, dg, **kw):
    import torch
    lab = G.cc(dg, options=G.Options(**kw))
    torch.cuda.synchronize()
    return G.to_u32(lab)


def test_union_find_rules_all_samplers(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        for sample in SAMPLERS:
            say(f"[uf] graph={name} n={C.n} m={C.m} sample={sample}")
            for link, find, splice in UF_RULES:
                for ac in (False, True):  # compression writes as stores / as CAS
                    got = _labels(G, dg, sample=sample, link=link, find=find, splice=splice,
                                  atomic_compress=ac)
                    assert np.array_equal(got, want), (name, sample, link, find, splice, ac)


def test_xcd_kout_every_union_rule(cases):
    """The XCD-bucketed k-out schedule (pre-link, flatten, per-XCD record
    groups) with every union-find rule: the oracle's labels, sampled-edge
    count, L_max and active set, and -- for the root-based rules -- a valid
    forest filling exactly the non-minimum slots."""
    import torch
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        roots_mask = want != np.arange(C.n, dtype=np.uint32)
        for k in (1, 2):
            lab_s, e_s = oracle.sample_kout(C.n, C.offsets, C.nbrs, k)
            say(f"[xcd] graph={name} n={C.n} m={C.m} k={k}")
            for link, find, splice in UF_RULES:
                for ac in (False, True):
                    o = G.Options(sample="kout", link=link, find=find, splice=splice, k=k,
                                  schedule="xcd", atomic_compress=ac)
                    lab, st = G.cc(dg, options=o, stats=True)
                    got = G.to_u32(lab)
                    assert np.array_equal(got, want), (name, k, link, find, splice, ac)
                    if C.m:
                        assert st["sampled_edges"] == e_s, (name, k, link)
                if splice == "splice_atomic":
                    continue
                o = G.Options(sample="kout", link=link, find=find, splice=splice, k=k,
                              schedule="xcd")
                fu, fv, lab = G.spanning_forest(dg, want_labels=True, options=o)
                torch.cuda.synchronize()
                assert np.array_equal(G.to_u32(lab), want), (name, k, link, "forest labels")
                fu, fv = G.to_u32(fu), G.to_u32(fv)
                oracle.check_forest(C.n, C.offsets, C.nbrs, fu, fv, want)
                assert np.array_equal(fu != G.EMPTY, roots_mask), (name, k, link)
            if C.m:
                L = oracle.lmax(lab_s, 1024, 1)
                lab, st = G.cc(dg, options=G.Options(sample="kout", link="rem_cas", k=k,
                                                     splice="split_one", schedule="xcd"),
                               stats=True)
                assert st["lmax"] == L, (name, k)
                assert st["active_vertices"] == oracle.active_count(C.n, C.offsets, lab_s, L)
                assert st["finish_edges"] == oracle.active_edges(C.n, C.offsets, lab_s, L)


def test_sv_and_label_propagation_all_samplers(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        for sample in SAMPLERS:
            say(f"[sv/lp] graph={name} sample={sample}")
            for link in ("sv", "lp"):
                got = _labels(G, dg, sample=sample, link=link)
                assert np.array_equal(got, want), (name, sample, link)


@pytest.mark.parametrize("variant", LT_VARIANTS)
def test_liu_tarjan_variants(cases, variant):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        for sample in SAMPLERS:
            say(f"[lt] variant={variant} graph={name} sample={sample}")
            got = _labels(G, dg, sample=sample, link="lt", lt_variant=variant)
            assert np.array_equal(got, want), (name, sample, variant)


def test_spanning_forest_valid_and_slot_exact(cases):
    import torch
    from paper_2008_11839_amd import gconn as G
    rules = [r for r in UF_RULES if r[2] != "splice_atomic"] + [("sv", "split", "split_one")]
    C, dg, _ = cases["er"]
    with pytest.raises(G.GconnError) as e:  # Rem's splice links non-roots: no forest
        G.spanning_forest(dg, options=G.Options(link="rem_cas", splice="splice_atomic"))
    assert e.value.status == -7
    for name, (C, dg, want) in cases.items():
        roots_mask = want != np.arange(C.n, dtype=np.uint32)
        for sample in SAMPLERS:
            say(f"[sf] graph={name} sample={sample}")
            for link, find, splice in rules:
                for with_labels in (True, False):
                    fu, fv, lab = G.spanning_forest(dg, want_labels=with_labels,
                                                    options=G.Options(sample=sample, link=link,
                                                                      find=find, splice=splice))
                    torch.cuda.synchronize()
                    fu, fv = G.to_u32(fu), G.to_u32(fv)
                    oracle.check_forest(C.n, C.offsets, C.nbrs, fu, fv, want)
                    if sample != "bfs":
                        assert np.array_equal(fu != G.EMPTY, roots_mask), (name, sample, link)
                    if with_labels:
                        assert np.array_equal(G.to_u32(lab), want)


def test_sampling_intermediates_match_oracle(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        if C.m == 0:
            continue
        for sample in ("kout", "hb"):
            if sample == "kout":
                s_lab, e = oracle.sample_kout(C.n, C.offsets, C.nbrs, 2)
            else:
                s_lab, e = oracle.sample_hb(C.n, C.offsets, C.nbrs, 4)
            L = oracle.lmax(s_lab, 1024, 1)
            for link in ("async", "rem_cas", "sv"):
                say(f"[stats] graph={name} sample={sample} link={link}")
                lab, st = G.cc(dg, options=G.Options(sample=sample, link=link), stats=True)
                assert st["sampled_edges"] == e
                assert st["lmax"] == L
                assert st["active_vertices"] == oracle.active_count(C.n, C.offsets, s_lab, L)
                assert st["finish_edges"] == oracle.active_edges(C.n, C.offsets, s_lab, L)
                assert np.array_equal(G.to_u32(lab), want)
        # BFS: the source is the largest-degree vertex, smallest id on ties
        b_lab, src = oracle.sample_bfs(C.n, C.offsets, C.nbrs)
        lab, st = G.cc(dg, options=G.Options(sample="bfs"), stats=True)
        assert st["bfs_source"] == src
        assert st["lmax"] == oracle.lmax(b_lab, 1024, 1)
        assert np.array_equal(G.to_u32(lab), want)


def test_no_sampling_hooks_count_is_n_minus_c(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        c = int((want == np.arange(C.n, dtype=np.uint32)).sum())
        for link, find, splice in UF_RULES:
            lab, st = G.cc(dg, options=G.Options(sample="none", link=link, find=find,
                                                 splice=splice), stats=True)
            assert st["hooks"] == C.n - c, (name, link, find)


def test_coo_input(cases):
    from paper_2008_11839_amd import gconn as G
    import torch
    for name, (C, dg, want) in cases.items():
        src, dst = C.coo()
        half = src < dst  # one entry per undirected edge is enough for COO
        for s_, d_ in ((src, dst), (src[half], dst[half])):
            g = G.coo(s_, d_, C.n)
            say(f"[coo] graph={name} m={g.m}")
            for link, find, splice in UF_RULES + [("sv", "split", "split_one"),
                                                  ("lp", "split", "split_one"),
                                                  ("lt", "split", "split_one")]:
                lab = G.cc(g, options=G.Options(link=link, find=find, splice=splice))
                torch.cuda.synchronize()
                assert np.array_equal(G.to_u32(lab), want), (name, link, find)
            fu, fv, lab = G.spanning_forest(g, options=G.Options(link="rem_cas"))
            torch.cuda.synchronize()
            oracle.check_forest(C.n, C.offsets, C.nbrs, G.to_u32(fu), G.to_u32(fv), want)


def test_uint64_offsets(cases):
    from paper_2008_11839_amd import gconn as G
    for name in ("rmat14", "grid2d", "hub_segments"):
        C, _, want = cases[name]
        dg = G.csr(C.offsets, C.nbrs, C.n, offsets64=True)
        for sample in SAMPLERS:
            for link in ("async", "rem_cas", "sv", "lt"):
                assert np.array_equal(_labels(G, dg, sample=sample, link=link), want)


def test_block_shapes(cases):
    from paper_2008_11839_amd import gconn as G
    C, dg, want = cases["rmat14"]
    for block in (64, 128, 512, 1024):
        for sample in SAMPLERS:
            assert np.array_equal(_labels(G, dg, sample=sample, link="rem_cas", block=block), want)


def test_repeated_runs_under_contention(cases):
    from paper_2008_11839_amd import gconn as G
    for name in ("star_center_max", "star_center_0", "clique", "hub_segments", "path_desc"):
        C, dg, want = cases[name]
        say(f"[repeat] graph={name}")
        for rep in range(40):
            for link, find, splice in (("async", "split", "split_one"), ("rem_cas", "split", "split_one"),
                                       ("hooks", "naive", "split_one"), ("early", "halve", "split_one"),
                                       ("rem_cas", "halve", "halve_one")):
                got = _labels(G, dg, sample="none", link=link, find=find, splice=splice,
                              atomic_compress=rep % 2 == 1)
                assert np.array_equal(got, want), (name, rep, link)


def test_validation_rejects_bad_ids():
    from paper_2008_11839_amd import gconn as G
    off = np.array([0, 1, 2], np.uint64)
    nb = np.array([1, 7], np.uint32)  # id 7 >= n = 2
    dg = G.csr(off, nb, 2)
    with pytest.raises(G.GconnError) as e:
        G.cc(dg, options=G.Options(validate=True))
    assert e.value.status == -1
    g = G.coo(np.array([0, 5], np.uint32), np.array([1, 1], np.uint32), 3)
    with pytest.raises(G.GconnError):
        G.cc(g, options=G.Options(validate=True))


def test_host_pointer_is_rejected():
    import torch
    from paper_2008_11839_amd import gconn as G
    C = tg.csr(4, [(0, 1)])
    dg = G.csr(C.offsets, C.nbrs, 4)
    with pytest.raises(ValueError):
        G.cc(dg, labels=torch.empty(4, dtype=torch.int32))  # CPU tensor


def test_incremental_batches_match_oracle_after_every_batch():
    import torch
    from paper_2008_11839_amd import gconn as G
    n = 20000
    src, dst = graphgen.rmat_edges(15, 60000, 21, n=n)
    graphgen.shuffle_edges(src, dst, 21)
    bounds = [0, 1, 10, 1000, 1001, 7000, 20000, 45000, len(src)]
    for i_rule, (link, find, splice) in enumerate(UF_RULES):
        ac = i_rule % 2 == 1  # alternate store / CAS compression writes
        say(f"[inc] link={link} find={find} splice={splice} atomic_compress={ac}")
        inc = G.Incremental(n, options=G.Options(sample="none", link=link, find=find,
                                                 splice=splice, atomic_compress=ac))
        uf = oracle.UnionFind(n)
        for i in range(len(bounds) - 1):
            lo, hi = bounds[i], bounds[i + 1]
            s_t = torch.from_numpy(src[lo:hi].view(np.int32)).cuda()
            d_t = torch.from_numpy(dst[lo:hi].view(np.int32)).cuda()
            inc.insert(s_t, d_t)
            uf.insert(src[lo:hi], dst[lo:hi])
            a, b = graphgen.uniform_pairs(n, 5000, 21, i)
            # include the endpoints of just-inserted edges
            a = np.concatenate([a, src[lo:hi][:500]])
            b = np.concatenate([b, dst[lo:hi][:500]])
            out = inc.query(torch.from_numpy(a.view(np.int32)).cuda(),
                            torch.from_numpy(b.view(np.int32)).cuda())
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), uf.query(a, b)), (link, i)
            assert np.array_equal(G.to_u32(inc.labels()), uf.labels()), (link, i)
        inc.close()


def test_incremental_with_initial_graph():
    import torch
    from paper_2008_11839_amd import gconn as G
    C = graphgen.rmat(13, 8, 6)
    n_max = C.n + 500
    extra_s, extra_d = graphgen.er_edges(n_max, 3000, 6)
    for sample in ("none", "kout"):
        inc = G.Incremental(n_max, initial=G.csr(C.offsets, C.nbrs, C.n),
                            options=G.Options(sample=sample, link="async"))
        uf = oracle.UnionFind(n_max)
        s0, d0 = C.coo()
        uf.insert(s0, d0)
        assert np.array_equal(G.to_u32(inc.labels()), uf.labels())
        inc.insert(torch.from_numpy(extra_s.view(np.int32)).cuda(),
                   torch.from_numpy(extra_d.view(np.int32)).cuda())
        uf.insert(extra_s, extra_d)
        torch.cuda.synchronize()
        assert np.array_equal(G.to_u32(inc.labels()), uf.labels())
        inc.close()


def test_incremental_validation():
    import torch
    from paper_2008_11839_amd import gconn as G
    inc = G.Incremental(10, options=G.Options(sample="none", validate=True))
    with pytest.raises(G.GconnError):
        inc.insert(torch.tensor([1, 12], dtype=torch.int32, device="cuda"),
                   torch.tensor([2, 3], dtype=torch.int32, device="cuda"))
    inc.insert(torch.tensor([1, 4], dtype=torch.int32, device="cuda"),
               torch.tensor([2, 3], dtype=torch.int32, device="cuda"))
    out = inc.query(torch.tensor([1, 1], dtype=torch.int32, device="cuda"),
                    torch.tensor([2, 3], dtype=torch.int32, device="cuda"))
    assert out.cpu().tolist() == [1, 0]


def test_kout_rem_cas_schedules_agree(cases):
    """The lane-refill step machine and the one-lane-per-vertex loop give the
    oracle's labels, a valid forest and the oracle's sampled-edge count."""
    import torch
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        roots_mask = want != np.arange(C.n, dtype=np.uint32)
        for k in (1, 2, 3):
            _, e_s = oracle.sample_kout(C.n, C.offsets, C.nbrs, k)
            for find in ("naive", "split", "halve"):
                for splice in ("split_one", "halve_one"):
                    for sched in ("auto", "lane", "step", "pipe", "twopass", "flat", "xcd"):
                        say(f"[sched] graph={name} k={k} find={find} splice={splice} sched={sched}")
                        o = G.Options(sample="kout", link="rem_cas", find=find, splice=splice,
                                      k=k, schedule=sched)
                        lab, st = G.cc(dg, options=o, stats=True)
                        assert np.array_equal(G.to_u32(lab), want), (name, k, find, splice, sched)
                        if C.m:
                            assert st["sampled_edges"] == e_s
                        fu, fv, _ = G.spanning_forest(dg, want_labels=False, options=o)
                        torch.cuda.synchronize()
                        fu, fv = G.to_u32(fu), G.to_u32(fv)
                        oracle.check_forest(C.n, C.offsets, C.nbrs, fu, fv, want)
                        assert np.array_equal(fu != G.EMPTY, roots_mask)


def test_hooks_count_is_n_minus_c_with_sampling(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        c = int((want == np.arange(C.n, dtype=np.uint32)).sum())
        for sched in ("auto", "lane", "step", "pipe", "twopass", "flat", "xcd"):
            lab, st = G.cc(dg, options=G.Options(sample="kout", link="rem_cas", schedule=sched),
                           stats=True)
            assert st["hooks"] == C.n - c, (name, sched)


def test_random_kout_and_larger_k(cases):
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        for k in (1, 2, 3, 5):
            for random in (False, True):
                for link in ("async", "rem_cas", "early"):
                    for sched in ("auto", "lane"):
                        got = _labels(G, dg, sample="kout", k=k, kout_random=random, link=link,
                                      schedule=sched, seed=7)
                        assert np.array_equal(got, want), (name, k, random, link, sched)


def test_kout_local(cases):
    """k-out with the LDS local-first pass: labels, sampled-edge count, L_max,
    active set and hook count equal the oracle's; the spanning forest is valid
    and fills exactly the non-minimum slots (local links record their edge)."""
    import torch
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        c = int((want == np.arange(C.n, dtype=np.uint32)).sum())
        roots_mask = want != np.arange(C.n, dtype=np.uint32)
        for k in (1, 2):
            s_lab, e = oracle.sample_kout(C.n, C.offsets, C.nbrs, k)
            L = oracle.lmax(s_lab, 1024, 1)
            for link, find, splice in UF_RULES:
                say(f"[local] graph={name} k={k} link={link} find={find} splice={splice}")
                o = G.Options(sample="kout", link=link, find=find, splice=splice, k=k,
                              kout_local=True)
                lab, st = G.cc(dg, options=o, stats=True)
                assert np.array_equal(G.to_u32(lab), want), (name, k, link, find, splice)
                if C.m:
                    assert st["sampled_edges"] == e
                    assert st["lmax"] == L
                    assert st["active_vertices"] == oracle.active_count(C.n, C.offsets, s_lab, L)
                if link != "ecl":
                    assert st["hooks"] == C.n - c, (name, k, link)
                if link != "ecl" and splice != "splice_atomic":
                    fu, fv, _ = G.spanning_forest(dg, want_labels=False, options=o)
                    torch.cuda.synchronize()
                    fu, fv = G.to_u32(fu), G.to_u32(fv)
                    oracle.check_forest(C.n, C.offsets, C.nbrs, fu, fv, want)
                    assert np.array_equal(fu != G.EMPTY, roots_mask), (name, k, link)


def test_kout_prelink(cases):
    """k-out with the contention-free pre-link pass: labels, sampled-edge count,
    L_max, active set and hook count equal the oracle's; the spanning forest is
    valid and fills exactly the non-minimum slots; k = 3 and random picks fall
    back to one union per sampled edge."""
    import torch
    from paper_2008_11839_amd import gconn as G
    for name, (C, dg, want) in cases.items():
        c = int((want == np.arange(C.n, dtype=np.uint32)).sum())
        roots_mask = want != np.arange(C.n, dtype=np.uint32)
        for k in (1, 2):
            s_lab, e = oracle.sample_kout(C.n, C.offsets, C.nbrs, k)
            L = oracle.lmax(s_lab, 1024, 1)
            for link, find, splice in UF_RULES + [("sv", "split", "split_one")]:
                for ac in (False, True):
                    say(f"[prelink] graph={name} k={k} link={link} find={find} splice={splice} ac={ac}")
                    o = G.Options(sample="kout", link=link, find=find, splice=splice, k=k,
                                  atomic_compress=ac, kout_prelink=True)
                    lab, st = G.cc(dg, options=o, stats=True)
                    assert np.array_equal(G.to_u32(lab), want), (name, k, link, find, splice, ac)
                    if C.m:
                        assert st["sampled_edges"] == e
                        assert st["lmax"] == L
                        assert st["active_vertices"] == oracle.active_count(C.n, C.offsets, s_lab, L)
                    if link not in ("sv", "ecl"):
                        assert st["hooks"] == C.n - c, (name, k, link)
                    if link not in ("sv", "ecl") and splice != "splice_atomic":
                        fu, fv, _ = G.spanning_forest(dg, want_labels=False, options=o)
                        torch.cuda.synchronize()
                        fu, fv = G.to_u32(fu), G.to_u32(fv)
                        oracle.check_forest(C.n, C.offsets, C.nbrs, fu, fv, want)
                        assert np.array_equal(fu != G.EMPTY, roots_mask), (name, k, link)
        for k, random in ((3, False), (2, True)):
            got = _labels(G, dg, sample="kout", k=k, kout_random=random, kout_prelink=True)
            assert np.array_equal(got, want), (name, k, random)


@pytest.mark.parametrize("ratio", [1.0, 0.25, 8.0])
def test_incremental_mixed_batches_match_oracle(ratio):
    """Mixed insert/query batches (inserts of a batch first, then its queries):
    every answer equals the oracle's after every batch, for every root-based
    union rule, on an RMAT edge stream and on a Barabasi-Albert stream."""
    import torch
    from paper_2008_11839_amd import gconn as G
    n = 20000
    streams = {"rmat": graphgen.rmat_edges(15, 40000, 31, n=n),
               "ba": graphgen.ba_edges(n, 3, 32)}
    for sname, (src, dst) in streams.items():
        if sname == "rmat":
            graphgen.shuffle_edges(src, dst, 31)
        kind, a, b = graphgen.mixed_stream(src, dst, n, ratio, 33)
        bounds = [0, 1, 17, 5000, 5001, 30000, len(kind)]
        rules = UF_RULES if ratio == 1.0 else UF_RULES[::4]
        for link, find, splice in rules:
            say(f"[mixed] stream={sname} ratio={ratio} link={link} find={find} splice={splice}")
            inc = G.Incremental(n, options=G.Options(sample="none", link=link, find=find,
                                                     splice=splice))
            uf = oracle.UnionFind(n)
            for i in range(len(bounds) - 1):
                lo, hi = bounds[i], bounds[i + 1]
                kk, aa, bb = kind[lo:hi], a[lo:hi], b[lo:hi]
                ins = kk == 0
                uf.insert(aa[ins], bb[ins])
                want = np.zeros(hi - lo, np.uint8)
                want[~ins] = uf.query(aa[~ins], bb[~ins])
                out = inc.mixed(torch.from_numpy(kk).cuda(),
                                torch.from_numpy(aa.view(np.int32)).cuda(),
                                torch.from_numpy(bb.view(np.int32)).cuda())
                got = out.cpu().numpy()
                assert np.array_equal(got, want), (sname, ratio, link, find, splice, i)
            inc.close()


def test_incremental_mixed_validation():
    import torch
    from paper_2008_11839_amd import gconn as G
    inc = G.Incremental(10, options=G.Options(sample="none", validate=True))
    k = torch.tensor([0, 2], dtype=torch.uint8, device="cuda")
    a = torch.tensor([1, 2], dtype=torch.int32, device="cuda")
    with pytest.raises(G.GconnError):
        inc.mixed(k, a, a)
    with pytest.raises(G.GconnError):
        inc.mixed(torch.tensor([0, 1], dtype=torch.uint8, device="cuda"), a,
                  torch.tensor([1, 12], dtype=torch.int32, device="cuda"))
    out = inc.mixed(torch.tensor([0, 1, 1], dtype=torch.uint8, device="cuda"),
                    torch.tensor([1, 1, 3], dtype=torch.int32, device="cuda"),
                    torch.tensor([2, 2, 4], dtype=torch.int32, device="cuda"))
    assert out.cpu().tolist() == [0, 1, 0]
    inc.close()
