"""Captured pipelines (gconn_cc_capture, gconn_cc_batch_capture): every
replay, with eager work and synchronisations between replays, equals the
oracle; a replay reads the input buffers' current contents; pipelines with a
host round trip are refused."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs as tg

pytestmark = pytest.mark.gpu

RULES = [dict(sample="kout", link="rem_cas", find="split", splice="splice_atomic"),
         dict(sample="kout", link="rem_cas", find="split", splice="split_one"),
         dict(sample="kout", link="async", find="halve"),
         dict(sample="kout", link="rem_cas", find="halve", kout_prelink=True),
         dict(sample="hb", link="early", find="split"),
         dict(sample="none", link="hooks", find="naive"),
         dict(sample="none", link="rem_lock", find="split"),
         dict(sample="kout", link="afforest"),
         dict(sample="kout", link="ecl")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _graphs():
    return {"rmat14": graphgen.rmat(14, 16, 3), "er": graphgen.er(20000, 60000, 4),
            "grid2d": graphgen.grid2d(150, 120, 0.6, 5),
            "star": tg.csr(3000, tg.star(3000, 2999))}


def test_captured_cc_replays_match_oracle(gpu_available):
    import torch
    from paper_2008_11839_amd import gconn as G
    other = graphgen.rmat(12, 8, 9)
    d_other = G.csr(other.offsets, other.nbrs, other.n)
    want_other = oracle.cc(other.n, other.offsets, other.nbrs)
    for name, C in _graphs().items():
        want = oracle.cc(C.n, C.offsets, C.nbrs)
        dg = G.csr(C.offsets, C.nbrs, C.n)
        for cfg in RULES:
            say(f"[capture] graph={name} {cfg}")
            o = G.Options(**cfg)
            lab = torch.empty(C.n, dtype=torch.int32, device="cuda")
            ex = G.capture_cc(dg, lab, options=o)
            for rep in range(4):
                lab.fill_(-1)                      # eager work between replays
                ex.launch()
                got_o = G.cc(d_other, options=o)   # an eager run on the same stream
                torch.cuda.synchronize()
                assert np.array_equal(G.to_u32(lab), want), (name, cfg, rep)
                assert np.array_equal(G.to_u32(got_o), want_other), (name, cfg, rep)
            ex.close()


def test_replay_reads_current_inputs(gpu_available):
    """Two relabellings of one graph (same n and m): after copying the second
    one's CSR into the captured buffers, a replay returns its labels."""
    import torch
    from paper_2008_11839_amd import gconn as G
    base = graphgen.rmat(12, 8, 11)
    src, dst = base.coo()
    pairs = list(zip(src.tolist(), dst.tolist()))
    A = tg.csr(base.n, tg.relabel(base.n, pairs, 1)[0])
    B = tg.csr(base.n, tg.relabel(base.n, pairs, 2)[0])
    assert A.m == B.m
    da, db = G.csr(A.offsets, A.nbrs, A.n), G.csr(B.offsets, B.nbrs, B.n)
    cap = G.csr(A.offsets, A.nbrs, A.n)  # the buffers the captured run reads
    lab = torch.empty(A.n, dtype=torch.int32, device="cuda")
    ex = G.capture_cc(cap, lab, options=G.Options(sample="kout", link="rem_cas"))
    for rep, (C, src_dev) in enumerate([(A, da), (B, db), (A, da), (B, db)]):
        cap.offsets.copy_(src_dev.offsets)
        cap.nbrs.copy_(src_dev.nbrs)
        ex.launch()
        torch.cuda.synchronize()
        assert np.array_equal(G.to_u32(lab), oracle.cc(C.n, C.offsets, C.nbrs)), rep
    ex.close()


def test_capture_refuses_host_round_trips(gpu_available):
    import torch
    from paper_2008_11839_amd import gconn as G
    C = graphgen.rmat(10, 8, 1)
    dg = G.csr(C.offsets, C.nbrs, C.n)
    lab = torch.empty(C.n, dtype=torch.int32, device="cuda")
    for cfg in (dict(link="sv"), dict(link="lt"), dict(link="lp"), dict(sample="bfs"),
                dict(validate=True)):
        with pytest.raises(G.GconnError) as e:
            G.capture_cc(dg, lab, options=G.Options(**cfg))
        assert e.value.status == -7, cfg
    G.profile_enable(True)
    try:
        with pytest.raises(G.GconnError):
            G.capture_cc(dg, lab, options=G.Options())
    finally:
        G.profile_enable(False)


def test_captured_batch_replays_match_eager(gpu_available):
    import torch
    from paper_2008_11839_amd import batch as B
    specs = graphgen.batched_specs(40, 7, n_lo=100, n_hi=30000, ef_lo=2, ef_hi=20)
    gs = [graphgen.batched_graph(*sp) for sp in specs]
    want = [oracle.cc(g.n, g.offsets, g.nbrs) for g in gs]
    hb = B.concat(gs)
    rng = np.random.default_rng(2)
    classes = [dict(sample="kout", link="rem_cas", find="split"),
               dict(sample="none", link="async", find="halve")]
    db = B.upload(hb, graph_class=rng.integers(0, 2, size=len(gs)))
    lab = torch.empty(hb.n, dtype=torch.int32, device="cuda")
    ex = B.capture_batch(db, classes, lab)
    for rep in range(4):
        lab.fill_(-1)
        ex.launch()
        eager = B.cc_batch(db, classes)
        torch.cuda.synchronize()
        got = lab.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, eager.cpu().numpy().view(np.uint32)), rep
        for i, g in enumerate(gs):
            lo = int(hb.vbase[i])
            assert np.array_equal(got[lo:lo + g.n], want[i]), (rep, i)
    ex.close()
