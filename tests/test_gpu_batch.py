"""GPU parity of the many-graph batch (gconn_cc_batch) and the autotuner:
every graph's local labels equal the oracle's, whatever class options it runs
with, and the per-class choices the autotuner makes give the same labels."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import graphgen
import oracle
from tests import graphs as tg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _graphs():
    gs = [tg.csr(1, []), tg.csr(64, tg.path(64)), tg.csr(65, tg.cycle(65)), tg.csr(200, []),
          tg.csr(2000, tg.star(2000, 1999))]
    specs = graphgen.batched_specs(60, 5, n_lo=100, n_hi=20000, ef_lo=2, ef_hi=24)
    for kind, n, ef, seed in specs:
        gs.append(graphgen.batched_graph(kind, n, ef, seed))
    gs.append(graphgen.grid2d(90, 70, 0.55, 3))
    return gs


CLASS_SETS = [
    [dict(sample="kout", link="rem_cas", find="split", splice="split_one", k=2)],
    [dict(sample="none", link="async", find="split"),
     dict(sample="kout", link="async", find="halve", k=2),
     dict(sample="kout", link="rem_cas", find="halve", splice="halve_one", k=3),
     dict(sample="kout", link="early", find="naive", k=1),
     dict(sample="none", link="rem_cas", find="naive", splice="split_one")],
    [dict(sample="kout", link="rem_cas", find="split", splice="splice_atomic", k=2),
     dict(sample="none", link="rem_cas", find="halve", splice="splice_atomic"),
     dict(sample="kout", link="rem_cas", find="naive", splice="splice_atomic", k=3)],
    [dict(sample="hb", link="rem_cas", find="split", splice="split_one", hb_n=4),
     dict(sample="hb", link="async", find="halve", hb_n=2),
     dict(sample="kout", link="rem_cas", find="split", splice="split_one", k=2),
     dict(sample="none", link="early", find="split")],
]


@pytest.fixture(scope="module")
def batch_case(gpu_available):
    gs = _graphs()
    want = [oracle.cc(g.n, g.offsets, g.nbrs) for g in gs]
    return gs, want


def _check(hb, gs, want, labels):
    lab = labels.cpu().numpy().view(np.uint32)
    for i, g in enumerate(gs):
        lo = int(hb.vbase[i])
        assert np.array_equal(lab[lo:lo + g.n], want[i]), f"graph {i} (n={g.n})"
        pad = lab[lo + g.n:int(hb.vbase[i + 1])]
        assert np.array_equal(pad, np.arange(g.n, g.n + len(pad), dtype=np.uint32))


def test_batch_labels_match_oracle_per_graph(batch_case):
    import torch
    from paper_2008_11839_amd import batch as B
    gs, want = batch_case
    hb = B.concat(gs)
    rng = np.random.default_rng(3)
    for ci, classes in enumerate(CLASS_SETS):
        gclass = rng.integers(0, len(classes), size=len(gs))
        db = B.upload(hb, graph_class=gclass if len(classes) > 1 else None,
                      block=(0, 512, 128)[ci % 3])
        say(f"[batch] graphs={len(gs)} n={hb.n} m={hb.m} class_set={ci}")
        for rep in range(3):
            lab, st = B.cc_batch(db, classes, stats=True)
            torch.cuda.synchronize()
            _check(hb, gs, want, lab)
            c_total = sum(int((w == np.arange(len(w), dtype=np.uint32)).sum()) for w in want)
            assert st["hooks"] == sum(g.n for g in gs) - c_total


@pytest.mark.parametrize("hb_n", [1, 4])
def test_batch_hook_based_sampled_count(batch_case, hb_n):
    """A batch whose graphs all sample hook-based: per-graph labels equal the
    oracle's, and the sampled entries add up to the oracle's count of the
    same sampler over every graph."""
    import torch
    from paper_2008_11839_amd import batch as B
    gs, want = batch_case
    hb = B.concat(gs)
    db = B.upload(hb)
    lab, st = B.cc_batch(db, [dict(sample="hb", link="rem_cas", find="split", hb_n=hb_n)],
                         stats=True)
    torch.cuda.synchronize()
    _check(hb, gs, want, lab)
    assert st["sampled_edges"] == sum(oracle.sample_hb(g.n, g.offsets, g.nbrs, hb_n)[1]
                                      for g in gs)


def test_batch_single_graph_equals_gconn_cc(batch_case):
    import torch
    from paper_2008_11839_amd import batch as B
    from paper_2008_11839_amd import gconn as G
    C = graphgen.rmat(14, 16, 9)
    want = oracle.cc(C.n, C.offsets, C.nbrs)
    hb = B.concat([C])
    db = B.upload(hb)
    lab = B.cc_batch(db, [dict(sample="kout", link="rem_cas", find="split")])
    single = G.cc(G.csr(C.offsets, C.nbrs, C.n))
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy().view(np.uint32)[:C.n], want)
    assert np.array_equal(G.to_u32(single), want)


def test_autotuner_choices_give_oracle_labels(batch_case, tmp_path):
    import torch
    from paper_2008_11839_amd import batch as B
    gs, want = batch_case
    tuner = B.Autotuner(str(tmp_path / "table.json"), reps=1, per_class=2)
    keys = tuner.tune(gs)
    assert len(keys) == len(gs) and len(tuner.table) >= 2
    for k, rec in tuner.table.items():
        choice = dict(rec["choice"])
        assert choice.pop("block") in B.BLOCKS and choice in B.CANDIDATES
        assert len(rec["times_ms"]) == len(B.CANDIDATES)
        assert len(rec["block_times_ms"]) == len(B.BLOCKS)
    classes, gclass = tuner.classes_for(keys)
    hb = B.concat(gs)
    db = B.upload(hb, graph_class=gclass, block=tuner.batch_block(keys, gs))
    lab = B.cc_batch(db, classes)
    torch.cuda.synchronize()
    _check(hb, gs, want, lab)
    # the launch shape timed on the whole batch: every shape tried, the
    # fastest kept, labels unchanged
    import ctypes
    from paper_2008_11839_amd import gconn as G
    bb = ctypes.c_size_t()
    G._check(G.lib().gconn_cc_batch_workspace_size(ctypes.byref(db.c), ctypes.byref(bb)))
    ws = G.alloc_workspace(bb.value)
    block, times = B.Autotuner.tune_batch_block(db, classes, lab, ws, reps=1)
    assert sorted(times) == sorted(B.BLOCKS) and block == min(times, key=times.get)
    assert int(db.c.block) == block
    lab = B.cc_batch(db, classes, workspace=ws)
    torch.cuda.synchronize()
    _check(hb, gs, want, lab)
    # the cached table is reused without re-timing
    again = B.Autotuner(str(tmp_path / "table.json"))
    assert again.table.keys() == tuner.table.keys()


def test_batch_rejects_bad_layouts(batch_case):
    import ctypes
    from paper_2008_11839_amd import batch as B
    from paper_2008_11839_amd import gconn as G
    gs, _ = batch_case
    db = B.upload(B.concat(gs[:3]))
    db.c.n = db.c.n - 1  # not a multiple of 64
    with pytest.raises(G.GconnError):
        B.cc_batch(db, [dict()])
    db = B.upload(B.concat(gs[:3]), block=96)  # not a multiple of 64
    with pytest.raises(G.GconnError):
        B.cc_batch(db, [dict()])
    db = B.upload(B.concat(gs[:3]))
    with pytest.raises(G.GconnError):
        B.cc_batch(db, [dict(sample="bfs")])
    with pytest.raises(G.GconnError):
        B.cc_batch(db, [dict(link="sv")])
