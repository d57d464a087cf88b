"""gconn_cc_noalloc (the entry point that allocates nothing) against gconn_cc
with a caller workspace: identical labels, element by element, on two calls
in a row -- the second on a smaller graph, so it runs on scratch memory that
still holds the first call's state -- and the documented size limit."""
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


CONFIGS = [
    dict(sample="kout", link="rem_cas", find="split", splice="splice_atomic"),
    dict(sample="kout", link="rem_cas", find="split", splice="split_one", schedule="flat"),
    dict(sample="hb", link="async", find="halve"),
    dict(sample="none", link="rem_cas", find="split", splice="split_one"),
]


@pytest.mark.parametrize("cfg", CONFIGS, ids=lambda c: "-".join(str(v) for v in c.values()))
def test_noalloc_matches_workspace_entry_point(gpu_available, cfg):
    import torch
    from paper_2008_11839_amd import gconn as G
    torch.cuda.set_device(0)
    big = graphgen.rmat(18, 16, 11)          # n = 262,144
    small = graphgen.er(5000, 12000, 12)     # second call: smaller input
    opts = G.Options(**cfg)
    for name, C in (("rmat18", big), ("er5000", small)):
        say(f"[noalloc] {cfg} on {name} n={C.n} m={C.m}")
        dg = G.csr(C.offsets, C.nbrs, C.n)
        want_dev = G.cc(dg, options=opts)
        got = torch.full((C.n,), -1, dtype=torch.int32, device="cuda")
        G.cc_noalloc(dg, got, options=opts)
        torch.cuda.synchronize()
        want = G.to_u32(want_dev)
        assert np.array_equal(G.to_u32(got), want), f"{name}: labels differ from gconn_cc"
        assert np.array_equal(want, oracle.cc(C.n, C.offsets, C.nbrs)), name


def test_noalloc_coo_and_stats(gpu_available):
    import torch
    from paper_2008_11839_amd import gconn as G
    torch.cuda.set_device(0)
    n = 40000
    src, dst = graphgen.er_edges(n, 90000, 13)
    dg = G.coo(src, dst, n)
    opts = G.Options(sample="none", link="async", find="split")
    got = torch.empty(n, dtype=torch.int32, device="cuda")
    lab, st = G.cc_noalloc(dg, got, options=opts, stats=True)
    want, st2 = G.cc(dg, options=opts, stats=True)
    torch.cuda.synchronize()
    assert np.array_equal(G.to_u32(lab), G.to_u32(want))
    assert st["active_vertices"] == st2["active_vertices"]


def test_noalloc_rejects_graphs_beyond_its_scratch(gpu_available):
    import torch
    from paper_2008_11839_amd import gconn as G
    torch.cuda.set_device(0)
    n = 12_000_000                           # default k-out pipeline: > 64 MiB of scratch
    off = torch.zeros(n + 1, dtype=torch.int32, device="cuda")
    off[-1] = 1                              # vertex n-1 has the one edge (n-1, 0)
    nbrs = torch.zeros(1, dtype=torch.int32, device="cuda")
    dg = G.csr(off, nbrs, n)
    need = G.workspace_size(dg, G.Options())
    assert need > G.NOALLOC_SCRATCH_BYTES
    labels = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    with pytest.raises(G.GconnError) as e:
        G.cc_noalloc(dg, labels, options=G.Options())
    assert e.value.status == -2  # GCONN_ENOMEM
    torch.cuda.synchronize()
    assert int((labels != -7).sum()) == 0    # nothing ran
