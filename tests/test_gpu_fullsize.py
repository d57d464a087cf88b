"""Parity at the workloads' full sizes, against records the oracle wrote
(tests/golden, make_golden.py): the SHA-256 of all labels, the component
count, and the sampling intermediates (sampled entries, L_max, active
vertices and their entries) of k-out and hook-based sampling -- for the
benchmark configuration and its neighbours on RMAT-24, and for the ER and
percolation-grid workloads."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
WORK = {"rmat24_ef16_s1": lambda: graphgen.rmat(24, 16, 1),
        "er_n100000_m1000000_s1": lambda: graphgen.er(100_000, 1_000_000, 1),
        "grid2d_4096_p07_s1": lambda: graphgen.grid2d(4096, 4096, 0.7, 1),
        "grid3d_256_p06_s1": lambda: graphgen.grid3d(256, 256, 256, 0.6, 1)}
CONFIGS = [dict(sample="kout", link="rem_cas", find="split", splice="splice_atomic"),  # benchmark
           dict(sample="kout", link="rem_cas", find="split", splice="split_one"),  # its forest
           dict(sample="kout", link="rem_cas", find="split", splice="split_one", schedule="xcd"),
           dict(sample="kout", link="rem_cas", find="split", splice="splice_atomic",
                schedule="xcd"),
           dict(sample="kout", link="rem_cas", find="split", splice="split_one", schedule="flat"),
           dict(sample="kout", link="rem_cas", find="halve", kout_prelink=True),
           dict(sample="kout", link="rem_cas", find="split", kout_local=True),
           dict(sample="kout", link="rem_cas", find="split", schedule="twopass"),
           dict(sample="kout", link="async", find="split"),
           dict(sample="hb", link="async", find="split"),
           dict(sample="none", link="rem_cas", find="split"),
           dict(sample="kout", link="sv"),
           dict(sample="kout", link="lt", lt_variant="PRF"),
           dict(sample="kout", link="jtb", find="two_try_split"),
           dict(sample="kout", link="afforest"),
           dict(sample="kout", link="hooks", find="split")]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sha(x) -> str:
    return hashlib.sha256(np.ascontiguousarray(x, dtype="<u4").tobytes()).hexdigest()


@pytest.mark.parametrize("name", list(WORK))
def test_full_size_labels_and_sampling_match_golden(gpu_available, name):
    import torch
    from paper_2008_11839_amd import gconn as G
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        gold = json.load(f)
    C = WORK[name]()
    assert (C.n, C.m) == (gold["n"], gold["m"])
    dg = G.csr(C.offsets, C.nbrs, C.n)
    lab = torch.empty(C.n, dtype=torch.int32, device="cuda")
    for cfg in CONFIGS:
        say(f"[full] {name} {cfg}")
        o = G.Options(**cfg)
        ws = G.alloc_workspace(G.workspace_size(dg, o))
        _, st = G.cc(dg, labels=lab, options=o, workspace=ws, stats=True)
        got = G.to_u32(lab)
        assert sha(got) == gold["labels_sha256"], (name, cfg)
        assert int((got == np.arange(C.n, dtype=np.uint32)).sum()) == gold["components"]
        if cfg["sample"] in ("kout", "hb") and cfg["link"] not in ("sv", "lt"):
            g = gold[cfg["sample"]]
            assert st["sampled_edges"] == g["sampled_edges"], (name, cfg)
            if cfg["link"] != "jtb":  # JTB's L_max is its tree's root, not the minimum
                assert st["lmax"] == g["lmax"], (name, cfg)
            assert st["active_vertices"] == g["active_vertices"], (name, cfg)
            assert st["finish_edges"] == g["active_edges"], (name, cfg)
        del ws
