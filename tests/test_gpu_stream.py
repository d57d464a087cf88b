"""Parity of the incremental serving workload at its full size (RMAT-26,
edge factor 16, both directions: 2.15e9 updates in insert batches of
1e4..1e7 with query batches of 1e5 pairs between them), against the record
the oracle wrote of the same stream (tests/golden/make_golden.py): every
query batch's answers, in order, and the final canonical labels."""
from __future__ import annotations

import hashlib
import json
import os
import sys

import numpy as np
import pytest

import graphgen

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "stream_rmat26_ef16_s1.json")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def sha16(x) -> str:
    return hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest()[:16]


@pytest.mark.timeout(600)
def test_stream_answers_and_labels_match_oracle_record(gpu_available):
    import torch
    from paper_2008_11839_amd import gconn as G
    with open(GOLDEN) as f:
        gold = json.load(f)
    say("[stream] generating the RMAT-26 update stream")
    n, src, dst, reqs = graphgen.update_stream(26, 16, 1)
    assert n == gold["n"] and len(src) == gold["stream_edges"] and len(reqs) == gold["requests"]
    dev = torch.device("cuda", 0)
    s_d = torch.from_numpy(src.view(np.int32)).to(dev)
    d_d = torch.from_numpy(dst.view(np.int32)).to(dev)
    del src, dst
    queries = [(a, b) for k, a, b in reqs if k == 1]
    qlen = [len(a) for a, _ in queries]
    qoff = np.concatenate([[0], np.cumsum(qlen)]).astype(np.int64)
    qa = torch.from_numpy(np.concatenate([a for a, _ in queries]).view(np.int32)).to(dev)
    qb = torch.from_numpy(np.concatenate([b for _, b in queries]).view(np.int32)).to(dev)
    out = torch.empty(int(qoff[-1]), dtype=torch.uint8, device=dev)
    for rule in (dict(link="async", find="split"),
                 dict(link="rem_cas", find="split", splice="splice_atomic")):
        say(f"[stream] replay {rule}")
        inc = G.Incremental(n, options=G.Options(sample="none", **rule))
        qi = 0
        for k, x, y in reqs:
            if k == 0:
                a, b = graphgen.insert_slices(s_d, d_d, x, y)
                inc.insert(a, b)
            else:
                lo, hi = int(qoff[qi]), int(qoff[qi + 1])
                inc.query(qa[lo:hi], qb[lo:hi], out=out[lo:hi])
                qi += 1
        ans = out.cpu().numpy()
        got = [sha16(ans[qoff[i]:qoff[i + 1]]) for i in range(len(qlen))]
        bad = [i for i, (g, w) in enumerate(zip(got, gold["query_answers_sha16"])) if g != w]
        assert not bad, f"{rule}: query batches {bad[:10]} differ from the oracle's answers"
        assert int(ans.sum()) == gold["connected_answers"]
        lab = G.to_u32(inc.labels())
        inc.close()
        assert int((lab == np.arange(n, dtype=np.uint32)).sum()) == gold["components"], rule
        assert hashlib.sha256(np.ascontiguousarray(lab, dtype="<u4").tobytes()).hexdigest() \
            == gold["labels_sha256"], rule
        del lab
