"""Write tests/golden/<config>.json from the CPU oracle alone.

Each static record pins, for one seeded full-size workload: its size, the
number of components, the largest component, a SHA-256 of the canonical
labels (uint32 little-endian), and the sampling-phase intermediates (L_max
over the default seeded sample of 1024 vertices with seed 1, active vertices
and active edges) for k-out (k = 2) and hook-based (N = 4) sampling.

Two more records cover the other full-size workloads:
  * stream_rmat26_ef16_s1: the incremental serving stream (graphgen's
    update_stream at scale 26), replayed through the oracle's sequential
    union-find: the first 16 hex digits of the SHA-256 of every query batch's
    answers (uint8, 1 = connected) in request order, the number of connected
    answers, and the final canonical labels' SHA-256 and component count.
  * batch2000_s1: the 2,000-graph batch (graphgen's batched_specs), each graph
    through the oracle: its size, component count and the first 16 hex digits
    of its labels' SHA-256.

Only `graphgen` (inputs) and `oracle` are used.

    python tests/golden/make_golden.py [config ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

CONFIGS = {
    "er_n100000_m1000000_s1": lambda: graphgen.er(100_000, 1_000_000, 1),
    "rmat24_ef16_s1": lambda: graphgen.rmat(24, 16, 1),
    # the other seeds of the headline graph (the benchmark reports the spread)
    **{f"rmat24_ef16_s{s}": (lambda s=s: graphgen.rmat(24, 16, s)) for s in (2, 3, 4, 5)},
    "grid2d_4096_p07_s1": lambda: graphgen.grid2d(4096, 4096, 0.7, 1),
    "grid3d_256_p06_s1": lambda: graphgen.grid3d(256, 256, 256, 0.6, 1),
    # the Barabasi-Albert stream of the mixed-batch measurement, as a graph
    "ba22_k10_s1": lambda: graphgen.csr_from_edges(1 << 22, *graphgen.ba_edges(1 << 22, 10, 1),
                                                   True, "ba22_k10_s1"),
}
LMAX_SAMPLES, LMAX_SEED = 1024, 1
STREAMS = {"stream_rmat26_ef16_s1": (26, 16, 1)}
BATCHES = {"batch2000_s1": (2000, 1, 1e3, 1e6)}


def sha(labels: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(labels, dtype="<u4").tobytes()).hexdigest()


def record(name: str) -> dict:
    t0 = time.time()
    G = CONFIGS[name]()
    t1 = time.time()
    lab = oracle.cc(G.n, G.offsets, G.nbrs)
    t2 = time.time()
    roots = lab == np.arange(G.n, dtype=np.uint32)
    sizes = np.bincount(lab.astype(np.int64), minlength=G.n)
    rec = {
        "config": name, "n": G.n, "m": G.m,
        "components": int(roots.sum()), "largest_component": int(sizes.max()),
        "labels_sha256": sha(lab),
        "isolated": int((G.degrees() == 0).sum()),
        "oracle_cc_seconds": round(t2 - t1, 2), "generate_seconds": round(t1 - t0, 2),
    }
    for sampler in ("kout", "hb"):
        if sampler == "kout":
            s_lab, e = oracle.sample_kout(G.n, G.offsets, G.nbrs, 2)
        else:
            s_lab, e = oracle.sample_hb(G.n, G.offsets, G.nbrs, 4)
        L = oracle.lmax(s_lab, LMAX_SAMPLES, LMAX_SEED)
        rec[sampler] = {"sampled_edges": e, "lmax": L,
                        "active_vertices": oracle.active_count(G.n, G.offsets, s_lab, L),
                        "active_edges": oracle.active_edges(G.n, G.offsets, s_lab, L),
                        "sampled_labels_sha256": sha(s_lab)}
    return rec


def sha16(x: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(x).tobytes()).hexdigest()[:16]


def stream_record(name: str) -> dict:
    scale, ef, seed = STREAMS[name]
    t0 = time.time()
    n, src, dst, reqs = graphgen.update_stream(scale, ef, seed)
    t1 = time.time()
    uf = oracle.UnionFind(n)
    qh, ones, updates = [], 0, 0
    for kind, x, y in reqs:
        if kind == 0:
            a, b = graphgen.insert_slices(src, dst, x, y)
            uf.insert(a, b)
            updates += y - x
        else:
            ans = uf.query(x, y)
            ones += int(ans.sum())
            qh.append(sha16(ans.astype(np.uint8)))
    lab = uf.labels()
    t2 = time.time()
    return {"config": name, "n": n, "stream_edges": len(src), "updates": updates,
            "requests": len(reqs), "insert_batches": len(reqs) - len(qh),
            "query_batches": len(qh), "connected_answers": ones,
            "components": int((lab == np.arange(n, dtype=np.uint32)).sum()),
            "labels_sha256": sha(lab), "query_answers_sha16": qh,
            "oracle_seconds": round(t2 - t1, 2), "generate_seconds": round(t1 - t0, 2)}


def batch_record(name: str) -> dict:
    from concurrent.futures import ThreadPoolExecutor
    count, seed, n_lo, n_hi = BATCHES[name]
    specs = graphgen.batched_specs(count, seed, n_lo=n_lo, n_hi=n_hi)

    def one(sp):
        g = graphgen.batched_graph(*sp)
        lab = oracle.cc(g.n, g.offsets, g.nbrs)
        return [g.n, g.m, int((lab == np.arange(g.n, dtype=np.uint32)).sum()), sha16(lab)]

    t0 = time.time()
    with ThreadPoolExecutor(max_workers=8) as ex:  # generator and oracle release the GIL
        graphs = list(ex.map(one, specs))
    return {"config": name, "graphs": count, "n_range": [n_lo, n_hi],
            "n": sum(g[0] for g in graphs), "m": sum(g[1] for g in graphs),
            "per_graph": graphs, "seconds": round(time.time() - t0, 2)}


def main(names):
    out_dir = os.path.dirname(os.path.abspath(__file__))
    for name in names:
        if name in STREAMS:
            rec = stream_record(name)
        elif name in BATCHES:
            rec = batch_record(name)
        else:
            rec = record(name)
        with open(os.path.join(out_dir, name + ".json"), "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
        print(json.dumps(rec)[:2000], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CONFIGS) + list(STREAMS) + list(BATCHES))
