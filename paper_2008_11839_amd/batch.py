"""Many-graph batches (gconn_cc_batch) and the per-class autotuner.

A batch concatenates graphs into one CSR with global ids, each graph's vertex
range padded to a multiple of 64.  Graph classes are derived from observable
statistics only (size decade, average degree, degree skew); the autotuner
times candidate option sets on representative graphs of each class with the
library's gconn_autotune and caches the winners in a JSON table.
"""
from __future__ import annotations

import ctypes
import json
import math
import os
from dataclasses import dataclass, field

import numpy as np
import torch

from . import gconn as G

# Candidate option sets per class (the batched kernels support these rules).
BLOCKS = (128, 256, 512, 1024)  # workgroup shapes tried for each class's chosen rule

CANDIDATES = [
    dict(sample="kout", link="rem_cas", find="split", splice="split_one"),
    dict(sample="kout", link="rem_cas", find="naive", splice="split_one"),
    dict(sample="kout", link="async", find="split"),
    dict(sample="kout", link="async", find="halve"),
    dict(sample="none", link="rem_cas", find="split", splice="split_one"),
    dict(sample="none", link="async", find="split"),
    dict(sample="none", link="async", find="halve"),
    dict(sample="kout", link="early", find="split"),
    dict(sample="hb", link="rem_cas", find="split", splice="split_one", hb_n=4),
    dict(sample="hb", link="async", find="halve", hb_n=4),
]


# Candidates for one graph on its own (gconn_cc): the whole design space the
# single-graph pipeline offers -- the automatic k-out schedule (local-first
# passes on graphs whose ids follow their geometry), hook-based and BFS
# sampling, no sampling, and the round-based finishes for high-diameter
# graphs.
SINGLE_CANDIDATES = [
    dict(sample="kout", link="rem_cas", find="split", splice="splice_atomic"),
    dict(sample="kout", link="rem_cas", find="split", splice="split_one"),
    dict(sample="kout", link="rem_cas", find="naive", splice="split_one"),
    dict(sample="kout", link="async", find="halve"),
    dict(sample="hb", link="rem_cas", find="split", splice="split_one"),
    dict(sample="hb", link="async", find="halve"),
    dict(sample="bfs", link="rem_cas", find="split", splice="split_one"),
    dict(sample="none", link="rem_cas", find="split", splice="split_one"),
    dict(sample="none", link="async", find="halve"),
    dict(sample="kout", link="sv"),
    dict(sample="kout", link="lt", lt_variant="PRF"),
]


def graph_class_key(n: int, m: int, max_deg: int) -> str:
    """Class of a graph from its size decade, average degree and skew."""
    size = int(math.floor(math.log10(max(n, 1))))
    avg = m / max(n, 1)
    dens = "dense" if avg > 24 else "sparse"
    skew = "skewed" if max_deg > 8 * max(avg, 1.0) else "flat"
    return f"n1e{size}-{dens}-{skew}"


@dataclass
class HostBatch:
    """Concatenated host CSR of several graphs (global ids, 64-aligned ranges)."""
    n: int
    offsets: np.ndarray          # uint64[n+1]
    nbrs: np.ndarray             # uint32[m]
    vbase: np.ndarray            # uint32[G+1]
    sizes: list = field(default_factory=list)   # real vertex count per graph

    @property
    def m(self) -> int:
        return int(self.offsets[-1])

    @property
    def num_graphs(self) -> int:
        return len(self.vbase) - 1


def concat(graphs) -> HostBatch:
    """graphs: iterable of objects with n, offsets (uint64[n+1]), nbrs (uint32[m])."""
    graphs = list(graphs)
    vbase = [0]
    for g in graphs:
        vbase.append(vbase[-1] + ((g.n + 63) // 64) * 64)
    n = vbase[-1]
    m = sum(int(g.offsets[-1]) for g in graphs)
    offsets = np.zeros(n + 1, np.uint64)
    nbrs = np.empty(m, np.uint32)
    e0 = 0
    for i, g in enumerate(graphs):
        lo, hi = vbase[i], vbase[i + 1]
        gm = int(g.offsets[-1])
        offsets[lo:lo + g.n + 1] = g.offsets.astype(np.uint64) + np.uint64(e0)
        offsets[lo + g.n:hi + 1] = e0 + gm          # padding vertices: empty rows
        nbrs[e0:e0 + gm] = g.nbrs + np.uint32(lo)
        e0 += gm
    return HostBatch(n, offsets, nbrs, np.asarray(vbase, np.uint32), [g.n for g in graphs])


@dataclass
class DeviceBatch:
    host: HostBatch
    offsets: torch.Tensor
    nbrs: torch.Tensor
    vbase: torch.Tensor
    graph_class: torch.Tensor | None
    c: G._Batch


def upload(hb: HostBatch, graph_class=None, device="cuda", block: int = 0) -> DeviceBatch:
    off = torch.from_numpy(hb.offsets.view(np.int64)).to(device)
    nb = torch.from_numpy(hb.nbrs.view(np.int32)).to(device)
    vb = torch.from_numpy(hb.vbase.view(np.int32)).to(device)
    gc = None
    if graph_class is not None:
        gc = torch.from_numpy(np.asarray(graph_class, np.uint8)).to(device)
    c = G._Batch()
    c.num_graphs, c.n, c.m = hb.num_graphs, hb.n, hb.m
    c.offsets, c.nbrs, c.vbase = off.data_ptr(), (nb.data_ptr() if hb.m else None), vb.data_ptr()
    c.graph_class = gc.data_ptr() if gc is not None else None
    c.block = block
    return DeviceBatch(hb, off, nb, vb, gc, c)


def class_options(spec: dict) -> G._ClassOptions:
    c = G._ClassOptions()
    c.sample = G.SAMPLE[spec.get("sample", "kout")]
    c.link = G.LINK[spec.get("link", "async")]
    c.find = G.FIND[spec.get("find", "split")]
    c.splice = G.SPLICE[spec.get("splice", "split_one")]
    # hook-based classes carry N (the edges of step 2) in k
    c.k = spec.get("hb_n", 4) if spec.get("sample") == "hb" else spec.get("k", 2)
    return c


def cc_batch(db: DeviceBatch, classes: list, labels: torch.Tensor | None = None,
             workspace: torch.Tensor | None = None, lmax_samples: int = 1024, seed: int = 1,
             stats: bool = False, stream=None):
    """Per-graph local labels (int32 tensor over the concatenated vertices)."""
    lib = G.lib()
    if labels is None:
        labels = torch.empty(max(db.host.n, 1), dtype=torch.int32, device=db.offsets.device)[: db.host.n]
    if workspace is None:
        b = ctypes.c_size_t()
        G._check(lib.gconn_cc_batch_workspace_size(ctypes.byref(db.c), ctypes.byref(b)))
        workspace = G.alloc_workspace(b.value, db.offsets.device)
    arr = (G._ClassOptions * len(classes))(*[class_options(c) for c in classes])
    st = G._Stats() if stats else None
    G._check(lib.gconn_cc_batch(ctypes.byref(db.c), labels.data_ptr() if db.host.n else None,
                                workspace.data_ptr(), workspace.numel(), arr, len(classes),
                                lmax_samples, seed, ctypes.byref(st) if st else None,
                                G._stream(stream)))
    return (labels, G._stats_dict(st)) if stats else labels


def capture_batch(db: DeviceBatch, classes: list, labels: torch.Tensor,
                  workspace: torch.Tensor | None = None, lmax_samples: int = 1024,
                  seed: int = 1) -> "G.Exec":
    """Record one gconn_cc_batch run into a HIP graph; Exec.launch() replays it."""
    lib = G.lib()
    if workspace is None:
        b = ctypes.c_size_t()
        G._check(lib.gconn_cc_batch_workspace_size(ctypes.byref(db.c), ctypes.byref(b)))
        workspace = G.alloc_workspace(b.value, db.offsets.device)
    arr = (G._ClassOptions * len(classes))(*[class_options(c) for c in classes])
    h = ctypes.c_void_p()
    G._check(lib.gconn_cc_batch_capture(ctypes.byref(db.c), labels.data_ptr() if db.host.n else None,
                                        workspace.data_ptr(), workspace.numel(), arr, len(classes),
                                        lmax_samples, seed, ctypes.byref(h)))
    return G.Exec(h, (db, labels, workspace, arr))


def autotune(device_graphs: list, candidates=CANDIDATES, reps: int = 3, stream=None):
    """Index of the fastest candidate over the given graphs, and the totals (ms)."""
    lib = G.lib()
    opts = (G._Options * len(candidates))(*[G.Options(**c).to_c() for c in candidates])
    gs = (G._Graph * len(device_graphs))(*[g.c for g in device_graphs])
    need = max(G.workspace_size(g, G.Options(**c)) for g in device_graphs for c in candidates)
    ws = G.alloc_workspace(need)
    scratch = torch.empty(max(g.n for g in device_graphs), dtype=torch.int32, device="cuda")
    best = ctypes.c_uint32()
    times = (ctypes.c_double * len(candidates))()
    G._check(lib.gconn_autotune(gs, len(device_graphs), opts, len(candidates), reps,
                                scratch.data_ptr(), ws.data_ptr(), ws.numel(), G._stream(stream),
                                ctypes.byref(best), times))
    return best.value, list(times)


def tune_single(device_graph, candidates=SINGLE_CANDIDATES, reps: int = 3, stream=None):
    """The fastest option set for one graph: (options dict, times in ms per
    candidate, in candidate order), timed with gconn_autotune."""
    best, times = autotune([device_graph], candidates, reps, stream)
    return dict(candidates[best]), times


class Autotuner:
    """Per-class choice of sampling / link / find, cached in a JSON table."""

    def __init__(self, table_path: str | None = None, reps: int = 3, per_class: int = 3):
        self.table_path = table_path
        self.reps = reps
        self.per_class = per_class
        self.table = {}
        if table_path and os.path.exists(table_path):
            with open(table_path) as f:
                self.table = json.load(f)

    def tune(self, host_graphs: list) -> list:
        """Classify the graphs, tune every class not yet in the table, and
        return the class key of each graph."""
        keys = []
        by_class = {}
        for i, g in enumerate(host_graphs):
            deg = np.diff(g.offsets.astype(np.int64))
            key = graph_class_key(g.n, int(g.offsets[-1]), int(deg.max()) if g.n else 0)
            keys.append(key)
            by_class.setdefault(key, []).append(i)
        for key, idx in by_class.items():
            if key in self.table:
                continue
            # representatives: the largest graphs of the class dominate its cost
            reps_idx = sorted(idx, key=lambda i: -int(host_graphs[i].offsets[-1]))[: self.per_class]
            dgs = [G.csr(host_graphs[i].offsets, host_graphs[i].nbrs, host_graphs[i].n)
                   for i in reps_idx]
            best, times = autotune(dgs, CANDIDATES, self.reps)
            # then the workgroup shape for the chosen rule
            shapes = [dict(CANDIDATES[best], block=b) for b in BLOCKS]
            bbest, btimes = autotune(dgs, shapes, self.reps)
            self.table[key] = {"choice": shapes[bbest], "times_ms": times,
                               "block_times_ms": dict(zip(map(str, BLOCKS), btimes))}
        if self.table_path:
            with open(self.table_path, "w") as f:
                json.dump(self.table, f, indent=1)
        return keys

    def batch_block(self, keys: list, host_graphs: list) -> int:
        """Workgroup shape for one batch launch: the tuned shape of the class
        that holds the most edges (one launch has one shape)."""
        edges = {}
        for k, g in zip(keys, host_graphs):
            edges[k] = edges.get(k, 0) + int(g.offsets[-1])
        top = max(edges, key=edges.get)
        return int(self.table[top]["choice"].get("block", 256))

    @staticmethod
    def tune_batch_block(db: "DeviceBatch", classes: list, labels: torch.Tensor,
                         workspace: torch.Tensor, reps: int = 3) -> tuple:
        """Workgroup shape for one batch launch, timed on the batch itself:
        every shape in BLOCKS runs the whole batch reps times (HIP events) and
        the fastest is kept in db.  The per-class shapes come from each class's
        own graphs timed alone, but in the batch every class's unions run
        beside the others'.  Returns (shape, {shape: mean ms})."""
        times = {}
        keep = int(db.c.block)
        try:
            for b in BLOCKS:
                db.c.block = b
                cc_batch(db, classes, labels=labels, workspace=workspace)  # warm
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    cc_batch(db, classes, labels=labels, workspace=workspace)
                e1.record()
                torch.cuda.synchronize()
                times[b] = e0.elapsed_time(e1) / reps
        finally:
            db.c.block = keep
        best = min(times, key=times.get)
        db.c.block = best
        return best, times

    def classes_for(self, keys: list):
        """(class option list, per-graph class index) for cc_batch."""
        uniq = sorted(set(keys))
        if len(uniq) > 64:
            raise ValueError("more than 64 graph classes")
        index = {k: i for i, k in enumerate(uniq)}
        return [self.table[k]["choice"] for k in uniq], [index[k] for k in keys]
