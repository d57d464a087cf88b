"""CPU oracle for the connectivity hot path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the benchmark's ``cpu_baseline`` leg
may import this package.  The GPU library never links, loads or calls it, and
it shares no code with the GPU path (the only common module is the seeded input
generator, which computes no connectivity).

Every function wraps plain sequential C in ``oracle.c`` (built with gcc -O2).
Cited passages are in that file's header; in short:
  * ``cc``             canonical labels = minimum vertex id per component
                       (Preliminaries: union-find links larger id under smaller)
  * ``spanning_forest``one recorded edge per root that was linked (Static
                       Spanning Forest paragraph)
  * ``UnionFind``      incremental insert / query batches (Incremental
                       Connectivity Support)
  * ``sample_kout`` / ``sample_hb`` / ``sample_bfs``  sampled partitions
                       (Sampling Algorithms; Appendix A.1)
  * ``lmax`` / ``active_count`` / ``active_edges``  most frequent label over a
                       seeded sample and the vertex-gathering set (Iterative GPU
                       Optimizations, vertex gathering)
  * ``check_forest``   spanning-forest validity (several forests are correct)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None
EMPTY = 0xFFFFFFFF


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        c32, c64 = ctypes.c_uint32, ctypes.c_uint64
        sig = {
            "oracle_uf_init": (None, [u32p, c32]),
            "oracle_uf_insert": (ctypes.c_int64, [u32p, c32, c64, u32p, u32p, u32p, u32p]),
            "oracle_uf_query": (ctypes.c_int, [u32p, c32, c64, u32p, u32p, u8p]),
            "oracle_uf_labels": (None, [u32p, c32, u32p]),
            "oracle_cc_csr": (ctypes.c_int, [c32, u64p, u32p, u32p]),
            "oracle_cc_coo": (ctypes.c_int, [c32, c64, u32p, u32p, u32p]),
            "oracle_sf_csr": (ctypes.c_int64, [c32, u64p, u32p, u32p, u32p]),
            "oracle_sample_kout": (ctypes.c_int64, [c32, u64p, u32p, c32, u32p]),
            "oracle_sample_hb": (ctypes.c_int64, [c32, u64p, u32p, c32, u32p]),
            "oracle_sample_bfs": (ctypes.c_int64, [c32, u64p, u32p, u32p]),
            "oracle_splitmix64": (c64, [c64, c64]),
            "oracle_lmax": (ctypes.c_int64, [u32p, c32, c32, c64]),
            "oracle_active_count": (ctypes.c_int64, [c32, u64p, u32p, c32]),
            "oracle_active_edges": (ctypes.c_int64, [c32, u64p, u32p, c32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _u32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint32)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint64)


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _csr(offsets, nbrs):
    off = _u64(offsets)
    nb = _u32(nbrs)
    if len(nb) == 0:
        nb = np.zeros(1, np.uint32)
    return off, nb


def cc(n: int, offsets, nbrs) -> np.ndarray:
    off, nb = _csr(offsets, nbrs)
    labels = np.empty(max(n, 1), np.uint32)
    rc = _load().oracle_cc_csr(n, _p(off, ctypes.c_uint64), _p(nb, ctypes.c_uint32),
                               _p(labels, ctypes.c_uint32))
    if rc != 0:
        raise ValueError(f"oracle_cc_csr failed ({rc})")
    return labels[:n]


def cc_coo(n: int, src, dst) -> np.ndarray:
    s, d = _u32(src), _u32(dst)
    m = len(s)
    if m == 0:
        s = d = np.zeros(1, np.uint32)
    labels = np.empty(max(n, 1), np.uint32)
    rc = _load().oracle_cc_coo(n, m, _p(s, ctypes.c_uint32), _p(d, ctypes.c_uint32),
                               _p(labels, ctypes.c_uint32))
    if rc != 0:
        raise ValueError(f"oracle_cc_coo failed ({rc})")
    return labels[:n]


def spanning_forest(n: int, offsets, nbrs):
    off, nb = _csr(offsets, nbrs)
    fu = np.empty(max(n, 1), np.uint32)
    fv = np.empty(max(n, 1), np.uint32)
    k = _load().oracle_sf_csr(n, _p(off, ctypes.c_uint64), _p(nb, ctypes.c_uint32),
                              _p(fu, ctypes.c_uint32), _p(fv, ctypes.c_uint32))
    if k < 0:
        raise ValueError("oracle_sf_csr failed")
    return fu[:n], fv[:n]


class UnionFind:
    """Sequential union-find kept across insert / query batches."""

    def __init__(self, n: int):
        self.n = n
        self.P = np.empty(max(n, 1), np.uint32)
        _load().oracle_uf_init(_p(self.P, ctypes.c_uint32), n)

    def insert(self, src, dst, record: bool = False):
        s, d = _u32(src), _u32(dst)
        k = len(s)
        if k == 0:
            return 0
        fu = fv = None
        if record:
            fu = np.full(self.n, EMPTY, np.uint32)
            fv = np.full(self.n, EMPTY, np.uint32)
        r = _load().oracle_uf_insert(_p(self.P, ctypes.c_uint32), self.n, k,
                                     _p(s, ctypes.c_uint32), _p(d, ctypes.c_uint32),
                                     _p(fu, ctypes.c_uint32) if record else None,
                                     _p(fv, ctypes.c_uint32) if record else None)
        if r < 0:
            raise ValueError("oracle_uf_insert: vertex id out of range")
        return (r, fu, fv) if record else r

    def query(self, a, b) -> np.ndarray:
        x, y = _u32(a), _u32(b)
        q = len(x)
        out = np.empty(max(q, 1), np.uint8)
        if q:
            rc = _load().oracle_uf_query(_p(self.P, ctypes.c_uint32), self.n, q,
                                         _p(x, ctypes.c_uint32), _p(y, ctypes.c_uint32),
                                         _p(out, ctypes.c_uint8))
            if rc != 0:
                raise ValueError("oracle_uf_query: vertex id out of range")
        return out[:q]

    def labels(self) -> np.ndarray:
        out = np.empty(max(self.n, 1), np.uint32)
        _load().oracle_uf_labels(_p(self.P, ctypes.c_uint32), self.n, _p(out, ctypes.c_uint32))
        return out[:self.n]


def sample_kout(n, offsets, nbrs, k: int = 2):
    off, nb = _csr(offsets, nbrs)
    labels = np.empty(max(n, 1), np.uint32)
    e = _load().oracle_sample_kout(n, _p(off, ctypes.c_uint64), _p(nb, ctypes.c_uint32), k,
                                   _p(labels, ctypes.c_uint32))
    if e < 0:
        raise ValueError("oracle_sample_kout failed")
    return labels[:n], int(e)


def sample_hb(n, offsets, nbrs, N: int = 4):
    off, nb = _csr(offsets, nbrs)
    labels = np.empty(max(n, 1), np.uint32)
    e = _load().oracle_sample_hb(n, _p(off, ctypes.c_uint64), _p(nb, ctypes.c_uint32), N,
                                 _p(labels, ctypes.c_uint32))
    if e < 0:
        raise ValueError("oracle_sample_hb failed")
    return labels[:n], int(e)


def sample_bfs(n, offsets, nbrs):
    off, nb = _csr(offsets, nbrs)
    labels = np.empty(max(n, 1), np.uint32)
    s = _load().oracle_sample_bfs(n, _p(off, ctypes.c_uint64), _p(nb, ctypes.c_uint32),
                                  _p(labels, ctypes.c_uint32))
    if s < 0:
        raise ValueError("oracle_sample_bfs failed")
    return labels[:n], int(s)


def splitmix64(state0: int, i: int) -> int:
    return int(_load().oracle_splitmix64(state0, i))


def lmax(labels, samples: int, seed: int) -> int:
    lab = _u32(labels)
    r = _load().oracle_lmax(_p(lab, ctypes.c_uint32), len(lab), samples, seed)
    if r < 0:
        raise ValueError("oracle_lmax failed")
    return int(r)


def active_count(n, offsets, labels, lmax_label: int) -> int:
    off, lab = _u64(offsets), _u32(labels)
    return int(_load().oracle_active_count(n, _p(off, ctypes.c_uint64),
                                           _p(lab, ctypes.c_uint32), lmax_label))


def active_edges(n, offsets, labels, lmax_label: int) -> int:
    off, lab = _u64(offsets), _u32(labels)
    return int(_load().oracle_active_edges(n, _p(off, ctypes.c_uint64),
                                           _p(lab, ctypes.c_uint32), lmax_label))


def check_forest(n: int, offsets, nbrs, fu, fv, labels=None) -> dict:
    """Validate a spanning forest given as per-slot edges (EMPTY = no edge).

    A valid result (Static Spanning Forest paragraph) is any acyclic subset of
    the input edges with the same partition as the graph: exactly n - c edges,
    every edge an input edge, no edge closing a cycle, and the forest's own
    components equal to the graph's.  Raises AssertionError on a violation and
    returns summary counts.
    """
    off, nb = _u64(offsets), _u32(nbrs)
    fu, fv = _u32(fu), _u32(fv)
    if labels is None:
        labels = cc(n, off, nb)
    labels = _u32(labels)
    used = fu != EMPTY
    assert np.array_equal(used, fv != EMPTY), "half-filled forest slot"
    eu, ev = fu[used], fv[used]
    c = int(np.count_nonzero(labels == np.arange(n, dtype=np.uint32)))
    assert len(eu) == n - c, f"forest has {len(eu)} edges, expected n-c = {n - c}"
    if len(eu):
        assert eu.max() < n and ev.max() < n, "forest edge endpoint out of range"
        # every forest edge is an input edge: vectorised lower-bound search for
        # v in u's sorted row
        lo = off[eu.astype(np.int64)].astype(np.int64)
        hi = off[eu.astype(np.int64) + 1].astype(np.int64)
        while True:
            open_ = lo < hi
            if not open_.any():
                break
            mid = (lo + hi) // 2
            go_right = open_ & (nb[np.minimum(mid, len(nb) - 1)] < ev)
            lo = np.where(go_right, mid + 1, lo)
            hi = np.where(open_ & ~go_right, mid, hi)
        found = (lo < off[eu.astype(np.int64) + 1].astype(np.int64))
        found &= nb[np.minimum(lo, len(nb) - 1)] == ev
        assert found.all(), f"{int((~found).sum())} forest edges are not graph edges"
    # acyclic: inserting the forest edges links on every single edge
    uf = UnionFind(n)
    links = uf.insert(eu, ev) if len(eu) else 0
    assert links == len(eu), "forest contains a cycle"
    # same partition as the graph
    assert np.array_equal(uf.labels(), labels), "forest partition differs from the graph's"
    return {"edges": int(len(eu)), "components": c}
