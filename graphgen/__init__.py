"""Seeded synthetic graph generators (input side only, shared by every consumer).

The generators draw the paper's graph classes as synthetic stand-ins (the
paper's evaluation uses symmetric real graphs in CSR and unsorted COO edge
batches; see its Graph Notation section and the input table):

* ``er``       Erdos-Renyi: m uniform endpoint pairs, self-loops dropped,
               duplicates kept, symmetrised to CSR with sorted rows.
* ``rmat``     RMAT with quadrant probabilities (a, b, c, 1-a-b-c), optional
               seeded bijective id scramble, symmetrised CSR.
* ``grid2d`` / ``grid3d``  bond-percolation lattices (each lattice edge kept
               i.i.d. with probability p): high diameter, many components.

All randomness is SplitMix64 (Steele, Lea, Flood, OOPSLA 2014) indexed by a
counter, implemented in ``graphgen.cpp``.  Nothing here computes connectivity.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile libgraphgen.so in-tree with g++ (OpenMP, portable flags)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
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
        lib.gg_key.restype = ctypes.c_uint64
        lib.gg_key.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_draw.restype = ctypes.c_uint64
        lib.gg_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_splitmix64_next.restype = ctypes.c_uint64
        lib.gg_splitmix64_next.argtypes = [u64p]
        lib.gg_er_edges.restype = ctypes.c_int64
        lib.gg_er_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, u32p, u32p]
        lib.gg_rmat_edges.restype = ctypes.c_int64
        lib.gg_rmat_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_uint64, ctypes.c_int, u32p, u32p]
        lib.gg_grid2d_edges.restype = ctypes.c_int64
        lib.gg_grid2d_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_double,
                                        ctypes.c_uint64, u32p, u32p]
        lib.gg_grid3d_edges.restype = ctypes.c_int64
        lib.gg_grid3d_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_double, ctypes.c_uint64, u32p, u32p]
        lib.gg_csr_from_edges.restype = ctypes.c_int64
        lib.gg_csr_from_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint64, u32p, u32p,
                                          ctypes.c_int, u64p, u32p]
        lib.gg_shuffle_edges.restype = None
        lib.gg_shuffle_edges.argtypes = [ctypes.c_uint64, ctypes.c_uint64, u32p, u32p]
        lib.gg_ba_edges.restype = ctypes.c_int64
        lib.gg_ba_edges.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64, u32p, u32p]
        lib.gg_uniform_pairs.restype = None
        lib.gg_uniform_pairs.argtypes = [ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint64, u32p, u32p]
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))


def _p64(a: np.ndarray):
    assert a.dtype == np.uint64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


@dataclass
class CSR:
    """Symmetric CSR graph: ``offsets`` uint64[n+1], ``nbrs`` uint32[m], rows sorted."""
    n: int
    offsets: np.ndarray
    nbrs: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.offsets[-1]) if self.n > 0 else 0

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int64)

    def coo(self):
        """Directed COO view (src, dst) of every CSR entry."""
        src = np.repeat(np.arange(self.n, dtype=np.uint32), self.degrees())
        return src, self.nbrs


# ---------------------------------------------------------------- raw draws
def key(seed: int, stream: int) -> int:
    return int(_load().gg_key(seed, stream))


def draw(k: int, i: int) -> int:
    return int(_load().gg_draw(k, i))


def splitmix64_sequence(state: int, count: int) -> list[int]:
    """First ``count`` outputs of SplitMix64 started at ``state``."""
    s = ctypes.c_uint64(state)
    lib = _load()
    return [int(lib.gg_splitmix64_next(ctypes.byref(s))) for _ in range(count)]


# ---------------------------------------------------------------- edge lists
def er_edges(n: int, m_draws: int, seed: int):
    src = np.empty(m_draws, np.uint32)
    dst = np.empty(m_draws, np.uint32)
    k = _load().gg_er_edges(n, m_draws, seed, _p32(src), _p32(dst))
    return src[:k].copy(), dst[:k].copy()


def rmat_edges(scale: int, m_draws: int, seed: int, a=0.57, b=0.19, c=0.19,
               scramble: bool = True, n: int | None = None):
    n = (1 << scale) if n is None else n
    src = np.empty(m_draws, np.uint32)
    dst = np.empty(m_draws, np.uint32)
    k = _load().gg_rmat_edges(scale, n, m_draws, a, b, c, seed, int(scramble), _p32(src), _p32(dst))
    if k < 0:
        raise ValueError("rmat: n exceeds 2^scale")
    if k == m_draws:
        return src, dst
    return src[:k].copy(), dst[:k].copy()


def grid2d_edges(W: int, H: int, p: float, seed: int):
    cap = max(0, (W - 1) * H) + max(0, W * (H - 1))
    src = np.empty(cap, np.uint32)
    dst = np.empty(cap, np.uint32)
    k = _load().gg_grid2d_edges(W, H, p, seed, _p32(src), _p32(dst))
    return src[:k].copy(), dst[:k].copy()


def grid3d_edges(X: int, Y: int, Z: int, p: float, seed: int):
    cap = max(0, (X - 1) * Y * Z) + max(0, X * (Y - 1) * Z) + max(0, X * Y * (Z - 1))
    src = np.empty(cap, np.uint32)
    dst = np.empty(cap, np.uint32)
    k = _load().gg_grid3d_edges(X, Y, Z, p, seed, _p32(src), _p32(dst))
    return src[:k].copy(), dst[:k].copy()


def csr_from_edges(n: int, src: np.ndarray, dst: np.ndarray, symmetrize: bool = True,
                   name: str = "") -> CSR:
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    k = len(src)
    offsets = np.empty(n + 1, np.uint64)
    nbrs = np.empty(k * (2 if symmetrize else 1), np.uint32)
    r = _load().gg_csr_from_edges(n, k, _p32(src), _p32(dst), int(symmetrize),
                                  _p64(offsets), _p32(nbrs))
    if r < 0:
        raise ValueError("csr_from_edges: vertex id out of range")
    return CSR(n, offsets, nbrs, name)


def shuffle_edges(src: np.ndarray, dst: np.ndarray, seed: int) -> None:
    _load().gg_shuffle_edges(len(src), seed, _p32(src), _p32(dst))


def ba_edges(n: int, k: int, seed: int):
    """Barabasi-Albert edges in arrival order: vertex v attaches k edges to
    earlier endpoints in proportion to degree (self-loops dropped)."""
    src = np.empty(max(n * k, 1), np.uint32)
    dst = np.empty(max(n * k, 1), np.uint32)
    w = _load().gg_ba_edges(n, k, seed, _p32(src), _p32(dst))
    return src[:w].copy(), dst[:w].copy()


def mixed_stream(src: np.ndarray, dst: np.ndarray, n: int, ratio: float, seed: int):
    """Insert edges shuffled together with uniform query pairs, 1/ratio queries
    per insert (ratio = inserts per query).  Returns (kind, a, b) with kind 0 for
    an insert and 1 for a query, in stream order."""
    k = len(src)
    q = int(round(k / ratio)) if ratio > 0 else 0
    qa, qb = uniform_pairs(n, q, seed, 77)
    kind = np.concatenate([np.zeros(k, np.uint32), np.ones(q, np.uint32)])
    a = np.concatenate([src, qa])
    b = np.concatenate([dst, qb])
    # one permutation applied to all three arrays: shuffle (kind, index) pairs
    idx = np.arange(k + q, dtype=np.uint32)
    tag = kind.copy()
    shuffle_edges(idx, tag, seed)
    return kind[idx].astype(np.uint8), a[idx], b[idx]


def uniform_pairs(n: int, q: int, seed: int, stream: int = 0):
    a = np.empty(q, np.uint32)
    b = np.empty(q, np.uint32)
    _load().gg_uniform_pairs(n, q, seed, stream, _p32(a), _p32(b))
    return a, b


# ---------------------------------------------------------------- workloads
def update_stream(scale: int, edge_factor: int, seed: int, max_requests: int = 0):
    """The incremental serving workload: an RMAT edge stream (scale, edge
    factor, stream seed seed + 100, shuffled) played in both directions, so
    every directed CSR entry is one update, cut into requests: each request is
    an insert batch of log-uniform size in [1e4, 1e7] (kept inside one
    direction's pass) or a batch of 1e5 uniform query pairs, with probability
    1/2 each (numpy's default_rng(seed)), until the updates run out or
    max_requests (> 0) requests exist.

    Returns (n, src, dst, reqs): inserts are (0, lo, hi), update indices of
    the two-pass stream (see insert_slices); queries are (1, a, b)."""
    n = 1 << scale
    src, dst = rmat_edges(scale, edge_factor * n, seed + 100)
    shuffle_edges(src, dst, seed + 100)
    E = len(src)
    rng = np.random.default_rng(seed)
    reqs, e = [], 0
    while e < 2 * E:
        if rng.random() < 0.5:
            k = int(10 ** rng.uniform(4, 7))
            lo, hi = e, min(e + k, 2 * E)
            if lo < E < hi:
                hi = E
            reqs.append((0, lo, hi))
            e = hi
        else:
            a, b = uniform_pairs(n, 100_000, seed, len(reqs))
            reqs.append((1, a, b))
        if max_requests and len(reqs) >= max_requests:
            break
    return n, src, dst, reqs


def insert_slices(src, dst, lo: int, hi: int):
    """Updates lo..hi of the two-pass stream: (src, dst) first, then (dst, src).
    Works on numpy arrays and on torch tensors alike (slicing only)."""
    E = len(src)
    if lo >= E:
        return dst[lo - E:hi - E], src[lo - E:hi - E]
    return src[lo:hi], dst[lo:hi]


def er(n: int, m_draws: int, seed: int = 1) -> CSR:
    s, d = er_edges(n, m_draws, seed)
    return csr_from_edges(n, s, d, True, f"er_n{n}_m{m_draws}_s{seed}")


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, a=0.57, b=0.19, c=0.19,
         scramble: bool = True, n: int | None = None) -> CSR:
    n = (1 << scale) if n is None else n
    s, d = rmat_edges(scale, edge_factor * n, seed, a, b, c, scramble, n)
    return csr_from_edges(n, s, d, True, f"rmat{scale}_ef{edge_factor}_s{seed}")


def grid2d(W: int, H: int, p: float, seed: int = 1) -> CSR:
    s, d = grid2d_edges(W, H, p, seed)
    return csr_from_edges(W * H, s, d, True, f"grid2d_{W}x{H}_p{p}_s{seed}")


def grid3d(X: int, Y: int, Z: int, p: float, seed: int = 1) -> CSR:
    s, d = grid3d_edges(X, Y, Z, p, seed)
    return csr_from_edges(X * Y * Z, s, d, True, f"grid3d_{X}x{Y}x{Z}_p{p}_s{seed}")


def from_pairs(n: int, pairs, name: str = "") -> CSR:
    """Symmetric CSR from an explicit list of undirected pairs (small test graphs)."""
    arr = np.asarray(list(pairs), dtype=np.uint32).reshape(-1, 2)
    return csr_from_edges(n, arr[:, 0].copy(), arr[:, 1].copy(), True, name)


def batched_specs(count: int, seed: int, n_lo: float = 1e3, n_hi: float = 1e6,
                  ef_lo: int = 8, ef_hi: int = 32):
    """Per-graph (kind, n, edge_factor, seed) for the many-graph workload:
    n log-uniform in [n_lo, n_hi], ER or RMAT by coin flip, edge factor uniform
    integer in [ef_lo, ef_hi]."""
    k = key(seed, 77)
    out = []
    lo, hi = math.log10(n_lo), math.log10(n_hi)
    for i in range(count):
        r0, r1, r2 = draw(k, 3 * i), draw(k, 3 * i + 1), draw(k, 3 * i + 2)
        u = (r0 >> 11) * (1.0 / (1 << 53))
        n = int(round(10 ** (lo + (hi - lo) * u)))
        kind = "rmat" if (r1 & 1) else "er"
        ef = ef_lo + int(((r2 & 0xFFFFFFFF) * (ef_hi - ef_lo + 1)) >> 32)
        out.append((kind, n, ef, seed * 100003 + i))
    return out


def batched_graph(kind: str, n: int, ef: int, gseed: int) -> CSR:
    if kind == "er":
        return er(n, ef * n, gseed)
    scale = max(1, int(math.ceil(math.log2(n))))
    return rmat(scale, ef, gseed, n=n)
