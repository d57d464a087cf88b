"""ctypes binding of libgconn.so (the C ABI in include/gconn.h).

Argument marshalling only: torch tensors provide device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  Vertex-id tensors are int32 tensors holding uint32 bit patterns
(0xFFFFFFFF, the empty forest slot, reads as -1).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgconn.so")
EMPTY = 0xFFFFFFFF

SAMPLE = {"none": 0, "kout": 1, "hb": 2, "bfs": 3}
LINK = {"async": 0, "hooks": 1, "early": 2, "rem_cas": 3, "ecl": 4, "sv": 5, "lt": 6, "lp": 7,
        "afforest": 8, "rem_lock": 9, "jtb": 10}
FIND = {"naive": 0, "split": 1, "halve": 2, "compress": 3, "two_try_split": 4}
SPLICE = {"split_one": 0, "halve_one": 1, "splice_atomic": 2}
SCHEDULE = {"auto": 0, "lane": 1, "step": 2, "pipe": 3, "twopass": 4, "flat": 5, "xcd": 6}
LT_VARIANTS = ["CUSA", "CRSA", "PUSA", "PRSA", "PUS", "PRS", "EUSA", "EUS",
               "CUFA", "CRFA", "PUFA", "PRFA", "PUF", "PRF", "EUFA", "EUF"]
STATUS = {0: "GCONN_OK", -1: "GCONN_EINVAL", -2: "GCONN_ENOMEM", -3: "GCONN_EDEVICE",
          -4: "GCONN_ENODEV", -5: "GCONN_EBUSY", -6: "GCONN_ETIMEOUT", -7: "GCONN_EUNSUPPORTED"}


class GconnError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class _Graph(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("offsets_64", ctypes.c_int32),
                ("n", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("m", ctypes.c_uint64), ("offsets", ctypes.c_void_p),
                ("nbrs", ctypes.c_void_p), ("dst", ctypes.c_void_p)]


class _Options(ctypes.Structure):
    _fields_ = [("sample", ctypes.c_int32), ("link", ctypes.c_int32), ("find", ctypes.c_int32),
                ("splice", ctypes.c_int32), ("lt_variant", ctypes.c_int32),
                ("k", ctypes.c_uint32), ("hb_n", ctypes.c_uint32),
                ("lmax_samples", ctypes.c_uint32), ("seed", ctypes.c_uint64),
                ("kout_random", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("block", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("atomic_compress", ctypes.c_int32), ("kout_prelink", ctypes.c_int32),
                ("kout_local", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("sampled_edges", ctypes.c_uint64), ("active_vertices", ctypes.c_uint64),
                ("finish_edges", ctypes.c_uint64), ("hooks", ctypes.c_uint64),
                ("rounds", ctypes.c_uint64), ("lmax", ctypes.c_uint32),
                ("bfs_source", ctypes.c_uint32)]


class _Batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_uint32), ("n", ctypes.c_uint32), ("m", ctypes.c_uint64),
                ("offsets", ctypes.c_void_p), ("nbrs", ctypes.c_void_p), ("vbase", ctypes.c_void_p),
                ("graph_class", ctypes.c_void_p), ("block", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class _ClassOptions(ctypes.Structure):
    _fields_ = [("sample", ctypes.c_int32), ("link", ctypes.c_int32), ("find", ctypes.c_int32),
                ("splice", ctypes.c_int32), ("k", ctypes.c_uint32), ("reserved", ctypes.c_uint32)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("n_max", ctypes.c_uint32), ("streams", ctypes.c_uint32),
                ("arena_bytes", ctypes.c_uint64), ("options", _Options)]


class _RequestInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("status", ctypes.c_int32), ("count", ctypes.c_uint64),
                ("epoch", ctypes.c_uint64), ("submit_us", ctypes.c_double),
                ("admit_us", ctypes.c_double), ("done_us", ctypes.c_double)]


class _PhaseTimes(ctypes.Structure):
    _fields_ = [("init_ms", ctypes.c_double), ("sample_ms", ctypes.c_double),
                ("compress_ms", ctypes.c_double), ("lmax_ms", ctypes.c_double),
                ("gather_ms", ctypes.c_double), ("finish_ms", ctypes.c_double),
                ("finalize_ms", ctypes.c_double), ("runs", ctypes.c_uint64)]


EXPORTS = ["gconn_server_create", "gconn_server_submit", "gconn_server_wait",
           "gconn_server_drain", "gconn_server_destroy", "gconn_cc_batch_workspace_size", "gconn_cc_batch", "gconn_autotune",
           "gconn_profile_enable", "gconn_profile_read", "gconn_options_default", "gconn_workspace_size", "gconn_cc", "gconn_cc_noalloc", "gconn_spanning_forest",
           "gconn_inc_workspace_size", "gconn_inc_create", "gconn_inc_insert_batch",
           "gconn_inc_query_batch", "gconn_inc_mixed_batch", "gconn_inc_labels", "gconn_inc_destroy",
           "gconn_cc_capture", "gconn_cc_batch_capture", "gconn_exec_launch", "gconn_exec_destroy",
           "gconn_status_string", "gconn_last_error", "gconn_version", "gconn_diag_random_access"]

_lib = None


def lib() -> ctypes.CDLL:
    """Load libgconn.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2008_11839_amd.build` (no CPU fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        gp, op, stp = ctypes.POINTER(_Graph), ctypes.POINTER(_Options), ctypes.POINTER(_Stats)
        L.gconn_options_default.restype = None
        L.gconn_options_default.argtypes = [op]
        L.gconn_workspace_size.restype = ctypes.c_int
        L.gconn_workspace_size.argtypes = [gp, op, ctypes.c_int, ctypes.c_int, ctypes.POINTER(sz)]
        L.gconn_cc.restype = ctypes.c_int
        L.gconn_cc.argtypes = [gp, vp, vp, sz, op, stp, vp]
        L.gconn_cc_noalloc.restype = ctypes.c_int
        L.gconn_cc_noalloc.argtypes = [gp, vp, op, stp, vp]
        L.gconn_diag_random_access.restype = ctypes.c_int
        L.gconn_diag_random_access.argtypes = [vp, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64,
                                               vp, ctypes.c_uint32, vp]
        L.gconn_spanning_forest.restype = ctypes.c_int
        L.gconn_spanning_forest.argtypes = [gp, vp, vp, vp, vp, sz, op, stp, vp]
        L.gconn_inc_workspace_size.restype = ctypes.c_int
        L.gconn_inc_workspace_size.argtypes = [ctypes.c_uint32, gp, op, ctypes.POINTER(sz)]
        L.gconn_inc_create.restype = ctypes.c_int
        L.gconn_inc_create.argtypes = [ctypes.c_uint32, vp, gp, vp, sz, op, vp,
                                       ctypes.POINTER(vp)]
        L.gconn_inc_insert_batch.restype = ctypes.c_int
        L.gconn_inc_insert_batch.argtypes = [vp, vp, vp, ctypes.c_uint64, vp]
        L.gconn_inc_query_batch.restype = ctypes.c_int
        L.gconn_inc_query_batch.argtypes = [vp, vp, vp, ctypes.c_uint64, vp, vp]
        L.gconn_inc_mixed_batch.restype = ctypes.c_int
        L.gconn_inc_mixed_batch.argtypes = [vp, vp, vp, vp, ctypes.c_uint64, vp, vp]
        L.gconn_cc_capture.restype = ctypes.c_int
        L.gconn_cc_capture.argtypes = [gp, vp, vp, sz, op, ctypes.POINTER(vp)]
        L.gconn_exec_launch.restype = ctypes.c_int
        L.gconn_exec_launch.argtypes = [vp, vp]
        L.gconn_exec_destroy.restype = ctypes.c_int
        L.gconn_exec_destroy.argtypes = [vp]
        L.gconn_inc_labels.restype = ctypes.c_int
        L.gconn_inc_labels.argtypes = [vp, vp, vp]
        L.gconn_inc_destroy.restype = ctypes.c_int
        L.gconn_inc_destroy.argtypes = [vp]
        bp, cp = ctypes.POINTER(_Batch), ctypes.POINTER(_ClassOptions)
        L.gconn_cc_batch_workspace_size.restype = ctypes.c_int
        L.gconn_cc_batch_workspace_size.argtypes = [bp, ctypes.POINTER(sz)]
        L.gconn_cc_batch.restype = ctypes.c_int
        L.gconn_cc_batch.argtypes = [bp, vp, vp, sz, cp, ctypes.c_uint32, ctypes.c_uint32,
                                     ctypes.c_uint64, stp, vp]
        L.gconn_cc_batch_capture.restype = ctypes.c_int
        L.gconn_cc_batch_capture.argtypes = [bp, vp, vp, sz, cp, ctypes.c_uint32, ctypes.c_uint32,
                                             ctypes.c_uint64, ctypes.POINTER(vp)]
        L.gconn_autotune.restype = ctypes.c_int
        L.gconn_autotune.argtypes = [gp, ctypes.c_uint32, op, ctypes.c_uint32, ctypes.c_uint32, vp,
                                     vp, sz, vp, ctypes.POINTER(ctypes.c_uint32),
                                     ctypes.POINTER(ctypes.c_double)]
        L.gconn_server_create.restype = ctypes.c_int
        L.gconn_server_create.argtypes = [ctypes.POINTER(_ServerConfig), vp, vp, ctypes.POINTER(vp)]
        L.gconn_server_submit.restype = ctypes.c_int
        L.gconn_server_submit.argtypes = [vp, ctypes.c_int, vp, vp, ctypes.c_uint64, vp,
                                          ctypes.POINTER(ctypes.c_uint64)]
        L.gconn_server_wait.restype = ctypes.c_int
        L.gconn_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.c_double,
                                        ctypes.POINTER(_RequestInfo)]
        L.gconn_server_drain.restype = ctypes.c_int
        L.gconn_server_drain.argtypes = [vp]
        L.gconn_server_destroy.restype = ctypes.c_int
        L.gconn_server_destroy.argtypes = [vp]
        L.gconn_profile_enable.restype = ctypes.c_int
        L.gconn_profile_enable.argtypes = [ctypes.c_int]
        L.gconn_profile_read.restype = ctypes.c_int
        L.gconn_profile_read.argtypes = [ctypes.POINTER(_PhaseTimes), ctypes.c_int]
        L.gconn_status_string.restype = ctypes.c_char_p
        L.gconn_status_string.argtypes = [ctypes.c_int]
        L.gconn_last_error.restype = ctypes.c_char_p
        L.gconn_last_error.argtypes = []
        L.gconn_version.restype = ctypes.c_char_p
        L.gconn_version.argtypes = []
        _lib = L
    return _lib


def _check(status: int) -> None:
    if status != 0:
        msg = lib().gconn_last_error().decode(errors="replace")
        raise GconnError(status, msg)


@dataclass
class Options:
    """Python view of gconn_options (names instead of enum values)."""
    sample: str = "kout"
    link: str = "async"
    find: str = "split"
    splice: str = "split_one"
    lt_variant: str = "PRF"
    k: int = 2
    hb_n: int = 4
    lmax_samples: int = 1024
    seed: int = 1
    kout_random: bool = False
    validate: bool = False
    block: int = 256
    schedule: str = "auto"
    atomic_compress: bool = True
    kout_prelink: bool = False
    kout_local: bool = False

    def to_c(self) -> _Options:
        o = _Options()
        lib().gconn_options_default(ctypes.byref(o))
        o.sample = SAMPLE[self.sample]
        o.link = LINK[self.link]
        o.find = FIND[self.find]
        o.splice = SPLICE[self.splice]
        o.lt_variant = LT_VARIANTS.index(self.lt_variant)
        o.k, o.hb_n, o.lmax_samples = self.k, self.hb_n, self.lmax_samples
        o.seed = self.seed
        o.kout_random = int(self.kout_random)
        o.validate = int(self.validate)
        o.block = self.block
        o.schedule = SCHEDULE[self.schedule]
        o.atomic_compress = int(self.atomic_compress)
        o.kout_prelink = int(self.kout_prelink)
        o.kout_local = int(self.kout_local)
        return o


def _ptr(t: torch.Tensor | None) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


@dataclass
class DeviceGraph:
    """A graph resident in device memory (CSR or COO) plus its C descriptor."""
    n: int
    m: int
    fmt: str
    offsets: torch.Tensor | None = None
    nbrs: torch.Tensor | None = None
    dst: torch.Tensor | None = None
    c: _Graph = field(default_factory=_Graph)

    def __post_init__(self):
        g = self.c
        g.format = 0 if self.fmt == "csr" else 1
        g.n = self.n
        g.m = self.m
        g.offsets_64 = int(self.offsets is not None and self.offsets.dtype == torch.int64)
        g.offsets = _ptr(self.offsets) if self.offsets is not None else None
        g.nbrs = _ptr(self.nbrs) if self.nbrs is not None and self.nbrs.numel() else None
        g.dst = _ptr(self.dst) if self.dst is not None and self.dst.numel() else None


def csr(offsets, nbrs, n: int | None = None, device="cuda", offsets64: bool | None = None) -> DeviceGraph:
    """Upload (or wrap) a CSR graph.  offsets: n+1 entries; nbrs: m ids."""
    if isinstance(offsets, np.ndarray):
        m = int(offsets[-1]) if len(offsets) else 0
        if offsets64 is None:
            offsets64 = m > 0xFFFFFFFF
        off = torch.from_numpy(offsets.astype(np.int64 if offsets64 else np.uint32).view(
            np.int64 if offsets64 else np.int32)).to(device)
    else:
        off = offsets
    if isinstance(nbrs, np.ndarray):
        nb = torch.from_numpy(np.ascontiguousarray(nbrs, dtype=np.uint32).view(np.int32)).to(device)
    else:
        nb = nbrs
    n = off.numel() - 1 if n is None else n
    return DeviceGraph(n=n, m=nb.numel(), fmt="csr", offsets=off, nbrs=nb)


def coo(src, dst, n: int, device="cuda") -> DeviceGraph:
    conv = lambda a: (torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).to(device)
                      if isinstance(a, np.ndarray) else a)
    s, d = conv(src), conv(dst)
    return DeviceGraph(n=n, m=s.numel(), fmt="coo", nbrs=s, dst=d)


def workspace_size(g: DeviceGraph, options: Options | None = None, forest: bool = False,
                   labels: bool = True) -> int:
    o = (options or Options()).to_c()
    b = ctypes.c_size_t(0)
    _check(lib().gconn_workspace_size(ctypes.byref(g.c), ctypes.byref(o), int(forest), int(labels),
                                      ctypes.byref(b)))
    return b.value


def alloc_workspace(nbytes: int, device="cuda") -> torch.Tensor:
    """Device buffer of at least nbytes whose data_ptr is 256-byte aligned."""
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + nbytes]


def _stats_dict(s: _Stats) -> dict:
    return {f: getattr(s, f) for f, _ in _Stats._fields_}


def cc(g: DeviceGraph, labels: torch.Tensor | None = None, options: Options | None = None,
       workspace: torch.Tensor | None = None, stats: bool = False, stream=None):
    """Connected-component labels (minimum vertex id per component), int32 tensor."""
    o = (options or Options()).to_c()
    if labels is None:
        labels = torch.empty(max(g.n, 1), dtype=torch.int32, device=g.nbrs.device if g.nbrs is not None else "cuda")[: g.n]
    if workspace is None:
        workspace = alloc_workspace(workspace_size(g, options))
    st = _Stats() if stats else None
    _check(lib().gconn_cc(ctypes.byref(g.c), _ptr(labels) if g.n else None, workspace.data_ptr(),
                          workspace.numel(), ctypes.byref(o), ctypes.byref(st) if st else None,
                          _stream(stream)))
    return (labels, _stats_dict(st)) if stats else labels


def diag_random_access(table: torch.Tensor, kind: int, accesses: int, sink: torch.Tensor,
                       stream=None) -> None:
    """gconn_diag_random_access: one kernel of `accesses` random 4-byte
    accesses to `table` (kind 0 cached loads, 1 coherent loads, 2 CAS)."""
    _check(lib().gconn_diag_random_access(_ptr(table), table.numel(), kind, accesses, _ptr(sink),
                                          sink.numel(), _stream(stream)))


NOALLOC_SCRATCH_BYTES = 64 << 20  # GCONN_NOALLOC_SCRATCH_BYTES


def cc_noalloc(g: DeviceGraph, labels: torch.Tensor, options: Options | None = None,
               stats: bool = False, stream=None):
    """gconn_cc_noalloc: gconn_cc without a workspace (the library's own
    per-device scratch array; raises GconnError with GCONN_ENOMEM when the
    graph needs more than NOALLOC_SCRATCH_BYTES)."""
    o = (options or Options()).to_c()
    st = _Stats() if stats else None
    _check(lib().gconn_cc_noalloc(ctypes.byref(g.c), _ptr(labels) if g.n else None,
                                  ctypes.byref(o), ctypes.byref(st) if st else None,
                                  _stream(stream)))
    return (labels, _stats_dict(st)) if stats else labels


class Exec:
    """A captured pipeline (gconn_cc_capture / gconn_cc_batch_capture): launch()
    replays it on a stream.  Holds references to every buffer it reads or
    writes, so they outlive the handle."""

    def __init__(self, handle: ctypes.c_void_p, keep: tuple):
        self._h = handle
        self._keep = keep

    def launch(self, stream=None) -> None:
        _check(lib().gconn_exec_launch(self._h, _stream(stream)))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().gconn_exec_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def capture_cc(g: DeviceGraph, labels: torch.Tensor, options: Options | None = None,
               workspace: torch.Tensor | None = None) -> Exec:
    """Record one gconn_cc run into a HIP graph; Exec.launch() replays it."""
    o = (options or Options()).to_c()
    if workspace is None:
        workspace = alloc_workspace(workspace_size(g, options))
    h = ctypes.c_void_p()
    _check(lib().gconn_cc_capture(ctypes.byref(g.c), _ptr(labels) if g.n else None,
                                  workspace.data_ptr(), workspace.numel(), ctypes.byref(o),
                                  ctypes.byref(h)))
    return Exec(h, (g, labels, workspace))


def spanning_forest(g: DeviceGraph, want_labels: bool = True, options: Options | None = None,
                    workspace: torch.Tensor | None = None, stats: bool = False, stream=None):
    """Per-slot forest edges (fu, fv) (-1 = empty slot) and optional labels."""
    o = (options or Options()).to_c()
    dev = g.nbrs.device if g.nbrs is not None else torch.device("cuda")
    fu = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)[: g.n]
    fv = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)[: g.n]
    labels = torch.empty(max(g.n, 1), dtype=torch.int32, device=dev)[: g.n] if want_labels else None
    if workspace is None:
        workspace = alloc_workspace(workspace_size(g, options, forest=True, labels=want_labels))
    st = _Stats() if stats else None
    _check(lib().gconn_spanning_forest(ctypes.byref(g.c), _ptr(fu) if g.n else None,
                                       _ptr(fv) if g.n else None,
                                       _ptr(labels) if (labels is not None and g.n) else None,
                                       workspace.data_ptr(), workspace.numel(), ctypes.byref(o),
                                       ctypes.byref(st) if st else None, _stream(stream)))
    out = (fu, fv, labels)
    return (*out, _stats_dict(st)) if stats else out


class Incremental:
    """Handle over gconn_inc_*: batched edge insertion and connectivity queries."""

    def __init__(self, n_max: int, initial: DeviceGraph | None = None,
                 options: Options | None = None, device="cuda", stream=None):
        self.options = options or Options(sample="none")
        o = self.options.to_c()
        self.n_max = n_max
        self.parent = torch.empty(max(n_max, 1), dtype=torch.int32, device=device)
        b = ctypes.c_size_t(0)
        gp = ctypes.byref(initial.c) if initial is not None else None
        _check(lib().gconn_inc_workspace_size(n_max, gp, ctypes.byref(o), ctypes.byref(b)))
        self.workspace = alloc_workspace(b.value, device)
        self._initial = initial  # keep device buffers alive while the handle is
        h = ctypes.c_void_p()
        _check(lib().gconn_inc_create(n_max, self.parent.data_ptr(), gp, self.workspace.data_ptr(),
                                      self.workspace.numel(), ctypes.byref(o), _stream(stream),
                                      ctypes.byref(h)))
        self._h = h

    def insert(self, src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
        _check(lib().gconn_inc_insert_batch(self._h, _ptr(src), _ptr(dst), src.numel(),
                                            _stream(stream)))

    def query(self, a: torch.Tensor, b: torch.Tensor, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(max(a.numel(), 1), dtype=torch.uint8, device=a.device)[: a.numel()]
        _check(lib().gconn_inc_query_batch(self._h, _ptr(a), _ptr(b), a.numel(),
                                           _ptr(out) if a.numel() else None, _stream(stream)))
        return out

    def mixed(self, kind: torch.Tensor, a: torch.Tensor, b: torch.Tensor,
              out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Mixed batch: kind (uint8, 0 insert / 1 query); the batch's inserts are
        applied first, then out[i] = 1 iff query i's endpoints are connected."""
        if kind.dtype != torch.uint8:
            raise ValueError("kind must be uint8")
        if out is None:
            out = torch.empty(max(a.numel(), 1), dtype=torch.uint8, device=a.device)[: a.numel()]
        _check(lib().gconn_inc_mixed_batch(self._h, _ptr(kind), _ptr(a), _ptr(b), a.numel(),
                                           _ptr(out) if a.numel() else None, _stream(stream)))
        return out

    def labels(self, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        if out is None:
            out = torch.empty(max(self.n_max, 1), dtype=torch.int32, device=self.parent.device)[: self.n_max]
        _check(lib().gconn_inc_labels(self._h, _ptr(out) if self.n_max else None, _stream(stream)))
        return out

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().gconn_inc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def profile_enable(on: bool = True) -> None:
    """Per-phase HIP-event timing of the pipeline on this thread (see gconn.h)."""
    _check(lib().gconn_profile_enable(int(on)))


PHASES = ["init", "sample", "compress", "lmax", "gather", "finish", "finalize"]


def profile_phases(names) -> None:
    """Profile only the named phases (two HIP events per phase per run)."""
    mask = 0
    for nm in names:
        mask |= 1 << (PHASES.index(nm) + 1)
    _check(lib().gconn_profile_enable(mask))


def profile_read(reset: bool = True) -> dict:
    t = _PhaseTimes()
    _check(lib().gconn_profile_read(ctypes.byref(t), int(reset)))
    return {f: getattr(t, f) for f, _ in _PhaseTimes._fields_}


INSERT, QUERY = 0, 1


class Server:
    """Handle over gconn_server_*: a continuous-batching request loop over one
    resident parent array.  submit() takes host numpy arrays (kept referenced
    here until waited on); wait() returns the request record and, for queries,
    the answers."""

    def __init__(self, n_max: int, streams: int = 4, arena_bytes: int = 64 << 20,
                 options: Options | None = None, device="cuda"):
        cfg = _ServerConfig()
        cfg.n_max, cfg.streams, cfg.arena_bytes = n_max, streams, arena_bytes
        cfg.options = (options or Options(sample="none")).to_c()
        self.parent = torch.empty(n_max, dtype=torch.int32, device=device)
        self.arena = alloc_workspace(arena_bytes, device)
        h = ctypes.c_void_p()
        _check(lib().gconn_server_create(ctypes.byref(cfg), self.parent.data_ptr(),
                                         self.arena.data_ptr(), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, kind: int, a: np.ndarray, b: np.ndarray,
               out: np.ndarray | None = None) -> int:
        """a, b (and out, queries) stay referenced until wait(); arrays over
        pinned host memory (e.g. torch pin_memory tensors' .numpy()) are
        transferred without the server's staging copy."""
        a = np.ascontiguousarray(a, dtype=np.uint32)
        b = np.ascontiguousarray(b, dtype=np.uint32)
        if kind == QUERY and out is None:
            out = np.zeros(len(a), np.uint8)
        if out is not None and (out.dtype != np.uint8 or not out.flags.c_contiguous
                                or len(out) < len(a)):
            raise ValueError("out must be a contiguous uint8 array of len(a) entries")
        t = ctypes.c_uint64()
        _check(lib().gconn_server_submit(self._h, kind, a.ctypes.data if len(a) else None,
                                         b.ctypes.data if len(b) else None, len(a),
                                         out.ctypes.data if out is not None and len(a) else None,
                                         ctypes.byref(t)))
        self._keep[t.value] = (a, b, out)
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0):
        info = _RequestInfo()
        st = lib().gconn_server_wait(self._h, ticket, timeout, ctypes.byref(info))
        _check(st)
        a, b, out = self._keep.pop(ticket)
        rec = {f: getattr(info, f) for f, _ in _RequestInfo._fields_}
        return rec, out

    def drain(self) -> None:
        _check(lib().gconn_server_drain(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().gconn_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_u32(t: torch.Tensor) -> np.ndarray:
    """Device int32 tensor -> host uint32 array (bit pattern preserved)."""
    return t.detach().cpu().numpy().view(np.uint32)
