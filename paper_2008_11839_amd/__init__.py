"""MI355X (gfx950) graph connectivity: HIP kernels behind the C ABI in
include/gconn.h, with a thin ctypes binding (``gconn``)."""
from . import gconn
from .gconn import (Options, DeviceGraph, Incremental, GconnError, csr, coo, cc,
                    spanning_forest, workspace_size, alloc_workspace, to_u32, EMPTY)

__all__ = ["gconn", "Options", "DeviceGraph", "Incremental", "GconnError", "csr", "coo", "cc",
           "spanning_forest", "workspace_size", "alloc_workspace", "to_u32", "EMPTY"]
