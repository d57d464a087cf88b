"""Build libgconn.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2008_11839_amd.build   (or build() from Python)
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgconn.so")
OBJDIR = os.path.join(ROOT, "_build", "gconn")
SOURCES = ["gconn_static.hip", "gconn_jtb.hip", "gconn_batch.hip", "gconn_server.hip",
           "gconn_api.hip", "gconn_diag.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"),
]


def _compile(src: str, defines=(), objdir: str = OBJDIR) -> str:
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC, *FLAGS, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-6000:]}")
    err = "\n".join(l for l in r.stderr.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if "warning" in err or "error" in err:
        sys.stderr.write(err + "\n")
    return obj


def build(verbose: bool = False, defines=(), out: str = LIB) -> str:
    """Compile every source and link `out` (the library; a diagnostic variant
    when `defines` are given, e.g. -DGCONN_COUNT_OPS=1 for the rules'
    operation counters)."""
    objdir = OBJDIR if not defines else os.path.join(ROOT, "_build", "gconn_variant")
    os.makedirs(objdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        objs = list(ex.map(lambda src: _compile(src, defines, objdir), SOURCES))
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-6000:]}")
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--op-counts", metavar="OUT.so",
                    help="build the diagnostic variant that counts the union-find rules' "
                         "parent reads, CASes and failed CASes (slow; counts only)")
    a = ap.parse_args()
    if a.op_counts:
        build(verbose=True, defines=("-DGCONN_COUNT_OPS=1",), out=os.path.abspath(a.op_counts))
    else:
        build(verbose=True)
