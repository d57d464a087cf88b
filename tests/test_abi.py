"""The C ABI without a GPU: the library loads, exports every symbol the header
declares, and its host-side logic (defaults, workspace sizing, argument and
device checks) behaves as documented.  No compute call reaches a kernel."""
from __future__ import annotations

import ctypes
import os
import re
import subprocess

import pytest

from paper_2008_11839_amd import gconn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gconn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gconn_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_documented_entry_points():
    names = declared_functions()
    for required in ["gconn_cc", "gconn_spanning_forest", "gconn_inc_create",
                     "gconn_inc_insert_batch", "gconn_inc_query_batch", "gconn_inc_labels",
                     "gconn_inc_destroy", "gconn_workspace_size", "gconn_status_string"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = gconn.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", gconn.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (gconn_\w+)", out))
    assert set(declared_functions()) <= exported
    assert set(gconn.EXPORTS) <= exported


def test_header_compiles_as_plain_c(tmp_path):
    src = tmp_path / "use.c"
    src.write_text('#include "gconn.h"\nint main(void){gconn_options o; gconn_options_default(&o);'
                   'return o.k == 2 ? 0 : 1;}\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER),
                    "-c", str(src), "-o", str(tmp_path / "use.o")], check=True)


def test_defaults_and_status_strings():
    o = gconn._Options()
    gconn.lib().gconn_options_default(ctypes.byref(o))
    assert (o.sample, o.link, o.find, o.splice, o.k, o.hb_n, o.lmax_samples, o.block) == \
        (1, 0, 1, 0, 2, 4, 1024, 256)
    for code in gconn.STATUS:
        s = gconn.lib().gconn_status_string(code).decode()
        assert s.startswith(gconn.STATUS[code])
    assert gconn.lib().gconn_version().decode().startswith("gconn")


def _graph(n, m, fmt=0, o64=0):
    g = gconn._Graph()
    g.format, g.n, g.m, g.offsets_64 = fmt, n, m, o64
    return g


def _ws(g, **kw):
    o = gconn.Options(**kw).to_c()
    b = ctypes.c_size_t()
    st = gconn.lib().gconn_workspace_size(ctypes.byref(g), ctypes.byref(o), 0, 1, ctypes.byref(b))
    return st, b.value


def test_workspace_sizes_scale_with_the_plan():
    n, m = 1 << 20, 1 << 24
    st, base = _ws(_graph(n, m))
    assert st == 0
    assert base >= 4 * n + 8 * (m // 33)          # small list + segments
    st, hooks = _ws(_graph(n, m), link="hooks")
    assert hooks - base >= 4 * n
    st, sv = _ws(_graph(n, m), link="sv")
    assert sv - base >= 4 * n + 8 * m             # prev + materialised edges
    st, none = _ws(_graph(n, m), sample="none")
    st, bfs = _ws(_graph(n, m), sample="bfs")
    assert bfs - none >= 8 * n                    # two queues
    # the automatic k-out schedule keeps room for the local-first records
    # (two per vertex, both endpoints); the one-pass kernel alone needs none
    st, lane = _ws(_graph(n, m), schedule="lane")
    assert base - lane >= 16 * n
    st, coo = _ws(_graph(n, m, fmt=1))
    assert coo < 32768                            # COO union-find needs control only


def test_option_errors_are_reported_on_the_host():
    g = _graph(10, 20)
    o = gconn.Options().to_c()
    o.link = 99
    b = ctypes.c_size_t()
    assert gconn.lib().gconn_workspace_size(ctypes.byref(g), ctypes.byref(o), 0, 1, ctypes.byref(b)) == -1
    assert b"link" in gconn.lib().gconn_last_error()
    o = gconn.Options(link="rem_cas", find="compress").to_c()
    assert gconn.lib().gconn_workspace_size(ctypes.byref(g), ctypes.byref(o), 0, 1, ctypes.byref(b)) == -7
    o = gconn.Options(block=100).to_c()
    assert gconn.lib().gconn_workspace_size(ctypes.byref(g), ctypes.byref(o), 0, 1, ctypes.byref(b)) == -1


def test_forest_with_label_propagation_is_unsupported():
    g = _graph(10, 20)
    o = gconn.Options(link="lp").to_c()
    st = gconn.lib().gconn_spanning_forest(ctypes.byref(g), None, None, None, None, 0,
                                           ctypes.byref(o), None, None)
    assert st == -7


def test_incremental_rejects_non_union_find_rules():
    o = gconn.Options(link="sv").to_c()
    h = ctypes.c_void_p()
    st = gconn.lib().gconn_inc_create(10, None, None, None, 0, ctypes.byref(o), None,
                                      ctypes.byref(h))
    assert st == -7 and not h.value


def test_compute_without_a_gpu_fails_loudly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = _graph(10, 20)
    st = gconn.lib().gconn_cc(ctypes.byref(g), None, None, 0, None, None, None)
    assert st == -4  # GCONN_ENODEV: there is no CPU fallback
    h = ctypes.c_void_p()
    st = gconn.lib().gconn_inc_create(10, None, None, None, 0, None, None, ctypes.byref(h))
    assert st in (-4, -7)


def test_jtb_options_and_workspace():
    g = _graph(1000, 8000)
    b = ctypes.c_size_t()

    def status(**kw):
        o = gconn.Options(**kw).to_c()
        return gconn.lib().gconn_workspace_size(ctypes.byref(g), ctypes.byref(o), 0, 1,
                                                ctypes.byref(b))
    assert status(link="jtb", find="naive") == 0
    assert status(link="jtb", find="two_try_split", sample="kout") == 0
    assert status(link="jtb", find="two_try_split", sample="none") == 0
    for find in ("split", "halve", "compress"):
        assert status(link="jtb", find=find) == -7
    for sample in ("hb", "bfs"):
        assert status(link="jtb", find="naive", sample=sample) == -7
    assert status(link="async", find="two_try_split") == -7
    # the words (8 bytes per vertex) and the root array (4) are in the plan
    n, m = 1 << 20, 1 << 22
    st, base = _ws(_graph(n, m), link="async", schedule="lane")
    st2, jtb = _ws(_graph(n, m), link="jtb", find="naive")
    assert st == 0 and st2 == 0 and jtb - base >= 12 * n
    # the incremental handle keeps the words in its workspace
    o = gconn.Options(link="jtb", find="naive", sample="none").to_c()
    assert gconn.lib().gconn_inc_workspace_size(n, None, ctypes.byref(o), ctypes.byref(b)) == 0
    assert b.value >= 8 * n
