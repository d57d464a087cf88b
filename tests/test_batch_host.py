"""Host-side batch layout and graph classification (no GPU)."""
import numpy as np

import graphgen
from paper_2008_11839_amd import batch as B
from tests import graphs as tg


def test_concat_layout_is_global_and_64_aligned():
    gs = [tg.csr(1, []), graphgen.er(100, 300, 1), tg.csr(64, tg.path(64)), graphgen.rmat(7, 8, 2)]
    hb = B.concat(gs)
    assert hb.vbase.tolist() == [0, 64, 192, 256, 384]
    assert hb.n == 384 and hb.m == sum(g.m for g in gs)
    assert np.all(hb.vbase % 64 == 0)
    off = hb.offsets.astype(np.int64)
    assert off[0] == 0 and off[-1] == hb.m and np.all(np.diff(off) >= 0)
    for i, g in enumerate(gs):
        lo, hi = int(hb.vbase[i]), int(hb.vbase[i + 1])
        rows = off[lo:lo + g.n + 1] - off[lo]
        assert np.array_equal(rows, g.offsets.astype(np.int64))
        seg = hb.nbrs[off[lo]:off[lo + g.n]]
        assert np.array_equal(seg - lo, g.nbrs)              # global ids = local + base
        assert np.all((seg >= lo) & (seg < lo + g.n))
        assert np.all(np.diff(off[lo + g.n:hi + 1]) == 0)   # padding rows are empty


def test_graph_classes_from_statistics():
    assert B.graph_class_key(1500, 20000, 30) == "n1e3-sparse-flat"
    assert B.graph_class_key(150000, 150000 * 40, 5000) == "n1e5-dense-skewed"
    er = graphgen.er(20000, 200000, 1)
    rm = graphgen.rmat(15, 16, 1)
    k_er = B.graph_class_key(er.n, er.m, int(er.degrees().max()))
    k_rm = B.graph_class_key(rm.n, rm.m, int(rm.degrees().max()))
    assert k_er.endswith("flat") and k_rm.endswith("skewed")
