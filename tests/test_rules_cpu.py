"""The library's union-find rules (gconn_rules.hpp, gconn_jtb.hpp) compiled
for the host and run concurrently from many threads: labels equal the
oracle's, every parent points to a smaller id (Union-JTB: to a vertex above it
in the rank order), and exactly n - c links succeed, with compression writes
as CAS and as relaxed stores -- and with the rules' cached parent reads
returning stale values (a per-thread copy that models an XCD's incoherent
L2), which the memory-model argument of gconn_rules.hpp says is harmless."""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import graphgen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "rules_stress.hip")
BIN = os.path.join(ROOT, "_build", "tests", "rules_stress")
RULES = list(range(28))


@pytest.fixture(scope="module")
def harness():
    os.makedirs(os.path.dirname(BIN), exist_ok=True)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    tmp = f"{BIN}.{os.getpid()}"  # parallel workers each build, then rename
    subprocess.run([hipcc, "-O2", "-std=c++17", "-pthread", "--offload-arch=gfx950",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    SRC, "-o", tmp], check=True, capture_output=True)
    os.replace(tmp, BIN)
    return BIN


def _graphs():
    yield "star_max", 3000, np.array([[2999, v] for v in range(2999)], np.uint32)
    yield "path_desc", 2000, np.array([[i + 1, i] for i in range(1999)][::-1], np.uint32)
    perm = np.random.default_rng(5).permutation(3000).astype(np.uint32)
    path = np.stack([perm[:-1], perm[1:]], 1)
    yield "path_shuffled", 3000, path[np.random.default_rng(6).permutation(len(path))]
    s, d = graphgen.rmat_edges(13, 80000, 4)
    yield "rmat13", 1 << 13, np.stack([s, d], 1)
    s, d = graphgen.er_edges(20000, 30000, 5)
    yield "er", 20000, np.stack([s, d], 1)
    g = graphgen.grid2d(100, 80, 0.6, 6)
    src, dst = g.coo()
    yield "grid", g.n, np.stack([src, dst], 1)


@pytest.mark.parametrize("atomic_compress", [1, 0])
@pytest.mark.parametrize("rule", RULES)
def test_rules_concurrent_on_cpu(harness, tmp_path, rule, atomic_compress):
    for name, n, edges in _graphs():
        ef = tmp_path / f"{name}.bin"
        edges.astype(np.uint32).tofile(ef)
        want = oracle.cc_coo(n, edges[:, 0], edges[:, 1])
        c = int((want == np.arange(n, dtype=np.uint32)).sum())
        for threads in (2, 8, 32):
            out = tmp_path / "labels.bin"
            r = subprocess.run([harness, str(ef), str(n), str(rule), str(threads), str(out),
                                str(atomic_compress)],
                               capture_output=True, text=True, timeout=120)
            assert r.returncode == 0, (name, rule, threads, r.returncode)
            got = np.fromfile(out, np.uint32)
            assert np.array_equal(got, want), (name, rule, threads)
            assert int(r.stdout.strip()) == n - c, (name, rule, threads)


# Union-JTB keeps its own 64-bit reads; the 32-bit rules all read through ld()
STALE_RULES = [r for r in RULES if r not in (26, 27)]


@pytest.mark.parametrize("stale", [30, 90])
@pytest.mark.parametrize("rule", STALE_RULES)
def test_rules_with_stale_cached_reads(harness, tmp_path, rule, stale):
    for name, n, edges in _graphs():
        ef = tmp_path / f"{name}.bin"
        edges.astype(np.uint32).tofile(ef)
        want = oracle.cc_coo(n, edges[:, 0], edges[:, 1])
        c = int((want == np.arange(n, dtype=np.uint32)).sum())
        for threads in (4, 32):
            out = tmp_path / "labels.bin"
            r = subprocess.run([harness, str(ef), str(n), str(rule), str(threads), str(out),
                                "1", str(stale)],
                               capture_output=True, text=True, timeout=120)
            assert r.returncode == 0, (name, rule, threads, stale, r.returncode)
            got = np.fromfile(out, np.uint32)
            assert np.array_equal(got, want), (name, rule, threads, stale)
            assert int(r.stdout.strip()) == n - c, (name, rule, threads, stale)
