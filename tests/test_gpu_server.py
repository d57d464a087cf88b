"""GPU tests of the serving loop: every query batch's answers equal the
oracle's for exactly the inserts submitted before it, whether the requests
run one at a time or mixed and overlapping, under an in-flight budget far
smaller than the offered work, with several client threads."""
from __future__ import annotations

import sys
import threading
import time

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _stream(n, seed, batches=40):
    """Seeded request list: (kind, a, b); batch sizes log-uniform 1..20000."""
    src, dst = graphgen.rmat_edges(15, 150_000, seed, n=n)
    graphgen.shuffle_edges(src, dst, seed)
    rng = np.random.default_rng(seed)
    reqs, e = [], 0
    while e < len(src) and len(reqs) < batches:
        if rng.random() < 0.5:
            k = int(10 ** rng.uniform(0, 4.3))
            reqs.append((0, src[e:e + k].copy(), dst[e:e + k].copy()))
            e += k
        else:
            a, b = graphgen.uniform_pairs(n, int(rng.integers(1, 3000)), seed, len(reqs))
            # also ask about endpoints of edges inserted so far, and of later ones
            j = rng.integers(0, len(src), size=200)
            a = np.concatenate([a, src[j]])
            b = np.concatenate([b, dst[j]])
            reqs.append((1, a, b))
    return reqs


def _oracle_answers(n, reqs):
    uf = oracle.UnionFind(n)
    ans = []
    for kind, a, b in reqs:
        if kind == 0:
            uf.insert(a, b)
            ans.append(None)
        else:
            ans.append(uf.query(a, b))
    return ans


@pytest.mark.parametrize("link,find", [("async", "split"), ("rem_cas", "split"),
                                       ("early", "halve"), ("ecl", "halve")])
def test_server_mixed_equals_alone_equals_oracle(gpu_available, link, find):
    from paper_2008_11839_amd import gconn as G
    n = 20000
    reqs = _stream(n, 11)
    want = _oracle_answers(n, reqs)
    opts = G.Options(sample="none", link=link, find=find)
    # alone: one request at a time, each waited for before the next
    srv = G.Server(n, streams=1, arena_bytes=1 << 20, options=opts)
    alone = []
    for kind, a, b in reqs:
        rec, out = srv.wait(srv.submit(kind, a, b))
        assert rec["status"] == 0
        alone.append(out)
    srv.close()
    # mixed: all submitted at once, four streams, a budget of ~3 requests
    srv = G.Server(n, streams=4, arena_bytes=600 << 10, options=opts)
    tickets = [srv.submit(kind, a, b) for kind, a, b in reqs]
    mixed, epochs, overlapped = [], [], 0
    recs = []
    for t in tickets:
        rec, out = srv.wait(t, timeout=60.0)
        assert rec["status"] == 0
        mixed.append(out)
        recs.append(rec)
    srv.close()
    for i, (kind, a, b) in enumerate(reqs):
        if kind == 1:
            assert np.array_equal(alone[i], want[i]), (link, i)
            assert np.array_equal(mixed[i], want[i]), (link, i)
    # epochs follow kind changes in submission order
    kinds = [k for k, _, _ in reqs]
    expect_epoch, e = [], 0
    for i, k in enumerate(kinds):
        if i == 0 or k != kinds[i - 1]:
            e += 1
        expect_epoch.append(e)
    assert [r["epoch"] for r in recs] == expect_epoch
    # admission happened while earlier requests were still running
    for i in range(1, len(recs)):
        if recs[i]["admit_us"] < recs[i - 1]["done_us"]:
            overlapped += 1
    say(f"[server] link={link} requests={len(reqs)} overlapped_admissions={overlapped}")
    assert overlapped > 0


def test_server_multithreaded_clients_total_order(gpu_available):
    """Requests from several threads: the server orders them by submission;
    replaying the recorded order through the oracle gives every answer."""
    from paper_2008_11839_amd import gconn as G
    n = 5000
    srv = G.Server(n, streams=4, arena_bytes=256 << 10, options=G.Options(sample="none"))
    lock = threading.Lock()
    log = []  # (ticket, kind, a, b)

    def client(seed):
        reqs = _stream(n, seed, batches=25)
        for kind, a, b in reqs:
            with lock:  # record the submission order as the server sees it
                t = srv.submit(kind, a, b)
                log.append((t, kind, a, b))
            time.sleep(0.0005 * (seed % 3))

    threads = [threading.Thread(target=client, args=(s,)) for s in (21, 22, 23)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    got = {}
    for t, kind, a, b in log:
        rec, out = srv.wait(t, timeout=60.0)
        assert rec["status"] == 0
        got[t] = out
    srv.close()
    log.sort(key=lambda r: r[0])
    want = _oracle_answers(n, [(k, a, b) for _, k, a, b in log])
    for (t, kind, a, b), w in zip(log, want):
        if kind == 1:
            assert np.array_equal(got[t], w)


def test_server_rejects_oversized_and_bad_requests(gpu_available):
    from paper_2008_11839_amd import gconn as G
    srv = G.Server(100, streams=2, arena_bytes=4096, options=G.Options(sample="none"))
    with pytest.raises(G.GconnError):
        srv.submit(0, np.zeros(1000, np.uint32), np.zeros(1000, np.uint32))  # 8000 B > arena
    t = srv.submit(0, np.array([1, 2], np.uint32), np.array([2, 3], np.uint32))
    rec, _ = srv.wait(t)
    rec, out = srv.wait(srv.submit(1, np.array([1, 1], np.uint32), np.array([3, 4], np.uint32)))
    assert out.tolist() == [1, 0]
    srv.close()
    with pytest.raises(G.GconnError):
        G.Server(100, options=G.Options(sample="none", link="sv"))


def test_server_pinned_buffers_skip_staging(gpu_available):
    """Requests whose buffers are pinned host memory (read and written by the
    copy engines directly) mixed with pageable ones: every answer equals the
    oracle's, run alone and overlapped."""
    import torch
    from paper_2008_11839_amd import gconn as G

    def pinned(x, dtype):
        t = torch.empty(max(len(x), 1), dtype=dtype, pin_memory=True)
        arr = t.numpy()[: len(x)]
        arr[:] = x.view(arr.dtype) if x.dtype != arr.dtype else x
        return t, arr

    n = 20000
    reqs = _stream(n, 13)
    want = _oracle_answers(n, reqs)
    keep, staged = [], []
    for i, (kind, a, b) in enumerate(reqs):
        if i % 3 == 2:  # every third request stays pageable
            staged.append((kind, a, b, None))
            continue
        ta, pa = pinned(a, torch.int32)
        tb, pb = pinned(b, torch.int32)
        out = None
        if kind == 1:
            to, out = pinned(np.zeros(len(a), np.uint8), torch.uint8)
            keep.append(to)
        keep += [ta, tb]
        staged.append((kind, pa.view(np.uint32), pb.view(np.uint32), out))
    for streams, arena in ((1, 1 << 20), (4, 600 << 10)):
        say(f"[server-pinned] streams={streams} arena={arena}")
        srv = G.Server(n, streams=streams, arena_bytes=arena,
                       options=G.Options(sample="none", link="async", find="split"))
        tickets = [srv.submit(k, a, b, out) for k, a, b, out in staged]
        for i, t in enumerate(tickets):
            rec, out = srv.wait(t, timeout=60.0)
            assert rec["status"] == 0
            if reqs[i][0] == 1:
                assert np.array_equal(out, want[i]), (streams, i)
        srv.close()


def test_server_rejects_out_of_range_ids(gpu_available):
    """A request holding a vertex id >= n_max is refused at submission
    (GCONN_EINVAL) and never reaches the device; the server keeps serving the
    other requests, whose answers equal the oracle's.  The bad id is planted
    at the start, the middle and the end of a request large enough for the
    threaded scan."""
    from paper_2008_11839_amd import gconn as G

    n = 5000
    srv = G.Server(n, streams=2, arena_bytes=64 << 20,
                   options=G.Options(sample="none", link="rem_cas", find="split"))
    rng = np.random.default_rng(3)
    big = 3 << 20
    for kind in (G.INSERT, G.QUERY):
        for where in (0, big // 2, big - 1):
            a = rng.integers(0, n, size=big).astype(np.uint32)
            b = rng.integers(0, n, size=big).astype(np.uint32)
            (a if where % 2 == 0 else b)[where] = n  # one id just out of range
            say(f"[server-ids] kind={kind} bad at {where}")
            with pytest.raises(G.GconnError) as e:
                srv.submit(kind, a, b)
            assert e.value.status == -1  # GCONN_EINVAL
        with pytest.raises(G.GconnError):
            srv.submit(kind, np.array([0xFFFFFFFF], np.uint32), np.array([0], np.uint32))
    # the server still works: a path over the first 100 ids, then queries
    src = np.arange(0, 99, dtype=np.uint32)
    dst = src + 1
    t = srv.submit(G.INSERT, src, dst)
    rec, _ = srv.wait(t, timeout=60.0)
    assert rec["status"] == 0
    qa = np.array([0, 0, 5, 100, 4999], np.uint32)
    qb = np.array([99, 100, 50, 101, 0], np.uint32)
    t = srv.submit(G.QUERY, qa, qb)
    rec, out = srv.wait(t, timeout=60.0)
    assert rec["status"] == 0
    assert out.tolist() == [1, 0, 1, 0, 0]
    srv.close()
