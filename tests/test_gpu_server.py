"""Served form (ann_server_*) through the C ABI.

Requests of uneven size and per-query nprobe are submitted from several
threads so that the scheduler coalesces them into shared launches on several
streams; every request's result must be bit-identical to the same request
searched alone (ann_search) and to the CPU oracle.  Also: admission under an
HBM budget that holds a single launch, statistics, and argument errors.
"""
import re
import threading

import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-server]", *a, flush=True)


@pytest.fixture(scope="module")
def ann():
    from paper_2409_16576_amd import ann as A
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    A.lib()
    return A


@pytest.fixture(scope="module")
def setup(tmp_path_factory, orc, ann):
    d = tmp_path_factory.mktemp("srvidx")
    X = fx.mixture(51, 20000, 32, "u8", n_centres=16, hi=255)
    p, _ = fx.built(d, "u8s", X, "u8", nlist=64, M=8)
    Q = fx.mixture(52, 600, 32, "u8", n_centres=16, hi=255).astype(np.float32)
    g = ann.Index(p, 0)
    yield orc.read_index(p), g, Q
    g.close()


def _requests(seed, Q, n_req, max_nq, kn=((10, 100),)):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        nq = int(rng.integers(1, max_nq + 1))
        rows = rng.integers(0, len(Q), size=nq)
        npq = rng.integers(1, 21, size=nq).astype(np.int32)
        k, n = kn[i % len(kn)]
        reqs.append((Q[rows], npq, k, n))
    return reqs


def _alone(g, q, npq, k, n):
    ids, d = g.search(torch.from_numpy(q).cuda(), torch.from_numpy(npq).cuda(), k, n)
    torch.cuda.synchronize()
    return ids.cpu().numpy(), d.cpu().numpy()


def _serve_all(srv, reqs, n_threads=4):
    out = [None] * len(reqs)
    tickets = [None] * len(reqs)

    def worker(t):
        for i in range(t, len(reqs), n_threads):
            q, npq, k, n = reqs[i]
            tickets[i] = srv.submit(q, npq, k, n)
    th = [threading.Thread(target=worker, args=(t,)) for t in range(n_threads)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for i, t in enumerate(tickets):
        out[i] = srv.poll(t, wait=True)
    return out


def test_results_same_alone_and_in_mix(ann, setup, orc):
    ix, g, Q = setup
    reqs = _requests(1, Q, 48, 40, kn=((10, 100), (10, 100), (5, 300)))
    _say("mix of", len(reqs), "requests")
    srv = ann.Server(g, max_slots=4, max_batch=96, max_nprobe=32, max_k=16, max_rerank_n=512)
    try:
        got = _serve_all(srv, reqs)
        st = srv.stats()
    finally:
        srv.stop()
    for (q, npq, k, n), (ids, d) in zip(reqs, got):
        a_ids, a_d = _alone(g, q, npq, k, n)
        assert np.array_equal(ids, a_ids) and np.array_equal(d, a_d)
        r = orc.search(ix, q, npq, k, n)
        assert np.array_equal(ids, r.ids) and np.array_equal(d, r.dists)
    assert st["requests_done"] == len(reqs)
    assert st["queries_done"] == sum(r[0].shape[0] for r in reqs)
    assert 1 <= st["launches"] <= len(reqs)
    assert st["launches"] < len(reqs), "waiting requests were never coalesced"
    assert st["max_in_flight"] >= 2, "launches never overlapped"
    assert 0 < st["peak_bytes"] <= st["budget_bytes"]
    assert 0 < st["latency_p50_ms"] <= st["latency_p99_ms"] <= st["latency_max_ms"]


def test_budget_of_one_launch(ann, setup, orc):
    """A budget that holds one launch of max_batch queries: admission waits for
    memory, results are unchanged, the peak never exceeds the budget."""
    ix, g, Q = setup
    with pytest.raises(ann.AnnError) as e:
        ann.Server(g, hbm_budget_bytes=4096, max_slots=4, max_batch=64, max_nprobe=32, max_k=16,
                   max_rerank_n=256)
    need = int(re.search(r"\((\d+) bytes\)", str(e.value)).group(1))
    _say("one launch needs", need, "bytes")
    srv = ann.Server(g, hbm_budget_bytes=need, max_slots=4, max_batch=64, max_nprobe=32,
                     max_k=16, max_rerank_n=256)
    reqs = _requests(2, Q, 30, 64, kn=((10, 256),))
    try:
        got = _serve_all(srv, reqs, n_threads=3)
        st = srv.stats(reset=True)
        assert srv.stats()["requests_done"] == 0
    finally:
        srv.stop()
    for (q, npq, k, n), (ids, d) in zip(reqs, got):
        r = orc.search(ix, q, npq, k, n)
        assert np.array_equal(ids, r.ids) and np.array_equal(d, r.dists)
    assert st["peak_bytes"] <= need
    assert st["requests_done"] == len(reqs)


def test_single_slot_and_sequential_use(ann, setup, orc):
    ix, g, Q = setup
    srv = ann.Server(g, max_slots=1, max_batch=32, max_nprobe=8, max_k=10, max_rerank_n=64)
    try:
        for i in range(5):
            q = Q[i * 7:i * 7 + 7]
            t = srv.submit(q, 8, 10, 64)
            ids, d = srv.poll(t, wait=True)
            r = orc.search(ix, q, np.full(len(q), 8, np.int32), 10, 64)
            assert np.array_equal(ids, r.ids) and np.array_equal(d, r.dists)
        assert srv.stats()["max_in_flight"] == 1
    finally:
        srv.stop()


def test_server_errors(ann, setup):
    _, g, Q = setup
    srv = ann.Server(g, max_slots=2, max_batch=16, max_nprobe=8, max_k=10, max_rerank_n=64)
    try:
        with pytest.raises(ann.AnnError):
            srv.submit(Q[:17], 4, 10, 64)        # more than max_batch
        with pytest.raises(ann.AnnError):
            srv.submit(Q[:4], 9, 10, 64)         # nprobe above the limit
        with pytest.raises(ann.AnnError):
            srv.submit(Q[:4], 4, 11, 64)         # k above the limit
        with pytest.raises(ann.AnnError):
            srv.submit(Q[:4], 4, 10, 5)          # rerank_n < k
        t = srv.submit(Q[:4], 4, 10, 64)
        assert srv.poll(t, wait=True) is not None
        with pytest.raises(ann.AnnError):
            srv.poll(t, wait=True)               # already collected
        with pytest.raises(ann.AnnError):
            srv.poll(12345, wait=False)          # never issued
    finally:
        srv.stop()
    with pytest.raises(ann.AnnError):
        ann.Server(g, max_slots=17)
    with pytest.raises(ann.AnnError):
        ann.Server(g, max_batch=10 ** 7)


def test_server_rejects_limits_beyond_the_scan_lds(ann, tmp_path):
    """Limits whose largest request would need more scan LDS than a block has
    are refused at start (an int8 index with 50 subspaces: its float32 table
    alone is 52 KiB; nprobe 4096 with rerank_n 4096 does not fit), instead of
    failing the server at the first such request; smaller limits start."""
    X = fx.mixture(53, 6000, 100, "i8", n_centres=8, lo=-128, hi=127)
    p, _ = fx.built(tmp_path, "i8s", X, "i8", nlist=40, M=50)
    g = ann.Index(p, 0)
    try:
        with pytest.raises(ann.AnnError):
            ann.Server(g, max_batch=16, max_nprobe=4096, max_k=10, max_rerank_n=4096)
        srv = ann.Server(g, max_batch=16, max_nprobe=64, max_k=10, max_rerank_n=400)
        try:
            Q = fx.mixture(54, 8, 100, "i8", n_centres=8, lo=-128, hi=127).astype(np.float32)
            t = srv.submit(Q, 16, 10, 400)
            assert srv.poll(t, wait=True) is not None
        finally:
            srv.stop()
    finally:
        g.close()
