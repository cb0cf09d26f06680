"""Host-memory raw tier (Sec. 4.3) through the C ABI.

An index loaded with raw_tier 1 keeps its raw vectors on pages of pinned
host memory, bucketed by nearest list; re-ranking reads whole pages, one read
per page per query (merging inside a mini-batch, reuse across mini-batches).
IDs, distances, candidates re-ranked and pages read must equal the CPU
oracle's (its page layout and read count are pinned by the paper's worked
example), and the results must equal the same index kept in HBM.
"""
import json
import os

import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GOLD = os.path.join(os.path.dirname(__file__), "golden", "page_dedup_example.json")


def _say(*a):
    print("[gpu-pages]", *a, flush=True)


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def ann():
    from paper_2409_16576_amd import ann as A
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    A.lib()
    return A


@pytest.fixture(scope="module")
def setup(tmp_path_factory, orc, ann):
    d = tmp_path_factory.mktemp("pageidx")
    out = {}
    X = fx.mixture(101, 20000, 32, "u8", n_centres=16, hi=255)
    out["u8"] = (fx.built(d, "u8", X, "u8", nlist=64, M=8)[0],
                 fx.mixture(102, 120, 32, "u8", n_centres=16, hi=255))
    X = fx.mixture(103, 12000, 100, "i8", n_centres=10, lo=-128, hi=127)
    out["i8"] = (fx.built(d, "i8", X, "i8", nlist=40, M=50)[0],
                 fx.mixture(104, 90, 100, "i8", n_centres=10, lo=-128, hi=127))
    X = fx.mixture(105, 15000, 64, "f32", n_centres=12)
    out["f32"] = (fx.built(d, "f32", X, "f32", nlist=48, M=16, R=3, eps=0.25)[0],
                  fx.mixture(106, 80, 64, "f32", n_centres=12))
    res = {}
    for name, (p, Q) in out.items():
        res[name] = (orc.read_index(p), p, Q.astype(np.float32), ann.Index(p, 0))
    yield res
    for _, _, _, g in res.values():
        g.close()


@pytest.mark.parametrize("name", ["u8", "i8", "f32"])
@pytest.mark.parametrize("page_bytes", [256, 4096])
def test_pages_fixed_and_heuristic_equal_oracle(ann, setup, orc, name, page_bytes):
    ix, path, Qh, g_hbm = setup[name]
    row = ix.dim * (4 if ix.kind == "f32" else 1)
    if row > page_bytes:
        pytest.skip("a vector does not fit the page")
    g = ann.Index(path, 0, raw_tier=1, page_bytes=page_bytes)
    try:
        assert g.desc["raw_tier"] == 1 and g.desc["page_bytes"] == page_bytes
        lay = orc.index_page_layout(ix, page_bytes)
        assert g.desc["pages"] == lay.pages
        rng = np.random.default_rng(3)
        npq = rng.integers(1, 20, size=len(Qh)).astype(np.int32)
        Q, NP = _cuda(Qh), _cuda(npq)
        for k, n, heur in ((10, 100, None), (7, 600, None), (10, 400, (50, 0.0, 2)),
                           (10, 2048, (300, 0.05, 1)), (5, 64, (1, 0.0, 3))):
            _say(name, page_bytes, k, n, heur)
            bs, eps, beta = heur if heur else (0, 0.0, 1)
            ids, d, rr, pr = g.search_pages(Q, NP, k, n, bs, eps, beta)
            torch.cuda.synchronize()
            r = orc.search(ix, Qh, npq, k, n, heuristic=heur, pages=lay)
            assert np.array_equal(ids.cpu().numpy(), r.ids), (k, n, heur)
            assert np.array_equal(d.cpu().numpy(), r.dists), (k, n, heur)
            assert np.array_equal(rr.cpu().numpy().astype(np.int64), r.reranked), (k, n, heur)
            assert np.array_equal(pr.cpu().numpy().astype(np.int64), r.page_reads), (k, n, heur)
            # the same results as the index kept in HBM
            if heur:
                h_ids, h_d, _ = g_hbm.search_heuristic(Q, NP, k, n, *heur)
            else:
                h_ids, h_d = g_hbm.search(Q, NP, k, n)
            torch.cuda.synchronize()
            assert torch.equal(ids, h_ids) and torch.equal(d.view(torch.int32), h_d.view(torch.int32))
        # ann_search / ann_search_heuristic on the host tier: same as HBM
        ids, d = g.search(Q, NP, 10, 300)
        h_ids, h_d = g_hbm.search(Q, NP, 10, 300)
        torch.cuda.synchronize()
        assert torch.equal(ids, h_ids) and torch.equal(d.view(torch.int32), h_d.view(torch.int32))
    finally:
        g.close()


def test_paper_worked_example_on_gpu(ann, orc, tmp_path):
    """The paper's example (Sec. 4.3): mini-batch 0 re-ranks V2, V4, V6 and
    reads P0 and P2 (V2 and V6 share P0); mini-batch 1 re-ranks V5, V8, V9,
    finds P2 in the buffer and reads P1 and P3.  Here with 64-dimensional
    uint8 vectors on 128-byte pages (two per page) and a codebook that decodes
    every vector exactly (subspace 0 holds the value of dimension 0)."""
    g = json.load(open(GOLD))
    dim = 64
    a = np.array(g["a"])
    X = np.zeros((10, dim), dtype=np.uint8)
    X[:, 0] = a
    M = 16
    cb = np.zeros((M, 256, 4), dtype=np.float32)
    cb[0, :, 0] = np.arange(256)
    codes = np.zeros((10, M), dtype=np.uint8)
    codes[:, 0] = a
    cent = np.zeros((5, dim), dtype=np.float32)
    cent[:, 0] = [2, 6, 3, 8, 9]
    assign = np.stack([np.array(g["bucket"]), -np.ones(10, dtype=np.int64)], axis=1)
    p, _ = fx.write_arrays(tmp_path, "example", "u8", cent, cb, codes, X, assign)
    ix = orc.read_index(p)
    lay = orc.index_page_layout(ix, 128)
    for name, pg in g["expect"]["page_of"].items():
        assert lay.page[int(name[1:])] == pg, name
    e = g["expect"]
    gi = ann.Index(p, 0, raw_tier=1, page_bytes=128)
    try:
        q = torch.zeros((1, dim), dtype=torch.float32, device="cuda")
        bs = e["minibatch_size"]
        ids, d, rr, pr = gi.search_pages(q, 5, 3, 6)  # fixed re-rank of the six tasks
        torch.cuda.synchronize()
        assert int(pr[0]) == e["reads_fixed_rerank_of_6"] and int(rr[0]) == 6
        assert ids[0].tolist() == e["tasks"][:3]
        ids, d, rr, pr = gi.search_pages(q, 5, 3, 6, bs, 0.0, 100)  # both mini-batches
        torch.cuda.synchronize()
        assert int(rr[0]) == 6
        assert int(pr[0]) == e["reads_minibatch_0"] + e["reads_minibatch_1"]
        ids, d, rr, pr = gi.search_pages(q, 5, 3, 6, bs, 1.0, 1)  # stops after mini-batch 0
        torch.cuda.synchronize()
        assert int(rr[0]) == 3 and int(pr[0]) == e["reads_minibatch_0"]
    finally:
        gi.close()


def test_pages_errors(ann, setup):
    ix, path, Qh, g_hbm = setup["u8"]
    Q = _cuda(Qh[:4])
    with pytest.raises(Exception):
        g_hbm.search_pages(Q, 4, 10, 100)  # raw vectors in HBM: no pages
    g = ann.Index(path, 0, raw_tier=1, page_bytes=4096)
    try:
        with pytest.raises(Exception):
            g.search_pages(Q, 4, 10, 4096)  # rerank_n above 2048
        with pytest.raises(Exception):
            g.rerank(Q, torch.zeros((4, 20), dtype=torch.int32, device="cuda"), 10)
    finally:
        g.close()
    with pytest.raises(Exception):
        ann.Index(path, 0, raw_tier=1, page_bytes=16)  # a 32-byte vector exceeds the page
