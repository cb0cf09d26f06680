"""Pins of the oracle's raw-vector pages (Sec. 4.3): the page layout rule and
the page reads of re-ranking with intra- and inter-mini-batch de-duplication.

The paper's worked example (two mini-batches reading 2 pages each) is the
golden fixture; the rest are invariants any correct layout and count must
satisfy, each chosen so that a plausible slip (no merging inside a mini-batch,
no buffer across mini-batches, a tail split over two pages, a page overfilled)
fails one of them."""
import json
import os

import numpy as np
import pytest

from tests import fixtures as fx

GOLD = os.path.join(os.path.dirname(__file__), "golden", "page_dedup_example.json")


def _example_index(tmp_path):
    g = json.load(open(GOLD))
    dim = g["dim"]
    X = np.zeros((10, dim), dtype=np.uint8)
    X[:, 0] = g["a"]
    cb = np.tile(np.arange(256, dtype=np.float32).reshape(1, 256, 1), (dim, 1, 1))
    cent = np.zeros((5, dim), dtype=np.float32)
    cent[:, 0] = [2, 6, 3, 8, 9]
    assign = np.stack([np.array(g["bucket"]), -np.ones(10, dtype=np.int64)], axis=1)
    p, _ = fx.write_arrays(tmp_path, "pages", "u8", cent, cb, X.copy(), X, assign)
    return g, p


def test_paper_worked_example(orc, tmp_path):
    g, p = _example_index(tmp_path)
    ix = orc.read_index(p)
    lay = orc.index_page_layout(ix, g["page_bytes"])
    assert lay.per_page == 2 and lay.pages == 5
    for name, pg in g["expect"]["page_of"].items():
        assert lay.page[int(name[1:])] == pg, name
    e = g["expect"]
    q = np.zeros((1, g["dim"]), dtype=np.float32)
    # fixed re-rank of the six tasks: one mini-batch, P0 and P2 merged
    r = orc.search(ix, q, 5, 3, 6, pages=lay)
    assert list(r.topn_ids[0]) == e["tasks"]
    assert r.page_reads[0] == e["reads_fixed_rerank_of_6"]
    # Alg. 1 with mini-batches of 3 that never stops early: both mini-batches
    bs = e["minibatch_size"]
    r = orc.search(ix, q, 5, 3, 6, heuristic=(bs, 0.0, 100), pages=lay)
    assert r.reranked[0] == 6
    assert r.page_reads[0] == e["reads_minibatch_0"] + e["reads_minibatch_1"]
    # ... and one that stops after mini-batch 0 (every ID changed: rate 1 <= eps 1)
    r = orc.search(ix, q, 5, 3, 6, heuristic=(bs, 1.0, 1), pages=lay)
    assert r.reranked[0] == 3
    assert r.page_reads[0] == e["reads_minibatch_0"]


def test_layout_packs_tails_largest_first(orc):
    """Hand-worked: 10 vectors per page; buckets of 27, 15, 4, 3, 11 vectors
    have 2, 1, 0, 0, 1 full pages and tails 7, 5, 4, 3, 1.  The tail pages
    take 7 then the largest that fits (3), then 5 then 4 then 1."""
    sizes = [27, 15, 4, 3, 11]
    b = np.repeat(np.arange(5), sizes).astype(np.int32)
    lay = orc.page_layout(b, 5, row_bytes=100, page_bytes=1000)
    assert lay.per_page == 10 and lay.pages == 4 + 2
    start = np.concatenate([[0], np.cumsum(sizes)])
    members = [np.arange(start[i], start[i + 1]) for i in range(5)]
    # full pages: bucket 0 on pages 0-1, bucket 1 on page 2, bucket 4 on page 3, in ID order
    assert list(lay.page[members[0][:20]]) == [0] * 10 + [1] * 10
    assert list(lay.slot[members[0][:20]]) == list(range(10)) * 2
    assert (lay.page[members[1][:10]] == 2).all() and (lay.page[members[4][:10]] == 3).all()
    # tails: page 4 = bucket 0's 7 + bucket 3's 3; page 5 = bucket 1's 5 + bucket 2's 4 + bucket 4's 1
    assert (lay.page[members[0][20:]] == 4).all() and (lay.page[members[3]] == 4).all()
    assert (lay.page[members[1][10:]] == 5).all() and (lay.page[members[2]] == 5).all()
    assert (lay.page[members[4][10:]] == 5).all()
    assert list(lay.slot[members[0][20:]]) == list(range(7))
    assert list(lay.slot[members[3]]) == [7, 8, 9]


@pytest.mark.parametrize("seed,row,page", [(1, 100, 4096), (2, 384, 4096), (3, 128, 4096),
                                           (4, 1000, 4096)])
def test_layout_invariants(orc, seed, row, page):
    rng = np.random.default_rng(seed)
    nb = 300
    sizes = rng.integers(0, 200, size=nb)
    b = np.repeat(np.arange(nb), sizes).astype(np.int32)
    rng.shuffle(b)  # bucket membership is by ID, not position
    lay = orc.page_layout(b, nb, row, page)
    P = page // row
    n = len(b)
    assert lay.per_page == P
    assert (lay.slot >= 0).all() and (lay.slot < P).all()
    assert (lay.page >= 0).all() and (lay.page < lay.pages).all()
    where = lay.page.astype(np.int64) * P + lay.slot
    assert len(np.unique(where)) == n  # no slot holds two vectors
    full = int((sizes // P).sum())
    tails = sizes % P
    assert lay.pages >= full + int(np.ceil(tails.sum() / P))
    assert lay.pages <= full + int((tails > 0).sum())
    for i in range(nb):
        m = np.flatnonzero(b == i)
        if len(m) == 0:
            continue
        nfull = len(m) // P * P
        # the bucket's full pages hold its lowest IDs in order; its tail is on one page
        assert (np.diff(where[m[:nfull]]) == 1).all() if nfull > 1 else True
        assert len(np.unique(lay.page[m[nfull:]])) <= 1
        if nfull and len(m) > nfull:
            assert lay.page[m[nfull]] >= full  # tails live after all full pages


def test_page_reads_are_distinct_pages_of_reranked(orc, tmp_path):
    """With a per-query buffer that keeps every page read, a query's reads are
    the distinct pages of the candidates it re-ranked, however the mini-batches
    fall (fixed re-rank and Alg. 1 alike); and never more than the candidates."""
    X = fx.mixture(31, 6000, 32, "u8", n_centres=12, hi=255)
    p, _ = fx.built(tmp_path, "pg", X, "u8", nlist=64, M=8)
    ix = orc.read_index(p)
    lay = orc.index_page_layout(ix, 4096)
    Q = fx.mixture(32, 40, 32, "u8", n_centres=12, hi=255).astype(np.float32)
    for heur in (None, (25, 0.0, 2), (10, 0.1, 1)):
        r = orc.search(ix, Q, 8, 10, 200, heuristic=heur, pages=lay)
        for i in range(len(Q)):
            used = int(r.reranked[i])
            ids = r.topn_ids[i][:used]
            assert r.page_reads[i] == len(set(lay.page[ids].tolist()))
            assert r.page_reads[i] <= used
        assert (r.page_reads < r.reranked).any()  # candidates do share pages
