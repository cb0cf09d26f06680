"""Batched form (ann_graph_*, ann_autotune) through the C ABI.

A captured graph is replayed several times with the program's own eager work
and synchronisations between replays; every replay must equal the eager
ann_search result and the CPU oracle bit for bit.  Rewriting the query tensor
in place changes the next replay's results accordingly.  The autotuner's
choice never changes results.
"""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-batched]", *a, flush=True)


@pytest.fixture(scope="module")
def ann():
    from paper_2409_16576_amd import ann as A
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    A.lib()
    return A


@pytest.fixture(scope="module")
def setup(tmp_path_factory, orc, ann):
    d = tmp_path_factory.mktemp("batchidx")
    out = {}
    X = fx.mixture(61, 20000, 32, "u8", n_centres=16, hi=255)
    p, _ = fx.built(d, "u8b", X, "u8", nlist=64, M=8)
    out["u8"] = (orc.read_index(p), ann.Index(p, 0),
                 fx.mixture(62, 300, 32, "u8", n_centres=16, hi=255).astype(np.float32))
    X = fx.mixture(63, 15000, 64, "f32", n_centres=12)
    p, _ = fx.built(d, "f32b", X, "f32", nlist=48, M=16, R=3, eps=0.25)
    out["f32"] = (orc.read_index(p), ann.Index(p, 0),
                  fx.mixture(64, 200, 64, "f32", n_centres=12).astype(np.float32))
    yield out
    for _, g, _ in out.values():
        g.close()


@pytest.mark.parametrize("name", ["u8", "f32"])
def test_graph_replays_equal_eager_and_oracle(ann, setup, orc, name):
    ix, g, Qh = setup[name]
    rng = np.random.default_rng(5)
    npq = rng.integers(1, 25, size=len(Qh)).astype(np.int32)
    Q = torch.from_numpy(Qh).cuda()
    NP = torch.from_numpy(npq).cuda()
    k, n = 10, 300
    r = orc.search(ix, Qh, npq, k, n)
    e_ids, e_d = g.search(Q, NP, k, n)
    torch.cuda.synchronize()
    assert np.array_equal(e_ids.cpu().numpy(), r.ids) and np.array_equal(e_d.cpu().numpy(), r.dists)
    gr = ann.Graph(g, Q, NP, k, n)
    try:
        for rep in range(4):
            _say("replay", name, rep)
            gr.ids.fill_(-7)
            ids, d = gr.launch()
            torch.cuda.synchronize()
            assert np.array_equal(ids.cpu().numpy(), r.ids), rep
            assert np.array_equal(d.cpu().numpy(), r.dists), rep
            # the program's own eager work between replays
            g.search(Q[:17], 5, 3, 40)
            (Q * 2).sum().item()
            torch.cuda.synchronize()
        # new queries written in place: the next replay searches them
        Q2h = Qh[::-1].copy()
        gr.Q.copy_(torch.from_numpy(Q2h).cuda())
        ids, d = gr.launch()
        torch.cuda.synchronize()
        r2 = orc.search(ix, Q2h, npq, k, n)
        assert np.array_equal(ids.cpu().numpy(), r2.ids) and np.array_equal(d.cpu().numpy(), r2.dists)
    finally:
        gr.close()


def test_graph_over_several_chunks(ann, setup, orc):
    """More queries than one chunk (16384): the graph holds several chunks."""
    ix, g, Qh = setup["u8"]
    Qbig = np.tile(Qh, (56, 1))[:16500]
    Q = torch.from_numpy(Qbig).cuda()
    gr = ann.Graph(g, Q, 4, 10, 64)
    try:
        _say("multi-chunk graph", Qbig.shape)
        for _ in range(2):
            ids, d = gr.launch()
            torch.cuda.synchronize()
            r = orc.search(ix, Qbig, np.full(len(Qbig), 4, np.int32), 10, 64)
            assert np.array_equal(ids.cpu().numpy(), r.ids) and np.array_equal(d.cpu().numpy(), r.dists)
    finally:
        gr.close()


def test_autotune_keeps_results(ann, setup, orc):
    ix, g, Qh = setup["f32"]
    Q = torch.from_numpy(Qh).cuda()
    _say("autotune")
    res = ann.autotune(g, Q, 20, 10, 200, reps=1)
    try:
        assert res["tried"] >= 20 and res["ms"] > 0
        assert g.get_option(g.OPT_SCAN_TILE) == res["tile"]
        assert g.get_option(g.OPT_SCAN_SPLIT) == res["split"]
        ids, d = g.search(Q, 20, 10, 200)
        r = orc.search(ix, Qh, np.full(len(Qh), 20, np.int32), 10, 200)
        assert np.array_equal(ids.cpu().numpy(), r.ids) and np.array_equal(d.cpu().numpy(), r.dists)
    finally:
        g.set_option(g.OPT_SCAN_TILE, 65536)
        g.set_option(g.OPT_SCAN_SPLIT, 16)


def test_graph_errors(ann, setup):
    _, g, Qh = setup["u8"]
    Q = torch.from_numpy(Qh).cuda()
    with pytest.raises(ann.AnnError):
        ann.Graph(g, Q, 4, 10, 5)      # rerank_n < k
    with pytest.raises(ann.AnnError):
        ann.Graph(g, Q[:0], 4, 10, 64)  # empty batch
    with pytest.raises(ann.AnnError):
        ann.autotune(g, Q, 4, 10, 64, reps=0)


@pytest.fixture(scope="module")
def zipf(orc, ann):
    """A small copy of the skewed batched-form workload: unit-norm float32,
    Zipf(1.1) list sizes (one list holds a large share of the vectors),
    per-query nprobe drawn from U{8..128} (clamped to the 64 lists)."""
    from paper_2409_16576_amd import workloads
    w = workloads.scaled(workloads.ZIPF_F32_5M, n=40000, nlist=64, n_centres=16, nq=150)
    path = workloads.ensure_index(w)
    ix = orc.read_index(path)
    g = ann.Index(path, 0)
    yield ix, g, workloads.queries(w), workloads.nprobe_per_query(w)
    g.close()


@pytest.mark.parametrize("lut16", [0, 1])
def test_skewed_lists_split_graph_and_tuning(ann, zipf, orc, lut16):
    ix, g, Qh, npq = zipf
    sizes = np.diff(ix.offsets)
    assert sizes.max() > 8 * np.median(sizes)  # the skew the form is for
    Q = torch.from_numpy(Qh).cuda()
    NP = torch.from_numpy(npq).cuda()
    k, n = 10, 400
    r = orc.search(ix, Qh, npq, k, n, lut_f16=bool(lut16))
    g.set_option(g.OPT_LUT_F16, lut16)
    try:
        for tile, split in ((512, 16), (4096, 4), (1 << 30, 1)):
            _say("zipf", lut16, tile, split)
            g.set_option(g.OPT_SCAN_TILE, tile)
            g.set_option(g.OPT_SCAN_SPLIT, split)
            ids, d = g.search(Q, NP, k, n)
            assert np.array_equal(ids.cpu().numpy(), r.ids) and np.array_equal(d.cpu().numpy(), r.dists)
        ann.autotune(g, Q, NP, k, n, reps=1)
        gr = ann.Graph(g, Q, NP, k, n)
        try:
            for _ in range(3):
                ids, d = gr.launch()
                torch.cuda.synchronize()
                assert np.array_equal(ids.cpu().numpy(), r.ids)
                assert np.array_equal(d.cpu().numpy(), r.dists)
        finally:
            gr.close()
    finally:
        g.set_option(g.OPT_LUT_F16, 0)
        g.set_option(g.OPT_SCAN_TILE, 65536)
        g.set_option(g.OPT_SCAN_SPLIT, 16)
