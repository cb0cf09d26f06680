"""List-major batched search (ANN_OPT_LIST_MAJOR) through the C ABI.

The batched form inverts a chunk's (query, probed list) pairs into per-list
query groups and scores each list's code rows once per group -- on the int8
matrix cores for integer-grid indexes, by interleaved LDS tables (float32 or
binary16) for float indexes -- leaving the replica entries, short lists and a
few leading lists per query to the per-query scan.  Every result -- final IDs and
distances, the top-n with its Eq. 1 values, the candidate counts, the
heuristic re-ranking -- must equal the plain per-query form's and the CPU
oracle's bit for bit, whatever the tuning (alpha, rows per work item, number
of persistent blocks), including queries whose list-major output overflows
and falls back to the per-query scan, groups split over several row tiles,
lists probed by more than 16 queries, nprobe 0 and nprobe > nlist.
"""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

OPT_LIST_MAJOR, OPT_LM_ALPHA, OPT_LM_TILE, OPT_LM_BLOCKS, OPT_LM_CAP = 5, 6, 7, 8, 9
OPT_LUT_F16, OPT_LM_MIN_ROWS = 3, 10


def _say(*a):
    print("[gpu-lmajor]", *a, flush=True)


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
    """Integer-grid indexes covering every supported subspace width (dsub 1,
    2, 4, 8) and K-chunk count (dim_pad 64, 128, 256), and a uniform-data index
    whose weak thresholds overflow the list-major output."""
    d = tmp_path_factory.mktemp("lmidx")
    out = {}

    def add(name, path, Q):
        out[name] = (orc.read_index(path), ann.Index(path, 0), Q.astype(np.float32))

    # uint8, dsub 4, dim_pad 64; 64 lists, 600 queries: ~100+ queries per list
    X = fx.mixture(81, 20000, 32, "u8", n_centres=16, hi=255)
    add("u8d4", fx.built(d, "u8d4", X, "u8", nlist=64, M=8)[0],
        fx.mixture(82, 600, 32, "u8", n_centres=16, hi=255))
    # int8, dsub 2, M = 50 (52-byte rows), dim 100 -> dim_pad 128
    X = fx.mixture(83, 12000, 100, "i8", n_centres=10, lo=-128, hi=127)
    add("i8d2", fx.built(d, "i8d2", X, "i8", nlist=40, M=50)[0],
        fx.mixture(84, 300, 100, "i8", n_centres=10, lo=-128, hi=127))
    # uint8, dsub 8, dim 64, R = 3 (rank-2 replica entries)
    X = fx.mixture(85, 15000, 64, "u8", n_centres=12, hi=255)
    add("u8d8", fx.built(d, "u8d8", X, "u8", nlist=48, M=8, R=3, eps=0.25)[0],
        fx.mixture(86, 250, 64, "u8", n_centres=12, hi=255))
    # uint8, dim 200 (dim_pad 256: four K chunks), dsub 4
    X = fx.mixture(87, 8000, 200, "u8", n_centres=8, hi=255)
    add("u8k4", fx.built(d, "u8k4", X, "u8", nlist=32, M=50)[0],
        fx.mixture(88, 200, 200, "u8", n_centres=8, hi=255))
    # lossless uint8 (dsub 1: every byte a codeword)
    p, _ = fx.lossless_u8(d, "lossless", n=3000, dim=16, nlist=8)
    rng = np.random.default_rng(89)
    add("u8d1", p, rng.integers(0, 256, size=(150, 16)))
    # uniform uint8 data: the leading list's n-th distance is a weak bound
    rng = np.random.default_rng(90)
    X = rng.integers(0, 256, size=(40000, 16)).astype(np.uint8)
    add("uniform", fx.built(d, "uniform", X, "u8", nlist=16, M=4)[0],
        rng.integers(0, 256, size=(64, 16)))
    yield out
    for _, g, _ in out.values():
        g.close()


def _set_lm(g, on, alpha=2, tile=4096, blocks=0):
    g.set_option(OPT_LIST_MAJOR, 1 if on else 0)
    g.set_option(OPT_LM_ALPHA, alpha)
    g.set_option(OPT_LM_TILE, tile)
    g.set_option(OPT_LM_BLOCKS, blocks)


NAMES = ["u8d4", "i8d2", "u8d8", "u8k4", "u8d1"]
TUNINGS = [(2, 4096, 0), (1, 64, 0), (8, 256, 7), (64, 4096, 1)]


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("tuning", TUNINGS)
def test_list_major_search_equals_plain_and_oracle(setup, orc, name, tuning):
    ix, g, Qh = setup[name]
    rng = np.random.default_rng(7)
    npq = rng.integers(0, min(ix.nlist, 24) + 1, size=len(Qh)).astype(np.int32)
    npq[:3] = (0, ix.nlist, ix.nlist)
    npmax = int(npq.max())
    Q, NP = _cuda(Qh), _cuda(npq)
    for k, n in ((10, 100), (7, 333), (10, 1400)):
        _set_lm(g, False)
        p_ids, p_d = g.search(Q, NP, k, n)
        _set_lm(g, True, *tuning)
        _say(name, tuning, k, n)
        l_ids, l_d = g.search(Q, NP, k, n)
        torch.cuda.synchronize()
        _set_lm(g, False)
        r = orc.search(ix, Qh, np.minimum(npq, npmax), k, n)
        assert np.array_equal(l_ids.cpu().numpy(), r.ids), (k, n)
        assert np.array_equal(l_d.cpu().numpy(), r.dists), (k, n)
        assert torch.equal(l_ids, p_ids)
        assert torch.equal(l_d.view(torch.int32), p_d.view(torch.int32))


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("n", [10, 257, 4096])
def test_list_major_topn_and_counts(setup, orc, name, n):
    """Top-n IDs with their Eq. 1 values, and the candidates scored per query."""
    ix, g, Qh = setup[name]
    _set_lm(g, True, 2, 512, 0)
    _say("topn", name, n)
    ids, adc, nc, nw = g.search_topn(_cuda(Qh), 13, n, walked=True)
    torch.cuda.synchronize()
    _set_lm(g, False)
    _, _, pnc, pnw = g.search_topn(_cuda(Qh), 13, n, walked=True)
    torch.cuda.synchronize()
    r = orc.search(ix, Qh, 13, 1, n)
    assert np.array_equal(ids.cpu().numpy(), r.topn_ids)
    assert np.array_equal(adc.cpu().numpy(), r.topn_adc)
    assert np.array_equal(nc.cpu().numpy(), r.ncand)
    assert torch.equal(nw, pnw)  # entries walked: the same entries, split two ways


@pytest.mark.parametrize("name", ["u8d4", "i8d2", "uniform"])
@pytest.mark.parametrize("cap", [1, 64, 700])
def test_list_major_overflow_falls_back(setup, orc, name, cap):
    """A small list-major capacity (ANN_OPT_LM_CAP) makes some or all queries
    overflow; those are searched again by the per-query scan: same results.
    (Uniform data: the leading list's n-th key is a weak bound.)"""
    ix, g, Qh = setup[name]
    Q = _cuda(Qh)
    for n in (10, 200):
        _set_lm(g, True, 1, 4096, 0)
        g.set_option(OPT_LM_CAP, cap)
        _say("overflow", name, cap, n)
        ids, d = g.search(Q, 16, 10, n)
        torch.cuda.synchronize()
        g.set_option(OPT_LM_CAP, 0)
        _set_lm(g, False)
        r = orc.search(ix, Qh, 16, 10, n)
        assert np.array_equal(ids.cpu().numpy(), r.ids)
        assert np.array_equal(d.cpu().numpy(), r.dists)


@pytest.mark.parametrize("name", ["u8d4", "i8d2"])
def test_list_major_graph_and_heuristic(ann, setup, orc, name):
    """Graphs created with the list-major option replay the list-major search
    (replays interleaved with eager work); the heuristic re-ranking on top of
    it is unchanged."""
    ix, g, Qh = setup[name]
    rng = np.random.default_rng(11)
    npq = rng.integers(1, 20, size=len(Qh)).astype(np.int32)
    Q, NP = _cuda(Qh), _cuda(npq)
    k, n = 10, 300
    r = orc.search(ix, Qh, npq, k, n)
    _set_lm(g, True, 2, 256, 0)
    gr = ann.Graph(g, Q, NP, k, n)
    try:
        for rep in range(3):
            _say("graph replay", name, rep)
            ids, d = gr.launch()
            torch.cuda.synchronize()
            assert np.array_equal(ids.cpu().numpy(), r.ids), rep
            assert np.array_equal(d.cpu().numpy(), r.dists), rep
            e_ids, _ = g.search(Q[:50], 5, k, n)  # eager work between replays
            torch.cuda.synchronize()
    finally:
        gr.close()
    h_ids, h_d, h_rr = g.search_heuristic(Q, NP, k, 400, 50, 0.0, 2)
    torch.cuda.synchronize()
    _set_lm(g, False)
    rh = orc.search(ix, Qh, npq, k, 400, heuristic=(50, 0.0, 2))
    assert np.array_equal(h_ids.cpu().numpy(), rh.ids)
    assert np.array_equal(h_d.cpu().numpy(), rh.dists)
    assert np.array_equal(h_rr.cpu().numpy().astype(np.int64), rh.reranked)


@pytest.fixture(scope="module")
def fsetup(tmp_path_factory, orc, ann):
    """Float indexes: R = 3 (64-d, M 16), 96-d M 24 with empty lists, 30-d M 10
    (3-d subspaces), and a Zipf-skewed unit-norm index (one list holds a large
    share of the vectors; per-query nprobe U{8..128})."""
    from paper_2409_16576_amd import workloads
    d = tmp_path_factory.mktemp("lmf")
    out = {}

    def add(name, path, Q, npq=None):
        out[name] = (orc.read_index(path), ann.Index(path, 0), Q.astype(np.float32), npq)

    X = fx.mixture(93, 15000, 64, "f32", n_centres=12)
    add("f32r3", fx.built(d, "f32r3", X, "f32", nlist=48, M=16, R=3, eps=0.25)[0],
        fx.mixture(94, 200, 64, "f32", n_centres=12))
    X = fx.mixture(95, 6000, 96, "f32", n_centres=4)
    add("f32m24", fx.built(d, "f32m24", X, "f32", nlist=96, M=24)[0],
        fx.mixture(96, 160, 96, "f32", n_centres=4))
    X = fx.mixture(97, 8000, 30, "f32", n_centres=8)
    add("f32d30", fx.built(d, "f32d30", X, "f32", nlist=32, M=10)[0],
        fx.mixture(98, 130, 30, "f32", n_centres=8))
    w = workloads.scaled(workloads.ZIPF_F32_5M, n=40000, nlist=64, n_centres=16, nq=300)
    add("zipf", workloads.ensure_index(w), workloads.queries(w), workloads.nprobe_per_query(w))
    yield out
    for _, g, _, _ in out.values():
        g.close()


FNAMES = ["f32r3", "f32m24", "f32d30", "zipf"]
FTUNINGS = [(2, 4096, 0, 0), (1, 1 << 24, 0, 0), (8, 256, 3, 500), (1, 64, 1, 3000)]


@pytest.mark.parametrize("name", FNAMES)
@pytest.mark.parametrize("tuning", FTUNINGS)
@pytest.mark.parametrize("lut16", [0, 1])
def test_list_major_float_tables_equal_plain_and_oracle(fsetup, orc, name, tuning, lut16):
    """Float indexes: four float32 (or eight binary16) tables side by side;
    lists shorter than the minimum stay per query; results bit-identical."""
    ix, g, Qh, npq = fsetup[name]
    if npq is None:
        rng = np.random.default_rng(13)
        npq = rng.integers(0, min(ix.nlist, 30) + 1, size=len(Qh)).astype(np.int32)
        npq[:2] = (0, ix.nlist)
    npq = np.minimum(npq, ix.nlist).astype(np.int32)
    Q, NP = _cuda(Qh), _cuda(npq)
    alpha, tile, blocks, min_rows = tuning
    g.set_option(OPT_LUT_F16, lut16)
    try:
        for k, n in ((10, 100), (10, 700)):
            _set_lm(g, False)
            p_ids, p_d = g.search(Q, NP, k, n)
            _set_lm(g, True, alpha, tile, blocks)
            g.set_option(OPT_LM_MIN_ROWS, min_rows)
            _say("float", name, tuning, lut16, k, n)
            l_ids, l_d = g.search(Q, NP, k, n)
            torch.cuda.synchronize()
            g.set_option(OPT_LM_MIN_ROWS, 0)
            _set_lm(g, False)
            r = orc.search(ix, Qh, npq, k, n, lut_f16=bool(lut16))
            assert np.array_equal(l_ids.cpu().numpy(), r.ids), (k, n)
            assert np.array_equal(l_d.cpu().numpy(), r.dists), (k, n)
            assert torch.equal(l_ids, p_ids)
            assert torch.equal(l_d.view(torch.int32), p_d.view(torch.int32))
    finally:
        g.set_option(OPT_LUT_F16, 0)


@pytest.mark.parametrize("lut16", [0, 1])
def test_list_major_float_topn_graph(ann, fsetup, orc, lut16):
    """Zipf index: top-n with its Eq. 1 values and candidate counts, and a
    graph replaying the list-major search, equal the oracle's."""
    ix, g, Qh, npq = fsetup["zipf"]
    Q, NP = _cuda(Qh), _cuda(npq)
    g.set_option(OPT_LUT_F16, lut16)
    try:
        _set_lm(g, True, 1, 2048, 0)
        g.set_option(OPT_LM_MIN_ROWS, 200)
        ids, adc, nc = g.search_topn(Q, NP, 300)
        torch.cuda.synchronize()
        r = orc.search(ix, Qh, npq, 1, 300, lut_f16=bool(lut16))
        assert np.array_equal(ids.cpu().numpy(), r.topn_ids)
        assert np.array_equal(adc.cpu().numpy(), r.topn_adc)
        assert np.array_equal(nc.cpu().numpy(), r.ncand)
        r = orc.search(ix, Qh, npq, 10, 400, lut_f16=bool(lut16))
        gr = ann.Graph(g, Q, NP, 10, 400)
        try:
            for rep in range(3):
                ids, d = gr.launch()
                torch.cuda.synchronize()
                assert np.array_equal(ids.cpu().numpy(), r.ids), rep
                assert np.array_equal(d.cpu().numpy(), r.dists), rep
        finally:
            gr.close()
    finally:
        g.set_option(OPT_LUT_F16, 0)
        g.set_option(OPT_LM_MIN_ROWS, 0)
        _set_lm(g, False)
