"""The fused probe (batches of >= 4096 queries on integer-grid indexes) at
list counts of a few thousand, whose last 128-list tile is ragged: lists and
distances bit-exact against the oracle's exact probe for both query-tile
widths (nprobe up to 64 and up to 128) and both K depths (dimension 32 and
100), and the whole search on top."""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-probe-fused]", *a, flush=True)


@pytest.fixture(scope="module")
def ann():
    from paper_2409_16576_amd import ann as A
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    A.lib()
    return A


@pytest.fixture(scope="module")
def idx(tmp_path_factory, orc):
    d = tmp_path_factory.mktemp("partsidx")
    out = {}
    # 3000 lists: the last tile holds 56
    X = fx.mixture(501, 30000, 32, "u8", n_centres=64, hi=255)
    out["u8_3000"] = (fx.built(d, "u8", X, "u8", nlist=3000, M=8, kmeans_iters=4)[0], "u8", 32)
    # 2100 lists: the last tile holds 52
    X = fx.mixture(503, 21000, 100, "i8", n_centres=64, lo=-128, hi=127)
    out["i8_2100"] = (fx.built(d, "i8", X, "i8", nlist=2100, M=50, kmeans_iters=4)[0], "i8", 100)
    return {k: (orc.read_index(p), p, kind, dim) for k, (p, kind, dim) in out.items()}


@pytest.mark.parametrize("name", ["u8_3000", "i8_2100"])
@pytest.mark.parametrize("npmax", [40, 128])
def test_probe_parts_bit_exact(ann, orc, idx, name, npmax):
    ix, path, kind, dim = idx[name]
    g = ann.Index(path, 0)
    try:
        rng = np.random.default_rng(23)
        lo, hi = (0, 255) if kind == "u8" else (-128, 127)
        Q = np.clip(np.rint(rng.uniform(lo, hi, size=(4500, dim))), lo, hi).astype(np.float32)
        npr = rng.integers(0, npmax + 1, size=len(Q)).astype(np.int32)
        npr[:2] = (0, npmax)
        _say(name, npmax)
        lists, d = g.probe(torch.from_numpy(Q).cuda(), torch.from_numpy(npr).cuda())
        torch.cuda.synchronize()
        ol, od = orc.probe(ix, Q, npr)
        w = ol.shape[1]
        assert np.array_equal(lists.cpu().numpy()[:, :w], ol)
        assert np.array_equal(d.cpu().numpy()[:, :w].view(np.int32), od.view(np.int32))
        assert (lists.cpu().numpy()[:, w:] == -1).all()
        # the whole search on top
        ids, dd = g.search(torch.from_numpy(Q).cuda(), torch.from_numpy(npr).cuda(), 10, 50)
        r = orc.search(ix, Q, npr, 10, 50)
        assert np.array_equal(ids.cpu().numpy(), r.ids)
        assert np.array_equal(dd.cpu().numpy().view(np.int32), r.dists.view(np.int32))
    finally:
        g.close()
