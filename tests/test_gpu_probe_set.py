"""The scan's probed-list set for large list counts (more than 16,384 lists:
the probed lists sorted in LDS instead of a bitmap over all lists), with the
run slots that frees: results bit-equal to the oracle for small and large
nprobe (surviving replica groups as runs, and queries whose groups exceed
the run slots and test their entries one by one) and for vectors in up to
three lists (entries whose second list must be tested too)."""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[gpu-probe-set]", *a, flush=True)


@pytest.fixture(scope="module")
def ann():
    from paper_2409_16576_amd import ann as A
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    A.lib()
    return A


@pytest.fixture(scope="module")
def idx(tmp_path_factory, orc):
    d = tmp_path_factory.mktemp("setidx")
    X = fx.mixture(701, 120000, 32, "u8", n_centres=256, hi=255, sigma=12.0)
    out = {}
    for R, eps in ((2, 0.2), (3, 0.3)):
        p, _ = fx.built(d, f"u8R{R}", X, "u8", nlist=17000, M=8, R=R, eps=eps, kmeans_iters=3)
        out[R] = (orc.read_index(p), p)
    Q = fx.mixture(702, 150, 32, "u8", n_centres=256, hi=255, sigma=12.0).astype(np.float32)
    return out, Q


@pytest.mark.parametrize("R", [2, 3])
def test_sorted_probe_set_search_equals_oracle(ann, orc, idx, R):
    (ixs, Q) = idx
    ix, path = ixs[R]
    assert ix.nlist > 16384
    g = ann.Index(path, 0)
    try:
        rng = np.random.default_rng(R)
        for npmax in (8, 64, 300):
            npq = rng.integers(1, npmax + 1, size=len(Q)).astype(np.int32)
            npq[0] = npmax
            _say("R", R, "nprobe", npmax)
            Qd, NP = torch.from_numpy(Q).cuda(), torch.from_numpy(npq).cuda()
            ids, dd = g.search(Qd, NP, 10, 100)
            tids, tadc, nc = g.search_topn(Qd, NP, 100)
            torch.cuda.synchronize()
            r = orc.search(ix, Q, npq, 10, 100)
            assert np.array_equal(ids.cpu().numpy(), r.ids), npmax
            assert np.array_equal(dd.cpu().numpy().view(np.int32), r.dists.view(np.int32)), npmax
            assert np.array_equal(tids.cpu().numpy(), r.topn_ids), npmax
            assert np.array_equal(nc.cpu().numpy(), r.ncand), npmax
    finally:
        g.close()
