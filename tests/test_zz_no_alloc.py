"""ann_search_noalloc (the allocation-free variant of ann_search) through the
C ABI: bit-identical to ann_search on two calls in a row, the first large
enough to be searched in several chunks of the fixed scratch array, the
second smaller (the array keeps the first call's contents)."""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[no-alloc]", *a, flush=True)


@pytest.fixture(scope="module")
def ann():
    from paper_2409_16576_amd import ann as A
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    A.lib()
    return A


@pytest.fixture(scope="module")
def index_paths(tmp_path_factory):
    d = tmp_path_factory.mktemp("noalloc")
    out = {}
    # uint8, 2048 lists: a query's working buffers take ~40 KB at rerank_n 256,
    # so 6000 queries need several chunks of the 128 MiB array
    X = fx.mixture(71, 40000, 32, "u8", n_centres=64, hi=255)
    out["u8"] = (fx.built(d, "u8", X, "u8", nlist=2048, M=8)[0],
                 fx.mixture(72, 6000, 32, "u8", n_centres=64, hi=255).astype(np.float32))
    X = fx.mixture(73, 12000, 48, "f32", n_centres=12)
    out["f32"] = (fx.built(d, "f32", X, "f32", nlist=64, M=12, R=3, eps=0.25)[0],
                  fx.mixture(74, 900, 48, "f32", n_centres=12).astype(np.float32))
    return out


def test_scratch_size_is_stated(ann):
    assert ann.lib().ann_noalloc_scratch_bytes() == 128 << 20


@pytest.mark.parametrize("name,nprobe,k,n", [("u8", 24, 10, 256), ("f32", 9, 7, 60)])
def test_noalloc_equals_search_on_two_calls(ann, index_paths, name, nprobe, k, n):
    path, Qh = index_paths[name]
    g = ann.Index(path, 0)
    try:
        Q = torch.from_numpy(Qh).cuda()
        rng = np.random.default_rng(5)
        npq = torch.from_numpy(rng.integers(1, nprobe + 1, size=len(Qh)).astype(np.int32)).cuda()
        for call, (nq, npa) in enumerate([(len(Qh), npq), (len(Qh) // 7, nprobe)]):
            npa_c = npa if isinstance(npa, int) else npa[:nq]
            _say(f"{name}: call {call}, {nq} queries, nprobe {'per query' if not isinstance(npa, int) else npa}")
            ids_a, d_a = g.search_noalloc(Q[:nq], npa_c, k, n)
            ids_b, d_b = g.search(Q[:nq], npa_c, k, n)
            torch.cuda.synchronize()
            assert torch.equal(ids_a, ids_b), f"call {call}: ids differ"
            assert torch.equal(d_a.view(torch.int32), d_b.view(torch.int32)), f"call {call}: dists differ"
            assert int((ids_a >= 0).sum()) > 0
    finally:
        g.close()


def test_noalloc_rejects_bad_arguments(ann, index_paths):
    path, Qh = index_paths["f32"]
    g = ann.Index(path, 0)
    try:
        Q = torch.from_numpy(Qh[:4]).cuda()
        with pytest.raises(Exception):
            g.search_noalloc(Q, 4, 10, 5)  # rerank_n < k
        with pytest.raises(Exception):
            g.search_noalloc(Q, 0, 10, 20)  # nprobe_max < 1
    finally:
        g.close()
