"""Run layout of the scan through the C ABI.

A probed list's replica entries are grouped by their vector's first list;
the scan skips a group whole when that first list is probed too (its
entries are owned there).  The surviving groups become runs of their own
when the block's run slots hold them (always, when the index's worst case
fits 1024 slots; else two slots per probed list, checked per query), and
otherwise each list's replica entries are one run tested entry by entry.
Both layouts must give the oracle's results bit for bit; the entries the
scan reports walked must be those of the layout the rule picks.
"""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MAX_SEG_RUNS = 1024  # the scan's run slots when every group may survive


def _say(*a):
    print("[gpu-walk]", *a, flush=True)


@pytest.fixture(scope="module")
def ann():
    from paper_2409_16576_amd import ann as A
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    A.lib()
    return A


@pytest.fixture(scope="module")
def setup(tmp_path_factory, orc, ann):
    d = tmp_path_factory.mktemp("walkidx")
    out = {}
    X = fx.mixture(71, 30000, 32, "u8", n_centres=16, hi=255)
    p, _ = fx.built(d, "many", X, "u8", nlist=256, M=8, eps=1.0)   # many groups per list
    out["many"] = (orc.read_index(p), ann.Index(p, 0))
    p, _ = fx.built(d, "few", X, "u8", nlist=64, M=8)               # few groups per list
    out["few"] = (orc.read_index(p), ann.Index(p, 0))
    yield out
    for _, g in out.values():
        g.close()


def _expected_walk(ix, lists, np_max):
    """Per query (entries walked by the rule, groups layout used?)."""
    lid = np.repeat(np.arange(ix.nlist), np.diff(ix.offsets))
    first = ix.assign[ix.entries, 0]
    groups = [np.unique(first[(lid == l) & (first != l)]) for l in range(ix.nlist)]
    max_segs = max(len(g) for g in groups)
    worst = np_max * (1 + max_segs)
    cap = worst if worst <= MAX_SEG_RUNS else 2 * np_max
    walk, used = [], []
    for row in lists:
        L = row[row >= 0]
        probed = np.zeros(ix.nlist, bool)
        probed[L] = True
        runs, seg_w, all_w = len(L), 0, 0
        for l in L:
            f = first[lid == l]
            all_w += len(f)
            rep = f[f != l]
            seg_w += int((f == l).sum() + (~probed[rep]).sum())
            runs += int((~probed[groups[l]]).sum())
        use = runs <= cap
        walk.append(seg_w if use else all_w)
        used.append(use)
    return np.array(walk), np.array(used)


@pytest.mark.parametrize("name,npb", [("many", 64), ("many", 100), ("many", 16), ("few", 12)])
def test_run_layouts_parity_and_walk(ann, setup, orc, name, npb):
    ix, g = setup[name]
    Qh = fx.mixture(72, 200, 32, "u8", n_centres=16, hi=255).astype(np.float32)
    rng = np.random.default_rng(npb)
    npq = rng.integers(max(1, npb // 2), npb + 1, size=len(Qh)).astype(np.int32)
    npq[0] = npb
    _say(name, "nprobe up to", npb)
    Q = torch.from_numpy(Qh).cuda()
    NP = torch.from_numpy(npq).cuda()
    r = orc.search(ix, Qh, npq, 10, 200)
    ids, d = g.search(Q, NP, 10, 200)
    assert np.array_equal(ids.cpu().numpy(), r.ids) and np.array_equal(d.cpu().numpy(), r.dists)
    tid, tadc, nc, nw = g.search_topn(Q, NP, 200, walked=True)
    torch.cuda.synchronize()
    assert np.array_equal(nc.cpu().numpy(), r.ncand)
    lists, _ = orc.probe(ix, Qh, npq)
    want, used = _expected_walk(ix, lists, int(npq.max()))
    assert np.array_equal(nw.cpu().numpy(), want)
    if name == "many" and npb >= 64:  # both layouts occur in this batch
        assert used.any() and not used.all(), used.mean()
    if name == "few":
        assert used.all()
