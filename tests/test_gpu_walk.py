"""Run layout of the scan through the C ABI.

A probed list's replica entries are grouped by their vector's first list;
the scan skips a group whole when that first list is probed too (its
entries are owned there).  The surviving groups become runs of their own
when the block's run slots hold them (always, when the index's worst case
fits 1024 slots; else as many slots as keep two scan blocks in a CU's LDS
next to the smallest top-n buffer, at least two per probed list, checked
per query), and otherwise each list's replica entries are one run tested
entry by entry.
Both layouts must give the oracle's results bit for bit; the entries the
scan reports walked must be those of the layout the rule picks.
"""
import numpy as np
import pytest

from tests import fixtures as fx

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MAX_SEG_RUNS = 1024  # the scan's run slots when every group may survive
TWO_PER_CU = 80 * 1024  # LDS of a scan block that still fits twice in a CU


def _a16(x):
    return (x + 15) // 16 * 16


def _scan_lds(ix, np_max, runs, cap):
    """LDS bytes of a scan block: the distance table, the probed-list set
    (bitmap over all lists, or the probed lists sorted and padded to a power
    of two when the bitmap would exceed both 512 words and nprobe_max
    entries), the probed lists, the run
    starts and offsets, the top-n buffer, per-wave sums, selection scratch."""
    words = (ix.nlist + 31) // 32
    p2 = 1 << max(0, (np_max - 1).bit_length())
    o = _a16(((ix.M + 3) // 4) * 4 * 256 * 4)
    o = _a16(o + ((p2 * 4 if words > 512 and words > np_max else words * 4) if ix.R > 1 else 0))
    o = _a16(o + np_max * 4)
    o = _a16(o + runs * 4)
    o = _a16(o + (runs + 1) * 4)
    o = _a16(o + cap * 8)
    o = _a16(o + 17 * 4)
    o = _a16(o + 1064)
    return _a16(o + 32)


def _run_slots(ix, np_max, max_segs, n):
    worst = np_max * (1 + max_segs)
    if worst <= MAX_SEG_RUNS:
        return worst
    fixed = _scan_lds(ix, np_max, 0, n + 1024)  # n + one round (1024 threads, one entry each)
    fit = (TWO_PER_CU - 64 - fixed) // 8 - 8 if fixed + 64 < TWO_PER_CU else 0
    return max(2 * np_max, min(worst, fit // 64 * 64))


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
    # 64 subspaces: the 64 KB table (with the buffer of n = 800) leaves no
    # room for extra run slots, so queries with many surviving groups test
    # their entries one by one
    X = fx.mixture(73, 30000, 64, "u8", n_centres=16, hi=255)
    p, _ = fx.built(d, "tight", X, "u8", nlist=256, M=64, eps=1.0)
    out["tight"] = (orc.read_index(p), ann.Index(p, 0))
    yield out
    for _, g in out.values():
        g.close()


def _expected_walk(ix, lists, np_max, n):
    """Per query (entries walked by the rule, groups layout used?)."""
    lid = np.repeat(np.arange(ix.nlist), np.diff(ix.offsets))
    first = ix.assign[ix.entries, 0]
    groups = [np.unique(first[(lid == l) & (first != l)]) for l in range(ix.nlist)]
    max_segs = max(len(g) for g in groups)
    cap = _run_slots(ix, np_max, max_segs, n)
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


@pytest.mark.parametrize("name,npb", [("many", 64), ("many", 100), ("many", 16), ("tight", 64),
                                      ("tight", 100), ("few", 12)])
def test_run_layouts_parity_and_walk(ann, setup, orc, name, npb):
    ix, g = setup[name]
    dim = 64 if name == "tight" else 32
    Qh = fx.mixture(72, 200, dim, "u8", n_centres=16, hi=255).astype(np.float32)
    rng = np.random.default_rng(npb)
    npq = rng.integers(max(1, npb // 2), npb + 1, size=len(Qh)).astype(np.int32)
    npq[0] = npb
    _say(name, "nprobe up to", npb)
    Q = torch.from_numpy(Qh).cuda()
    NP = torch.from_numpy(npq).cuda()
    # "tight": the 64 KB table and a top-n buffer of n = 800 (+ one round)
    # leave no LDS for run slots past two per probed list
    n = 800 if name == "tight" else 200
    r = orc.search(ix, Qh, npq, 10, n)
    ids, d = g.search(Q, NP, 10, n)
    assert np.array_equal(ids.cpu().numpy(), r.ids) and np.array_equal(d.cpu().numpy(), r.dists)
    tid, tadc, nc, nw = g.search_topn(Q, NP, n, walked=True)
    torch.cuda.synchronize()
    assert np.array_equal(nc.cpu().numpy(), r.ncand)
    lists, _ = orc.probe(ix, Qh, npq)
    want, used = _expected_walk(ix, lists, int(npq.max()), n)
    assert np.array_equal(nw.cpu().numpy(), want)
    if name == "tight" and npb >= 64:  # both layouts occur in this batch
        assert used.any() and not used.all(), used.mean()
    if name in ("few", "many"):  # the run slots hold every query's surviving groups
        assert used.all()
