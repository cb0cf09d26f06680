"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test names the property it pins and what it rules out.  None of them
re-derives an expected value through the oracle itself.
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

from tests import fixtures as fx

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _toy(tmp_path):
    g = json.load(open(os.path.join(GOLDEN, "toy_adc_search.json")))
    path, _ = fx.write_arrays(tmp_path, "toy", "f32", np.array(g["centroids"], np.float32),
                              np.array(g["codebooks"], np.float32), np.array(g["codes"], np.uint8),
                              np.array(g["vectors"], np.float32), np.array(g["assign"], np.int32))
    return g, path


def test_toy_hand_worked_example(tmp_path, orc):
    """Hand-computed table, Eq. 1 sums, dedup, tie-break and re-rank (golden fixture)."""
    g, path = _toy(tmp_path)
    e = g["expect"]
    ix = orc.read_index(path)
    q = np.array([g["query"]], np.float32)
    lists, d = orc.probe(ix, q, 2)
    assert lists[0].tolist() == [0, 1] and d[0].tolist() == e["coarse_dists"]
    l32, l64 = orc.lut(ix, q)
    assert l32[0].tolist() == e["lut"]
    assert orc.adc(ix, l32[0], np.arange(5)).tolist() == e["adc"]
    assert orc.exact(ix, q[0], np.arange(5)).tolist() == e["exact"]
    for l, want in enumerate(e["lists"]):
        assert ix.entries[ix.offsets[l]:ix.offsets[l + 1]].tolist() == want
    u, gsz = orc.gather_dedup(ix, [0])
    assert u.tolist() == e["nprobe1"]["unique"] and gsz == e["nprobe1"]["gathered"]
    u, gsz = orc.gather_dedup(ix, [0, 1])
    assert u.tolist() == e["nprobe2"]["unique"] and gsz == e["nprobe2"]["gathered"]
    for key, n in (("search_nprobe2_n3_k2", 3), ("search_nprobe2_n2_k2", 2)):
        r = orc.search(ix, q, 2, 2, n)
        assert r.topn_ids[0].tolist() == e[key]["topn_ids"]
        assert r.topn_adc[0].tolist() == e[key]["topn_adc"]
        assert r.ids[0].tolist() == e[key]["ids"] and r.dists[0].tolist() == e[key]["dists"]
    ids, dd = orc.bruteforce(ix, q, 3)
    assert ids[0].tolist() == e["bruteforce_k3"]["ids"] and dd[0].tolist() == e["bruteforce_k3"]["dists"]


@pytest.mark.parametrize("kind", ["f32", "u8", "i8"])
def test_eq1_identity_table_sum_is_decoded_distance(tmp_path, orc, kind):
    """Eq. 1 with dist = squared L2: sum_m L[m][code_m] == ||q - decode(v)||^2.

    decode(v) concatenates the codewords named by the code; the right-hand
    side is computed on whole vectors with numpy, so a wrong subspace offset,
    a transposed codebook or a dropped subspace breaks the equality.
    """
    lo, hi = (-128, 127) if kind == "i8" else (0, 255 if kind == "u8" else 100)
    X = fx.mixture(3, 3000, 32, kind, lo=lo, hi=hi)
    path, _ = fx.built(tmp_path, "eq1", X, kind, nlist=16, M=8)
    ix = orc.read_index(path)
    Q = fx.mixture(5, 7, 32, kind, lo=lo, hi=hi).astype(np.float32)
    l32, l64 = orc.lut(ix, Q)
    ids = np.arange(0, 3000, 7, dtype=np.int32)
    dec = np.concatenate([ix.codebooks[m][ix.codes[ids, m]] for m in range(ix.M)], axis=1)
    for i in range(len(Q)):
        a32, a64 = orc.adc(ix, l32[i], ids, l64[i])
        ref = ((Q[i].astype(np.float64)[None, :] - dec.astype(np.float64)) ** 2).sum(1)
        np.testing.assert_allclose(a64, ref, rtol=1e-12, atol=1e-9)
        # float32 sum of M correctly rounded terms: relative error <= M * 2^-24
        np.testing.assert_allclose(a32, ref, rtol=ix.M * 2.0 ** -23)
        if kind != "f32":  # integer grid: every value exact
            assert np.array_equal(a32.astype(np.float64), ref)


def test_table_is_zero_at_the_query_codeword(tmp_path, orc):
    """dist(q_m, c) >= 0 with equality exactly where the subvector is a codeword."""
    X = fx.mixture(4, 2000, 16, "f32")
    path, _ = fx.built(tmp_path, "zero", X, "f32", nlist=8, M=4)
    ix = orc.read_index(path)
    j = np.array([5, 17, 200, 255])
    q = np.concatenate([ix.codebooks[m][j[m]] for m in range(4)])[None].astype(np.float32)
    l32, _ = orc.lut(ix, q)
    assert (l32 >= 0).all()
    for m in range(4):
        assert l32[0, m, j[m]] == 0.0
        assert np.count_nonzero(l32[0, m] == 0.0) == np.count_nonzero(
            (ix.codebooks[m] == ix.codebooks[m][j[m]]).all(1))


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_probe_is_sorted_nearest_lists(tmp_path, orc, kind):
    """Step 2: the m nearest centroids, ordered by (distance, list id) — scipy cdist."""
    X = fx.mixture(6, 4000, 16, kind, hi=255)
    path, _ = fx.built(tmp_path, "probe", X, kind, nlist=64, M=4)
    ix = orc.read_index(path)
    Q = fx.mixture(8, 25, 16, kind, hi=255).astype(np.float32)
    lists, d = orc.probe(ix, Q, 10)
    D = cdist(Q.astype(np.float64), ix.centroids.astype(np.float64), "sqeuclidean")
    for i in range(len(Q)):
        if kind == "u8":  # integers: cdist is exact, so the order must match exactly
            want = np.lexsort((np.arange(ix.nlist), D[i]))[:10]
            assert lists[i].tolist() == want.tolist()
            assert np.array_equal(d[i], D[i][want].astype(np.float32))
        else:
            np.testing.assert_allclose(d[i], D[i][lists[i]], rtol=1e-6)
            assert (np.diff(d[i]) >= 0).all()
            rest = np.setdiff1d(np.arange(ix.nlist), lists[i])
            assert D[i][rest].min() >= d[i][-1] * (1 - 1e-6)


def test_probe_pads_and_clamps(tmp_path, orc):
    X = fx.mixture(9, 500, 8, "u8", hi=255)
    path, _ = fx.built(tmp_path, "pad", X, "u8", nlist=4, M=2)
    ix = orc.read_index(path)
    Q = X[:3].astype(np.float32)
    lists, d = orc.probe(ix, Q, np.array([2, 9, 4], np.int32))
    assert (lists[0, 2:] == -1).all() and np.isinf(d[0, 2:]).all()
    assert sorted(lists[1, :4].tolist()) == [0, 1, 2, 3] and (lists[1, 4:] == -1).all()


def test_dedup_closed_forms(tmp_path, orc):
    """Steps 3+5: probing every list gathers E entries and yields all N IDs once;
    with R = 1 the multiset already is a set."""
    X = fx.mixture(10, 3000, 16, "f32")
    path, _ = fx.built(tmp_path, "dd", X, "f32", nlist=32, M=4, R=3, eps=0.3)
    ix = orc.read_index(path)
    u, g = orc.gather_dedup(ix, np.arange(ix.nlist))
    assert g == ix.entries.shape[0] and g > ix.n  # replication happened
    assert np.array_equal(u, np.arange(ix.n))
    lists = [3, 30, 7, 12]
    u, g = orc.gather_dedup(ix, lists)
    cat = np.concatenate([ix.entries[ix.offsets[l]:ix.offsets[l + 1]] for l in lists])
    assert g == len(cat) and np.array_equal(u, np.unique(cat))
    path1, _ = fx.built(tmp_path, "dd1", X, "f32", nlist=32, M=4, R=1)
    ix1 = orc.read_index(path1)
    u, g = orc.gather_dedup(ix1, np.arange(0, 32, 3))
    assert len(u) == g


def test_lossless_pq_adc_top_k_is_exact_knn(tmp_path, orc):
    """dsub = 1 and every byte value a codeword: ADC equals the exact distance,
    so the ADC top-k with rerank_n = k is the brute-force top-k, bit for bit."""
    path, _ = fx.lossless_u8(tmp_path, "lossless")
    ix = orc.read_index(path)
    rng = np.random.default_rng(1)
    Q = rng.integers(0, 256, size=(20, ix.dim)).astype(np.float32)
    r = orc.search(ix, Q, ix.nlist, 10, 10)
    bi, bd = orc.bruteforce(ix, Q, 10)
    assert np.array_equal(r.topn_ids.astype(np.int64), bi)
    assert np.array_equal(r.topn_adc, bd)
    assert np.array_equal(r.ids, bi) and np.array_equal(r.dists, bd)


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_exhaustive_search_is_bruteforce(tmp_path, orc, kind):
    """nprobe = nlist and rerank_n >= N re-rank everything: search == brute force."""
    X = fx.mixture(12, 700, 16, kind, hi=255)
    path, _ = fx.built(tmp_path, "exh", X, kind, nlist=8, M=4)
    ix = orc.read_index(path)
    Q = fx.mixture(13, 15, 16, kind, hi=255).astype(np.float32)
    r = orc.search(ix, Q, ix.nlist, 10, ix.n)
    bi, bd = orc.bruteforce(ix, Q, 10)
    assert np.array_equal(r.ids, bi) and np.array_equal(r.dists, bd)
    assert (r.ncand == ix.n).all()


def test_bruteforce_matches_numpy_exact(tmp_path, orc):
    """Brute force on uint8 data vs numpy integer distances and lexsort."""
    X = fx.mixture(14, 900, 24, "u8", hi=255)
    path, _ = fx.built(tmp_path, "bf", X, "u8", nlist=4, M=6)
    ix = orc.read_index(path)
    Q = fx.mixture(15, 12, 24, "u8", hi=255).astype(np.float32)
    bi, bd = orc.bruteforce(ix, Q, 7)
    D = ((Q[:, None, :].astype(np.int64) - X[None].astype(np.int64)) ** 2).sum(-1)
    for i in range(len(Q)):
        want = np.lexsort((np.arange(len(X)), D[i]))[:7]
        assert bi[i].tolist() == want.tolist()
        assert bd[i].tolist() == D[i][want].astype(np.float32).tolist()


def test_identical_vectors_break_ties_by_lower_id(tmp_path, orc):
    """All vectors equal: every distance ties, so the results are IDs 0..k-1."""
    X = np.full((50, 8), 7, np.uint8)
    cb = np.tile(np.arange(256, dtype=np.float32).reshape(1, 256, 1), (8, 1, 1))
    assign = np.stack([np.arange(50) % 3, -np.ones(50, int)], 1)
    cent = np.full((3, 8), 7, np.float32)
    path, _ = fx.write_arrays(tmp_path, "same", "u8", cent, cb, X.copy(), X, assign)
    ix = orc.read_index(path)
    Q = np.array([[0] * 8, [9] * 8], np.float32)
    r = orc.search(ix, Q, 3, 5, 20)
    assert r.ids.tolist() == [[0, 1, 2, 3, 4]] * 2
    assert r.topn_ids.tolist() == [list(range(20))] * 2
    bi, _ = orc.bruteforce(ix, Q, 4)
    assert bi.tolist() == [[0, 1, 2, 3]] * 2


def test_topn_and_rerank_are_valid_selections(tmp_path, orc):
    """Step 7 keeps the n smallest (adc, id) of the deduplicated candidates;
    step 8 returns them re-ordered by (exact distance, id)."""
    X = fx.mixture(16, 5000, 32, "u8", hi=255)
    path, _ = fx.built(tmp_path, "sel", X, "u8", nlist=32, M=8)
    ix = orc.read_index(path)
    Q = fx.mixture(17, 10, 32, "u8", hi=255).astype(np.float32)
    n, k, npb = 40, 10, 5
    r = orc.search(ix, Q, npb, k, n)
    lists, _ = orc.probe(ix, Q, npb)
    l32, l64 = orc.lut(ix, Q)
    for i in range(len(Q)):
        cand = np.unique(np.concatenate([ix.entries[ix.offsets[l]:ix.offsets[l + 1]] for l in lists[i]]))
        assert r.ncand[i] == len(cand)
        dec = np.concatenate([ix.codebooks[m][ix.codes[cand, m]] for m in range(ix.M)], axis=1)
        adc = ((Q[i][None].astype(np.float64) - dec) ** 2).sum(1)  # integers: exact
        want = cand[np.lexsort((cand, adc))][:n]
        assert r.topn_ids[i].tolist() == want.tolist()
        ex = ((Q[i][None].astype(np.int64) - X[want].astype(np.int64)) ** 2).sum(1)
        order = np.lexsort((want, ex))[:k]
        assert r.ids[i].tolist() == want[order].tolist()
        assert r.dists[i].tolist() == ex[order].astype(np.float32).tolist()


def test_integer_queries_are_rounded_and_saturated(tmp_path, orc):
    """uint8 index: a query is rounded half to even and clipped before use."""
    path, _ = fx.lossless_u8(tmp_path, "conv", n=64, dim=4)
    ix = orc.read_index(path)
    raw = np.array([[2.5, 3.5, -7.0, 300.0]], np.float32)
    conv = np.array([[2.0, 4.0, 0.0, 255.0]], np.float32)
    l_raw, _ = orc.lut(ix, raw)
    l_conv, _ = orc.lut(ix, conv)
    assert np.array_equal(l_raw, l_conv)
    assert np.array_equal(orc.bruteforce(ix, raw, 5)[0], orc.bruteforce(ix, conv, 5)[0])


def test_padding_when_fewer_candidates_than_k(tmp_path, orc):
    g, path = _toy(tmp_path)
    ix = orc.read_index(path)
    r = orc.search(ix, np.array([g["query"]], np.float32), 1, 8, 6)
    assert r.ids[0].tolist()[:4] == [0, 3, 1, 4] and r.ids[0].tolist()[4:] == [-1] * 4
    assert np.isinf(r.dists[0, 4:]).all()
    assert r.topn_ids[0].tolist()[4:] == [-1, -1]


def test_recall_rises_to_one_with_rerank_n(tmp_path, orc):
    """More re-ranked candidates never lose recall at fixed nprobe (same top-n prefix)."""
    X = fx.mixture(18, 20000, 32, "f32", n_centres=32)
    path, _ = fx.built(tmp_path, "rec", X, "f32", nlist=128, M=8)
    ix = orc.read_index(path)
    Q = fx.mixture(19, 40, 32, "f32", n_centres=32).astype(np.float32)
    bi, _ = orc.bruteforce(ix, Q, 10)
    rec = [orc.recall_at_k(orc.search(ix, Q, 128, 10, n).ids, bi, 10) for n in (10, 50, 200, 20000)]
    assert all(a <= b + 1e-12 for a, b in zip(rec, rec[1:]))
    assert rec[-1] == 1.0


def test_binary16_rounding_matches_numpy(orc):
    """The half-precision table variant rounds each float32 entry to the
    nearest binary16 value, ties to even; numpy's float16 conversion is an
    independent implementation of the same IEEE rounding.  Covers exact
    half-way points (where truncation or ties-away would differ), the
    subnormal range, the largest finite value and overflow."""
    rng = np.random.default_rng(3)
    x = np.concatenate([
        rng.uniform(0, 70000, 20000), 10.0 ** rng.uniform(-9, 6, 20000),
        rng.uniform(-100, 100, 2000),
        [0.0, -0.0, 65504.0, 65519.99, 65520.0, 65535.0, 1e30, 2.0 ** -24, 2.0 ** -25,
         3 * 2.0 ** -26, 2.0 ** -14, 2.0 ** -14 - 2.0 ** -25],
    ]).astype(np.float32)
    h = np.arange(0, 0x7C00, dtype=np.uint16).view(np.float16).astype(np.float32)
    mids = ((h[:-1].astype(np.float64) + h[1:]) / 2).astype(np.float32)  # exact in float32
    x = np.concatenate([x, mids, h])
    want = x.astype(np.float16).astype(np.float32)
    got = orc.round_half(x)
    assert np.array_equal(np.isinf(got), np.isinf(want))
    fin = ~np.isinf(want)
    assert np.array_equal(got[fin].view(np.uint32), want[fin].view(np.uint32))


def test_half_table_variant(tmp_path, orc):
    """f16 table = binary16 rounding of the float32 table (numpy float16);
    where every entry is exactly representable (small integers) the f16 search
    is the float32 search bit for bit; otherwise its top-n is the valid
    selection under the rounded table."""
    path, _ = fx.lossless_u8(tmp_path, "h16", n=400, dim=8)
    ix = orc.read_index(path)
    rng = np.random.default_rng(8)
    Q = rng.integers(0, 40, size=(12, 8)).astype(np.float32)  # entries (q - c)^2 <= 2048 for c <= 85
    X = ix.vectors.astype(np.int64)
    l32, _ = orc.lut(ix, Q)
    l16, _ = orc.lut(ix, Q, f16=True)
    assert np.array_equal(l16, l32.astype(np.float16).astype(np.float32))
    small = (l32 <= 2048).all(axis=(1, 2))
    r32 = orc.search(ix, Q, 4, 5, 30)
    r16 = orc.search(ix, Q, 4, 5, 30, lut_f16=True)
    for i in range(len(Q)):
        if small[i]:
            assert r16.topn_ids[i].tolist() == r32.topn_ids[i].tolist()
    X = fx.mixture(21, 4000, 32, "f32", n_centres=8, hi=1.0, sigma=0.05)
    path, _ = fx.built(tmp_path, "h16f", X, "f32", nlist=16, M=8)
    ix = orc.read_index(path)
    Q = fx.mixture(22, 6, 32, "f32", n_centres=8, hi=1.0, sigma=0.05).astype(np.float32)
    n = 50
    r = orc.search(ix, Q, 4, 10, n, lut_f16=True)
    lists, _ = orc.probe(ix, Q, 4)
    l32, _ = orc.lut(ix, Q)
    t16 = l32.astype(np.float16).astype(np.float32)
    for i in range(len(Q)):
        cand = np.unique(np.concatenate([ix.entries[ix.offsets[l]:ix.offsets[l + 1]] for l in lists[i]]))
        adc = np.zeros(len(cand), np.float32)
        for m in range(ix.M):  # float32 sum in subspace order, as Eq. 1's reading
            adc = (adc + t16[i, m, ix.codes[cand, m]]).astype(np.float32)
        want = cand[np.lexsort((cand, adc))][:n]
        assert r.topn_ids[i].tolist() == want.tolist()
        assert r.topn_adc[i].tolist() == np.sort(adc)[:n].tolist()


def _prefix_topk(Q, X, cand, k):
    """Exact top-k (distance, id) of each prefix length, by numpy (integers)."""
    ex = ((Q[None, :].astype(np.int64) - X[cand].astype(np.int64)) ** 2).sum(1)
    return ex


def test_heuristic_rerank_reductions_and_rule(tmp_path, orc):
    """Heuristic re-ranking (Alg. 1, change rate of Eq. 3), pinned three ways:
    (a) beta larger than the number of mini-batches never stops early, so the
        result is the fixed-n re-rank; (b) eps >= 1 with beta = 1 stops after
        the first mini-batch, so the result is the exact top-k of the first
        batch_size candidates; (c) for other settings the result is the exact
        top-k of the first T candidates and T is where the stopping rule,
        re-derived here with numpy sets of prefix top-k IDs, first fires."""
    X = fx.mixture(23, 6000, 32, "u8", n_centres=8, hi=255)
    path, _ = fx.built(tmp_path, "heur", X, "u8", nlist=16, M=8)
    ix = orc.read_index(path)
    Q = fx.mixture(24, 12, 32, "u8", n_centres=8, hi=255).astype(np.float32)
    k, n = 10, 300
    fixed = orc.search(ix, Q, 6, k, n)
    never = orc.search(ix, Q, 6, k, n, heuristic=(32, 0.0, 10 ** 6))
    assert np.array_equal(never.ids, fixed.ids) and np.array_equal(never.dists, fixed.dists)
    assert (never.reranked == np.minimum(n, fixed.ncand)).all()
    # (8, 0.85, 1) and (6, 0.7, 2): after a first mini-batch smaller than k the
    # change rate is batch/k (Eq. 3 divides by k), below eps, while dividing
    # by the heap's size would give 1 -- so only the k reading stops there
    for B, eps, beta in ((40, 1.0, 1), (16, 0.0, 2), (8, 0.1, 3), (25, 0.2, 1), (8, 0.85, 1),
                         (6, 0.7, 2)):
        r = orc.search(ix, Q, 6, k, n, heuristic=(B, eps, beta))
        for i in range(len(Q)):
            cand = fixed.topn_ids[i][fixed.topn_ids[i] >= 0]
            ex = _prefix_topk(Q[i], X, cand, k)
            stop, stable, prev = len(cand), 0, set()
            for b0 in range(0, len(cand), B):
                t = min(len(cand), b0 + B)
                cur = set(cand[np.lexsort((cand[:t], ex[:t]))][:k].tolist())
                delta = len(cur - prev) / k
                prev = cur
                stable = stable + 1 if delta <= eps else 0
                if stable >= beta:
                    stop = t
                    break
            assert r.reranked[i] == stop, (B, eps, beta, i)
            o = np.lexsort((cand[:stop], ex[:stop]))[:k]
            assert r.ids[i][:len(o)].tolist() == cand[:stop][o].tolist()
            assert r.dists[i][:len(o)].tolist() == ex[:stop][o].astype(np.float32).tolist()
            if (B, eps, beta) == (40, 1.0, 1):
                assert stop == min(40, len(cand))
            if (B, eps, beta) == (8, 0.85, 1):
                assert stop == min(8, len(cand))


def test_int8_exact_and_bruteforce_match_numpy(tmp_path, orc):
    """int8 data (Table 1's 100-d int8 set): exact squared distances and brute
    force against numpy int64 arithmetic on signed values.  Rows hold negative
    values down to -128 and queries hit both saturation bounds, so reading the
    rows as unsigned bytes, or skipping the query's saturation, changes the
    distances."""
    rng = np.random.default_rng(31)
    n, dim = 1500, 20
    X = rng.integers(-128, 128, size=(n, dim)).astype(np.int8)
    X[::7, ::3] = -128
    cb = np.tile(np.arange(-128, 128, dtype=np.float32).reshape(1, 256, 1), (dim, 1, 1))
    cent = np.rint(rng.uniform(-128, 127, size=(4, dim))).astype(np.float32)
    d = ((X[:, None, :].astype(np.int64) - cent[None].astype(np.int64)) ** 2).sum(-1)
    assign = np.stack([np.argmin(d, axis=1), -np.ones(n, dtype=np.int64)], axis=1)
    codes = (X.astype(np.int16) + 128).astype(np.uint8)
    path, _ = fx.write_arrays(tmp_path, "i8x", "i8", cent, cb, codes, X, assign)
    ix = orc.read_index(path)
    Q = rng.integers(-128, 128, size=(9, dim)).astype(np.float32)
    Q[0, :5] = [-300.0, 250.0, -128.0, 127.0, -0.5]  # saturate / round half to even
    Qc = np.clip(np.rint(Q), -128, 127).astype(np.int64)
    D = ((Qc[:, None, :] - X[None].astype(np.int64)) ** 2).sum(-1)
    ids = np.arange(0, n, 3, dtype=np.int32)
    for i in range(len(Q)):
        got = orc.exact(ix, Q[i], ids)
        assert got.tolist() == D[i][ids].astype(np.float32).tolist()
    bi, bd = orc.bruteforce(ix, Q, 8)
    for i in range(len(Q)):
        want = np.lexsort((np.arange(n), D[i]))[:8]
        assert bi[i].tolist() == want.tolist()
        assert bd[i].tolist() == D[i][want].astype(np.float32).tolist()
    # lossless codebook (dsub = 1, every int8 value a codeword): ADC = exact
    r = orc.search(ix, Q, 4, 8, 8)
    assert np.array_equal(r.ids, bi) and np.array_equal(r.dists, bd)


def test_float_distances_are_one_rounding_of_the_exact_sum(tmp_path, orc):
    """Float data: every exact squared distance (probe, re-rank, brute force)
    and every table entry is the exact real sum rounded once to float32.

    Coordinates are multiples of 2^-4 below 64 in magnitude, so each squared
    difference is a multiple of 2^-8 below 2^14 and a sum over 128 dimensions
    needs up to 29 + 8 significant bits: float64 holds every partial sum
    exactly, float32 does not.  The exact value comes from integer
    arithmetic; a float32 running sum (or any second rounding) differs from it
    in the last bits for most vectors."""
    rng = np.random.default_rng(37)
    n, dim, nlist, M = 600, 128, 8, 16
    grid = lambda *s: (rng.integers(-1023, 1024, size=s) / 16.0).astype(np.float32)  # noqa: E731
    X, cent, cb = grid(n, dim), grid(nlist, dim), grid(M, 256, dim // M)
    Q = grid(11, dim)
    xi, ci, qi, cbi = ((a.astype(np.float64) * 16).astype(np.int64) for a in (X, cent, Q, cb))
    dc = ((xi[:, None, :] - ci[None]) ** 2).sum(-1)
    assign = np.stack([np.argmin(dc, axis=1), -np.ones(n, dtype=np.int64)], axis=1)
    codes = rng.integers(0, 256, size=(n, M)).astype(np.uint8)
    path, _ = fx.write_arrays(tmp_path, "grid", "f32", cent, cb, codes, X, assign)
    ix = orc.read_index(path)

    def once(S):  # integer multiple of 2^-8 -> float32, one rounding (S < 2^53)
        return (np.asarray(S, np.int64).astype(np.float64) / 256.0).astype(np.float32)

    DX = ((qi[:, None, :] - xi[None]) ** 2).sum(-1)
    DC = ((qi[:, None, :] - ci[None]) ** 2).sum(-1)
    ids = np.arange(n, dtype=np.int32)
    diff32 = 0
    for i in range(len(Q)):
        want = once(DX[i])
        assert orc.exact(ix, Q[i], ids).view(np.uint32).tolist() == want.view(np.uint32).tolist()
        acc = np.zeros(n, np.float32)  # the float32 running sum the reading rules out
        for t in range(dim):
            acc = (acc + ((Q[i, t] - X[:, t]) ** 2).astype(np.float32)).astype(np.float32)
        diff32 += int((acc != want).sum())
    assert diff32 > n  # the fixture separates the two accumulations
    lists, pd = orc.probe(ix, Q, nlist)
    for i in range(len(Q)):
        order = np.lexsort((np.arange(nlist), once(DC[i])))
        assert lists[i].tolist() == order.tolist()
        assert pd[i].view(np.uint32).tolist() == once(DC[i])[order].view(np.uint32).tolist()
    bi, bd = orc.bruteforce(ix, Q, 6)
    for i in range(len(Q)):
        w = once(DX[i])
        order = np.lexsort((np.arange(n), w))[:6]
        assert bi[i].tolist() == order.tolist()
        assert bd[i].view(np.uint32).tolist() == w[order].view(np.uint32).tolist()
    l32, _ = orc.lut(ix, Q)
    ds = dim // M
    for m in range(M):
        E = ((qi[:, None, m * ds:(m + 1) * ds] - cbi[m][None]) ** 2).sum(-1)  # [nq, 256]
        assert l32[:, m, :].view(np.uint32).tolist() == once(E).view(np.uint32).tolist()
