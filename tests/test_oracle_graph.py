"""Pins of the oracle's navigation-graph probe (Sec. 4.1) and of the builder's
graph, on the CPU.

The walk is pinned by a hand-worked example (a greedy walk that stops in a
local minimum with one slot and finds the nearest list with two), by the
closed forms "complete graph => exact probe for any beam >= m" and "beam >=
nlist on a graph reachable from its entries => exact probe", and by the
stopping property of a finished walk: with beam = m, every neighbour of a
returned list is either returned or farther than the last one returned.
"""
import json
import os

import numpy as np
import pytest

from tests import fixtures as fx

GOLD = os.path.join(os.path.dirname(__file__), "golden", "nav_graph_example.json")


def _line_index(tmp_path, xs):
    """A float32 index of dimension 1 whose list centroids are xs."""
    k = len(xs)
    cent = np.asarray(xs, dtype=np.float32).reshape(k, 1)
    cb = np.zeros((1, 256, 1), dtype=np.float32)
    X = cent.copy()
    codes = np.zeros((k, 1), dtype=np.uint8)
    assign = np.stack([np.arange(k), -np.ones(k, dtype=np.int64)], axis=1)
    p, _ = fx.write_arrays(tmp_path, "line", "f32", cent, cb, codes, X, assign)
    return p


@pytest.mark.parametrize("which", [0, 1])
def test_worked_examples(orc, tmp_path, which):
    g = json.load(open(GOLD))["examples"][which]
    ix = orc.read_index(_line_index(tmp_path, g["centroids_1d"]))
    adj = np.asarray(g["adj"], dtype=np.int32)
    q = np.array([[g["query"]]], dtype=np.float32)
    l_all, d_all = orc.probe(ix, q, ix.nlist)
    assert [g["squared_distances"][v] for v in l_all[0]] == d_all[0].tolist()
    for c in g["cases"]:
        G = orc.NavGraph(adj, np.asarray(c["entry"], dtype=np.int32), c["beam"])
        lists, d, nd = orc.graph_probe(ix, G, q, c["m"])
        assert lists[0].tolist() == c["lists"], c
        assert d[0].tolist() == c["dists"], c
        assert int(nd[0]) == c["computed"], c


def _small(tmp_path, kind="f32"):
    if kind == "f32":
        X = fx.mixture(301, 3000, 16, "f32", n_centres=12)
    else:
        X = fx.mixture(303, 3000, 16, "i8", n_centres=12, lo=-128, hi=127)
    p, _ = fx.built(tmp_path, "g" + kind, X, kind, nlist=48, M=4)
    Q = fx.mixture(302, 40, 16, "f32" if kind == "f32" else "i8", n_centres=12,
                   **({} if kind == "f32" else dict(lo=-128, hi=127))).astype(np.float32)
    return p, Q


@pytest.mark.parametrize("kind", ["f32", "i8"])
def test_complete_graph_gives_exact_probe(orc, tmp_path, kind):
    p, Q = _small(tmp_path, kind)
    ix = orc.read_index(p)
    k = ix.nlist
    adj = np.array([[u for u in range(k) if u != v] for v in range(k)], dtype=np.int32)
    rng = np.random.default_rng(5)
    for m in (1, 5, 16):
        ex_l, ex_d = orc.probe(ix, Q, m)
        for beam in (m, m + 3, k):
            entry = rng.choice(k, size=3, replace=False).astype(np.int32)
            lists, d, nd = orc.graph_probe(ix, orc.NavGraph(adj, entry, beam), Q, m)
            assert np.array_equal(lists, ex_l), (m, beam)
            assert np.array_equal(d, ex_d), (m, beam)
            assert (nd == k).all()  # everything is visited from the first expansion on


def _ring_graph(k, extra, seed):
    """A ring (every vertex reachable from any other) plus random chords."""
    rng = np.random.default_rng(seed)
    deg = 2 + extra
    adj = -np.ones((k, deg), dtype=np.int32)
    for v in range(k):
        row = [(v + 1) % k, (v - 1) % k]
        others = [u for u in rng.permutation(k) if u != v and u not in row][:extra]
        row += others
        adj[v, :len(row)] = row
    return adj


@pytest.mark.parametrize("kind", ["f32", "i8"])
def test_full_beam_gives_exact_probe(orc, tmp_path, kind):
    p, Q = _small(tmp_path, kind)
    ix = orc.read_index(p)
    adj = _ring_graph(ix.nlist, 2, 9)
    for m in (1, 7, ix.nlist):
        ex_l, ex_d = orc.probe(ix, Q, m)
        lists, d, nd = orc.graph_probe(ix, orc.NavGraph(adj, np.array([0], np.int32), ix.nlist),
                                       Q, m)
        assert np.array_equal(lists, ex_l) and np.array_equal(d, ex_d), m
        assert (nd == ix.nlist).all()


@pytest.mark.parametrize("kind", ["f32", "i8"])
def test_finished_walk_is_closed(orc, tmp_path, kind):
    """beam = m: every neighbour u of a returned list v was offered, so u is
    returned or its (distance, list) key is above the last returned key."""
    p, Q = _small(tmp_path, kind)
    ix = orc.read_index(p)
    _, full_d = orc.probe(ix, Q, ix.nlist)
    full_l, _ = orc.probe(ix, Q, ix.nlist)
    for seed, extra in ((1, 1), (2, 3)):
        adj = _ring_graph(ix.nlist, extra, seed)
        for m in (1, 4, 9):
            lists, d, nd = orc.graph_probe(ix, orc.NavGraph(adj, np.array([3], np.int32), m), Q, m)
            for i in range(len(Q)):
                dist = dict(zip(full_l[i].tolist(), full_d[i].tolist()))
                got = lists[i].tolist()
                assert d[i].tolist() == [dist[v] for v in got]  # exact distances
                keys = [(dist[v], v) for v in got]
                assert keys == sorted(keys)
                last = keys[-1]
                for v in got:
                    for u in adj[v]:
                        if u >= 0 and u not in got:
                            assert (dist[int(u)], int(u)) > last, (i, m, v, u)
                assert m <= nd[i] <= ix.nlist


def test_search_with_full_beam_equals_exact_search(orc, tmp_path):
    p, Q = _small(tmp_path, "i8")
    ix = orc.read_index(p)
    adj = _ring_graph(ix.nlist, 2, 4)
    G = orc.NavGraph(adj, np.array([0], np.int32), ix.nlist)
    a = orc.search(ix, Q, 6, 10, 50)
    b = orc.search(ix, Q, 6, 10, 50, graph=G)
    assert np.array_equal(a.ids, b.ids) and np.array_equal(a.dists, b.dists)
    assert np.array_equal(a.ncand, b.ncand)
    # a narrow walk: the search scans exactly the lists the walk returns
    G1 = orc.NavGraph(adj, np.array([0], np.int32), 1)
    lists, _, _ = orc.graph_probe(ix, G1, Q, 6)
    c = orc.search(ix, Q, 6, 10, 50, graph=G1)
    for i in range(len(Q)):
        uniq, _ = orc.gather_dedup(ix, lists[i])
        assert c.ncand[i] == len(uniq)


def test_builder_graph_shape_and_reachability(tmp_path):
    from paper_2409_16576_amd import builder as B
    rng = np.random.default_rng(3)
    for k, deg, rule in ((300, 16, True), (300, 16, False), (50, 64, True), (2, 4, True)):
        C = rng.standard_normal((k, 12)).astype(np.float32) * 10
        adj, entry = B.build_nav_graph(C, deg=deg, seed=1, rng=rule)
        assert adj.shape == (k, min(deg, k - 1))
        d = ((C[:, None, :].astype(np.float64) - C[None].astype(np.float64)) ** 2).sum(-1)
        for v in range(k):
            row = adj[v][adj[v] >= 0]
            assert len(set(row.tolist())) == len(row) and v not in row
            if not rule:
                assert np.all(np.diff(d[v, row]) >= -1e-3)  # nearest first
            else:  # the leading edges satisfy the relative neighbourhood rule
                lead = []
                for u in row:
                    if all(d[u, x] >= d[v, u] * (1 - 1e-5) for x in lead):
                        lead.append(int(u))
                    else:
                        break
                assert len(lead) >= 1
        seen = np.zeros(k, bool)
        front = list(entry)
        seen[front] = True
        while front:
            nxt = []
            for v in front:
                for u in adj[v]:
                    if u >= 0 and not seen[u]:
                        seen[u] = True
                        nxt.append(int(u))
            front = nxt
        assert seen.all()
        assert len(set(entry.tolist())) == len(entry)
