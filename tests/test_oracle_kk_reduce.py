"""Pins of the oracle's cluster/decluster speed-up for Kamada-Kawai (sec.
3.1: contract nodes with one edge, replace nodes with two edges by one edge,
lay out, decluster).

A hand-worked example fixes which nodes go (tests/golden/closed_forms.json);
the reduced graph, rebuilt explicitly with weighted chain edges, has the
same distances as the full one (the reason the kept nodes can use the full
hop distances); a path comes back as its exact straight embedding; a star's
leaves come back at distance l, evenly around the centre.
"""
import json
import math
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def graph(orc, n, edges):
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    rp, col, _ = orc.build_csr(n, e[:, 0], e[:, 1])
    return rp, col


def test_worked_example(orc):
    g = GOLD["kk_reduce_example"]
    rp, col = graph(orc, g["n"], g["edges"])
    kept, chains, leaves = orc.kk_reduce(rp, col)
    assert np.nonzero(kept)[0].tolist() == g["kept"]
    assert [list(map(int, r)) for r in chains] == g["chain_records"]
    assert [list(map(int, r)) for r in leaves] == g["leaf_records"]


def weighted_distances(n, wedges):
    d = np.full((n, n), np.inf)
    np.fill_diagonal(d, 0.0)
    for a, b, w in wedges:
        d[a, b] = min(d[a, b], w)
        d[b, a] = min(d[b, a], w)
    for k in range(n):
        d = np.minimum(d, d[:, k:k + 1] + d[k:k + 1, :])
    return d


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_reduced_graph_keeps_distances(orc, seed):
    from paper_2403_03504_amd import workloads as w
    g = w.small_component(seed * 31, 120)
    rp, col, _ = orc.build_csr(g.n, g.src, g.dst)
    kept, chains, _ = orc.kk_reduce(rp, col)
    assert 0 < kept.sum() < g.n
    # the reduced graph: edges between kept nodes, plus one edge of length
    # k + 1 per removed chain of k nodes
    wedges = [(i, j, 1) for i in range(g.n) for j in col[rp[i]:rp[i + 1]] if kept[i] and kept[j]]
    per_chain = {}
    for v, a, b, i, k in chains:
        per_chain[(a, b)] = k
    wedges += [(a, b, k + 1) for (a, b), k in per_chain.items()]
    D = orc.hop_distances(rp, col).astype(float)
    R = weighted_distances(g.n, wedges)
    K = np.nonzero(kept)[0]
    assert np.array_equal(R[np.ix_(K, K)], D[np.ix_(K, K)])


def test_path_comes_back_straight(orc):
    rp, col = graph(orc, 7, [[i, i + 1] for i in range(6)])
    kept, chains, leaves = orc.kk_reduce(rp, col)
    assert np.nonzero(kept)[0].tolist() == [1, 5]
    rng = np.random.default_rng(3)
    x, y, _ = orc.kk_reduced_layout(rp, col, rng.normal(size=7), rng.normal(size=7), l=1.3, minimiser="newton",
                                    eps=1e-12)
    # exact straight embedding at spacing l: energy 0
    assert orc.kk_energy(orc.hop_distances(rp, col), x, y, 1.3) < 1e-18


def test_star_leaves_around_the_centre(orc):
    rp, col = graph(orc, 5, [[0, 1], [0, 2], [0, 3], [0, 4]])
    x, y, kept = orc.kk_reduced_layout(rp, col, np.full(5, 2.0), np.full(5, -1.0), l=0.7)
    assert kept.tolist() == [True, False, False, False, False]
    ang = np.arctan2(y[1:] + 1.0, x[1:] - 2.0) % (2 * np.pi)
    assert np.allclose(np.hypot(x[1:] - 2.0, y[1:] + 1.0), 0.7, rtol=1e-14)
    assert np.allclose(ang, 2 * np.pi * np.arange(4) / 4, atol=1e-12)


def test_decluster_places(orc):
    from paper_2403_03504_amd import workloads as w
    g = w.small_component(99, 150)
    rp, col, _ = orc.build_csr(g.n, g.src, g.dst)
    x, y, kept = orc.kk_reduced_layout(rp, col, g.x, g.y, l=1.0, minimiser="newton")
    _, chains, leaves = orc.kk_reduce(rp, col)
    for v, a, b, i, k in chains:
        t = i / (k + 1)
        assert x[v] == pytest.approx(x[a] + t * (x[b] - x[a]), abs=1e-12)
        assert y[v] == pytest.approx(y[a] + t * (y[b] - y[a]), abs=1e-12)
    placed = np.ones(g.n, bool)
    placed[[u for u, _, _, _ in leaves]] = False
    cx, cy = x[placed].mean(), y[placed].mean()
    for u, v, j, k in leaves:
        assert math.hypot(x[u] - x[v], y[u] - y[v]) == pytest.approx(1.0, rel=1e-12)
        if k == 1:  # straight away from the centre of gravity
            out = np.array([x[v] - cx, y[v] - cy])
            assert np.dot([x[u] - x[v], y[u] - y[v]], out) == pytest.approx(np.linalg.norm(out), rel=1e-9)


def test_switches_and_small_cases(orc):
    rp, col = graph(orc, 2, [[0, 1]])
    kept, _, _ = orc.kk_reduce(rp, col)
    assert kept.tolist() == [True, True]  # a 2-node component keeps both
    rp, col = graph(orc, 5, [[0, 1], [1, 2], [2, 3], [3, 4], [4, 0]])
    kept, chains, leaves = orc.kk_reduce(rp, col)
    assert kept.all() and not chains and not leaves  # a pure cycle stays
    rp, col = graph(orc, 5, [[i, i + 1] for i in range(4)])
    assert np.nonzero(orc.kk_reduce(rp, col, leaves=False)[0])[0].tolist() == [0, 4]
    assert np.nonzero(orc.kk_reduce(rp, col, chains=False)[0])[0].tolist() == [1, 2, 3]
