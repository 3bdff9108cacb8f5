"""Pins of the oracle's component assembly (sec. 4: rescale the component
layouts to a similar density, link the components into a tree, lay the tree
out by Kamada-Kawai, split and reassemble when it is large).

Each check rests on a hand-derived value (tests/golden/closed_forms.json), an
invariant of the construction, or an independent recomputation (parent walks
instead of the all-pairs algorithm, node centroids of the finished drawing
instead of the composed translations).
"""
import json
import math
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def square(cx, cy, h=1.0):
    return (np.array([cx - h, cx + h, cx - h, cx + h]), np.array([cy - h, cy - h, cy + h, cy + h]))


# --- density rescaling ----------------------------------------------------------

def test_frame_of_square_matches_hand_values(orc):
    g = GOLD["assembly_square_frame"]
    p = np.array(g["nodes"])
    cen, s, R = orc.component_frames(p[:, 0], p[:, 1], [0, 4], g["density"])
    assert np.allclose(cen[0], g["centroid"], rtol=0, atol=1e-15)
    assert s[0] == pytest.approx(g["scale"], rel=1e-14)
    assert R[0] == pytest.approx(g["radius"], rel=1e-14)


def test_uniform_disc_lands_at_target_density(orc):
    # nodes spread uniformly over a disc: after rescaling, nodes per unit area
    # of the disc they fill must be the target density (the reading's intent)
    rng = np.random.default_rng(5)
    n = 40000
    r = 7.0 * np.sqrt(rng.random(n))
    a = 2 * np.pi * rng.random(n)
    x, y = 3.0 + r * np.cos(a), -1.0 + r * np.sin(a)
    for dens in (0.25, 1.0, 4.0):
        cen, s, R = orc.component_frames(x, y, [0, n], dens)
        assert n / (math.pi * R[0] ** 2) == pytest.approx(dens, rel=0.01)
        assert np.allclose(cen[0], (3.0, -1.0), atol=0.1)


def test_frames_of_degenerate_components(orc):
    # one node, and three coincident nodes: no spread, so no scaling, radius 0
    x = np.array([5.0, 1.0, 1.0, 1.0, -2.0, 0.0])
    y = np.array([6.0, 2.0, 2.0, 2.0, 0.0, 0.0])
    cen, s, R = orc.component_frames(x, y, [0, 1, 4, 6], 1.0)
    assert list(s[:2]) == [1.0, 1.0] and list(R[:2]) == [0.0, 0.0]
    assert np.array_equal(cen[:2], [[5.0, 6.0], [1.0, 2.0]])
    # two nodes 2 apart: rho = 1, area 2 pi, s = sqrt(2 / (2 pi)) = 1/sqrt(pi)
    assert s[2] == pytest.approx(1 / math.sqrt(math.pi), rel=1e-14)
    assert R[2] == pytest.approx(1 / math.sqrt(math.pi), rel=1e-14)


def test_frames_scale_free(orc):
    # the same shape at any size and place gives the same radius
    rng = np.random.default_rng(9)
    x, y = rng.normal(size=50), rng.normal(size=50)
    _, s1, R1 = orc.component_frames(x, y, [0, 50], 2.0)
    _, s2, R2 = orc.component_frames(7.5 * x - 4, 7.5 * y + 11, [0, 50], 2.0)
    assert R2[0] == pytest.approx(R1[0], rel=1e-13)
    assert s2[0] == pytest.approx(s1[0] / 7.5, rel=1e-13)


# --- the meta-graph ---------------------------------------------------------------

def test_meta_tree_worked_example(orc):
    g = GOLD["assembly_meta_tree_example"]
    par, el = orc.meta_tree(np.array(g["nodes"]), np.array(g["radius"]), g["gap"])
    assert par.tolist() == g["parent"]
    assert np.allclose(el, g["edge"], rtol=0, atol=1e-15)
    D = orc.tree_distances(par, el)
    for i, j, d in g["pairs"]:
        assert D[i, j] == pytest.approx(d, abs=1e-13)
        assert D[j, i] == D[i, j]


def path_to_root(par, el, t):
    acc, out = 0.0, {t: 0.0}
    while par[t] >= 0:
        acc += el[t]
        t = par[t]
        out[t] = acc
    return out


def test_meta_tree_invariants_and_distances(orc):
    rng = np.random.default_rng(21)
    g = 120
    w = rng.integers(1, 30, g)
    R = rng.random(g) * 3
    par, el = orc.meta_tree(w, R, 0.7)
    assert par[0] == -1 and np.all(par[1:] >= 0) and np.all(par[1:] < np.arange(1, g))
    for t in range(1, g):
        # a largest of the previous items, and no earlier item as large
        assert w[par[t]] == w[:t].max() and np.all(w[:par[t]] < w[par[t]])
        assert el[t] == pytest.approx(R[t] + R[par[t]] + 0.7, abs=1e-14)
    # distances by walking both items up to their lowest common ancestor
    D = orc.tree_distances(par, el)
    for _ in range(300):
        i, j = rng.integers(0, g, 2)
        ui, uj = path_to_root(par, el, i), path_to_root(par, el, j)
        ref = min(ui[a] + uj[a] for a in ui if a in uj)
        assert D[i, j] == pytest.approx(ref, rel=1e-13)


# --- Kamada-Kawai with real lengths (sequential majorization) --------------------

def test_sweeps_two_items_exact_after_one_sweep(orc):
    D = np.array([[0.0, 3.25], [3.25, 0.0]])
    x, y = orc.kk_sweeps(D, [0.4, -1.0], [0.2, 2.5], 1)
    assert math.hypot(x[0] - x[1], y[0] - y[1]) == pytest.approx(3.25, rel=1e-14)


def test_sweeps_star_k13_reaches_closed_form(orc):
    r_ref = GOLD["kk_star_k13"]["radius_over_l"]
    D = np.array([[0, 1, 1, 1], [1, 0, 2, 2], [1, 2, 0, 2], [1, 2, 2, 0]], dtype=float)
    x, y = orc.kk_sweeps(D, [0.1, 1.0, -0.7, 0.2], [0.0, 0.3, 0.5, -1.1], 2000)
    r = np.hypot(x[1:] - x[0], y[1:] - y[0])
    assert np.allclose(r, r_ref, rtol=1e-9)
    for a, b in ((1, 2), (1, 3), (2, 3)):
        assert math.hypot(x[a] - x[b], y[a] - y[b]) == pytest.approx(r_ref * math.sqrt(3), rel=1e-9)


def test_sweeps_embed_a_path_exactly(orc):
    # path metrics embed on a line: that embedding (energy 0) is a fixed point
    # of a sweep, and sweeps from elsewhere head to it
    el = np.array([0.0, 1.5, 0.25, 2.0, 1.0, 0.75])
    par = np.array([-1, 0, 1, 2, 3, 4])
    D = orc.tree_distances(par, el)
    line = np.cumsum(el)
    x, y = orc.kk_sweeps(D, line, np.zeros(6), 1)
    assert np.abs(x - line).max() < 1e-14 and np.abs(y).max() == 0.0
    x0, y0 = orc.meta_initial(D)
    e = [orc.stress(D, *orc.kk_sweeps(D, x0, y0, s)) for s in (10, 100, 1000, 10000)]
    assert e[0] > e[1] > e[2] > e[3] and e[3] < 1e-6 * e[0]


def test_sweeps_never_raise_the_energy(orc):
    rng = np.random.default_rng(4)
    w = rng.integers(1, 100, 60)
    par, el = orc.meta_tree(w, rng.random(60) * 4, 1.0)
    D = orc.tree_distances(par, el)
    x, y = orc.meta_initial(D)
    e = orc.stress(D, x, y)
    for _ in range(30):
        x, y = orc.kk_sweeps(D, x, y, 1)
        e2 = orc.stress(D, x, y)
        assert e2 <= e * (1 + 1e-13)
        e = e2


def test_meta_initial_positions(orc):
    par, el = orc.meta_tree(np.array([5, 1, 1, 1]), np.zeros(4), 2.0)
    D = orc.tree_distances(par, el)
    x, y = orc.meta_initial(D)
    assert (x[0], y[0]) == (0.0, 0.0)
    assert np.allclose(np.hypot(x, y), D[0], rtol=1e-15)
    assert np.allclose(np.arctan2(y[1:], x[1:]) % (2 * np.pi), 2 * np.pi * np.arange(1, 4) / 4)


# --- the whole assembly -----------------------------------------------------------

def random_components(seed, K, lo=1, hi=40):
    rng = np.random.default_rng(seed)
    sizes = rng.integers(lo, hi, K)
    off = np.concatenate([[0], np.cumsum(sizes)])
    x = rng.normal(size=off[-1]) * rng.uniform(0.5, 20, K).repeat(sizes) + rng.uniform(-100, 100, K).repeat(sizes)
    y = rng.normal(size=off[-1]) * rng.uniform(0.5, 20, K).repeat(sizes) + rng.uniform(-100, 100, K).repeat(sizes)
    return off, x, y, rng.permutation(K)


def test_two_components_closed_form(orc):
    xa, ya = square(10.0, 4.0, 2.0)
    xb = np.array([-3.0, -1.0])
    yb = np.array([0.0, 0.0])
    x, y = np.concatenate([xa, xb]), np.concatenate([ya, yb])
    prm = orc.AssembleParams(density=0.5, gap=0.75, sweeps=5)
    A = orc.assemble(x, y, [0, 4, 6], [0, 1], prm)
    R0 = math.sqrt(2) / math.sqrt(math.pi * 0.5)  # square frame, hand value
    R1 = math.sqrt(2 / (2 * math.pi * 0.5))         # two nodes: rho = 1
    D = R0 + R1 + 0.75
    assert A.radius[0] == pytest.approx(R0, rel=1e-14) and A.radius[1] == pytest.approx(R1, rel=1e-14)
    assert np.allclose(A.shift[0], (2 * D / 6, 0.0), atol=1e-13)
    assert np.allclose(A.shift[1], (-4 * D / 6, 0.0), atol=1e-13)
    assert A.parent.tolist() == [-1, 0]


def test_single_component_is_centred_and_scaled(orc):
    rng = np.random.default_rng(2)
    x, y = rng.normal(size=30) * 5 + 40, rng.normal(size=30) * 5 - 7
    A = orc.assemble(x, y, [0, 30], [0])
    assert abs(A.x.mean()) < 1e-12 and abs(A.y.mean()) < 1e-12
    rho = math.sqrt(np.mean(A.x ** 2 + A.y ** 2))
    assert 30 / (2 * math.pi * rho ** 2) == pytest.approx(1.0, rel=1e-12)
    assert A.levels == 1 and A.groups == 1


@pytest.mark.parametrize("K,M", [(7, 256), (300, 64), (1000, 16)])
def test_assembly_invariants(orc, K, M):
    off, x, y, order = random_components(K + 3, K)
    prm = orc.AssembleParams(density=0.8, gap=1.5, max_group=M, sweeps=20)
    A = orc.assemble(x, y, off, order, prm)
    n = off[-1]
    ext = np.max(np.hypot(A.x, A.y))
    # the drawing is centred: node centroid at the origin
    assert abs(A.x.sum()) / n < 1e-12 * ext and abs(A.y.sum()) / n < 1e-12 * ext
    for k in range(K):
        a, b = off[k], off[k + 1]
        # every component keeps its shape, scaled by its own factor
        ia, ib = a, b - 1
        d0 = math.hypot(x[ia] - x[ib], y[ia] - y[ib])
        d1 = math.hypot(A.x[ia] - A.x[ib], A.y[ia] - A.y[ib])
        assert d1 == pytest.approx(A.scale[k] * d0, rel=1e-12, abs=1e-12 * ext)
        # its node centroid is its shift
        assert np.allclose([A.x[a:b].mean(), A.y[a:b].mean()], A.shift[k], rtol=0, atol=1e-11 * ext)
    levels = 1
    m = K
    while m > M:
        m = -(-m // M)
        levels += 1
    assert A.levels == levels
    # first-level links: within a group, to a largest earlier component
    nodes = np.diff(off)
    for t in range(K):
        k = order[t]
        if t % M == 0:
            assert A.parent[k] == -1
        else:
            g0 = t - t % M
            prev = nodes[order[g0:t]]
            assert nodes[A.parent[k]] == prev.max()


def test_assembly_places_groups_by_their_own_layout(orc):
    # two levels: the node centroid of every first-level group, relative to
    # the first group's, is where the second level placed that group
    K, M = 40, 8
    off, x, y, order = random_components(77, K)
    prm = orc.AssembleParams(gap=1.0, max_group=M, sweeps=15)
    A = orc.assemble(x, y, off, order, prm)
    assert A.levels == 2
    nodes = np.diff(off)
    groups = [order[a:a + M] for a in range(0, K, M)]
    cents = []
    for comps in groups:
        W = nodes[comps].sum()
        cents.append(np.array([np.sum(nodes[comps] * A.shift[comps, 0]), np.sum(nodes[comps] * A.shift[comps, 1])]) / W)
    # rebuild the second level independently from the group frames
    Wg = np.array([nodes[c].sum() for c in groups])
    Rg = []
    for comps, c in zip(groups, cents):
        Rg.append(max(math.hypot(*(A.shift[k] - c)) + A.radius[k] for k in comps))
    par, el = orc.meta_tree(Wg, np.array(Rg), 1.0)
    D = orc.tree_distances(par, el)
    px, py = orc.kk_sweeps(D, *orc.meta_initial(D), 15)
    for gi in range(1, len(groups)):
        assert np.allclose(cents[gi] - cents[0], (px[gi] - px[0], py[gi] - py[0]), rtol=1e-9, atol=1e-9)


def test_assembly_of_single_nodes(orc):
    K = 50
    off = np.arange(K + 1)
    rng = np.random.default_rng(8)
    x, y = rng.normal(size=K), rng.normal(size=K)
    A = orc.assemble(x, y, off, rng.permutation(K), orc.AssembleParams(gap=2.0, sweeps=10))
    assert np.all(A.scale == 1.0) and np.all(A.radius == 0.0)
    assert np.allclose(np.c_[A.x, A.y], A.shift, atol=1e-12)
