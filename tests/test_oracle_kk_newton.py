"""Pins of the oracle's Kamada-Kawai Newton-Raphson minimiser (sec. 3.1).

The derivatives are checked against finite differences of the energy; the
minimiser against hand-derived configurations (tests/golden/closed_forms.json)
and against its own stopping rule.
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
    return orc.hop_distances(rp, col)


def ring(k, r, phase=0.3):
    a = phase + 2 * np.pi * np.arange(k) / k
    return r * np.cos(a), r * np.sin(a)


def test_derivatives_match_finite_differences(orc):
    rng = np.random.default_rng(5)
    n = 10
    d = graph(orc, n, [[i, i + 1] for i in range(n - 1)] + [[0, 6], [3, 9]])
    x, y = rng.normal(size=n) * 3, rng.normal(size=n) * 3
    l, h = 1.3, 1e-5
    for m in range(n):
        gx, gy, hxx, hxy, hyy = orc.kk_grad_hess(d, x, y, m, l)

        def e_at(dx, dy):
            xx, yy = x.copy(), y.copy()
            xx[m] += dx
            yy[m] += dy
            return orc.kk_energy(d, xx, yy, l)

        def g_at(dx, dy):
            xx, yy = x.copy(), y.copy()
            xx[m] += dx
            yy[m] += dy
            return orc.kk_grad_hess(d, xx, yy, m, l)[:2]

        assert gx == pytest.approx((e_at(h, 0) - e_at(-h, 0)) / (2 * h), rel=1e-6, abs=1e-8)
        assert gy == pytest.approx((e_at(0, h) - e_at(0, -h)) / (2 * h), rel=1e-6, abs=1e-8)
        assert hxx == pytest.approx((g_at(h, 0)[0] - g_at(-h, 0)[0]) / (2 * h), rel=1e-5, abs=1e-7)
        assert hxy == pytest.approx((g_at(0, h)[0] - g_at(0, -h)[0]) / (2 * h), rel=1e-5, abs=1e-7)
        assert hxy == pytest.approx((g_at(h, 0)[1] - g_at(-h, 0)[1]) / (2 * h), rel=1e-5, abs=1e-7)
        assert hyy == pytest.approx((g_at(0, h)[1] - g_at(0, -h)[1]) / (2 * h), rel=1e-5, abs=1e-7)


def test_two_nodes_in_one_move(orc):
    # the gradient is radial and the radial second derivative is 2w, so the
    # Newton step lands the pair at distance l exactly
    d = graph(orc, 2, [[0, 1]])
    x, y, k = orc.kk_newton(d, [0.3, -2.0], [1.0, 0.5], l=1.7, eps=1e-9, moves=10)
    assert k == 1
    assert math.hypot(x[0] - x[1], y[0] - y[1]) == pytest.approx(1.7, rel=1e-14)


@pytest.mark.parametrize("l", [1.0, 2.5])
def test_reaches_closed_form_minima(orc, l):
    rng = np.random.default_rng(2)
    # square C4: side a = (8 + 2 sqrt2) l / 10
    d = graph(orc, 4, [[0, 1], [1, 2], [2, 3], [3, 0]])
    sx, sy = ring(4, 1.0)
    x, y, _ = orc.kk_newton(d, sx + 0.2 * rng.normal(size=4), sy + 0.2 * rng.normal(size=4), l, 1e-12, 5000)
    side = [math.hypot(x[i] - x[(i + 1) % 4], y[i] - y[(i + 1) % 4]) for i in range(4)]
    assert np.allclose(side, GOLD["kk_square_c4"]["side_over_l"] * l, rtol=1e-9)
    # star K13: leaves at r = (4 + 2 sqrt3) l / 7 from the centre, 120 degrees apart
    d = graph(orc, 4, [[0, 1], [0, 2], [0, 3]])
    lx, ly = ring(3, 1.0)
    x, y, _ = orc.kk_newton(d, np.r_[0.1, lx], np.r_[-0.1, ly] + 0.1 * rng.normal(size=4), l, 1e-12, 5000)
    r = np.hypot(x[1:] - x[0], y[1:] - y[0])
    assert np.allclose(r, GOLD["kk_star_k13"]["radius_over_l"] * l, rtol=1e-9)
    # path P5: collinear at spacing l (energy 0)
    d = graph(orc, 5, [[i, i + 1] for i in range(4)])
    x, y, _ = orc.kk_newton(d, np.arange(5) * 0.9 * l, 0.1 * rng.normal(size=5), l, 1e-12, 20000)
    assert orc.kk_energy(d, x, y, l) < 1e-16


def test_stops_by_its_rule(orc):
    from paper_2403_03504_amd import workloads as w
    g = w.small_component(77, 60)
    rp, col, _ = orc.build_csr(g.n, g.src, g.dst)
    d = orc.hop_distances(rp, col)
    rng = np.random.default_rng(3)
    x0, y0 = rng.uniform(-5, 5, g.n), rng.uniform(-5, 5, g.n)
    x, y, k = orc.kk_newton(d, x0, y0, 1.0, 1e-3, 100000)
    assert k < 100000
    assert max(math.hypot(*orc.kk_grad_hess(d, x, y, m)[:2]) for m in range(g.n)) < 1e-3
    # a budget of moves is honoured, and fewer moves leave a higher energy
    x1, y1, k1 = orc.kk_newton(d, x0, y0, 1.0, 1e-3, 10)
    assert k1 == 10 and orc.kk_energy(d, x1, y1) > orc.kk_energy(d, x, y)


def test_energy_never_rises(orc):
    # every accepted step lowers the moving node's energy, which is the part
    # of E that depends on it, so E falls move by move
    from paper_2403_03504_amd import workloads as w
    g = w.small_component(12, 40)
    rp, col, _ = orc.build_csr(g.n, g.src, g.dst)
    d = orc.hop_distances(rp, col)
    rng = np.random.default_rng(8)
    x0, y0 = rng.uniform(-4, 4, g.n), rng.uniform(-4, 4, g.n)
    e = [orc.kk_energy(d, *orc.kk_newton(d, x0, y0, 1.0, 1e-6, k)[:2]) for k in range(0, 60)]
    assert all(b <= a * (1 + 1e-14) for a, b in zip(e, e[1:]))
    assert e[-1] < 0.5 * e[0]
