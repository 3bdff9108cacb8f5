"""Pins of the oracle's Barnes-Hut repulsion (the O(N log N) method that
sec. 3.2.1 names as the FMM's predecessor; the comparator of the FMM).

theta = 0 reduces to the exact sum; an accepted cell is exactly its monopole
(closed form below, worked by hand); the error falls as theta falls; the
approximation does not depend on where the picture sits.
"""
import math

import numpy as np
import pytest


def blobs(seed, n, k=6, spread=4.0, radius=100.0):
    rng = np.random.default_rng(seed)
    c = rng.uniform(-radius, radius, (k, 2))
    w = rng.integers(0, k, n)
    p = c[w] + rng.normal(0, spread, (n, 2))
    return p[:, 0], p[:, 1], rng.integers(1, 30, n).astype(float)


@pytest.mark.parametrize("leaf", [1, 8, 64])
def test_theta_zero_is_the_exact_sum(orc, leaf):
    x, y, m = blobs(1, 1500)
    ex, ey = orc.repulsion_exact(x, y, m, 1.7)
    bx, by = orc.repulsion_bh(x, y, m, 1.7, theta=0.0, leaf_size=leaf)
    assert orc.rel_err(bx, by, ex, ey) < 1e-13


def test_far_pair_closed_form(orc):
    # target T (mass 1) at the origin; a pair A (mass 2) at (999, 1000) and
    # B (mass 3) at (1001, 1000).  Root side 1001; with leaf size 2 the root
    # splits and the pair is the leaf (1, 1) of level 1, side 500.5, centre
    # of mass (1000.2, 1000), at distance d = 1414.35 from T: s/d = 0.354.
    x = np.array([0.0, 999.0, 1001.0])
    y = np.array([0.0, 1000.0, 1000.0])
    m = np.array([1.0, 2.0, 3.0])
    com = np.array([1000.2, 1000.0])
    d2 = com @ com
    mono = -5.0 * com / d2
    pa = np.array([999.0, 1000.0])
    pb = np.array([1001.0, 1000.0])
    exact_t = -2.0 * pa / (pa @ pa) - 3.0 * pb / (pb @ pb)
    fx, fy = orc.repulsion_bh(x, y, m, 1.0, theta=0.5, leaf_size=2)
    assert np.allclose([fx[0], fy[0]], mono, rtol=1e-13, atol=0)
    fx, fy = orc.repulsion_bh(x, y, m, 1.0, theta=0.3, leaf_size=2)
    assert np.allclose([fx[0], fy[0]], exact_t, rtol=1e-13, atol=0)
    # A: its own leaf is opened (direct with B), T's single-particle leaf is
    # exact as a monopole, so A's force is exact at any theta
    ex, ey = orc.repulsion_exact(x, y, m)
    for th in (0.3, 0.5, 2.0):
        fx, fy = orc.repulsion_bh(x, y, m, 1.0, theta=th, leaf_size=2)
        assert fx[1] == pytest.approx(ex[1], rel=1e-13) and fy[1] == pytest.approx(ey[1], rel=1e-13)


def test_error_falls_with_theta(orc):
    x, y, m = blobs(2, 4000, spread=10.0)
    ex, ey = orc.repulsion_exact(x, y, m)
    errs = []
    for th in (1.2, 0.8, 0.5, 0.3, 0.15):
        bx, by = orc.repulsion_bh(x, y, m, theta=th, leaf_size=16)
        errs.append(orc.rel_err(bx, by, ex, ey))
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    # a monopole's error is second order in s/d: halving theta cuts it ~4x
    assert errs[2] / errs[4] > 4.0


def test_translation_invariance_and_targets(orc):
    x, y, m = blobs(3, 2000)
    x, y = np.round(x * 64) / 64, np.round(y * 64) / 64  # exact under the shift
    fx, fy = orc.repulsion_bh(x, y, m, theta=0.6, leaf_size=8)
    gx, gy = orc.repulsion_bh(x + 4096.0, y - 2048.0, m, theta=0.6, leaf_size=8)
    assert orc.rel_err(gx, gy, fx, fy) < 1e-11
    tg = np.array([5, 17, 1999, 0, 17])
    hx, hy = orc.repulsion_bh(x, y, m, theta=0.6, leaf_size=8, targets=tg)
    assert np.array_equal(hx, fx[tg]) and np.array_equal(hy, fy[tg])


def test_coincident_points_and_depth_cap(orc):
    # many copies of one point overflow a depth-capped leaf; the copies exert
    # no force on each other, as in the exact sum
    x = np.r_[np.zeros(50), np.linspace(1, 9, 30)]
    y = np.r_[np.zeros(50), np.linspace(3, -2, 30)]
    m = np.ones(80)
    ex, ey = orc.repulsion_exact(x, y, m)
    bx, by = orc.repulsion_bh(x, y, m, theta=0.0, leaf_size=4, bits=3)
    assert orc.rel_err(bx, by, ex, ey) < 1e-13
