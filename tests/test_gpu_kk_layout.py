"""GPU parity for the Kamada-Kawai path and the whole-layout pipeline.

Hop distances: bit-exact against the oracle's breadth-first search.  One KK
step: FP32 vs FP64 on identical positions, within 1e-5 (l + |p|) (a handful
of FP32 roundings of terms of size ~|p|).  Layout dispatch: each component's
result equals the same component laid out on its own (bitwise).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay
    return fa2lay


@pytest.fixture(scope="module")
def ctx(fl):
    c = fl.Context(0)
    yield c
    c.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def small_batch(n_comp, seed, lo=2, hi=200):
    from paper_2403_03504_amd import workloads as w
    sizes = np.clip(w.small_component_sizes(seed, n_comp, max(lo, 3), hi), lo, hi)
    parts = [w.small_component(seed * 1000 + i, int(s)) for i, s in enumerate(sizes)]
    g, offs = w.union(parts)
    return g, offs.astype(np.int32)


def test_hop_distances_bit_exact(ctx, fl, orc):
    _note("hop distances, 300 components")
    g, offs = small_batch(300, 31)
    G = ctx.build_csr(g.n, dev(g.src), dev(g.dst))
    dist, doff = ctx.hop_distances(G, offs)
    D = host(dist)
    rp, col, deg = orc.build_csr(g.n, g.src, g.dst)
    for k in range(len(offs) - 1):
        a, b = offs[k], offs[k + 1]
        n = b - a
        lrp = rp[a:b + 1] - rp[a]
        lcol = col[rp[a]:rp[b]] - a
        ref = orc.hop_distances(lrp, lcol)
        assert np.array_equal(D[doff[k]:doff[k] + n * n].reshape(n, n), ref), k


def test_hop_distances_rejects_bad_ranges(ctx, fl):
    _note("hop distances, disconnected range")
    src = np.array([0, 2], np.int32)
    dst = np.array([1, 3], np.int32)
    G = ctx.build_csr(4, dev(src), dev(dst))
    with pytest.raises(fl.FlError) as e:
        ctx.hop_distances(G, [0, 4])
    assert e.value.status == fl.FL_EINVAL


@pytest.mark.parametrize("l", [1.0, 2.5])
def test_kk_one_step_parity(ctx, fl, orc, l):
    _note("kk one step, l =", l)
    g, offs = small_batch(200, 37)
    G = ctx.build_csr(g.n, dev(g.src), dev(g.dst))
    dist, doff = ctx.hop_distances(G, offs)
    D = host(dist)
    x, y = dev(g.x), dev(g.y)
    ctx.kk_steps(offs, dist, x, y, fl.kk_params(l=l, steps=1))
    gx, gy = host(x), host(y)
    for k in range(len(offs) - 1):
        a, b = offs[k], offs[k + 1]
        n = b - a
        rx, ry = orc.kk_steps(D[doff[k]:doff[k] + n * n].reshape(n, n), g.x[a:b], g.y[a:b], l, 1)
        tol = 1e-5 * (l + np.abs(rx).max() + np.abs(ry).max())
        assert np.max(np.abs(gx[a:b] - rx)) <= tol and np.max(np.abs(gy[a:b] - ry)) <= tol, k


def test_kk_closed_form_fixed_points(ctx, fl, orc):
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
    _note("kk fixed points")
    l = 1.5
    a = gold["kk_square_c4"]["side_over_l"] * l
    ang = 0.3 + np.pi / 2 * np.arange(4)
    sx, sy = a / np.sqrt(2) * np.cos(ang), a / np.sqrt(2) * np.sin(ang)
    rr = gold["kk_star_k13"]["radius_over_l"] * l
    ang3 = 0.1 + 2 * np.pi / 3 * np.arange(3)
    # square (nodes 0..3) and star (nodes 4..7, centre 4) as two components
    src = np.array([0, 1, 2, 3, 4, 4, 4], np.int32)
    dst = np.array([1, 2, 3, 0, 5, 6, 7], np.int32)
    x = np.concatenate([sx, [0.0], rr * np.cos(ang3)]).astype(np.float32)
    y = np.concatenate([sy, [0.0], rr * np.sin(ang3)]).astype(np.float32)
    G = ctx.build_csr(8, dev(src), dev(dst))
    xd, yd = dev(x), dev(y)
    ctx.kk_layout(G, [0, 4, 8], xd, yd, fl.kk_params(l=l, steps=50))
    assert np.allclose(host(xd), x, atol=2e-5) and np.allclose(host(yd), y, atol=2e-5)


def test_kk_many_steps_reduce_stress(ctx, fl, orc):
    _note("kk 200 steps")
    g, offs = small_batch(100, 41)
    G = ctx.build_csr(g.n, dev(g.src), dev(g.dst))
    dist, doff = ctx.hop_distances(G, offs)
    D = host(dist)
    x, y = dev(g.x), dev(g.y)
    ctx.kk_steps(offs, dist, x, y, fl.kk_params(steps=200))
    gx, gy = host(x), host(y)
    for k in range(len(offs) - 1):
        a, b = offs[k], offs[k + 1]
        n = b - a
        Dk = D[doff[k]:doff[k] + n * n].reshape(n, n)
        e0 = orc.kk_energy(Dk, g.x[a:b], g.y[a:b], 1.0)
        e1 = orc.kk_energy(Dk, gx[a:b], gy[a:b], 1.0)
        assert e1 <= e0 + 1e-9


def test_layout_dispatch_matches_parts(ctx, fl, orc):
    """fl_layout on a mix of single nodes, small and large components gives
    each component exactly what it gets on its own."""
    from paper_2403_03504_amd import workloads as w
    _note("layout dispatch")
    parts = [w.small_component(900 + i, int(s)) for i, s in enumerate([3, 7, 40, 150, 2])]
    parts.append(w.scaled(77, 6000, hubs_per_4000=False))
    parts.append(w.scaled(78, 3000, hubs_per_4000=False))
    single = w.Graph(n=1, src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                     x=np.array([5.0], np.float32), y=np.array([-3.0], np.float32))
    parts.insert(2, single)
    # interleave node ids: shuffle the union so components are not contiguous
    g, offs = w.union(parts)
    rng = np.random.default_rng(5)
    perm = rng.permutation(g.n).astype(np.int32)  # new id of old node i
    src, dst = perm[g.src], perm[g.dst]
    x = np.empty_like(g.x)
    y = np.empty_like(g.y)
    x[perm], y[perm] = g.x, g.y
    G = ctx.build_csr(g.n, dev(src), dev(dst))
    xd, yd = dev(x), dev(y)
    fa2 = fl.default_params(repulsion=fl.REP_FMM, p=8, leaf_size=32)
    kk = fl.kk_params(steps=100)
    st = ctx.layout(G, xd, yd, fa2, 30, kk, kk_max_nodes=256, fmm_min_nodes=4096)
    _note("  stats", st)
    assert st["n_comp"] == len(parts) and st["n_single"] == 1 and st["n_fa2"] == 2
    lx, ly = host(xd), host(yd)
    # each part alone
    for k, part in enumerate(parts):
        ids = perm[offs[k]:offs[k + 1]]  # new ids of this part's nodes, in the part's order
        if part.n == 1:
            assert lx[ids[0]] == 0.0 and ly[ids[0]] == 0.0
            continue
        Gp = ctx.build_csr(part.n, dev(part.src), dev(part.dst))
        # the layout numbers a component's nodes by ascending id: do the same
        order = np.argsort(ids, kind="stable")
        inv = np.empty_like(order)
        inv[order] = np.arange(part.n)
        Gp = ctx.build_csr(part.n, dev(inv[part.src].astype(np.int32)), dev(inv[part.dst].astype(np.int32)))
        px, py = dev(part.x[order]), dev(part.y[order])
        if part.n <= 256:
            ctx.kk_layout(Gp, [0, part.n], px, py, kk)
        else:
            p = fa2 if part.n >= 4096 else fl.default_params(repulsion=fl.REP_EXACT, p=8, leaf_size=32)
            ctx.fa2_run(Gp, px, py, fl.FA2State.zeros(part.n, "cuda"), p, 30)
        assert np.array_equal(host(px), lx[ids[order]]), k
        assert np.array_equal(host(py), ly[ids[order]]), k


def test_kk_pairs_land_at_l(ctx, fl):
    # 2-node components: one majorization step puts each pair at distance l
    # about its midpoint (closed form), and further steps keep it there
    _note("kk pairs")
    rng = np.random.default_rng(9)
    k = 50
    src = np.arange(0, 2 * k, 2, dtype=np.int32)
    dst = src + 1
    x = rng.uniform(-3, 3, 2 * k).astype(np.float32)
    y = rng.uniform(-3, 3, 2 * k).astype(np.float32)
    G = ctx.build_csr(2 * k, dev(src), dev(dst))
    offs = np.arange(0, 2 * k + 1, 2, dtype=np.int32)
    for steps in (1, 200):
        xd, yd = dev(x), dev(y)
        ctx.kk_layout(G, offs, xd, yd, fl.kk_params(l=1.25, steps=steps))
        px, py = host(xd), host(yd)
        r = np.hypot(px[0::2] - px[1::2], py[0::2] - py[1::2])
        assert np.allclose(r, 1.25, rtol=1e-5)
        assert np.allclose((px[0::2] + px[1::2]) / 2, (x[0::2] + x[1::2]) / 2, atol=1e-5)
