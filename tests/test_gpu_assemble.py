"""GPU parity of the component assembly (sec. 4) against the oracle.

Integer work (the first-level meta-graph links) must match bit for bit.
Component frames (centroid, scale, radius) are FP64 sums of the same FP32
positions in another order: 1e-12 relative.  The meta-graph layout runs in
FP32: with no sweeps (the starting layout) and after one sweep the shifts
must match the FP64 oracle within 2e-6 and 2e-5 of the drawing's extent;
after many sweeps (where rounding differences may steer the descent into a
different, equally good, neighbourhood) every group's layout must reach the
oracle's energy within 1e-3 and the shifts must stay within 1e-3 of the
extent, each component must keep its shape, and the drawing must be
centred.
"""
import math
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


def make_components(seed, sizes, spread=(0.5, 20.0), centre=100.0):
    """Nodes grouped by component (component k = nodes off[k]..off[k+1]),
    FP32 positions, labels = first node id of each component."""
    rng = np.random.default_rng(seed)
    sizes = np.asarray(sizes, dtype=np.int64)
    K = sizes.shape[0]
    off = np.concatenate([[0], np.cumsum(sizes)])
    sp = rng.uniform(*spread, K).repeat(sizes)
    x = (rng.normal(size=off[-1]) * sp + rng.uniform(-centre, centre, K).repeat(sizes)).astype(np.float32)
    y = (rng.normal(size=off[-1]) * sp + rng.uniform(-centre, centre, K).repeat(sizes)).astype(np.float32)
    label = off[:-1].repeat(sizes).astype(np.int32)
    return off, x, y, label, rng.permutation(K).astype(np.int32)


def power_law_sizes(seed, K, lo=1, hi=200, alpha=2.2):
    rng = np.random.default_rng(seed)
    u = rng.random(K)
    return np.clip(np.floor(lo * (1 - u) ** (-1 / (alpha - 1))), lo, hi).astype(np.int64)


def run_gpu(ctx, fl, off, x, y, label, order, **kw):
    K = len(off) - 1
    prm = fl.assemble_params(**kw)
    X, Y = dev(x), dev(y)
    frame = torch.empty(K * 6, dtype=torch.float64, device="cuda")
    parent = torch.empty(K, dtype=torch.int32, device="cuda")
    st = ctx.assemble(dev(label), K, order, X, Y, prm, frame, parent)
    return host(X), host(Y), host(frame).reshape(K, 6), host(parent), st


def oracle(orc, off, x, y, order, **kw):
    prm = orc.AssembleParams(**kw)
    return orc.assemble(x.astype(np.float64), y.astype(np.float64), off, order, prm)


def check_frames(F, A):
    ext = max(1.0, np.abs(A.centroid).max())
    assert np.allclose(F[:, 0:2], A.centroid, rtol=0, atol=1e-12 * ext)
    assert np.allclose(F[:, 2], A.scale, rtol=1e-12, atol=0)
    assert np.allclose(F[:, 3], A.radius, rtol=1e-12, atol=1e-300)


def check_shapes(x, y, off, x0, y0, F, tol):
    """Every node at s (p - c) + shift, with the frame the GPU reported."""
    sizes = np.diff(off)
    k = np.repeat(np.arange(len(sizes)), sizes)
    ex = F[k, 2] * (x0.astype(np.float64) - F[k, 0]) + F[k, 4]
    ey = F[k, 2] * (y0.astype(np.float64) - F[k, 1]) + F[k, 5]
    ext = max(1.0, np.abs(np.r_[ex, ey]).max())
    assert np.abs(x - ex).max() <= tol * ext and np.abs(y - ey).max() <= tol * ext


def group_stress(orc, order, nodes, radius, shift, M, gap):
    """Energy of every first-level group's layout, items placed at their
    components' shifts (a group's layout up to a translation)."""
    out = []
    K = len(order)
    for a in range(0, K, M):
        comps = order[a:a + M]
        par, el = orc.meta_tree(nodes[comps], radius[comps], gap)
        D = orc.tree_distances(par, el)
        out.append(orc.stress(D, shift[comps, 0], shift[comps, 1]) if len(comps) > 1 else 0.0)
    return np.array(out)


@pytest.mark.parametrize("sweeps,tol", [(0, 2e-6), (1, 2e-5)])
def test_frames_links_and_early_layout_match_oracle(ctx, fl, orc, sweeps, tol):
    sizes = power_law_sizes(3, 700)
    off, x, y, label, order = make_components(5, sizes)
    _note(f"assembly K=700 n={off[-1]} M=64 sweeps={sweeps}")
    gx, gy, F, par, st = run_gpu(ctx, fl, off, x, y, label, order, max_group=64, sweeps=sweeps, gap=1.5,
                                 density=0.8)
    A = oracle(orc, off, x, y, order, max_group=64, sweeps=sweeps, gap=1.5, density=0.8)
    assert st["levels"] == A.levels == 2 and st["groups"] == A.groups
    check_frames(F, A)
    assert np.array_equal(par, A.parent)
    ext = np.abs(A.shift).max()
    err = np.abs(F[:, 4:6] - A.shift).max() / ext
    print("shift error / extent", err)
    assert err <= tol
    assert np.abs(gx - A.x).max() <= tol * ext + 1e-6 * ext and np.abs(gy - A.y).max() <= tol * ext + 1e-6 * ext
    check_shapes(gx, gy, off, x, y, F, 2e-7)


def test_full_sweeps_reach_oracle_energy(ctx, fl, orc):
    sizes = power_law_sizes(7, 3000, lo=3)
    sizes[::500] = [5000, 20000, 7000, 12000, 3000, 9000]
    off, x, y, label, order = make_components(9, sizes)
    M, gap = 256, 1.0
    _note(f"assembly K=3000 n={off[-1]} M={M} sweeps=100")
    gx, gy, F, par, st = run_gpu(ctx, fl, off, x, y, label, order, max_group=M, sweeps=100, gap=gap)
    A = oracle(orc, off, x, y, order, max_group=M, sweeps=100, gap=gap)
    check_frames(F, A)
    assert np.array_equal(par, A.parent)
    nodes = np.diff(off)
    eg = group_stress(orc, order, nodes, A.radius, F[:, 4:6], M, gap)
    eo = group_stress(orc, order, nodes, A.radius, A.shift, M, gap)
    print("group energies gpu/oracle", np.round(eg / np.maximum(eo, 1e-300), 6))
    assert np.all(eg <= eo * (1 + 1e-3) + 1e-9)
    err = np.abs(F[:, 4:6] - A.shift).max() / np.abs(A.shift).max()
    print("shift error / extent", err)
    assert err <= 1e-3
    check_shapes(gx, gy, off, x, y, F, 2e-7)
    w = nodes.astype(np.float64)
    ext = np.abs(F[:, 4:6]).max()
    assert abs(np.sum(w * F[:, 4])) / w.sum() < 1e-9 * ext and abs(np.sum(w * F[:, 5])) / w.sum() < 1e-9 * ext


def test_large_components_span_many_tiles(ctx, fl, orc):
    sizes = np.array([50000, 3, 70001, 1, 2048, 2049, 4097])
    off, x, y, label, order = make_components(13, sizes, spread=(1.0, 300.0), centre=5000.0)
    _note(f"assembly K=7 n={off[-1]} (tiles)")
    gx, gy, F, par, st = run_gpu(ctx, fl, off, x, y, label, order, sweeps=30)
    A = oracle(orc, off, x, y, order, sweeps=30)
    check_frames(F, A)
    assert np.array_equal(par, A.parent)
    assert np.abs(F[:, 4:6] - A.shift).max() <= 1e-4 * np.abs(A.shift).max()
    check_shapes(gx, gy, off, x, y, F, 2e-7)


def test_shuffled_node_ids_and_labels(ctx, fl, orc):
    sizes = power_law_sizes(17, 400)
    off, x, y, _, order = make_components(19, sizes)
    n = off[-1]
    rng = np.random.default_rng(23)
    newid = rng.permutation(n)  # node i of the grouped layout gets id newid[i]
    comp = np.repeat(np.arange(len(sizes)), sizes)
    lab_by_comp = np.full(len(sizes), n)
    np.minimum.at(lab_by_comp, comp, newid)
    # components are numbered by ascending label: renumber, keep node order within
    rank = np.argsort(np.argsort(lab_by_comp, kind="stable"), kind="stable")
    xs = np.empty(n, np.float32)
    ys = np.empty(n, np.float32)
    xs[newid], ys[newid] = x, y
    label = np.empty(n, np.int32)
    label[newid] = lab_by_comp[comp]
    # oracle input: nodes grouped by the renumbered components, in id order
    ids = np.argsort(label, kind="stable")
    goff = np.concatenate([[0], np.cumsum(np.bincount(rank[comp], minlength=len(sizes)))])
    order2 = rng.permutation(len(sizes)).astype(np.int32)
    _note(f"assembly shuffled ids K={len(sizes)} n={n}")
    gx, gy, F, par, st = run_gpu(ctx, fl, goff, xs, ys, label, order2, max_group=32, sweeps=1)
    A = oracle(orc, goff, xs[ids], ys[ids], order2, max_group=32, sweeps=1)
    check_frames(F, A)
    assert np.array_equal(par, A.parent)
    ext = np.abs(A.shift).max()
    assert np.abs(gx[ids] - A.x).max() <= 2e-5 * ext and np.abs(gy[ids] - A.y).max() <= 2e-5 * ext


@pytest.mark.parametrize("K,M", [(1, 256), (257, 256), (50, 2), (1000, 3)])
def test_edge_shapes(ctx, fl, orc, K, M):
    sizes = power_law_sizes(K + M, K)
    off, x, y, label, order = make_components(K * 7 + M, sizes)
    _note(f"assembly edge K={K} M={M}")
    gx, gy, F, par, st = run_gpu(ctx, fl, off, x, y, label, order, max_group=M, sweeps=1)
    A = oracle(orc, off, x, y, order, max_group=M, sweeps=1)
    assert st["levels"] == A.levels and st["groups"] == A.groups
    check_frames(F, A)
    assert np.array_equal(par, A.parent)
    ext = max(np.abs(A.shift).max(), 1.0)
    assert np.abs(F[:, 4:6] - A.shift).max() <= 2e-5 * ext
    check_shapes(gx, gy, off, x, y, F, 2e-7)


def test_single_nodes_only(ctx, fl, orc):
    K = 5000
    off, x, y, label, order = make_components(29, np.ones(K, np.int64))
    _note("assembly of single nodes")
    gx, gy, F, par, st = run_gpu(ctx, fl, off, x, y, label, order, sweeps=0)
    A = oracle(orc, off, x, y, order, sweeps=0)
    assert np.all(F[:, 2] == 1.0) and np.all(F[:, 3] == 0.0)
    assert np.array_equal(par, A.parent)
    ext = np.abs(A.shift).max()
    assert np.abs(gx - A.x).max() <= 2e-6 * ext


def test_rejects_bad_input(ctx, fl):
    off, x, y, label, order = make_components(31, [3, 4, 5])
    X, Y = dev(x), dev(y)
    prm = fl.assemble_params()
    _note("assembly error paths")
    for bad_order in ([0, 1, 1], [0, 1, 3], [-1, 0, 1]):
        with pytest.raises(fl.FlError) as e:
            ctx.assemble(dev(label), 3, bad_order, X, Y, prm)
        assert e.value.status == fl.FL_EINVAL
    with pytest.raises(ValueError):
        ctx.assemble(dev(label), 3, [0, 1], X, Y, prm)
    with pytest.raises(fl.FlError) as e:
        ctx.assemble(dev(label), 4, [0, 1, 2, 3], X, Y, prm)
    assert e.value.status == fl.FL_EINVAL
    bad = label.copy()
    bad[2] = 12
    with pytest.raises(fl.FlError) as e:
        ctx.assemble(dev(bad), 3, order, X, Y, prm)
    assert e.value.status == fl.FL_EINVAL
    for kw in ({"gap": 0.0}, {"density": -1.0}, {"max_group": 1}, {"max_group": 257}, {"sweeps": -1}):
        with pytest.raises(fl.FlError) as e:
            ctx.assemble(dev(label), 3, order, X, Y, fl.assemble_params(**kw))
        assert e.value.status == fl.FL_EINVAL
    assert np.array_equal(host(X), x) and np.array_equal(host(Y), y)
