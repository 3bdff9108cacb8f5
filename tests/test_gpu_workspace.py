"""Workspace growth on the GPU: a context that grows its buffers (a small
graph, then a larger one) keeps the replaced buffers until a quiet point
and gives the larger graph exactly the result a fresh context gives
(tolerance: bitwise; the kernels are the same, only buffer addresses
differ)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _run(fl, c, g, prm, iters):
    G = c.build_csr(g.n, dev(g.src), dev(g.dst))
    x, y = dev(g.x), dev(g.y)
    c.fa2_run(G, x, y, fl.FA2State.zeros(g.n, "cuda"), prm, iters)
    return host(x), host(y)


def test_grown_workspace_matches_fresh_context():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    prm = fl.default_params(repulsion=fl.REP_FMM, p=8, leaf_size=64)
    small, large = w.scaled(701, 3000), w.scaled(702, 40000)
    grown = fl.Context(0)
    fresh = fl.Context(0)
    try:
        _note("small graph then a larger one on one context")
        _run(fl, grown, small, prm, 12)
        held_small = grown.workspace_bytes()
        gx, gy = _run(fl, grown, large, prm, 12)
        held = grown.workspace_bytes()
        assert held > held_small
        grown.synchronize()  # frees the buffers the growth replaced
        after = grown.workspace_bytes()
        assert 0 < after < held  # the replaced buffers are gone
        _note("the larger graph on a fresh context")
        fx, fy = _run(fl, fresh, large, prm, 12)
        assert np.array_equal(gx, fx) and np.array_equal(gy, fy)
        assert np.all(np.isfinite(gx))
        _note("the larger graph again on the grown context")
        hx, hy = _run(fl, grown, large, prm, 12)
        assert np.array_equal(hx, fx) and np.array_equal(hy, fy)
        assert grown.workspace_bytes() == after  # no growth the second time
    finally:
        grown.close()
        fresh.close()


def test_hash_table_reused_across_key_layouts():
    """One context builds a forest of two systems (a wider cell-hash key),
    then one small system (the key layout changes: the epoch restarts), then
    a larger single system whose table reaches slots the small build never
    used.  Every slot must have been cleared at the restart, or words left by
    the two-system forest pass the new epoch's test and hand out stale cell
    ids.  The larger run must equal a fresh context's bitwise."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    prm = fl.default_params(repulsion=fl.REP_FMM, p=8, leaf_size=32)
    two, _ = w.union([w.scaled(711, 30000), w.scaled(712, 30000)])
    small, large = w.scaled(713, 3000), w.scaled(714, 60000)
    reused = fl.Context(0)
    fresh = fl.Context(0)
    try:
        reused.set_graphs(False)  # the layout's forest is built on this context itself
        _note("two-system forest, then one small system, then a larger one, on one context")
        G2 = reused.build_csr(two.n, dev(two.src), dev(two.dst))
        x2, y2 = dev(two.x), dev(two.y)
        st = reused.layout(G2, x2, y2, prm, 1, fl.kk_params(), kk_max_nodes=256, fmm_min_nodes=4096)
        assert st["n_fa2"] == 2
        _run(fl, reused, small, prm, 1)
        rx, ry = _run(fl, reused, large, prm, 3)
        _note("the larger system on a fresh context")
        fx, fy = _run(fl, fresh, large, prm, 3)
        assert np.array_equal(rx, fx) and np.array_equal(ry, fy)
        assert np.all(np.isfinite(rx))
    finally:
        reused.close()
        fresh.close()
