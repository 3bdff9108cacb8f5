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
        assert 0 < after <= held
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
