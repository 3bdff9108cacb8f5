"""The allocation-free iteration (fl_fa2_step_noalloc) against fl_fa2_step
through the C ABI: the same kernels on the same inputs, only the workspace
differs (a fixed per-GPU scratch array instead of the context's grow-only
buffers), so every output must be equal bit for bit.  Two calls in a row,
the second with a smaller graph, on FMM and exact repulsion; a graph whose
buffers do not fit is rejected with FL_ENOMEM and leaves the caller's arrays
as they were; a context used only for these calls holds no workspace."""
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


def _state(fl, n, seed):
    """A state after a few iterations: nonzero previous forces and s_G."""
    rng = np.random.default_rng(seed)
    st = fl.FA2State.zeros(n, "cuda")
    st.fx_prev.copy_(torch.from_numpy(rng.normal(size=n).astype(np.float32)))
    st.fy_prev.copy_(torch.from_numpy(rng.normal(size=n).astype(np.float32)))
    st.scalars[0] = 0.37
    st.iter = 5
    return st


def _clone(fl, st):
    return fl.FA2State(st.fx_prev.clone(), st.fy_prev.clone(), st.scalars.clone(), st.iter)


@pytest.mark.parametrize("rep", ["fmm", "exact"])
def test_noalloc_step_equals_step(rep):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    ref, na = fl.Context(0), fl.Context(0)
    try:
        prm = fl.default_params(repulsion=fl.REP_FMM if rep == "fmm" else fl.REP_EXACT, p=8, leaf_size=64)
        # two calls in a row, the second with a smaller graph
        for seed, n in ((901, 60000), (902, 7000)):
            _note("noalloc vs step,", rep, "n =", n)
            g = w.scaled(seed, n)
            G = ref.build_csr(g.n, dev(g.src), dev(g.dst))
            st_a = _state(fl, g.n, seed)
            st_b = _clone(fl, st_a)
            xa, ya, xb, yb = dev(g.x), dev(g.y), dev(g.x), dev(g.y)
            sa = ref.fa2_step(G, xa, ya, st_a, prm)
            sb = na.fa2_step_noalloc(G, xb, yb, st_b, prm)
            assert sa == sb
            assert st_a.iter == st_b.iter == 6
            for a, b in ((xa, xb), (ya, yb), (st_a.fx_prev, st_b.fx_prev), (st_a.fy_prev, st_b.fy_prev),
                         (st_a.scalars, st_b.scalars)):
                assert np.array_equal(host(a), host(b))
            assert np.all(np.isfinite(host(xb)))
        assert na.workspace_bytes() == 0  # nothing was taken from the context's own workspace
    finally:
        ref.close()
        na.close()


def test_noalloc_systems_equal_step():
    """Independent systems in one state (component offsets): the forest
    build sorts them as segments, with its sort tiles carved from the same
    scratch array; bitwise fl_fa2_step's result."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    parts = [w.scaled(911, 9000), w.scaled(912, 4096, hubs_per_4000=False), w.small_component(913, 300)]
    g, offs = w.union(parts)
    ref, na = fl.Context(0), fl.Context(0)
    try:
        _note("noalloc vs step, systems", [p.n for p in parts])
        G = ref.build_csr(g.n, dev(g.src), dev(g.dst))
        prm = fl.default_params(repulsion=fl.REP_FMM, p=8, leaf_size=32)
        rng = np.random.default_rng(914)
        fx, fy = rng.normal(size=g.n).astype(np.float32), rng.normal(size=g.n).astype(np.float32)
        states = []
        for _ in range(2):
            st = fl.FA2State.zeros(g.n, "cuda", comp_offsets=offs)
            st.fx_prev.copy_(torch.from_numpy(fx))
            st.fy_prev.copy_(torch.from_numpy(fy))
            st.scalars[0::4] = torch.tensor([0.37, 0.5, 0.21], dtype=torch.float64)
            st.iter = 3
            states.append(st)
        xa, ya, xb, yb = dev(g.x), dev(g.y), dev(g.x), dev(g.y)
        ref.fa2_step(G, xa, ya, states[0], prm)
        na.fa2_step_noalloc(G, xb, yb, states[1], prm)
        for a, b in ((xa, xb), (ya, yb), (states[0].fx_prev, states[1].fx_prev),
                     (states[0].fy_prev, states[1].fy_prev), (states[0].scalars, states[1].scalars)):
            assert np.array_equal(host(a), host(b))
        assert na.workspace_bytes() == 0
    finally:
        ref.close()
        na.close()


def test_noalloc_rejects_what_does_not_fit():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    c = fl.Context(0)
    try:
        n = 1_500_000
        _note("noalloc past its scratch, n =", n)
        x, y = w.random_positions(77, n, 1000.0)
        empty = torch.zeros(0, dtype=torch.int32, device="cuda")
        G = c.build_csr(n, empty, empty)
        xd, yd = dev(x), dev(y)
        st = fl.FA2State.zeros(n, "cuda")
        with pytest.raises(fl.FlError) as e:
            c.fa2_step_noalloc(G, xd, yd, st, fl.default_params(repulsion=fl.REP_FMM))
        assert e.value.status == fl.FL_ENOMEM
        assert np.array_equal(host(xd), x) and np.array_equal(host(yd), y)
        assert st.iter == 0 and not host(st.fx_prev).any()
        # the context still works afterwards, with its own workspace
        small = w.scaled(903, 3000)
        Gs = c.build_csr(small.n, dev(small.src), dev(small.dst))
        xs, ys = dev(small.x), dev(small.y)
        c.fa2_step(Gs, xs, ys, fl.FA2State.zeros(small.n, "cuda"), fl.default_params())
        assert np.all(np.isfinite(host(xs)))
    finally:
        c.close()
