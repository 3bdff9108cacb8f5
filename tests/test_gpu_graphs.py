"""Graph replay and concurrent components.

fl_fa2_run captures one iteration into a HIP graph and replays it; fl_layout
replays one graph holding an iteration of every large component, spread over
branch streams.  An iteration has no floating-point atomics, so every result
must equal the eager one bit for bit.  Replays are checked after every call,
with eager launches, torch work and synchronisations between the calls.
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
def ctxs(fl):
    graph, eager = fl.Context(0), fl.Context(0)
    eager.set_graphs(False)
    yield graph, eager
    graph.close()
    eager.close()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("rep", ["fmm", "exact"])
def test_replay_equals_eager(ctxs, fl, rep):
    from paper_2403_03504_amd import workloads as w
    _note("graph replay vs eager,", rep)
    g = w.bipartite(21, 8000, 12000, 5, hub_deg=(500, 2000)) if rep == "fmm" else w.plain_2k()
    prm = fl.default_params(repulsion=fl.REP_FMM if rep == "fmm" else fl.REP_EXACT, p=8, leaf_size=32)
    runs = []
    for c in ctxs:
        G = c.build_csr(g.n, dev(g.src), dev(g.dst))
        runs.append(dict(c=c, G=G, x=dev(g.x), y=dev(g.y), st=fl.FA2State.zeros(g.n, "cuda")))
    # graph run, eager step, graph run, unrelated torch work, graph runs
    plan = [("run", 12), ("step", 1), ("run", 7), ("torch", 0), ("run", 5), ("run", 4)]
    for what, k in plan:
        for r in runs:
            if what == "run":
                r["c"].fa2_run(r["G"], r["x"], r["y"], r["st"], prm, k)
            elif what == "step":
                r["c"].fa2_step(r["G"], r["x"], r["y"], r["st"], prm)
            else:
                junk = torch.randn(1 << 20, device="cuda")
                (junk * 2).sum().item()
                torch.cuda.synchronize()
        a, b = runs
        assert a["st"].iter == b["st"].iter
        for key in ("x", "y"):
            assert np.array_equal(host(a[key]), host(b[key])), (what, k, key)
        for key in ("fx_prev", "fy_prev", "scalars"):
            assert np.array_equal(host(getattr(a["st"], key)), host(getattr(b["st"], key))), (what, k, key)


def _many_components(seed):
    """More large components than branch streams, exact and FMM ones, with
    small Kamada-Kawai components and single nodes between them, ids shuffled."""
    from paper_2403_03504_amd import workloads as w
    sizes = [9000, 6000, 5200, 4100, 3000, 1800, 900, 700, 520, 400, 300, 260]
    parts = [w.scaled(seed + i, s, hubs_per_4000=(i % 3 == 0)) for i, s in enumerate(sizes)]
    parts += [w.small_component(seed * 100 + i, s) for i, s in enumerate([5, 30, 120, 2])]
    single = w.Graph(n=1, src=np.zeros(0, np.int32), dst=np.zeros(0, np.int32),
                     x=np.array([1.0], np.float32), y=np.array([2.0], np.float32))
    parts.insert(5, single)
    g, offs = w.union(parts)
    perm = np.random.default_rng(seed).permutation(g.n).astype(np.int32)
    x = np.empty_like(g.x)
    y = np.empty_like(g.y)
    x[perm], y[perm] = g.x, g.y
    return parts, offs, perm, perm[g.src], perm[g.dst], x, y


@pytest.mark.parametrize("iters", [1, 2, 30])
def test_layout_concurrent_components_equal_alone(ctxs, fl, iters):
    from oracle import oracle as orc
    _note("layout, 12 ForceAtlas2 components on branch streams, iters =", iters)
    c, eager = ctxs
    parts, offs, perm, src, dst, x, y = _many_components(300 + iters)
    G = c.build_csr(len(x), dev(src), dev(dst))
    fa2 = fl.default_params(repulsion=fl.REP_FMM, p=8, leaf_size=32)
    kk = fl.kk_params(steps=50)
    results = []
    for _ in range(2):  # a second call reuses the branch contexts
        xd, yd = dev(x), dev(y)
        st = c.layout(G, xd, yd, fa2, iters, kk, kk_max_nodes=256, fmm_min_nodes=4096)
        results.append((host(xd), host(yd)))
    assert st["n_fa2"] == 12 and st["n_single"] == 1
    assert np.array_equal(results[0][0], results[1][0]) and np.array_equal(results[0][1], results[1][1])
    lx, ly = results[0]
    for k, part in enumerate(parts):
        if part.n <= 256:
            continue
        ids = perm[offs[k]:offs[k + 1]]
        order = np.argsort(ids, kind="stable")
        inv = np.empty_like(order)
        inv[order] = np.arange(part.n)
        psrc, pdst = inv[part.src].astype(np.int32), inv[part.dst].astype(np.int32)
        Gp = eager.build_csr(part.n, dev(psrc), dev(pdst))
        # the reference run's own inputs are checked too, so that a mismatch
        # names its side: the CSR against the oracle's, bit for bit
        rp, col, _ = orc.build_csr(part.n, psrc, pdst)
        assert np.array_equal(host(Gp.row_ptr), rp.astype(np.int32)), ("alone CSR rows", k)
        assert np.array_equal(host(Gp.col)[:len(col)], col.astype(np.int32)), ("alone CSR columns", k)
        p = fa2 if part.n >= 4096 else fl.default_params(repulsion=fl.REP_EXACT, p=8, leaf_size=32)
        alone = []
        for _ in range(2):  # and the reference run is itself reproducible
            px, py = dev(part.x[order]), dev(part.y[order])
            eager.fa2_run(Gp, px, py, fl.FA2State.zeros(part.n, "cuda"), p, iters)
            alone.append((host(px), host(py)))
        assert np.array_equal(alone[0][0], alone[1][0]) and np.array_equal(alone[0][1], alone[1][1]), \
            ("alone runs differ", k, part.n)
        assert np.array_equal(alone[0][0], lx[ids[order]]), (k, part.n)
        assert np.array_equal(alone[0][1], ly[ids[order]]), (k, part.n)


def test_fmm_stats_equal_across_schedules(fl):
    """The list statistics (read by the host only) are enqueued on the
    attraction branch in replayed and branch-stream iterations, and in line
    when phases are timed: both schedules give the same counts, and the same
    positions bit for bit."""
    from paper_2403_03504_amd import workloads as w
    _note("fmm statistics: branch schedule vs in-line schedule")
    g = w.bipartite(21, 8000, 12000, 5, hub_deg=(500, 2000))
    prm = fl.default_params(repulsion=fl.REP_FMM, p=8, leaf_size=32)
    iters = 12
    out = []
    for inline in (False, True):
        c = fl.Context(0)
        try:
            if inline:
                c.set_timing(True)
            G = c.build_csr(g.n, dev(g.src), dev(g.dst))
            x, y = dev(g.x), dev(g.y)
            st = fl.FA2State.zeros(g.n, "cuda")
            c.fmm_stats(reset=True)
            c.fa2_run(G, x, y, st, prm, iters)
            out.append((c.fmm_stats(), host(x), host(y)))
        finally:
            c.close()
    (s0, x0, y0), (s1, x1, y1) = out
    assert np.array_equal(x0, x1) and np.array_equal(y0, y1)
    assert s0["evaluations"] == iters and s0["total_particles"] == iters * g.n
    for k in ("cells", "leaves", "near_pairs", "v_entries", "total_near_pairs", "total_v_entries", "evaluations",
              "total_particles"):
        assert s0[k] == s1[k], (k, s0[k], s1[k])
    assert s0["total_near_pairs"] > 0
