#!/usr/bin/env python3
"""Throughput of the FMM-ForceAtlas2 iteration on one MI355X.

Workload: a synthetic bitcoin-like bipartite transaction graph of 2,000,000
nodes (40 % transactions, Zipf(2) input/output counts capped at 20, 500 hub
addresses of degree 5k-20k, re-attached into one component), positions
uniform in a square, FP32.  A step is one full ForceAtlas2 iteration:
Morton sort, quadtree, lists, FMM repulsion (P2M, M2M, M2L/P2L, L2L,
L2P/M2P/P2P), CSR attraction, gravity, FP64 swing/traction sums, speed and
update.  The metric is node-updates/s = nodes x iterations / wall time.

Also reported (same JSON line): GPU exact-direct repulsion at the same size
(the equal-accuracy comparator), the FMM's relative force error on a sampled
node subset against the FP64 exact sum, the roofline of the dominant kernel
(P2P/L2P/M2P evaluation, FP32 ALU) measured with HIP events over the timed
region, and the FP64 CPU oracle's throughput on the same workload.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FA2 node-updates/s at 2M nodes (FMM vs direct, ≤1e-3 err); p50/p99 latency"
FP32_PUBLISHED = 157.3e12                   # published FP32 vector peak, the roofline's denominator
FP32_VALU_PEAK = 256 * 4 * 16 * 2 * 2.4e9  # 78.6 TFLOP/s: unpacked FP32 FMA (packed FP32 is off in this build)
HBM_PEAK = 8.0e12


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def profiled_traffic(kernel: str = "k_p2p", source: str = "fl_fmm.hip", profile: str = "fa2_fmm_giant2m_p8.md"):
    """HBM bytes per launch of `kernel` from the committed PMC summary, or None
    if the kernel's source file changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", profile)
    src = os.path.join(ROOT, "paper_2403_03504_amd", "csrc", source)
    try:
        text = open(path).read()
        want = re.search(re.escape(source) + r"\)\[:16\] = ([0-9a-f]{16})", text).group(1)
        have = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
        if want != have:
            return None
        row = re.search(r"\| `" + re.escape(kernel) + r"` \| \d+ \| [\d.]+ \| [\d.]+ \| ([\d.]+) \|", text)
        return float(row.group(1)) * 1e6 if row else None
    except (OSError, AttributeError):
        return None


def serving(args, fl, w, np) -> dict:
    """Layout jobs arriving as a Poisson stream, n ~ round(exp(U(ln 100,
    ln 1e6))) bipartite graphs (40 % transactions, n/4000 hubs), each laid out
    with `serving_iters` iterations; once with continuous batching (several
    slots, admission by memory budget) and once one job at a time."""
    import math
    import threading
    rng = np.random.Generator(np.random.PCG64(5))
    J = args.serving_jobs
    sizes = np.round(np.exp(rng.uniform(math.log(100), math.log(1e6), size=J))).astype(np.int64)
    gaps = rng.exponential(1.0 / args.serving_rate, size=J)
    t = time.perf_counter()
    jobs = []
    for i, n in enumerate(sizes):
        jobs.append(w.scaled(5_000_000 + i, int(n)))
        if (i + 1) % 200 == 0 and J > 200:
            log(f"serving: {i + 1} of {J} jobs generated")
    log(f"serving: generated {J} jobs ({int(sizes.sum())} nodes) in {time.perf_counter() - t:.1f}s")
    prm = fl.default_params(p=args.p, leaf_size=args.leaf)
    out = {"jobs": J, "rate_per_s": args.serving_rate, "iters": args.serving_iters,
           "nodes_total": int(sizes.sum()), "sizes": "log-uniform 100..1e6", "budget_GiB": 32}

    def run(slots):
        srv = fl.Server(0, budget_bytes=32 << 30, slots=slots)
        ids = []

        def feeder():
            t_next = time.perf_counter()
            for g, dt in zip(jobs, gaps):  # arrival times fixed by the gaps, not by how long submit takes
                t_next += dt
                time.sleep(max(0.0, t_next - time.perf_counter()))
                ids.append(srv.submit(g.n, g.src, g.dst, g.x, g.y, args.serving_iters, prm))

        th = threading.Thread(target=feeder)
        t0 = time.perf_counter()
        th.start()
        th.join()
        times = []
        for k, i in enumerate(ids):
            assert srv.wait(i, 900.0) == fl.JOB_DONE
            times.append(srv.result(i)[2])
            if (k + 1) % 200 == 0 and len(ids) > 200:
                log(f"serving ({slots} slots): {k + 1} of {len(ids)} jobs done")
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        ta = np.array([v[0] for v in times])
        ts = np.array([v[1] for v in times])
        td = np.array([v[2] for v in times])
        lat = (td - ta) * 1e3
        wait = (ts - ta) * 1e3
        span = td.max() - ta.min()
        # share of the span during which at least one job ran
        ev = sorted([(a, 1) for a in ts] + [(b, -1) for b in td])
        busy, depth, last = 0.0, 0, None
        for t, dlt in ev:
            if depth > 0:
                busy += t - last
            depth += dlt
            last = t
        q = max(1, len(lat) // 5)
        return {"slots": slots, "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()), "queue_wait_p50_ms": float(np.percentile(wait, 50)),
                "queue_wait_p99_ms": float(np.percentile(wait, 99)),
                "node_updates_per_s": float(sizes.sum()) * args.serving_iters / span,
                "busy_fraction": busy / span, "span_s": float(span), "wall_s": wall,
                # latency drift with queue position: the first and the last fifth of the arrivals
                "first_fifth_p50_ms": float(np.percentile(lat[:q], 50)),
                "last_fifth_p50_ms": float(np.percentile(lat[-q:], 50)),
                "peak_bytes": st["peak_bytes"], "peak_held_bytes": st["peak_held_bytes"], "trims": st["trims"],
                "over_estimate": st["over_estimate"]}

    out["batched"] = run(args.serving_slots)
    b = out["batched"]
    log(f"serving ({args.serving_slots} slots): p50 {b['p50_ms']:.1f} ms, p99 {b['p99_ms']:.1f} ms, "
        f"{b['node_updates_per_s']:.3g} node-updates/s, busy {b['busy_fraction']:.2f}, "
        f"first/last fifth p50 {b['first_fifth_p50_ms']:.0f}/{b['last_fifth_p50_ms']:.0f} ms")
    if not args.serving_no_single:
        out["one_at_a_time"] = run(1)
        o = out["one_at_a_time"]
        log(f"serving (1 slot): p50 {o['p50_ms']:.1f} ms, p99 {o['p99_ms']:.1f} ms, "
            f"first/last fifth p50 {o['first_fifth_p50_ms']:.0f}/{o['last_fifth_p50_ms']:.0f} ms")
    return out


def batched(args, fl, w, np, torch) -> dict:
    """Many uneven components through one fl_layout call: power-law small
    components (sizes 3..200) laid out by Kamada-Kawai and a few large ones
    (log-uniform 5k..50k nodes) by ForceAtlas2; concurrent replayed graphs,
    then the same call with every component run eagerly one after the other."""
    t = time.perf_counter()
    g, offs = w.batched_components(3, args.batched_small, args.batched_large)
    sizes = np.diff(offs)
    log(f"batched: generated {sizes.size} components ({g.n} nodes) in {time.perf_counter() - t:.1f}s")
    dev = torch.device("cuda", 0)
    ctx = fl.Context(0)
    G = ctx.build_csr(g.n, torch.from_numpy(g.src).to(dev), torch.from_numpy(g.dst).to(dev))
    fa2 = fl.default_params(repulsion=fl.REP_FMM, p=args.p, leaf_size=args.leaf)
    kk = fl.kk_params(steps=args.batched_kk_steps)
    small = sizes[sizes <= 256]
    kk_pairs = float(np.sum(small * (small - 1))) * args.batched_kk_steps
    large = sizes[sizes > 256]
    out = {"components": int(sizes.size), "nodes": int(g.n), "kk_components": int(small.size),
           "fa2_components": int(large.size), "fa2_sizes": [int(v) for v in sorted(large)],
           "kk_steps": args.batched_kk_steps, "fa2_iters": args.batched_fa2_iters,
           "fmm_min_nodes": 4096}
    for mode in ("concurrent_graphs", "sequential_eager"):
        ctx.set_graphs(mode == "concurrent_graphs")
        best = None
        for _ in range(2):  # the first call sizes the workspaces
            x = torch.from_numpy(g.x).to(dev)
            y = torch.from_numpy(g.y).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = ctx.layout(G, x, y, fa2, args.batched_fa2_iters, kk, kk_max_nodes=256, fmm_min_nodes=4096)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if best is None or wall < best[0]:
                best = (wall, st)
        wall, st = best
        r = {"wall_ms": wall * 1e3, "setup_ms": st["ms_setup"], "kk_ms": st["ms_kk"], "fa2_ms": st["ms_fa2"],
             "kk_pair_updates_per_s": kk_pairs / (st["ms_kk"] * 1e-3),
             "fa2_node_updates_per_s": st["fa2_nodes"] * args.batched_fa2_iters / (st["ms_fa2"] * 1e-3)}
        out[mode] = r
        log(f"batched ({mode}): wall {r['wall_ms']:.1f} ms, KK {r['kk_ms']:.1f} ms "
            f"({r['kk_pair_updates_per_s']:.3g} pair-updates/s), FA2 {r['fa2_ms']:.1f} ms "
            f"({r['fa2_node_updates_per_s']:.3g} node-updates/s)")
    ctx.set_graphs(True)
    out["assembly"] = assembly(args, ctx, G, g, x, y, fl, np, torch)
    out["kk_minimisers"] = kk_minimisers(args, ctx, g, offs, fl, np, torch)
    ctx.close()
    return out


def kk_minimisers(args, ctx, g, offs, fl, np, torch) -> dict:
    """The batched workload's small components laid out from the same start by
    the two Kamada-Kawai minimisers, localized stress majorization (all nodes
    of a component at once, 200 steps) and the paper's Newton-Raphson (one
    node at a time, until every gradient norm < 1e-3 l, at most 200 moves per
    node), each also with the cluster/decluster reductions of sec. 3.1.  Time
    of the whole fl_kk_layout call (hop distances included) and the total
    energy of the result by the FP64 oracle."""
    from oracle import oracle as orc
    sizes = np.diff(offs)
    small = np.nonzero(sizes <= 256)[0]
    # the small components are a prefix of the batched workload
    assert np.all(small == np.arange(small.size))
    ns = int(offs[small.size])
    keep = (g.src < ns) & (g.dst < ns)
    dev = torch.device("cuda", 0)
    G = ctx.build_csr(ns, torch.from_numpy(g.src[keep]).to(dev), torch.from_numpy(g.dst[keep]).to(dev))
    coff = offs[: small.size + 1].astype(np.int32)
    dist, doff = ctx.hop_distances(G, coff)
    D = dist.cpu().numpy()
    out = {"components": int(small.size), "nodes": ns}
    variants = (("majorization", dict(minimiser=fl.KK_MAJORIZATION, steps=200)),
                ("majorization_reduced", dict(minimiser=fl.KK_MAJORIZATION, steps=200, reduce=3)),
                ("newton", dict(minimiser=fl.KK_NEWTON, steps=200, eps=1e-3)),
                ("newton_reduced", dict(minimiser=fl.KK_NEWTON, steps=200, eps=1e-3, reduce=3)))
    for name, kw in variants:
        best = None
        for _ in range(2):
            x = torch.from_numpy(g.x[:ns]).to(dev)
            y = torch.from_numpy(g.y[:ns]).to(dev)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.kk_layout(G, coff, x, y, fl.kk_params(**kw))
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if best is None or wall < best[0]:
                best = (wall, x.cpu().numpy(), y.cpu().numpy())
        wall, xh, yh = best
        energy = 0.0
        for k in range(small.size):
            a, b = coff[k], coff[k + 1]
            n = b - a
            energy += orc.kk_energy(D[doff[k]:doff[k] + n * n].reshape(n, n), xh[a:b], yh[a:b])
        out[name] = {"ms": wall * 1e3, "energy": energy}
        log(f"KK {name}: {wall * 1e3:.1f} ms for {small.size} components, total energy {energy:.6g}")
    out["newton_over_majorization_energy"] = out["newton"]["energy"] / out["majorization"]["energy"]
    return out


def assembly(args, ctx, G, g, xl, yl, fl, np, torch) -> dict:
    """The components just laid out, assembled into one drawing (density
    rescaling, meta-graph layout in groups of up to 256, placement); the
    oracle's assembly of the same components is timed beside it."""
    label, K = ctx.components(G)
    order = np.random.Generator(np.random.PCG64(args.seed + 101)).permutation(K).astype(np.int32)
    prm = fl.assemble_params()
    best = None
    for _ in range(3):  # the first call sizes the workspaces
        x, y = xl.clone(), yl.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ctx.assemble(label, K, order, x, y, prm)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if best is None or wall < best[0]:
            best = (wall, st)
    wall, st = best
    sizes, groups = [K], []
    while sizes[-1] > prm.max_group:
        sizes.append(-(-sizes[-1] // prm.max_group))
    pairs = 0
    for m in sizes:
        for a in range(0, m, prm.max_group):
            gsz = min(prm.max_group, m - a)
            pairs += gsz * (gsz - 1)
    out = {"components": K, "levels": st["levels"], "groups": st["groups"], "sweeps": prm.sweeps,
           "max_group": prm.max_group, "wall_ms": wall * 1e3,
           "meta_pair_updates": pairs * prm.sweeps}
    log(f"assembly: {K} components, {st['levels']} levels, {st['groups']} groups, wall {wall * 1e3:.2f} ms")
    if not args.no_cpu:
        from oracle import oracle as orc
        lab = label.cpu().numpy()
        ids = np.argsort(lab, kind="stable")
        off = np.concatenate([[0], np.cumsum(np.unique(lab, return_counts=True)[1])])
        t0 = time.perf_counter()
        orc.assemble(g.x[ids].astype(np.float64), g.y[ids].astype(np.float64), off, order,
                     orc.AssembleParams(sweeps=prm.sweeps, max_group=prm.max_group))
        out["oracle_ms"] = (time.perf_counter() - t0) * 1e3
        out["oracle_cores"] = 1  # the sweeps and the all-pairs loops run on one core
        log(f"assembly oracle: {out['oracle_ms']:.0f} ms")
    return out


def bh_comparison(args, ctx, G, x, y, tg, ex, ey, fl, orc, np, torch) -> dict:
    """Barnes-Hut (the O(N log N) method the FMM replaces) against the FMM on
    the same positions: repulsion time per evaluation (tree build included;
    HIP events around every phase on the context's stream) and the error
    against the FP64 exact sum on the sampled targets."""
    reps = 5

    def timed(fn):
        fn()  # sizes the workspace
        torch.cuda.synchronize()
        ctx.get_timing()
        ctx.set_timing(True)
        for _ in range(reps):
            out = fn()
        torch.cuda.synchronize()
        ctx.set_timing(False)
        return out, sum(v[0] for v in ctx.get_timing().values()) / reps

    def err(fx, fy):
        return orc.rel_err(fx.cpu().numpy()[tg], fy.cpu().numpy()[tg], ex, ey)

    res = {"fmm": [], "bh": [], "leaf_size": args.leaf, "sample_nodes": int(tg.size)}
    for p in (4, 8, 12):
        prm = fl.default_params(repulsion=fl.REP_FMM, p=p, leaf_size=args.leaf)
        out, ms = timed(lambda: ctx.fa2_forces(G, x, y, prm, components=False))
        res["fmm"].append({"p": p, "ms": ms, "rel_err": err(out["frx"], out["fry"])})
        log(f"FMM p={p}: {ms:.3f} ms per repulsion, error {res['fmm'][-1]['rel_err']:.2e}")
    for th in [float(v) for v in args.bh_thetas.split(",")]:
        (fx, fy), ms = timed(lambda: ctx.bh_repulsion(x, y, G.deg, 1.0, th, args.leaf))
        res["bh"].append({"theta": th, "ms": ms, "rel_err": err(fx, fy)})
        log(f"Barnes-Hut theta={th}: {ms:.3f} ms per repulsion, error {res['bh'][-1]['rel_err']:.2e}")
    eq = []
    for f in res["fmm"]:
        ok = [b for b in res["bh"] if b["rel_err"] <= f["rel_err"]]
        if ok:
            b = min(ok, key=lambda v: v["ms"])
            eq.append({"p": f["p"], "fmm_ms": f["ms"], "fmm_rel_err": f["rel_err"], "theta": b["theta"],
                       "bh_ms": b["ms"], "bh_rel_err": b["rel_err"], "bh_over_fmm_time": b["ms"] / f["ms"]})
        else:
            eq.append({"p": f["p"], "fmm_ms": f["ms"], "fmm_rel_err": f["rel_err"], "theta": None,
                       "note": "no theta tried reaches this error"})
    res["equal_error"] = eq
    fm = [f for f in res["fmm"] if f["rel_err"] <= 1e-3]
    bm = [b for b in res["bh"] if b["rel_err"] <= 1e-3]
    if fm and bm:
        f, b = min(fm, key=lambda v: v["ms"]), min(bm, key=lambda v: v["ms"])
        res["at_1e-3"] = {"fmm_p": f["p"], "fmm_ms": f["ms"], "theta": b["theta"], "bh_ms": b["ms"],
                          "bh_over_fmm_time": b["ms"] / f["ms"]}
        log(f"within 1e-3: FMM p={f['p']} {f['ms']:.3f} ms, Barnes-Hut theta={b['theta']} {b['ms']:.3f} ms "
            f"({b['ms'] / f['ms']:.1f}x)")
    return res


def precision_study(args, ctx, G, g, fl, orc, np, torch) -> dict:
    """Expansion order p in {4, 8, 12} on the full graph: each p runs its own
    trajectory from the initial positions; at iterations t in {0, 1, 100,
    last} the FMM repulsion and the GPU exact-direct repulsion are compared
    with the FP64 exact sum over all nodes on a fixed random sample of
    targets."""
    dev = torch.device("cuda", 0)
    deg = G.deg.cpu().numpy()
    rng = np.random.default_rng(4)
    tg = np.sort(rng.choice(g.n, size=min(args.precision_sample, g.n), replace=False))
    last = args.precision_iters - 1
    marks = sorted({0, 1, min(100, last), last})
    prm_d = fl.default_params(repulsion=fl.REP_EXACT)
    out = {"sample_nodes": int(tg.size), "iterations": args.precision_iters, "checkpoints": marks,
           "leaf_size": args.leaf, "reference": "FP64 exact sum over all nodes (oracle) on the sample",
           "orders": {}}
    for p in (4, 8, 12):
        prm = fl.default_params(repulsion=fl.REP_FMM, p=p, leaf_size=args.leaf)
        x = torch.from_numpy(g.x).to(dev)
        y = torch.from_numpy(g.y).to(dev)
        st = fl.FA2State.zeros(g.n, dev)
        rows, t_run, n_run = [], 0.0, 0
        for t in marks:
            k = t - st.iter
            if k > 0:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                ctx.fa2_run(G, x, y, st, prm, k)
                torch.cuda.synchronize()
                t_run += time.perf_counter() - t0
                n_run += k
            of = ctx.fa2_forces(G, x, y, prm, components=False)
            od = ctx.fa2_forces(G, x, y, prm_d, components=False)
            xs, ys = x.cpu().numpy(), y.cpu().numpy()
            ex, ey = orc.repulsion_exact(xs, ys, deg + 1.0, targets=tg)
            e_f = orc.rel_err(of["frx"].cpu().numpy()[tg], of["fry"].cpu().numpy()[tg], ex, ey)
            e_d = orc.rel_err(od["frx"].cpu().numpy()[tg], od["fry"].cpu().numpy()[tg], ex, ey)
            rows.append({"t": t, "fmm_rel_err": e_f, "direct_rel_err": e_d})
        ms = t_run * 1e3 / max(n_run, 1)
        out["orders"][str(p)] = {"errors": rows, "ms_per_step": ms, "node_updates_per_s": g.n / (ms * 1e-3),
                                 "max_fmm_rel_err": max(r["fmm_rel_err"] for r in rows)}
        log(f"precision p={p}: {ms:.3f} ms/iter, FMM error " +
            ", ".join(f"t={r['t']} {r['fmm_rel_err']:.2e}" for r in rows) +
            f" (direct {max(r['direct_rel_err'] for r in rows):.2e})")
    return out


def tuned_run(args, G, g, fl, np, torch, xl, yl) -> dict:
    """fl_autotune for the error bound on the points of the laid-out graph
    (xl, yl: positions after the main run, where hub clusters have formed and
    the FMM error is larger than on the random start), in a random order so
    that each size is a uniform subsample; then the timed iterations again,
    from the start, with FL_REP_AUTO."""
    dev = torch.device("cuda", 0)
    ctx = fl.Context(0)
    order = torch.from_numpy(np.random.default_rng(7).permutation(g.n)).to(dev)
    xs = xl[order].contiguous()
    ys = yl[order].contiguous()
    ds = G.deg[order].contiguous()
    sizes = [s for s in (1024, 4096, 16384, 65536, 262144, 1048576) if s < g.n] + [g.n]
    t0 = time.perf_counter()
    table, samples = ctx.autotune(xs, ys, ds, sizes, max_rel_err=args.tune_err, reps=3)
    tune_s = time.perf_counter() - t0
    log(f"autotune ({tune_s:.1f} s): crossover {table['fmm_min_nodes']}, (p, leaf) per size " +
        ", ".join(f"{s}: ({p}, {l})" for s, p, l in zip(sizes, table["p"], table["leaf_size"])))
    prm = fl.default_params(repulsion=fl.REP_AUTO)
    x = torch.from_numpy(g.x).to(dev)
    y = torch.from_numpy(g.y).to(dev)
    st = fl.FA2State.zeros(g.n, dev)
    ctx.fa2_run(G, x, y, st, prm, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.fa2_run(G, x, y, st, prm, args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.close()
    k = len(sizes) - 1
    pick = [q for q in samples if q["size"] == g.n and q["p"] == table["p"][k]
            and q["leaf_size"] == table["leaf_size"][k] and q["list_lanes"] == table["list_lanes"][k]]
    out = {"max_rel_err": args.tune_err, "sizes": sizes, "table": table, "tune_s": tune_s,
           "measurements": len(samples), "ms_per_step": wall * 1e3 / args.steps,
           "node_updates_per_s": g.n * args.steps / wall,
           "full_size_choice": {"p": table["p"][k], "leaf_size": table["leaf_size"][k],
                                "list_lanes": table["list_lanes"][k],
                                "rel_err_vs_gpu_exact": pick[0]["rel_err"] if pick else None}}
    log(f"tuned run: {out['ms_per_step']:.3f} ms/iter, {out['node_updates_per_s']:.4g} node-updates/s")
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--nodes", type=int, default=2_000_000)
    ap.add_argument("--hubs", type=int, default=500)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--list-lanes", type=int, default=0, help="lanes per cell of the list kernels (0: by size)")
    ap.add_argument("--phase-steps", type=int, default=50,
                    help="iterations of the eager pass that times every phase with HIP events")
    ap.add_argument("--direct-steps", type=int, default=1, help="exact-direct comparator iterations (0: skip)")
    ap.add_argument("--sample", type=int, default=1000, help="nodes in the force-error sample (0: skip)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--serving-jobs", type=int, default=100, help="jobs in the serving run (0: skip)")
    ap.add_argument("--serving-rate", type=float, default=20.0, help="Poisson arrival rate, jobs/s")
    ap.add_argument("--serving-slots", type=int, default=4)
    ap.add_argument("--serving-iters", type=int, default=200)
    ap.add_argument("--serving-no-single", action="store_true", help="skip the one-job-at-a-time comparison")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving section (no 2M-node run)")
    ap.add_argument("--batched-only", action="store_true",
                    help="run only the batched-components section (no 2M-node run)")
    ap.add_argument("--tune-err", type=float, default=1e-3,
                    help="error bound of the autotuned run (0: skip)")
    ap.add_argument("--precision-sample", type=int, default=500,
                    help="sample nodes of the p = 4/8/12 precision study (0: skip)")
    ap.add_argument("--precision-iters", type=int, default=300)
    ap.add_argument("--batched-small", type=int, default=10_000, help="small components in the batched run (0: skip)")
    ap.add_argument("--batched-large", type=int, default=20)
    ap.add_argument("--batched-kk-steps", type=int, default=200)
    ap.add_argument("--batched-fa2-iters", type=int, default=200)
    ap.add_argument("--bh-thetas", default="1.0,0.7,0.5,0.35,0.25,0.18,0.12",
                    help="Barnes-Hut opening angles compared with the FMM at equal error ('' skips)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="finish with a device-to-device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: this build runs on exactly one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "multi-GPU sharding is a design note only", file=sys.stderr)
        return 2

    import numpy as np

    from paper_2403_03504_amd import workloads as w

    if args.batched_only:  # the many-components workload alone
        import torch

        from paper_2403_03504_amd import fa2lay as fl
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 1
        print(json.dumps({"batched": batched(args, fl, w, np, torch)}), flush=True)
        return 0
    if args.serving_only:  # the serving study alone (long runs of many jobs)
        import torch

        from paper_2403_03504_amd import fa2lay as fl
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            return 1
        print(json.dumps({"serving": serving(args, fl, w, np)}), flush=True)
        return 0

    t = time.perf_counter()
    g = w.giant_2m(args.seed, args.nodes, args.hubs)
    log(f"generated {g.n} nodes / {g.m} edge records in {time.perf_counter() - t:.1f}s")

    import torch

    from paper_2403_03504_amd import fa2lay as fl

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    ctx = fl.Context(0)
    dev = torch.device("cuda", 0)
    src = torch.from_numpy(g.src).to(dev)
    dst = torch.from_numpy(g.dst).to(dev)
    torch.cuda.synchronize()
    t = time.perf_counter()
    G = ctx.build_csr(g.n, src, dst)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t
    nnz = int(G.row_ptr[-1].item())
    log(f"CSR built on GPU: nnz {nnz} in {setup_s * 1e3:.1f} ms")

    prm = fl.default_params(repulsion=fl.REP_FMM, p=args.p, leaf_size=args.leaf, list_lanes=args.list_lanes)
    x = torch.from_numpy(g.x).to(dev)
    y = torch.from_numpy(g.y).to(dev)
    st = fl.FA2State.zeros(g.n, dev)
    ctx.fa2_run(G, x, y, st, prm, args.warmup)
    torch.cuda.synchronize()
    log(f"warmup {args.warmup} iterations done")

    # ---- timed region: one fl_fa2_run call (one eager iteration, then a
    # captured iteration replayed as a HIP graph) ------------------------------
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.fa2_run(G, x, y, st, prm, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    value = g.n * args.steps / wall
    log(f"timed {args.steps} iterations: {wall * 1e3 / args.steps:.3f} ms/iter, {value:.4g} node-updates/s")

    # ---- per-kernel durations: an eager pass with HIP events around every
    # phase on the context's stream (the stream the kernels run on) ----------
    n_phase = min(args.steps, args.phase_steps)
    ctx.fmm_stats(reset=True)
    ctx.get_timing()
    ctx.set_timing(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ctx.fa2_run(G, x, y, st, prm, n_phase)
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t2) * 1e3 / max(n_phase, 1)
    ctx.set_timing(False)
    phases = ctx.get_timing()
    fst = ctx.fmm_stats()
    log(f"eager pass with phase events: {eager_ms:.3f} ms/iter over {n_phase} iterations")
    log("phases (ms/iter): " + ", ".join(f"{k} {v[0] / max(v[1], 1):.3f}" for k, v in phases.items() if v[1]))

    # roofline of the dominant kernel: P2P + L2P + M2P evaluation (FP32 ALU)
    evals = max(fst["evaluations"], 1)
    pairs_per_launch = fst["total_near_pairs"] / evals
    eval_ms = phases["eval"][0] / max(phases["eval"][1], 1)
    # near field (k_p2p): 11 FLOP per pair (2 sub, 3 for r^2, 1 reciprocal,
    # 1 mul, 4 for the two multiply-adds)
    eval_flop = 11.0 * pairs_per_launch
    achieved = eval_flop / (eval_ms * 1e-3)
    # far field (k_far): L2P, Horner of degree p-1 in complex arithmetic,
    # 8 FLOP per term per particle (the W-list terms not counted)
    far_ms = phases["far"][0] / max(phases["far"][1], 1)
    far_flop = 8.0 * args.p * g.n
    # M2L: per V-list entry one p-term outgoing-to-incoming conversion,
    # 4p^2 + 15p FLOP (p complex products rho^k a_k, the binomial sums, the
    # mass term and p complex multiply-adds by rho^l; the powers of rho come
    # from a table); the phase also holds the (small) L2L launch, so this is
    # a lower bound
    m2l_ms = phases["m2l"][0] / max(phases["m2l"][1], 1)
    v_per_launch = fst["total_v_entries"] / evals
    m2l_flop = v_per_launch * (4.0 * args.p * args.p + 15.0 * args.p)
    attract_ms = phases["attract"][0] / max(phases["attract"][1], 1)
    attract_bytes = 40.0 * g.n + 4.0 * nnz  # compulsory bytes of the attraction/combine pass
    # algorithmic bytes of the near field: every particle record read once
    # (16 B) and its near-field sum written once (8 B)
    p2p_bytes = 24.0 * g.n
    p2p_traffic = profiled_traffic("k_p2p") if args.p == 8 else None
    at_parts = [profiled_traffic(k, "fl_fa2.hip") for k in ("k_attract_chunks", "k_attract_rows")]
    at_traffic = sum(at_parts) if all(v is not None for v in at_parts) and args.p == 8 else None
    # compulsory bytes of the gathers alone: row offsets, column ids, the
    # (x, y) of every row and of every neighbour once, the FP64 sums written
    gather_bytes = 4.0 * (g.n + 1) + 4.0 * nnz + 8.0 * g.n + 16.0 * g.n
    roofline = {"kernel": "k_p2p (FMM near field)", "bound": "alu", "achieved": achieved / 1e12,
                "peak": FP32_PUBLISHED / 1e12, "unit": "TFLOP/s", "frac": achieved / FP32_PUBLISHED,
                "traffic": p2p_traffic,
                "algorithmic_bytes_per_launch": p2p_bytes,
                "traffic_ratio": p2p_traffic / p2p_bytes if p2p_traffic else None,
                "unpacked_fp32_peak": FP32_VALU_PEAK / 1e12,
                "frac_of_unpacked_peak": achieved / FP32_VALU_PEAK,
                # the pair loop's own ceiling: 8 wave instructions per pair
                # (the reciprocal included: the VALU counters show it issuing
                # at the full rate) for 11 FLOP, at one unpacked FP32
                # instruction per lane per 4 cycles
                "pair_loop_ceiling": 11.0 / 8.0 * FP32_VALU_PEAK / 2 / 1e12,
                "frac_of_pair_loop_ceiling": achieved / (11.0 / 8.0 * FP32_VALU_PEAK / 2),
                "flop_per_launch": eval_flop, "near_pairs_per_launch": pairs_per_launch,
                "launch_ms": eval_ms,
                "far": {"kernel": f"k_far<{args.p}>", "achieved_TFLOPs": far_flop / (far_ms * 1e-3) / 1e12,
                        "flop_per_launch": far_flop, "launch_ms": far_ms},
                "m2l": {"achieved_TFLOPs": m2l_flop / (m2l_ms * 1e-3) / 1e12, "flop_per_launch": m2l_flop,
                        "v_entries_per_launch": v_per_launch, "launch_ms": m2l_ms,
                        "frac": m2l_flop / (m2l_ms * 1e-3) / FP32_PUBLISHED},
                "attraction": {"achieved_GBps": attract_bytes / (attract_ms * 1e-3) / 1e9,
                               "bytes_per_launch": attract_bytes, "launch_ms": attract_ms,
                               "frac_hbm": attract_bytes / (attract_ms * 1e-3) / HBM_PEAK,
                               "gather_traffic": at_traffic, "gather_compulsory_bytes": gather_bytes,
                               "gather_traffic_ratio": at_traffic / gather_bytes if at_traffic else None}}
    # the whole iteration against its roofs: each step's algorithmic work at
    # its bound (ALU work at the FP32 peak, memory work at HBM bandwidth),
    # summed, over the measured time per iteration.  Tree and list building
    # are latency-bound and have no roof here (counted as zero).
    p_ = float(args.p)
    ideal_us = {
        "near_field": eval_flop / FP32_PUBLISHED * 1e6,
        "m2l": m2l_flop / FP32_PUBLISHED * 1e6,
        "p2m_l2p": 16.0 * p_ * g.n / FP32_PUBLISHED * 1e6,
        "m2m_l2l": 8.0 * (p_ + 1) ** 2 * fst["cells"] / FP32_PUBLISHED * 1e6,
        "attraction": (4.0 * (g.n + 1) + 4.0 * nnz + 16.0 * g.n) / HBM_PEAK * 1e6,
        "update_swing": 40.0 * g.n / HBM_PEAK * 1e6,
        "sort": 4 * 2 * 8.0 * g.n / HBM_PEAK * 1e6,
    }
    iter_us = wall * 1e6 / args.steps
    roofline["iteration"] = {"ideal_us": ideal_us, "ideal_total_us": sum(ideal_us.values()),
                             "measured_us": iter_us, "frac": sum(ideal_us.values()) / iter_us}

    result = {"metric": METRIC, "value": value, "unit": "node-updates/s", "n_gpus": 1, "steps": args.steps,
              "warmup": args.warmup, "ms_per_step": wall * 1e3 / args.steps, "higher_is_better": True,
              "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
              "config": {"workload": f"bipartite Zipf transaction graph, {g.n} nodes, {args.hubs} hubs, "
                                     f"{nnz // 2} edges; FMM p={args.p}, leaf<={args.leaf}",
                         "nodes": g.n, "edges": nnz // 2, "p": args.p, "leaf_size": args.leaf,
                         "fp64": "swing/traction sums, speeds, bounding square"},
              "roofline": roofline,
              "phases_ms_per_iter": {k: v[0] / max(v[1], 1) for k, v in phases.items() if v[1]},
              "phase_pass": {"iterations": n_phase, "ms_per_step_eager_with_events": eager_ms},
              "fmm": {k: fst[k] for k in ("cells", "leaves", "max_level", "near_pairs", "v_entries",
                                         "w_entries", "x_entries")},
              "setup_ms": setup_s * 1e3}

    # ---- accuracy on a sample, and the exact-direct comparator --------------
    from oracle import oracle as orc
    xs = x.detach().cpu().numpy()
    ys = y.detach().cpu().numpy()
    deg = G.deg.cpu().numpy()
    prm_d = fl.default_params(repulsion=fl.REP_EXACT)
    direct_rep_s = None
    if args.sample > 0:
        out_fmm = ctx.fa2_forces(G, x, y, prm, components=False)
        torch.cuda.synchronize()
        td = time.perf_counter()
        out_dir = ctx.fa2_forces(G, x, y, prm_d, components=False)
        torch.cuda.synchronize()
        direct_rep_s = time.perf_counter() - td
        rng = np.random.default_rng(12345)
        tg = np.sort(rng.choice(g.n, size=min(args.sample, g.n), replace=False))
        ex, ey = orc.repulsion_exact(xs, ys, deg + 1.0, targets=tg)
        fmx, fmy = out_fmm["frx"].cpu().numpy()[tg], out_fmm["fry"].cpu().numpy()[tg]
        dmx, dmy = out_dir["frx"].cpu().numpy()[tg], out_dir["fry"].cpu().numpy()[tg]
        result["accuracy"] = {"sample_nodes": int(tg.size), "positions": f"after {args.warmup + args.steps} iterations",
                              "fmm_rel_err": orc.rel_err(fmx, fmy, ex, ey),
                              "direct_rel_err": orc.rel_err(dmx, dmy, ex, ey),
                              "reference": "FP64 exact sum over all nodes (oracle)"}
        log(f"repulsion error on {tg.size} nodes: FMM {result['accuracy']['fmm_rel_err']:.2e}, "
            f"direct {result['accuracy']['direct_rel_err']:.2e}")
        if args.bh_thetas:
            result["barnes_hut"] = bh_comparison(args, ctx, G, x, y, tg, ex, ey, fl, orc, np, torch)
    if args.direct_steps > 0:
        xd, yd = x.clone(), y.clone()
        sd = fl.FA2State(st.fx_prev.clone(), st.fy_prev.clone(), st.scalars.clone(), st.iter)
        torch.cuda.synchronize()
        td = time.perf_counter()
        ctx.fa2_run(G, xd, yd, sd, prm_d, args.direct_steps)
        torch.cuda.synchronize()
        dwall = time.perf_counter() - td
        dv = g.n * args.direct_steps / dwall
        result["direct"] = {"node_updates_per_s": dv, "ms_per_step": dwall * 1e3 / args.direct_steps,
                            "steps": args.direct_steps, "fmm_speedup": value / dv,
                            "pairs_per_s": g.n * (g.n - 1) * args.direct_steps / dwall,
                            "repulsion_only_s": direct_rep_s}
        log(f"exact-direct: {dwall * 1e3 / args.direct_steps:.1f} ms/iter, FMM speedup {value / dv:.1f}x")

    # ---- CPU oracle baseline: one full FA2 iteration, FMM repulsion, FP64 ----
    if not args.no_cpu:
        rp, col, deg_o = orc.build_csr(g.n, g.src, g.dst)
        oprm = orc.FA2Params(repulsion="fmm", p=args.p, leaf_size=args.leaf)
        tc = time.perf_counter()
        orc.fa2_step(rp, col, deg_o, g.x, g.y, np.zeros(g.n), np.zeros(g.n), 0.0, 0, oprm)
        cs = time.perf_counter() - tc
        result["cpu_baseline"] = {"value": g.n / cs, "unit": "node-updates/s", "cores": orc.num_threads(),
                                  "kind": "oracle",
                                  "sample": f"one full FA2 iteration of the same {g.n}-node graph (FP64 FMM "
                                            f"repulsion p={args.p}, leaf<={args.leaf}), {cs:.1f} s"}
        log(f"cpu oracle: {cs:.1f}s per iteration on {orc.num_threads()} threads")
    if args.tune_err > 0:
        result["autotuned"] = tuned_run(args, G, g, fl, np, torch, x, y)
    if args.precision_sample > 0:
        result["precision"] = precision_study(args, ctx, G, g, fl, orc, np, torch)
    if args.batched_small > 0:
        result["batched"] = batched(args, fl, w, np, torch)
    if args.serving_jobs > 0:
        ctx.close()
        result["serving"] = serving(args, fl, w, np)
        ctx = fl.Context(0)
    if args.copy_calib_mb > 0:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale that turns the counters of the kernels above into bytes
        nbytes = args.copy_calib_mb << 20
        a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = nbytes
    ctx.close()
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
