"""Serving on the GPU: jobs of mixed sizes run concurrently give exactly the
result each gets alone (tolerance: bitwise; every kernel reduces in a fixed
order over the job's own data)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def test_results_alone_equal_results_in_the_mix():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    sizes = [300, 2500, 6000, 30000, 900, 12000, 150, 60000]
    jobs = [w.scaled(500 + i, n) for i, n in enumerate(sizes)]
    prm = fl.default_params(p=8, leaf_size=64)
    _note("mix of", len(jobs), "jobs on 4 slots")
    srv = fl.Server(0, budget_bytes=8 << 30, slots=4)
    ids = [srv.submit(g.n, g.src, g.dst, g.x, g.y, 40, prm) for g in jobs]
    mix = []
    for i, g in zip(ids, jobs):
        st_i = srv.wait(i, 120.0)
        if st_i != fl.JOB_DONE:
            _note("job", i, "of", g.n, "nodes ended in state", st_i)
        mix.append(srv.result(i))  # raises with the job's error message if it failed
        assert st_i == fl.JOB_DONE
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(jobs) and st["peak_bytes"] <= 8 << 30
    _note("alone, one slot")
    srv1 = fl.Server(0, budget_bytes=8 << 30, slots=1)
    for g, (mx, my, t) in zip(jobs, mix):
        j = srv1.submit(g.n, g.src, g.dst, g.x, g.y, 40, prm)
        st_j = srv1.wait(j, 120.0)
        ax, ay, _ = srv1.result(j)  # raises with the job's error message if it failed
        assert st_j == fl.JOB_DONE
        assert np.array_equal(ax, mx) and np.array_equal(ay, my), g.n
        assert np.all(np.isfinite(ax))
        assert t[0] <= t[1] <= t[2]
    srv1.close()


def test_failed_job_does_not_disturb_others():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    _note("failing job in the mix")
    good = w.scaled(601, 5000)
    bad = w.scaled(602, 3000)
    bad.x[17] = np.nan
    prm = fl.default_params()
    srv = fl.Server(0, budget_bytes=4 << 30, slots=2)
    a = srv.submit(good.n, good.src, good.dst, good.x, good.y, 20, prm)
    b = srv.submit(bad.n, bad.src, bad.dst, bad.x, bad.y, 20, prm)
    assert srv.wait(a, 60.0) == fl.JOB_DONE
    assert srv.wait(b, 60.0) == fl.JOB_FAILED
    x, y, _ = srv.result(a)
    assert np.all(np.isfinite(x))
    with pytest.raises(fl.FlError):
        srv.result(b)
    srv.close()


def test_held_memory_stays_within_the_budget():
    """Workers keep their workspace between jobs; the admission charges what
    they hold, and a worker past the budget gives its memory back.  After a
    mix of small and large jobs the measured bytes the workers hold stay
    within the budget, and so does every recorded peak."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_03504_amd import fa2lay as fl
    from paper_2403_03504_amd import workloads as w
    sizes = [60000, 2000, 40000, 500, 60000, 9000, 1200, 50000]
    jobs = [w.scaled(800 + i, n) for i, n in enumerate(sizes)]
    est = [700 * g.n + 48 * len(g.src) + (16 << 20) for g in jobs]
    budget = int(1.6 * max(est))  # room for one large job and a small one
    prm = fl.default_params(p=8, leaf_size=64)
    _note("held memory, budget", budget, "bytes, 3 slots")
    srv = fl.Server(0, budget_bytes=budget, slots=3)
    ids = [srv.submit(g.n, g.src, g.dst, g.x, g.y, 20, prm) for g in jobs]
    for i in ids:
        assert srv.wait(i, 120.0) == fl.JOB_DONE
        srv.result(i)
    st = srv.stats()
    srv.close()
    _note("stats", st)
    assert st["completed"] == len(jobs)
    assert 0 < st["held_bytes"] <= budget
    assert st["peak_held_bytes"] <= budget and st["peak_bytes"] <= budget
