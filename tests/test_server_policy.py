"""Admission policy of the layout server, on the host-only executor (no GPU):
FIFO order, memory budget never exceeded, no starvation of a large job at the
head, cancellation, rejection of jobs larger than the budget, time stamps."""
import time

import numpy as np
import pytest


@pytest.fixture(scope="module")
def fl():
    import os
    lib = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2403_03504_amd",
                       "libfa2lay.so")
    if not os.path.exists(lib):
        pytest.fail("libfa2lay.so is not built")
    from paper_2403_03504_amd import fa2lay
    return fa2lay


def job_bytes(n, m):  # the server's estimate (see fl_server.hip)
    return 700 * n + 48 * m + (16 << 20)


def submit(srv, fl, n, iters=10):
    z = np.zeros(n, np.float32)
    return srv.submit(n, np.zeros(0, np.int32), np.zeros(0, np.int32), z, z, iters, fl.default_params())


def test_budget_and_fifo(fl):
    sizes = [1000, 200_000, 1000, 1000, 50_000, 1000, 1000, 1000]
    budget = job_bytes(200_000, 0) + job_bytes(1000, 0)  # the big job plus one small one
    srv = fl.Server(budget_bytes=budget, slots=4, fake_ns_per_update=200.0)
    ids = [submit(srv, fl, n) for n in sizes]
    seen_peak = 0
    while any(srv.poll(i) < fl.JOB_DONE for i in ids):
        st = srv.stats()
        assert st["bytes_in_use"] <= budget
        seen_peak = max(seen_peak, st["bytes_in_use"])
        time.sleep(0.002)
    times = [srv.result(i)[2] for i in ids]
    starts = [t[1] for t in times]
    assert starts == sorted(starts)  # admitted in submission order
    for ta, ts, td in times:
        assert ta <= ts <= td
    st = srv.stats()
    assert st["completed"] == len(sizes) and st["failed"] == 0 and st["peak_bytes"] <= budget
    assert st["node_updates"] == sum(sizes) * 10
    srv.close()


def test_large_head_is_not_starved(fl):
    budget = job_bytes(100_000, 0) + 3 * job_bytes(2000, 0)
    srv = fl.Server(budget_bytes=budget, slots=4, fake_ns_per_update=500.0)
    first = [submit(srv, fl, 2000, iters=40) for _ in range(3)]
    big = submit(srv, fl, 100_000, iters=2)
    later = [submit(srv, fl, 2000, iters=1) for _ in range(3)]
    for i in first + [big] + later:
        srv.wait(i, 30.0)
    t_big = srv.result(big)[2]
    for i in later:  # nothing submitted after the big job starts before it
        assert srv.result(i)[2][1] >= t_big[1]
    for i in first:
        srv.result(i)
    srv.close()


def test_cancel_and_reject(fl):
    srv = fl.Server(budget_bytes=job_bytes(10_000, 0), slots=1, fake_ns_per_update=1000.0)
    a = submit(srv, fl, 10_000, iters=20)  # 0.2 s
    b = submit(srv, fl, 10_000)
    srv.cancel(b)
    assert srv.poll(b) == fl.JOB_CANCELED
    with pytest.raises(fl.FlError) as e:
        submit(srv, fl, 1_000_000)  # larger than the whole budget
    assert e.value.status == fl.FL_ENOMEM
    assert srv.wait(a, 30.0) == fl.JOB_DONE
    with pytest.raises(fl.FlError) as e:
        srv.result(b)
    assert e.value.status == fl.FL_ECANCELED
    st = srv.stats()
    assert st["canceled"] == 1 and st["completed"] == 1
    srv.close()


def test_concurrency_overlaps_jobs(fl):
    # 8 jobs of 0.1 s on 4 slots finish in about 0.2 s, not 0.8 s
    srv = fl.Server(budget_bytes=1 << 40, slots=4, fake_ns_per_update=1000.0)
    t0 = time.time()
    ids = [submit(srv, fl, 10_000, iters=10) for _ in range(8)]
    for i in ids:
        srv.wait(i, 30.0)
    assert time.time() - t0 < 0.6
    srv.close()
