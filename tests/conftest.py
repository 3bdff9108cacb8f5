import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as o
    o.build()
    return o


def per_node_errors(ax, ay, bx, by):
    """Per-node force error |F_a,i - F_b,i| / max(|F_b,i|, median_j |F_b,j|):
    relative to the node's own force, with the median force as the floor, so
    that a node whose forces nearly cancel (the exact sum near the middle of
    the cloud) is judged against a typical force rather than a tiny one."""
    import numpy as np
    ax, ay, bx, by = (np.asarray(v, dtype=np.float64) for v in (ax, ay, bx, by))
    fn = np.hypot(bx, by)
    floor = max(float(np.median(fn)), 1e-300)
    return np.hypot(ax - bx, ay - by) / np.maximum(fn, floor)


@pytest.fixture(scope="session")
def node_err():
    return per_node_errors
