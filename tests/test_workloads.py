"""The seeded synthetic workloads: deterministic, bipartite, one component,
Zipf degree law (the stand-in for the paper's bitcoin transaction graphs)."""
import numpy as np
from scipy import stats

from paper_2403_03504_amd import workloads as w


def test_deterministic_per_seed():
    a = w.bipartite(5, 300, 400, 2, hub_deg=(50, 100))
    b = w.bipartite(5, 300, 400, 2, hub_deg=(50, 100))
    c = w.bipartite(6, 300, 400, 2, hub_deg=(50, 100))
    assert np.array_equal(a.src, b.src) and np.array_equal(a.x, b.x)
    assert not np.array_equal(a.src, c.src)


def test_bipartite_single_component_and_hubs():
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    g = w.bipartite(3, 2000, 3000, 4, hub_deg=(300, 600))
    T = g.n_tx
    assert np.all((g.src < T) != (g.dst < T))  # every edge joins a tx and an address
    A = sp.coo_matrix((np.ones(g.m), (g.src, g.dst)), shape=(g.n, g.n))
    assert connected_components(A, directed=True, connection="weak")[0] == 1
    deg = np.bincount(np.concatenate([g.src, g.dst]), minlength=g.n)
    assert np.all(deg[T:T + 4] >= 300)
    assert g.x.dtype == np.float32 and np.abs(g.x).max() <= 100 * np.sqrt(5000 / 2000) + 1e-3


def test_zipf_counts_match_pmf():
    rng = np.random.Generator(np.random.PCG64(0))
    k = w.zipf_counts(rng, 200_000, 2.0, 20)
    obs = np.bincount(k, minlength=21)[1:]
    pmf = np.arange(1, 21, dtype=float) ** -2.0
    exp = pmf / pmf.sum() * k.size
    chi2 = np.sum((obs - exp) ** 2 / exp)
    assert chi2 < stats.chi2.ppf(0.999, df=19)


def test_named_workload_shapes():
    g = w.plain_2k()
    assert g.n == 2000 and 3500 < g.m < 6000
    assert np.abs(g.x).max() <= 100.0
    sizes = w.small_component_sizes(3, 10_000)
    assert sizes.min() >= 3 and sizes.max() <= 200 and 7 < sizes.mean() < 11
