"""Seeded synthetic workloads: bitcoin-like bipartite transaction graphs.

The paper lays out real bitcoin transaction graphs (section 2: a bipartite
graph of address and transaction vertices; an input edge joins an address to
a transaction that spends from it, an output edge joins a transaction to an
address it pays).  Those graphs are not available here, so every workload is
synthetic, with the shape of the paper's data:

* transactions draw their input and output counts from a Zipf law
  (pmf proportional to k^-s on {1..kmax}), endpoints uniform over addresses;
* a few "hub" addresses take part in thousands of transactions;
* components other than the largest are re-attached to it by one edge, so
  the graph is a single component (the giant-component workloads);
* initial positions are uniform in a square.

This module is deliberately free of the layout method's arithmetic.  It emits
the raw directed edge list (duplicates included: an address can be both input
and output of one transaction), which the method's own graph preparation must
then collapse.  Connected components for the re-attachment step come from
``scipy.sparse.csgraph``, a library routine shared by neither the oracle nor
the HIP path.  Both sides of every parity test take their inputs from here.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    """A directed edge list on ``n`` nodes plus FP32 initial positions."""

    n: int
    src: np.ndarray  # int32 [m]
    dst: np.ndarray  # int32 [m]
    x: np.ndarray  # float32 [n]
    y: np.ndarray  # float32 [n]
    n_tx: int = 0
    n_addr: int = 0

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def zipf_counts(rng: np.random.Generator, size: int, s: float, kmax: int) -> np.ndarray:
    """Draw ``size`` values from the truncated Zipf law on {1..kmax} by inverse CDF."""
    k = np.arange(1, kmax + 1, dtype=np.float64)
    pmf = k ** (-s)
    cdf = np.cumsum(pmf / pmf.sum())
    cdf[-1] = 1.0
    u = rng.random(size)
    return (np.searchsorted(cdf, u, side="right") + 1).astype(np.int64)


def _components(n: int, src: np.ndarray, dst: np.ndarray):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components

    a = sp.coo_matrix((np.ones(src.shape[0], dtype=np.int8), (src, dst)), shape=(n, n)).tocsr()
    return connected_components(a, directed=True, connection="weak")


def bipartite(seed: int, n_tx: int, n_addr: int, n_hubs: int = 0, *, zipf_s: float = 2.0,
              kmax: int = 20, hub_deg: tuple[int, int] = (5000, 20000),
              radius: float | None = None, reattach: bool = True) -> Graph:
    """Bipartite transaction graph generator (seeded, PCG64).

    Node ids: transactions ``0..n_tx-1``, addresses ``n_tx..n_tx+n_addr-1``.
    Hubs are the first ``n_hubs`` addresses; hub h joins ``D_h`` distinct
    transactions, ``D_h = round(exp(U(ln lo, ln hi)))`` capped at ``n_tx // 2``.
    ``radius`` defaults to ``100 * sqrt(n / 2000)`` (the density of a
    2000-node graph in [-100, 100]^2).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    T, A = int(n_tx), int(n_addr)
    n = T + A
    if T < 1 or A < 1:
        raise ValueError("need at least one transaction and one address")
    km = min(kmax, A)
    n_in = zipf_counts(rng, T, zipf_s, km)
    n_out = zipf_counts(rng, T, zipf_s, km)
    tx_in = np.repeat(np.arange(T, dtype=np.int64), n_in)
    tx_out = np.repeat(np.arange(T, dtype=np.int64), n_out)
    addr_in = rng.integers(0, A, size=tx_in.shape[0]) + T
    addr_out = rng.integers(0, A, size=tx_out.shape[0]) + T
    srcs = [addr_in, tx_out]  # inputs: address -> tx ; outputs: tx -> address
    dsts = [tx_in, addr_out]
    for h in range(min(n_hubs, A)):
        lo, hi = hub_deg
        d = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        d = max(1, min(d, T // 2 if T >= 2 else 1))
        txs = rng.choice(T, size=d, replace=False).astype(np.int64)
        srcs.append(np.full(d, T + h, dtype=np.int64))
        dsts.append(txs)
    src = np.concatenate(srcs)
    dst = np.concatenate(dsts)

    if reattach:
        ncomp, lab = _components(n, src, dst)
        if ncomp > 1:
            sizes = np.bincount(lab, minlength=ncomp)
            big = int(np.argmax(sizes))  # argmax takes the first maximum
            big_nodes = np.nonzero(lab == big)[0]
            big_tx = big_nodes[big_nodes < T]
            big_addr = big_nodes[big_nodes >= T]
            # representative of each other component: its min-id address, or
            # its min-id transaction when it holds no address
            ids = np.arange(n, dtype=np.int64)
            is_addr = ids >= T
            key_addr = np.where(is_addr, ids, np.int64(n + 1))
            min_addr = np.full(ncomp, n + 1, dtype=np.int64)
            np.minimum.at(min_addr, lab, key_addr)
            min_any = np.full(ncomp, n + 1, dtype=np.int64)
            np.minimum.at(min_any, lab, ids)
            others = np.array([c for c in range(ncomp) if c != big], dtype=np.int64)
            rep = np.where(min_addr[others] <= n, min_addr[others], min_any[others])
            rep_is_addr = rep >= T
            pick_tx = big_tx[rng.integers(0, big_tx.shape[0], size=others.shape[0])] if big_tx.size else None
            pick_addr = big_addr[rng.integers(0, big_addr.shape[0], size=others.shape[0])] if big_addr.size else None
            e_src = np.where(rep_is_addr, rep, pick_addr if pick_addr is not None else rep)
            e_dst = np.where(rep_is_addr, pick_tx if pick_tx is not None else rep, rep)
            src = np.concatenate([src, e_src])
            dst = np.concatenate([dst, e_dst])

    R = radius if radius is not None else 100.0 * math.sqrt(n / 2000.0)
    pos = rng.uniform(-R, R, size=(2, n))
    return Graph(n=n, src=src.astype(np.int32), dst=dst.astype(np.int32),
                 x=pos[0].astype(np.float32), y=pos[1].astype(np.float32), n_tx=T, n_addr=A)


# --- the named workloads -----------------------------------------------------

def plain_2k(seed: int = 1) -> Graph:
    """1,000 transactions + 1,000 addresses, Zipf(2) capped at 20, positions in [-100,100]^2."""
    return bipartite(seed, 1000, 1000, 0, radius=100.0)


def giant_200k(seed: int = 2) -> Graph:
    """80k transactions, 120k addresses, 50 hubs of degree 5k-20k."""
    return bipartite(seed, 80_000, 120_000, 50)


def giant_2m(seed: int = 4, n_nodes: int = 2_000_000, n_hubs: int = 500) -> Graph:
    """2M nodes (40% transactions), 500 hubs."""
    T = int(round(0.4 * n_nodes))
    return bipartite(seed, T, n_nodes - T, n_hubs)


def scaled(seed: int, n_nodes: int, hubs_per_4000: bool = True) -> Graph:
    """A bipartite graph of ``n_nodes`` nodes (40% transactions, floor(n/4000) hubs)."""
    T = max(1, int(round(0.4 * n_nodes)))
    A = max(1, n_nodes - T)
    H = n_nodes // 4000 if hubs_per_4000 else 0
    return bipartite(seed, T, A, H)


def small_component_sizes(seed: int, count: int, lo: int = 3, hi: int = 200, expo: float = 2.2) -> np.ndarray:
    """Component sizes with P(n) proportional to n^-expo on [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    k = np.arange(lo, hi + 1, dtype=np.float64)
    pmf = k ** (-expo)
    cdf = np.cumsum(pmf / pmf.sum())
    cdf[-1] = 1.0
    return (np.searchsorted(cdf, rng.random(count), side="right") + lo).astype(np.int64)


def small_component(seed: int, n: int, radius: float | None = None) -> Graph:
    """One small connected bipartite component of ``n`` nodes (``n >= 2``)."""
    T = max(1, int(round(0.4 * n)))
    A = max(1, n - T)
    r = radius if radius is not None else math.sqrt(n)
    return bipartite(seed, T, A, 0, radius=r)


def union(graphs: list[Graph]) -> tuple[Graph, np.ndarray]:
    """Disjoint union; returns the graph and the node offset of each part."""
    offs = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        offs[i + 1] = offs[i] + g.n
    src = np.concatenate([g.src.astype(np.int64) + offs[i] for i, g in enumerate(graphs)])
    dst = np.concatenate([g.dst.astype(np.int64) + offs[i] for i, g in enumerate(graphs)])
    x = np.concatenate([g.x for g in graphs])
    y = np.concatenate([g.y for g in graphs])
    return Graph(n=int(offs[-1]), src=src.astype(np.int32), dst=dst.astype(np.int32), x=x, y=y), offs


def batched_components(seed: int = 3, n_small: int = 10_000, n_large: int = 20,
                       large_lo: int = 5000, large_hi: int = 50_000) -> tuple[Graph, np.ndarray]:
    """Many small components (power-law sizes on [3, 200]) plus a few large ones."""
    sizes = small_component_sizes(seed, n_small)
    rng = np.random.Generator(np.random.PCG64(seed + 17))
    large = np.round(np.exp(rng.uniform(math.log(large_lo), math.log(large_hi), size=n_large))).astype(np.int64)
    parts = [small_component(3_000_000 + i, int(s)) for i, s in enumerate(sizes)]
    parts += [scaled(3_100_000 + i, int(s), hubs_per_4000=False) for i, s in enumerate(large)]
    return union(parts)


def random_positions(seed: int, n: int, radius: float) -> tuple[np.ndarray, np.ndarray]:
    rng = np.random.Generator(np.random.PCG64(seed))
    p = rng.uniform(-radius, radius, size=(2, n))
    return p[0].astype(np.float32), p[1].astype(np.float32)


def clustered_positions(seed: int, n: int, n_clusters: int, radius: float, spread: float) -> tuple[np.ndarray, np.ndarray]:
    """Gaussian blobs: a stand-in for the dense hub clusters a laid-out graph develops."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centers = rng.uniform(-radius, radius, size=(n_clusters, 2))
    which = rng.integers(0, n_clusters, size=n)
    p = centers[which] + rng.normal(0.0, spread, size=(n, 2))
    return p[:, 0].astype(np.float32), p[:, 1].astype(np.float32)
