"""Seeded synthetic Max-Cut inputs shared by the tests, the oracle checks and the benchmark.

This module only *generates graphs* (vertex count, edge endpoints, integer weights) from
numpy's seeded generator.  It holds none of the optimisation method's arithmetic: no fitness,
no Philox, no colouring, no GOM.  Both the CPU oracle and the GPU library receive the same
arrays produced here and nothing else.

The paper's benchmark sets (fully connected graphs, 2D tori and BIQMAC instances; Section 6.2)
are not available, so seeded stand-ins with the same structure are used:

* ``torus(L, ...)`` -- an L x L grid with wrap-around on both axes (the structure of set B:
  every vertex has exactly four neighbours, m = 2 L^2 edges).
* ``configuration_model(n, d, ...)`` -- a random d-regular multigraph from the configuration
  model with self-loops and repeated pairs removed (sparse, unstructured graphs in the regime
  of the larger set-C instances).

Weights are drawn after the structure from the same generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Graph:
    """A simple undirected edge-weighted graph as three aligned int32 edge arrays."""

    n: int
    u: np.ndarray
    v: np.ndarray
    w: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.u.shape[0])

    @property
    def total_weight(self) -> int:
        return int(self.w.astype(np.int64).sum())


def _as_graph(n: int, u, v, w, name: str) -> Graph:
    return Graph(n=int(n), u=np.ascontiguousarray(u, dtype=np.int32),
                 v=np.ascontiguousarray(v, dtype=np.int32),
                 w=np.ascontiguousarray(w, dtype=np.int32), name=name)


def torus(L: int, w_lo: int, w_hi: int, seed: int) -> Graph:
    """L x L torus; vertex id r*L + c; per vertex in row-major order its edge to the right,
    then its edge downwards (both with wrap-around).  Weights uniform in [w_lo, w_hi]."""
    if L < 3:
        raise ValueError("a simple L x L torus needs L >= 3")
    rng = np.random.default_rng(seed)
    r, c = np.divmod(np.arange(L * L, dtype=np.int64), L)
    vid = r * L + c
    right = r * L + (c + 1) % L
    down = ((r + 1) % L) * L + c
    u = np.stack([vid, vid], axis=1).reshape(-1)
    v = np.stack([right, down], axis=1).reshape(-1)
    w = rng.integers(w_lo, w_hi + 1, size=u.shape[0], dtype=np.int64)
    return _as_graph(L * L, u, v, w, f"torus{L}x{L}")


def signed_uniform(rng: np.random.Generator, size: int, mag: int) -> np.ndarray:
    """Integers uniform over {-mag..-1} U {1..mag} (zero excluded)."""
    k = rng.integers(0, 2 * mag, size=size, dtype=np.int64)
    return np.where(k < mag, k - mag, k - mag + 1)


def configuration_model(n: int, d: int, seed: int, weights: str = "signed50",
                        w_lo: int = 1, w_hi: int = 100) -> Graph:
    """Random d-regular graph from the configuration model: n*d stubs shuffled, consecutive
    stubs paired; self-loops and repeated unordered pairs are dropped (first occurrence
    kept), so a few vertices end with degree below d.  ``weights`` is ``"signed50"``
    (uniform over +-1..50, zero excluded) or ``"uniform"`` (uniform in [w_lo, w_hi])."""
    if (n * d) % 2:
        raise ValueError("n*d must be even")
    rng = np.random.default_rng(seed)
    stubs = np.repeat(np.arange(n, dtype=np.int64), d)
    rng.shuffle(stubs)
    a, b = stubs[0::2], stubs[1::2]
    keep = a != b
    a, b = a[keep], b[keep]
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = lo * n + hi
    _, first = np.unique(key, return_index=True)
    first.sort()
    a, b = a[first], b[first]
    if weights == "signed50":
        w = signed_uniform(rng, a.shape[0], 50)
    elif weights == "uniform":
        w = rng.integers(w_lo, w_hi + 1, size=a.shape[0], dtype=np.int64)
    else:
        raise ValueError(weights)
    return _as_graph(n, a, b, w, f"cm{n}d{d}")


def from_edges(n: int, edges, weights=None, name: str = "") -> Graph:
    """Graph from an explicit edge list (pairs), unit weights unless given."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    w = np.ones(e.shape[0], dtype=np.int64) if weights is None else np.asarray(weights)
    return _as_graph(n, e[:, 0], e[:, 1], w, name)


# Fully-specified workloads.  FOS kind: 0 = univariate, 1 = neighbourhood {v} U N(v),
# 2 = linkage tree by UPGMA on |w| with set sizes up to lt_bound (0 = the full tree).
@dataclass(frozen=True)
class Workload:
    name: str
    graph_fn: object = field(repr=False)
    fos: int
    pop: int
    max_gens: int
    to_total_weight: bool  # run until the elite reaches the total weight (bipartite tori)
    seeds: tuple = (1, 2, 3, 4, 5)
    lt_bound: int = 0

    def graph(self) -> Graph:
        return self.graph_fn()


def _c1():
    return torus(10, 1, 5, seed=1)


def _c2():
    return torus(100, 1, 100, seed=2)


def _t1000():
    return torus(1000, 1, 100, seed=7)


def _c3(d):
    return lambda: configuration_model(100_000, d, seed=3, weights="signed50")


WORKLOADS = {
    # 10x10 torus, weights U{1..5}, univariate FOS, population 16, 20 generations.
    "torus10_uni_p16": Workload("torus10_uni_p16", _c1, 0, 16, 20, False),
    # 100x100 torus, weights U{1..100}, neighbourhood FOS, population 64, to optimum or 500.
    "torus100_nbhd_p64": Workload("torus100_nbhd_p64", _c2, 1, 64, 500, True),
}
# 1000x1000 torus (10^6 vertices), weights U{1..100}: the HBM-bound size.
WORKLOADS["torus1000_uni_p64"] = Workload("torus1000_uni_p64", _t1000, 0, 64, 1000, True)
WORKLOADS["torus1000_nbhd_p64"] = Workload("torus1000_nbhd_p64", _t1000, 1, 64, 1000, True)
# Random 4- and 8-regular graphs with 10^6 vertices, weights U{1..100}, univariate FOS: the
# HBM-bound size beyond the torus (degree 8 is outside the bit-sliced sweep's degree limit).
for _d in (4, 8):
    WORKLOADS[f"cm1m_d{_d}_uni_p64"] = Workload(
        f"cm1m_d{_d}_uni_p64",
        (lambda d: lambda: configuration_model(1_000_000, d, seed=5, weights="uniform",
                                               w_lo=1, w_hi=100))(_d), 0, 64, 200, False)
# 3162x3162 torus (10^7 vertices), weights U{1..100}, univariate FOS: a working set (about
# 520 MB) larger than the 256 MB Infinity Cache, so the sweep's traffic reaches HBM.
WORKLOADS["torus3162_uni_p64"] = Workload("torus3162_uni_p64",
                                          lambda: torus(3162, 1, 100, seed=9), 0, 64, 100, True)
# 100x100 torus, weights U{1..100}, univariate FOS (the graph's own colouring: the classes of
# the colouring-parallel local search).
WORKLOADS["torus100_uni_p64"] = Workload("torus100_uni_p64", _c2, 0, 64, 500, True)
# 32x32 torus, weights U{1..100}, neighbourhood FOS: small enough to reach its optimum.
WORKLOADS["torus32_nbhd_p64"] = Workload("torus32_nbhd_p64", lambda: torus(32, 1, 100, seed=8),
                                         1, 64, 500, True)
# 48x48, 64x64 and 80x80 tori, weights U{1..100}, neighbourhood FOS: the sizes around the
# largest instance the automatic schedule choice keeps resident.
for _L in (48, 64, 80):
    WORKLOADS[f"torus{_L}_nbhd_p64"] = Workload(
        f"torus{_L}_nbhd_p64", (lambda L: lambda: torus(L, 1, 100, seed=8))(_L), 1, 64, 500, True)
# 100x100 torus with fixed linkage trees: the full tree and trees bounded to 10 and 100.
for _b in (0, 10, 100):
    _name = f"torus100_bflt{_b}_p64" if _b else "torus100_flt_p64"
    WORKLOADS[_name] = Workload(_name, _c2, 2, 64, 500, True, lt_bound=_b)
for _d in (3, 6, 12):
    for _k, _fn in ((0, "uni"), (1, "nbhd")):
        WORKLOADS[f"cm100k_d{_d}_{_fn}_p32"] = Workload(
            f"cm100k_d{_d}_{_fn}_p32", _c3(_d), _k, 32, 200, False)


@dataclass(frozen=True)
class BatchItem:
    graph: Graph
    fos: int
    pop: int
    seed: int
    to_total_weight: bool


def batch_mix(count: int = 256, seed: int = 4, n_lo: float = 1e3, n_hi: float = 1e5):
    """Many independent instances for batched runs: n log-uniform in [n_lo, n_hi]; even
    positions are L x L tori (L = n's square root rounded to an even number, >= 4), odd ones
    configuration-model graphs of degree 4 and 8 alternately; weights uniform in [1, 100];
    populations uniform in [16, 64]; univariate and neighbourhood FOS alternate in pairs.
    Tori have the total weight as their optimum (even torus, positive weights)."""
    rng = np.random.default_rng(seed)
    items = []
    for k in range(count):
        n = int(round(10 ** rng.uniform(np.log10(n_lo), np.log10(n_hi))))
        pop = int(rng.integers(16, 65))
        fos = 0 if k % 4 < 2 else 1
        if k % 2 == 0:
            L = max(4, 2 * int(round(np.sqrt(n) / 2)))
            g = torus(L, 1, 100, seed=10_000 + k)
            items.append(BatchItem(g, fos, pop, 1 + k, True))
        else:
            d = 4 if (k // 2) % 2 == 0 else 8
            g = configuration_model(n + (n * d) % 2, d, seed=10_000 + k, weights="uniform",
                                    w_lo=1, w_hi=100)
            items.append(BatchItem(g, fos, pop, 1 + k, False))
    return items


@dataclass(frozen=True)
class ServeJob:
    graph: Graph
    fos: int
    pop: int
    seed: int
    target: int           # total weight for tori (their optimum), else unreachable
    max_gens: int


def serve_stream(count: int = 200, seed: int = 5, max_gens: int = 1000,
                 sizes=("small", "medium", "large")):
    """Jobs of the serving workload: L x L tori with L in {100, 316, 1000} or configuration-
    model graphs with n in {10^4, 10^5, 10^6} and degree uniform in {4..8}, weights uniform in
    [1, 100], population 64; univariate and neighbourhood FOS alternate; tori run to their
    total weight (their optimum), the others to the generation limit.  `sizes` restricts the
    three size classes (small = 10^4 vertices, medium = 10^5, large = 10^6)."""
    rng = np.random.default_rng(seed)
    side = {"small": 100, "medium": 316, "large": 1000}
    verts = {"small": 10_000, "medium": 100_000, "large": 1_000_000}
    jobs = []
    for k in range(count):
        size = sizes[int(rng.integers(0, len(sizes)))]
        fos = k % 2
        gseed = 20_000 + k
        if rng.integers(0, 2) == 0:
            g = torus(side[size], 1, 100, seed=gseed)
            target = g.total_weight
        else:
            d = int(rng.integers(4, 9))
            n = verts[size]
            g = configuration_model(n + (n * d) % 2, d, seed=gseed, weights="uniform",
                                    w_lo=1, w_hi=100)
            target = 1 << 62
        jobs.append(ServeJob(g, fos, 64, 1000 + k, target, max_gens))
    return jobs


def poisson_arrivals(count: int, rate: float, seed: int = 5) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed + 1)
    return np.cumsum(rng.exponential(1.0 / rate, size=count))
