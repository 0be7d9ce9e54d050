"""Seeded synthetic inputs shared by the tests, the smoke check and the bench.

This module holds no PageRank arithmetic: it only produces inputs (edge
lists of small hand-made graphs, personalised-PageRank seed sets, random
start vectors, random network weights).  Both the CPU oracle and the HIP
path receive exactly the arrays returned here.  The R-MAT edge lists are not
made here: each side implements the counter-based R-MAT generator from its
published definition, and the two are compared bit for bit.
"""
from __future__ import annotations

import numpy as np

# Workload sizes of the benchmark graphs (R-MAT, edge factor 16, the seed
# equals the scale).
RMAT_EDGEFACTOR = 16
DAMPING = 0.85

# Web-shaped stand-in for the paper's web crawl (Section IV: 50.6 million
# pages, 1.9494 billion links, strong locality, high mean degree).  The
# parameters of the web-shaped generator (see GrM_web_edges): out-degrees
# min(4000, D(7)) with 17.75 % of pages without links; 5 % home links,
# 60 % local links at distance >= max(16, k_u), 35 % global links with
# popularity scale 1024.  At WEB_N vertices this generates 2,120,533,943
# links, about 1.93 billion after merging repeats (38.2 per vertex).
WEB_N = 50_600_000
WEB_SEED = 50
WEB_MODEL = {
    "kmin": 7, "kmax": 4000,
    "p_zero": 11633, "p_home": 3277, "p_local": 39322,
    "local_min": 16, "hub": 1024,
    "perm_a": 2654435761, "perm_b": 12345,
}
# The paper does not state its PageRank settings for the crawl; these are
# the GAP benchmark's (damping 0.85, tolerance 1e-4 on the L1 change).
WEB_TOL = 1e-4
WEB_ITERMAX = 100


def cycle(n: int):
    """Directed cycle 0->1->...->n-1->0."""
    src = np.arange(n, dtype=np.uint32)
    dst = ((np.arange(n) + 1) % n).astype(np.uint32)
    return n, src, dst


def complete(n: int):
    """Complete digraph without self-loops."""
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = i != j
    return n, i[keep].astype(np.uint32), j[keep].astype(np.uint32)


def empty(n: int):
    """n vertices, no edges."""
    return n, np.zeros(0, np.uint32), np.zeros(0, np.uint32)


def star_in(m: int):
    """Leaves 1..m each point to the centre 0."""
    leaves = np.arange(1, m + 1, dtype=np.uint32)
    return m + 1, leaves, np.zeros(m, np.uint32)


def star_out(m: int):
    """Centre 0 points to each leaf 1..m."""
    leaves = np.arange(1, m + 1, dtype=np.uint32)
    return m + 1, np.zeros(m, np.uint32), leaves


def star_both(m: int):
    """Centre 0 and every leaf linked in both directions."""
    leaves = np.arange(1, m + 1, dtype=np.uint32)
    z = np.zeros(m, np.uint32)
    return m + 1, np.concatenate([z, leaves]), np.concatenate([leaves, z])


def path2():
    """Two vertices, one edge 0->1."""
    return 2, np.array([0], np.uint32), np.array([1], np.uint32)


def random_edges(n: int, nedges: int, seed: int, self_loops: bool = True):
    """Uniform random directed edges (duplicates and, optionally, self-loops
    included) for brute-force checks of the CSR build."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, nedges, dtype=np.uint32)
    dst = rng.integers(0, n, nedges, dtype=np.uint32)
    if not self_loops:
        keep = src != dst
        src, dst = src[keep], dst[keep]
    return n, src, dst


def ppr_seed_sets(n: int, count: int, seed: int = 7, max_size: int = 16):
    """``count`` seed sets; each has a size drawn uniformly from 1..max_size
    and that many distinct vertices drawn uniformly from [0, n)."""
    rng = np.random.default_rng(seed)
    sets = []
    for _ in range(count):
        k = int(rng.integers(1, max_size + 1))
        sets.append(np.sort(rng.choice(n, size=k, replace=False)).astype(np.int32))
    return sets


def random_distribution(n: int, seed: int) -> np.ndarray:
    """A positive vector summing to one (a non-uniform start vector)."""
    rng = np.random.default_rng(seed)
    x = rng.random(n) + 0.05
    return x / x.sum()


def random_vector(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.random(n)


def _splitmix64_first(seed: int) -> int:
    """First output of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014)
    seeded with `seed`: one increment of the state, then the mix."""
    m = (1 << 64) - 1
    z = (seed + 0x9E3779B97F4A7C15) & m
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & m
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & m
    return z ^ (z >> 31)


def many_graph_specs(count: int = 256, base_seed: int = 3000, smin: int = 10,
                     smax: int = 16):
    """(scale, seed) of each graph of the many-small-graphs workload: graph
    i has seed base_seed + i and scale smin + (SplitMix64(base_seed + i) mod
    (smax - smin + 1)), the first draw of the generator seeded with the
    graph's seed."""
    k = smax - smin + 1
    return [(smin + _splitmix64_first(base_seed + i) % k, base_seed + i) for i in range(count)]
