"""Seeded synthetic inputs: community-structured graphs, target sets and partitions.

This module draws inputs only. It holds no step of the betweenness method: no
shortest paths, no path counts, no dependencies. The GPU path's tests and bench and
the oracle's tests all take their inputs from here, so both sides see the same arrays.

Every generator uses numpy's ``Generator(PCG64(...))``. Graphs are simple and
undirected: edges are drawn as unordered pairs, deduplicated, with no self-loops, and
an edge's weight is drawn once and stored on both of its arcs. The shapes follow the
paper's workloads: community-structured graphs whose planted communities serve as the
partition (Sec. 7, "Graph-partitioning"), and a uniformly random target set (Sec. 7,
"Datasets": 200 random targets on the real graphs).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 14064173


@dataclasses.dataclass
class Graph:
    """Symmetric CSR graph plus an optional planted partition and target set.

    ``row_ptr`` int64 [n+1], ``col`` int32 [nnz] sorted within each row, ``w`` int32
    [nnz] (>= 1) or None for unit weights. ``part`` int32 [n] in [0, k). ``S`` int32,
    distinct node ids.
    """

    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray | None
    part: np.ndarray | None = None
    k: int = 0
    S: np.ndarray | None = None
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Undirected edge count."""
        return self.nnz // 2

    def edges(self):
        """Each undirected edge once, as (u, v, w) with u < v."""
        u = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))
        v = self.col.astype(np.int64)
        keep = u < v
        w = self.w[keep] if self.w is not None else np.ones(int(keep.sum()), np.int64)
        return u[keep], v[keep], w


def rng_for(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


def csr_from_edges(n: int, u, v, w=None) -> tuple:
    """Symmetric CSR from unique undirected edges (u != v). Rows sorted by column."""
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, src + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    col = dst.astype(np.int32)
    if w is None:
        return row_ptr, col, None
    w = np.asarray(w, np.int64)
    ww = np.concatenate([w, w])[order].astype(np.int32)
    return row_ptr, col, ww


def graph_from_edges(n, u, v, w=None, **kw) -> Graph:
    u = np.asarray(u, np.int64)
    v = np.asarray(v, np.int64)
    a = np.minimum(u, v)
    b = np.maximum(u, v)
    keep = a != b
    a, b = a[keep], b[keep]
    key = a * n + b
    key, idx = np.unique(key, return_index=True)
    a, b = key // n, key % n
    if w is not None:
        w = np.asarray(w, np.int64)[keep][idx]
    row_ptr, col, ww = csr_from_edges(n, a, b, w)
    return Graph(n=n, row_ptr=row_ptr, col=col, w=ww, **kw)


# ----------------------------------------------------------------------------------
# pair samplers
# ----------------------------------------------------------------------------------

def _tri_unrank(idx: np.ndarray):
    """Map a rank in [0, s(s-1)/2) to the pair (i, j), 0 <= i < j."""
    idx = idx.astype(np.int64)
    j = ((1.0 + np.sqrt(1.0 + 8.0 * idx.astype(np.float64))) / 2.0).astype(np.int64)
    # correct float rounding on either side
    j = np.where(j * (j - 1) // 2 > idx, j - 1, j)
    j = np.where((j + 1) * j // 2 <= idx, j + 1, j)
    i = idx - j * (j - 1) // 2
    return i, j


def _block_pairs(rng, size: int, p: float):
    """Bernoulli(p) over the size*(size-1)/2 pairs of one block; local (i, j)."""
    npairs = size * (size - 1) // 2
    if npairs == 0 or p <= 0.0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    if p >= 1.0:
        cnt = npairs
        ranks = np.arange(npairs, dtype=np.int64)
    else:
        cnt = int(rng.binomial(npairs, p))
        ranks = rng.choice(npairs, size=cnt, replace=False)
    return _tri_unrank(np.asarray(ranks, np.int64))


def _cross_pairs(rng, n: int, label: np.ndarray, count: int):
    """`count` distinct unordered pairs with different labels, uniform over such pairs."""
    have = np.zeros(0, np.int64)
    while have.size < count:
        need = count - have.size
        draw = max(64, int(need * 1.3) + 16)
        a = rng.integers(0, n, draw, dtype=np.int64)
        b = rng.integers(0, n, draw, dtype=np.int64)
        ok = label[a] != label[b]
        a, b = a[ok], b[ok]
        key = np.minimum(a, b) * n + np.maximum(a, b)
        # keep first occurrences, in draw order, of keys not seen before
        _, first = np.unique(key, return_index=True)
        key = key[np.sort(first)]
        key = key[~np.isin(key, have)]
        have = np.concatenate([have, key[:need]])
    return have // n, have % n


def sbm(rng, sizes, p_in, n_cross: int, wmax: int | None, name: str = "") -> Graph:
    """Block graph: Bernoulli(p_in[c]) inside block c, `n_cross` uniform cross pairs.

    ``wmax`` None gives unit weights, else weights uniform in {1..wmax}.
    """
    sizes = np.asarray(sizes, np.int64)
    k = sizes.size
    n = int(sizes.sum())
    offs = np.concatenate([[0], np.cumsum(sizes)])
    label = np.repeat(np.arange(k, dtype=np.int32), sizes)
    p_in = np.broadcast_to(np.asarray(p_in, np.float64), (k,))
    us, vs = [], []
    for c in range(k):
        i, j = _block_pairs(rng, int(sizes[c]), float(p_in[c]))
        us.append(i + offs[c])
        vs.append(j + offs[c])
    a, b = _cross_pairs(rng, n, label, int(n_cross))
    us.append(a)
    vs.append(b)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    w = None if wmax is None else rng.integers(1, wmax + 1, u.size, dtype=np.int64)
    g = graph_from_edges(n, u, v, w, name=name)
    g.part = label
    g.k = k
    return g


def equal_sizes(n: int, k: int) -> np.ndarray:
    base = np.full(k, n // k, np.int64)
    base[: n % k] += 1
    return base


def cross_count_for(rng, sizes, p_out) -> int:
    sizes = np.asarray(sizes, np.int64)
    n = int(sizes.sum())
    pairs = n * (n - 1) // 2 - int((sizes * (sizes - 1) // 2).sum())
    return int(rng.binomial(pairs, p_out)) if pairs > 0 else 0


# ----------------------------------------------------------------------------------
# the five workload configurations and the small-cut paper-regime graph
# ----------------------------------------------------------------------------------

def planted_1k() -> Graph:
    """1,000 nodes in 8 communities of 125, p_in 0.05, p_out 0.0005, unit weights, S = V."""
    rng = rng_for(SEED_BASE + 0)
    sizes = equal_sizes(1000, 8)
    g = sbm(rng, sizes, 0.05, cross_count_for(rng, sizes, 0.0005), None, "planted_1k")
    g.S = np.arange(g.n, dtype=np.int32)
    return g


def sbm_10k() -> Graph:
    """10,000 nodes, 40 communities of 250, mean degree 10 with 90% of edges inside a
    community, weights uniform in {1..10}, S = V."""
    rng = rng_for(SEED_BASE + 1)
    sizes = equal_sizes(10000, 40)
    p_in = 9.0 / 249.0
    p_out = 1.0 / 9750.0
    g = sbm(rng, sizes, p_in, cross_count_for(rng, sizes, p_out), 10, "sbm_10k")
    g.S = np.arange(g.n, dtype=np.int32)
    return g


def _community_graph(rng, n, k, deg, intra, wmax, name, sizes=None):
    sizes = equal_sizes(n, k) if sizes is None else np.asarray(sizes, np.int64)
    p_in = np.minimum(1.0, intra * deg / np.maximum(sizes - 1, 1))
    n_cross = int(round(n * deg * (1.0 - intra) / 2.0))
    return sbm(rng, sizes, p_in, n_cross, wmax, name)


def batch_256(count: int = 256) -> list:
    """256 independent community graphs: n log-uniform in [200, 5000], 4..32 equal
    communities, mean degree uniform in [6, 12] with 90% of edges inside a community,
    unit weights; S = a uniform 5-20% of the nodes (at least 2)."""
    out = []
    for gi in range(count):
        rng = rng_for(SEED_BASE + 2, gi)
        n = int(round(math.exp(rng.uniform(math.log(200), math.log(5000)))))
        k = int(rng.integers(4, 33))
        deg = float(rng.uniform(6.0, 12.0))
        g = _community_graph(rng, n, k, deg, 0.9, None, f"batch_{gi}")
        ns = max(2, int(round(rng.uniform(0.05, 0.20) * n)))
        g.S = np.sort(rng.choice(n, ns, replace=False)).astype(np.int32)
        out.append(g)
    return out


def pareto_sizes(rng, total: int, k: int, alpha: float = 2.0, min_size: int = 2):
    """Community sizes (Pareto(alpha)+1), scaled to `total` by largest remainder."""
    raw = rng.pareto(alpha, k) + 1.0
    share = raw / raw.sum() * (total - min_size * k)
    base = np.floor(share).astype(np.int64)
    rem = total - min_size * k - int(base.sum())
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rem]] += 1
    return base + min_size


def pareto_100k() -> Graph:
    """100,000 nodes, 500 communities of Pareto(2) sizes, mean degree 8 with 85% of
    edges inside a community, weights uniform in {1..4}, |S| = 2000 uniform."""
    rng = rng_for(SEED_BASE + 3)
    sizes = pareto_sizes(rng, 100000, 500)
    p_in = np.minimum(1.0, 6.8 / np.maximum(sizes - 1, 1))
    g = sbm(rng, sizes, p_in, 60000, 4, "pareto_100k")
    g.S = np.sort(rng.choice(g.n, 2000, replace=False)).astype(np.int32)
    return g


def smallcut_100k() -> Graph:
    """Paper regime (small cuts between parts): 100,000 nodes in 2,000 communities of 50,
    mean degree 8 with 99% of edges inside a community (98% of the nodes in one
    connected component), weights uniform in {1..4}, |S| = 200."""
    rng = rng_for(SEED_BASE + 5)
    g = _community_graph(rng, 100000, 2000, 8.0, 0.99, 4, "smallcut_100k")
    g.S = np.sort(rng.choice(g.n, 200, replace=False)).astype(np.int32)
    return g


P1_INTRA = (0.9, 0.97, 0.99, 0.995, 0.998)


def p1_graph(intra: float) -> Graph:
    """Small-cut sweep: 100,000 nodes in 5,000 communities of 20, mean degree 8 with a
    fraction `intra` of the edges inside a community, weights uniform in {1..4},
    |S| = 200. The fraction sets the cut size, and with it how small the skeleton is."""
    rng = rng_for(SEED_BASE + 6, int(round(intra * 1000)))
    g = _community_graph(rng, 100000, 5000, 8.0, intra, 4, f"p1_{intra}")
    g.S = np.sort(rng.choice(g.n, 200, replace=False)).astype(np.int32)
    return g


def serving_pool(count: int = 64) -> list:
    """64 resident graphs: n log-uniform in [1e3, 5e4], max(4, n/200) equal
    communities, mean degree 8 with 85% of edges inside a community; unit weights for
    even indices, {1..10} for odd ones."""
    out = []
    for gi in range(count):
        rng = rng_for(SEED_BASE + 4, gi)
        n = int(round(math.exp(rng.uniform(math.log(1e3), math.log(5e4)))))
        k = max(4, int(round(n / 200)))
        wmax = None if gi % 2 == 0 else 10
        out.append(_community_graph(rng, n, k, 8.0, 0.85, wmax, f"pool_{gi}"))
    return out


def serving_stream(pool_sizes, rate: float = 200.0, seconds: float = 32.0, seed_extra: int = 0):
    """Open-loop Poisson arrivals: (arrival_s, graph index, S) with |S| log-uniform in
    [16, 4096] capped at the graph's node count."""
    rng = rng_for(SEED_BASE + 4, 1_000_000 + seed_extra)
    t = 0.0
    out = []
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= seconds:
            break
        gi = int(rng.integers(0, len(pool_sizes)))
        n = int(pool_sizes[gi])
        ns = min(n, int(round(math.exp(rng.uniform(math.log(16), math.log(4096))))))
        S = np.sort(rng.choice(n, ns, replace=False)).astype(np.int32)
        out.append((t, gi, S))
    return out


CONFIGS = {
    "planted_1k": planted_1k,
    "sbm_10k": sbm_10k,
    "pareto_100k": pareto_100k,
    "smallcut_100k": smallcut_100k,
}


# ----------------------------------------------------------------------------------
# small graph families for closed forms, edge cases and brute force
# ----------------------------------------------------------------------------------

def star(n: int) -> Graph:
    return graph_from_edges(n, np.zeros(n - 1, np.int64), np.arange(1, n), name=f"star{n}")


def path(n: int, w=None) -> Graph:
    return graph_from_edges(n, np.arange(n - 1), np.arange(1, n), w, name=f"path{n}")


def cycle(n: int) -> Graph:
    a = np.arange(n)
    return graph_from_edges(n, a, (a + 1) % n, name=f"cycle{n}")


def complete(n: int) -> Graph:
    i, j = np.triu_indices(n, 1)
    return graph_from_edges(n, i, j, name=f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    i, j = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return graph_from_edges(a + b, i.ravel(), j.ravel(), name=f"K{a},{b}")


def grid(r: int, c: int, w=None) -> Graph:
    """r x c grid, node (i, j) = i*c + j."""
    idx = np.arange(r * c).reshape(r, c)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return graph_from_edges(r * c, u, v, w, name=f"grid{r}x{c}")


def empty(n: int) -> Graph:
    return Graph(n=n, row_ptr=np.zeros(n + 1, np.int64), col=np.zeros(0, np.int32),
                 w=None, name=f"empty{n}")


def random_graph(seed: int, n: int, p: float, wmax: int | None = None, k: int = 0,
                 ns: int | None = None) -> Graph:
    """G(n, p) with weights in {1..wmax} (None = unit), a random partition into k parts
    (k = 0 picks 1..max(1, n//3)) and a random target set of size ns (None = random)."""
    rng = rng_for(SEED_BASE + 99, seed)
    i, j = np.triu_indices(n, 1)
    keep = rng.random(i.size) < p
    u, v = i[keep], j[keep]
    w = None if wmax is None else rng.integers(1, wmax + 1, u.size, dtype=np.int64)
    g = graph_from_edges(n, u, v, w, name=f"gnp{seed}")
    if k <= 0:
        k = int(rng.integers(1, max(1, n // 3) + 1))
    g.part = rng.integers(0, k, n).astype(np.int32)
    g.k = k
    if ns is None:
        ns = int(rng.integers(0, n + 1))
    g.S = np.sort(rng.choice(n, min(ns, n), replace=False)).astype(np.int32)
    return g


def random_targets(seed: int, n: int, ns: int) -> np.ndarray:
    rng = rng_for(SEED_BASE + 98, seed)
    return np.sort(rng.choice(n, ns, replace=False)).astype(np.int32)


def random_partition(seed: int, n: int, k: int) -> np.ndarray:
    rng = rng_for(SEED_BASE + 97, seed)
    return rng.integers(0, k, n).astype(np.int32)
