"""Seeded synthetic data graphs (undirected, simple) in CSR form.

This module only draws inputs.  It holds none of the counting method's
arithmetic and is shared by the oracle tests, the device tests and the
benchmark so that both sides see byte-identical graphs.

Every generator returns a ``Graph``: ``n`` vertices, ``row_ptr`` (int64,
n+1) and ``col`` (int32, 2m) with each undirected edge stored in both
directions, neighbour lists sorted by vertex id, no self-loops and no
duplicate edges.

Generators
----------
* ``erdos_renyi(n, avg_degree, seed)``  G(n, p) with p = avg_degree/(n-1).
* ``chung_lu(n, mean, gamma, w_max, seed)``  the random power-law model of
  the paper's analysis (Appendix A: edge (i, j) present independently with
  probability min(1, w_i w_j / sum(w))), sampled in O(n + m) by skipping
  over non-edges with geometric jumps (the Miller-Hagberg scheme).
* ``complete(n)``, ``from_edges(n, edges)`` and small helpers for tests.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[row_ptr[n]]
    name: str = ""

    @property
    def m(self) -> int:
        """Number of undirected edges."""
        return int(self.row_ptr[-1]) // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def edge_list(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64 array of shape (m, 2)."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]


def from_edges(n: int, edges, name: str = "") -> Graph:
    """Build a symmetric CSR from an undirected edge list.

    Self-loops are dropped and duplicate edges merged, so the result is
    always a simple graph."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size:
        if e.min() < 0 or e.max() >= n:
            raise ValueError("edge endpoint out of range")
    e = e[e[:, 0] != e[:, 1]]
    a = np.minimum(e[:, 0], e[:, 1])
    b = np.maximum(e[:, 0], e[:, 1])
    key = np.unique(a * n + b)
    a = key // n
    b = key % n
    src = np.concatenate([a, b])
    dst = np.concatenate([b, a])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return Graph(n=n, row_ptr=row_ptr, col=dst.astype(np.int32), name=name)


def permute(g: Graph, seed: int) -> Graph:
    """Relabel vertices by a seeded random permutation (same graph)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    perm = rng.permutation(g.n)
    e = g.edge_list()
    return from_edges(g.n, perm[e], name=g.name)


def erdos_renyi(n: int, avg_degree: float, seed: int) -> Graph:
    """G(n, p), p = avg_degree / (n - 1): every unordered pair independently."""
    p = avg_degree / (n - 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.shape[0]) < p
    return from_edges(n, np.stack([iu[keep], ju[keep]], axis=1),
                      name=f"er_n{n}_d{avg_degree:g}_s{seed}")


def power_law_weights(n: int, mean: float, gamma: float, w_max: float) -> np.ndarray:
    """Expected degrees w_i = c (i + i0)^(-1/(gamma-1)), i = 0..n-1.

    ``c`` and ``i0`` are fitted so that w_0 = w_max and mean(w) = mean.
    The exponent -1/(gamma-1) gives a degree distribution with tail
    P[deg >= d] ~ d^-(gamma-1)."""
    beta = 1.0 / (gamma - 1.0)
    idx = np.arange(n, dtype=np.float64)

    def mean_for(i0: float) -> float:
        return float(w_max * np.mean(((idx + i0) / i0) ** (-beta)))

    lo, hi = 1e-6, 1e12
    for _ in range(200):
        mid = math.sqrt(lo * hi)
        if mean_for(mid) < mean:
            lo = mid
        else:
            hi = mid
    i0 = math.sqrt(lo * hi)
    return w_max * ((idx + i0) / i0) ** (-beta)


def structural_cutoff(n: int, mean: float, cap: float = 1e4) -> float:
    """w_max = min(cap, sqrt(sum w)), so that w_i w_j / sum(w) <= 1."""
    return min(cap, math.sqrt(n * mean))


def chung_lu_from_weights(w: np.ndarray, seed: int, name: str = "") -> Graph:
    """Sample edge (i, j), i < j, independently with p = min(1, w_i w_j / S).

    ``w`` must be non-increasing.  For each row i the candidates j > i are
    visited with geometric skips under the current (non-increasing) bound p,
    and a visited candidate is kept with probability q/p where q is its own
    probability; this yields exactly the independent-edge model in O(n + m)
    expected draws.  All rows advance together, one vectorised step at a time,
    so the sequence of random draws is fixed by ``seed`` alone."""
    n = int(w.shape[0])
    if n < 2:
        return from_edges(n, np.zeros((0, 2), dtype=np.int64), name=name)
    if np.any(np.diff(w) > 0):
        raise ValueError("weights must be non-increasing")
    S = float(np.sum(w))
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.arange(n - 1, dtype=np.int64)
    v = u + 1
    p = np.minimum(w[u] * w[v] / S, 1.0)
    active = p > 0
    u, v, p = u[active], v[active], p[active]
    out_u, out_v = [], []
    while u.size:
        r = rng.random(u.size)
        skip = np.zeros(u.size, dtype=np.int64)
        lt1 = p < 1.0
        if np.any(lt1):
            with np.errstate(divide="ignore"):
                s = np.floor(np.log(r[lt1]) / np.log1p(-p[lt1]))
            s = np.minimum(s, float(n))
            skip[lt1] = s.astype(np.int64)
        v = v + skip
        inb = v < n
        q = np.zeros(u.size, dtype=np.float64)
        q[inb] = np.minimum(w[u[inb]] * w[v[inb]] / S, 1.0)
        r2 = rng.random(u.size)
        acc = inb & (r2 < q / p)
        out_u.append(u[acc])
        out_v.append(v[acc])
        p = q
        v = v + 1
        keep = inb & (v < n) & (p > 0)
        u, v, p = u[keep], v[keep], p[keep]
    e = np.stack([np.concatenate(out_u), np.concatenate(out_v)], axis=1)
    return from_edges(n, e, name=name)


def chung_lu(n: int, mean: float, gamma: float, w_max: float | None, seed: int,
             relabel: bool = True) -> Graph:
    """Chung-Lu power-law graph with vertex ids shuffled by ``seed``."""
    if w_max is None:
        w_max = structural_cutoff(n, mean)
    w = power_law_weights(n, mean, gamma, w_max)
    g = chung_lu_from_weights(w, seed,
                              name=f"chunglu_n{n}_mean{mean:g}_g{gamma:g}_s{seed}")
    if relabel:
        g = permute(g, seed ^ 0x5A5A5A5A)
        g.name = f"chunglu_n{n}_mean{mean:g}_g{gamma:g}_s{seed}"
    return g


def complete(n: int) -> Graph:
    iu, ju = np.triu_indices(n, k=1)
    return from_edges(n, np.stack([iu, ju], axis=1), name=f"K{n}")


def cycle_graph(n: int) -> Graph:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], name=f"C{n}")


def disjoint_union(a: Graph, b: Graph) -> Graph:
    e = np.concatenate([a.edge_list(), b.edge_list() + a.n])
    return from_edges(a.n + b.n, e, name=f"{a.name}+{b.name}")


def hub_and_clique(leaves: int, clique: int = 12):
    """A star (vertex 0 with `leaves` leaves 1..leaves) beside a clique on the
    next `clique` vertices, with a fixed colouring for k = clique - 1 colours:
    the hub colour 0, leaf i colour 1 + (i - 1) % (k - 1), clique vertex j
    colour j % k (colour 0 twice).  Returns (graph, colours)."""
    k = clique - 1
    e = [(0, i) for i in range(1, leaves + 1)]
    base = leaves + 1
    e += [(base + a, base + b) for a in range(clique) for b in range(a + 1, clique)]
    n = base + clique
    col = np.zeros(n, dtype=np.uint8)
    col[1:base] = [1 + (i - 1) % (k - 1) for i in range(1, base)]
    col[base:] = [j % k for j in range(clique)]
    return from_edges(n, np.array(e, dtype=np.int64), name=f"hub{leaves}+K{clique}"), col


# The benchmark workloads, by name.  Sizes follow the configurations the
# counting benchmark is quoted on; each is seeded and deterministic.
def workload_graph(name: str) -> Graph:
    if name == "er1000":
        return erdos_renyi(1000, 10.0, seed=1)
    if name == "cl1m":
        return chung_lu(1_000_000, 16.0, 2.1, 1e4, seed=2)
    if name == "cl2m":
        return chung_lu(2_000_000, 20.0, 2.2, None, seed=3)
    if name == "cl4m":
        return chung_lu(4_000_000, 20.0, 2.1, None, seed=4)
    raise KeyError(name)
