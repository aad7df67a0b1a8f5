"""Seeded query graphs (small, connected, simple; nodes 0..k-1).

Only inputs: no counting arithmetic lives here.

Named shapes used by the tests and the benchmark, plus a seeded generator of
treewidth <= 2 queries of 4-10 nodes drawn from four families: plain cycles,
cycles with one or two non-crossing chords, a cycle with a random tree on the
remaining nodes, and two cycles sharing a node or an edge.
"""
from __future__ import annotations

import numpy as np


def cycle(L: int):
    return L, [(i, (i + 1) % L) for i in range(L)]


def path(k: int):
    return k, [(i, i + 1) for i in range(k - 1)]


def star(k: int):
    """K_{1,k-1}: centre 0."""
    return k, [(0, i) for i in range(1, k)]


def cycle_pendant(L: int):
    """Cycle 0..L-1 plus one pendant node L attached to node 0."""
    k, e = cycle(L)
    return L + 1, e + [(0, L)]


def domino_tail():
    """Two 4-cycles sharing the edge (0,1), plus a 2-node tail at node 2:
    nodes a,b,c,d,e,f,t1,t2 = 0..7."""
    a, b, c, d, e, f, t1, t2 = range(8)
    return 8, [(a, b), (b, c), (c, d), (d, a), (b, e), (e, f), (f, a), (c, t1), (t1, t2)]


def satellite():
    """The worked decomposition example of Section 4.1, rebuilt from its
    text: blocks (a,b,c,d,e), (f,h), (a,f,g,c), (i,j,k) and root (i,f,g).
    Nodes a..k = 0..10."""
    a, b, c, d, e, f, g, h, i, j, k = range(11)
    E = [(a, b), (b, c), (c, d), (d, e), (e, a), (a, f), (f, g), (g, c), (f, h),
         (f, i), (g, i), (i, j), (j, k), (k, i)]
    return 11, E


def k4():
    return 4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def k23():
    """K_{2,3}: two hubs 0,1 joined through 2,3,4 (treewidth 2)."""
    return 5, [(0, 2), (2, 1), (0, 3), (3, 1), (0, 4), (4, 1)]


def k33():
    return 6, [(a, b) for a in range(3) for b in range(3, 6)]


def star_triangle(leaves: int = 8):
    """A star of `leaves` leaves whose centre (node 0) also lies on a
    triangle (nodes 0, leaves + 1, leaves + 2): k = leaves + 3."""
    k = leaves + 3
    E = [(0, i) for i in range(1, leaves + 1)]
    E += [(0, leaves + 1), (leaves + 1, leaves + 2), (leaves + 2, 0)]
    return k, E


def random_query(rng: np.random.Generator, kmin: int = 4, kmax: int = 10):
    """One treewidth <= 2 query; family uniform over four shapes."""
    k = int(rng.integers(kmin, kmax + 1))
    fam = int(rng.integers(0, 4))
    if fam == 0:                       # plain cycle
        return k, cycle(k)[1], "cycle"
    if fam == 1:                       # cycle with 1-2 non-crossing chords
        L = k
        E = cycle(L)[1]
        nch = 1 if L < 6 else int(rng.integers(1, 3))
        chords = []
        tries = 0
        while len(chords) < nch and tries < 100:
            tries += 1
            a, b = sorted(int(x) for x in rng.choice(L, size=2, replace=False))
            if b - a < 2 or (a == 0 and b == L - 1):
                continue
            ok = True
            for (c, d) in chords:
                # crossing iff exactly one endpoint of (c,d) strictly inside (a,b)
                inside = (a < c < b) != (a < d < b)
                if inside and len({a, b, c, d}) == 4:
                    ok = False
                if (a, b) == (c, d):
                    ok = False
            if ok:
                chords.append((a, b))
        if not chords:
            return k, E, "cycle"
        return k, E + chords, "chorded"
    if fam == 2:                       # cycle C_L plus a random tree on the rest
        L = int(rng.integers(3, k))
        E = cycle(L)[1]
        for v in range(L, k):
            E.append((int(rng.integers(0, v)), v))
        return k, E, "cycle+tree"
    # two cycles sharing a node or an edge
    share_edge = bool(rng.integers(0, 2))
    if share_edge and k >= 4:
        # cycle A: 0..L1-1 ; cycle B shares edge (0,1) and adds k-L1 nodes
        L1 = int(rng.integers(3, k))
        if k - L1 < 1:
            L1 = k - 1
        E = cycle(L1)[1]
        rest = list(range(L1, k))
        chain = [1] + rest + [0]
        for x, y in zip(chain, chain[1:]):
            E.append((x, y))
        return k, E, "two-cycles-edge"
    # share a node: cycle 0..L1-1, second cycle through node 0
    if k < 5:
        return k, cycle(k)[1], "cycle"
    L1 = int(rng.integers(3, k - 1))
    E = cycle(L1)[1]
    rest = list(range(L1, k))
    chain = [0] + rest + [0]
    for x, y in zip(chain, chain[1:]):
        E.append((x, y))
    return k, E, "two-cycles-node"


def random_queries(seed: int, count: int, kmin: int = 4, kmax: int = 10):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [random_query(rng, kmin, kmax) for _ in range(count)]


def random_series_parallel(rng: np.random.Generator, k: int):
    """A random connected treewidth <= 2 graph on k nodes built by series and
    parallel extensions: repeatedly subdivide an edge or add a pendant or a
    new path between the two ends of an existing edge."""
    E = {(0, 1)}
    nxt = 2
    while nxt < k:
        op = int(rng.integers(0, 3))
        e = sorted(E)[int(rng.integers(0, len(E)))]
        if op == 0:                    # pendant
            a = int(rng.integers(0, nxt))
            E.add((a, nxt))
        elif op == 1:                  # subdivide e
            E.discard(e)
            E.add((e[0], nxt))
            E.add((e[1], nxt))
        else:                          # parallel path of length 2 beside e
            E.add((e[0], nxt))
            E.add((e[1], nxt))
        nxt += 1
    return k, sorted(tuple(sorted(x)) for x in E)
