"""The seeded input generators (no GPU): the power-law weights hit their stated
maximum and mean, the Chung-Lu sampler realises the independent-edge model
(edge count and hub degree against their exact expectations), graphs are
simple and symmetric and fixed by their seed, and the generated queries have
the stated sizes and are connected."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from cc_inputs import graphs, queries as Q  # noqa: E402


def _edges(g):
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    return src, np.asarray(g.col, dtype=np.int64)


def _simple_symmetric(g):
    u, v = _edges(g)
    assert np.all(u != v)
    fwd = set(zip(u.tolist(), v.tolist()))
    assert len(fwd) == u.size  # no duplicates
    assert all((b, a) in fwd for a, b in fwd)


@pytest.mark.parametrize("n,mean,gamma,wmax", [(10_000, 16.0, 2.1, 1e3), (5000, 20.0, 2.2, None)])
def test_power_law_weights(n, mean, gamma, wmax):
    wmax = graphs.structural_cutoff(n, mean) if wmax is None else wmax
    w = graphs.power_law_weights(n, mean, gamma, wmax)
    assert w[0] == pytest.approx(wmax, rel=1e-9)
    assert float(np.mean(w)) == pytest.approx(mean, rel=1e-6)
    assert np.all(np.diff(w) <= 0)


def test_chung_lu_sampler_realises_the_edge_model():
    n, mean, gamma = 2000, 10.0, 2.1
    w = graphs.power_law_weights(n, mean, gamma, graphs.structural_cutoff(n, mean))
    S = float(w.sum())
    p = np.minimum(np.outer(w, w) / S, 1.0)
    np.fill_diagonal(p, 0.0)
    iu = np.triu_indices(n, 1)
    e_m, var_m = float(p[iu].sum()), float((p[iu] * (1 - p[iu])).sum())
    e_d0, var_d0 = float(p[0].sum()), float((p[0] * (1 - p[0])).sum())
    ms, d0s = [], []
    for seed in range(6):
        g = graphs.chung_lu_from_weights(w, seed)
        _simple_symmetric(g)
        ms.append(g.m)
        d0s.append(int(g.row_ptr[1] - g.row_ptr[0]))  # vertex 0 carries the largest weight
    # means of 6 independent draws within 5 standard errors of the exact expectations
    assert abs(np.mean(ms) - e_m) < 5 * np.sqrt(var_m / 6)
    assert abs(np.mean(d0s) - e_d0) < 5 * np.sqrt(var_d0 / 6)


def test_graphs_fixed_by_seed():
    a = graphs.chung_lu(3000, 8.0, 2.3, None, seed=11)
    b = graphs.chung_lu(3000, 8.0, 2.3, None, seed=11)
    c = graphs.chung_lu(3000, 8.0, 2.3, None, seed=12)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert not (np.array_equal(a.row_ptr, c.row_ptr) and np.array_equal(a.col, c.col))
    _simple_symmetric(a)


def test_erdos_renyi_mean_degree():
    g = graphs.workload_graph("er1000")
    _simple_symmetric(g)
    assert g.n == 1000
    assert 2 * g.m / g.n == pytest.approx(10.0, rel=0.05)


def _connected(k, E):
    adj = {i: set() for i in range(k)}
    for a, b in E:
        adj[a].add(b)
        adj[b].add(a)
    seen, stack = {0}, [0]
    while stack:
        for y in adj[stack.pop()]:
            if y not in seen:
                seen.add(y)
                stack.append(y)
    return len(seen) == k


def test_generated_queries():
    qs = Q.random_queries(204, 20, 4, 10)
    assert len(qs) == 20
    fams = set()
    for k, E, fam in qs:
        assert 4 <= k <= 10
        assert _connected(k, E)
        assert all(0 <= a < k and 0 <= b < k and a != b for a, b in E)
        assert len({tuple(sorted(e)) for e in map(tuple, E)}) == len(E)  # simple
        # treewidth <= 2 queries have at most 2k - 3 edges
        assert len(E) <= 2 * k - 3
        fams.add(fam)
    assert len(fams) >= 3
    # the same seed gives the same queries
    assert [(k, [tuple(map(int, e)) for e in E]) for k, E, _ in Q.random_queries(204, 20, 4, 10)] == \
           [(k, [tuple(map(int, e)) for e in E]) for k, E, _ in qs]
