"""Parity at the benchmark's sizes and on the shapes of the larger
configurations.

Full size (Chung-Lu n = 1e6, 6-cycle + pendant, k = 7): the device's
per-source shares (matches by their highest vertex) against the oracle's for
hubs of the first dense group, low-degree sources and mid-degree sources; the
shares sum to the device's total.  Scaled configurations (the same
generators, smaller n): the C2 shape at n = 30000, whose automatic tier
choice runs dense groups, the one-workgroup tier and its hand-backs in one
solve; domino + tail with all 64 colourings; the 20 generated queries with
all 16 colourings each.  Expected values that take the oracle minutes come
from tests/golden/scale_counts.json, written by
tests/golden/make_scale_golden.py (oracle only).  Overflow: a sum that leaves
64 bits is reported exactly in 128 bits and flagged; a table entry that
leaves 64 bits is flagged, also when the count itself is small."""
import json
import os

import numpy as np
import pytest

from cc_inputs import graphs, queries as Q
from oracle import oracle as O

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1602_04478_amd.cc")


@pytest.fixture(scope="module")
def cl1m():
    return graphs.workload_graph("cl1m")


def _gold(name):
    data = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "scale_counts.json")))
    return data[name]


def test_full_size_sampled_sources(cl1m):
    """Per-source shares at n = 1e6 against the oracle's: hubs of the first
    dense group (ranks 40-63 from the top of the degree order) and sixteen
    low-degree sources, from stored oracle values (the hubs take the oracle
    minutes each), plus mid-degree sources computed here."""
    g = cl1m
    k, E = Q.cycle_pendant(6)
    chi = O.colours(g.n, k, 102, 0)
    dg = cc.Graph.from_csr(g)
    q = cc.Query(k, E)
    print("[scale] cl1m C6+pendant per-source run", flush=True)
    counts, ovf, exact, per = cc.count_colors(dg, q, chi, per_source=True)
    st = cc.last_solve_stats()
    assert not ovf[0]
    per = per[0]
    assert sum(per) == exact[0]
    # the first dense group holds the 64 highest sources
    assert st["dense_sources"] >= 64 and st["group_sources"] == 64, st
    # the same total from the seeded path
    assert cc.count(dg, q, 102, 1)[2][0] == exact[0]
    gold = _gold("c2_sources")
    assert gold["seed"] == 102 and gold["trial"] == 0
    deg = g.degrees()
    order = np.lexsort((np.arange(g.n), deg))[::-1]  # highest (degree, id) first
    for r, s, v in zip(gold["ranks"], gold["sources"], gold["shares"]):
        assert int(order[r]) == s
        assert per[s] == int(v), (r, s, int(deg[s]))
    assert sum(1 for v in gold["shares"] if int(v) > 0) >= 20
    # sources of degree ~500, ~270 and ~170
    sample = list(order[3000:3008]) + list(order[6000:6008]) + list(order[10000:10004])
    print(f"[scale] oracle on {len(sample)} sources", flush=True)
    tot, vals = O.db(g, k, E, chi, reverse_ties=False, sources=sample)
    for s, v in zip(sample, vals):
        assert per[int(s)] == v, (int(s), int(deg[s]))
    assert any(v > 0 for v in vals)


def test_c2_shape_whole_solve_all_tiers():
    """The C2 shape (Chung-Lu, exponent 2.1, 6-cycle + pendant, k = 7)
    scaled to n = 30000: whole counts against the oracle's, with the
    library's own tier choice running dense groups, the one-workgroup tier
    and hand-backs from it in one solve."""
    import importlib.util
    spec = importlib.util.spec_from_file_location(
        "make_scale_golden", os.path.join(os.path.dirname(__file__), "golden", "make_scale_golden.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    g = mk.c2_scaled_graph()
    gold = _gold("c2_scaled")
    k, E = Q.cycle_pendant(6)
    dg = cc.Graph.from_csr(g)
    q = cc.Query(k, E)
    want = [int(x) for x in gold["counts"]]
    print(f"[scale] c2 shape n={g.n} m={g.m}: two colourings in one call", flush=True)
    counts, ovf, exact, _ = cc.count(dg, q, gold["seed"], len(want))
    assert [int(x) for x in exact] == want and not ovf.any()
    for t, w in enumerate(want):
        print(f"[scale] c2 shape: colouring {t} alone", flush=True)
        c1, o1, e1, _ = cc.count(dg, q, gold["seed"] + t, 1)
        assert e1[0] == w and not o1[0]
        st = cc.last_solve_stats()
        assert st["dense_sources"] > 0 and st["light_sources"] > 0 and st["handed_back"] > 0, st


def test_domino_tail_64_trials():
    """The C3 shape (domino + tail, k = 8, 64 colourings) at n = 5000: every
    colouring of the batched call and of the plain call against the oracle."""
    g = graphs.chung_lu(5000, 20.0, 2.2, None, seed=3)
    k, E = Q.domino_tail()
    dg = cc.Graph.from_csr(g)
    q = cc.Query(k, E)
    gold = _gold("c3_scaled")
    want = [int(x) for x in gold["counts"]]
    print("[scale] chung-lu 5000 domino+tail 64 colourings, batched", flush=True)
    counts, ovf, est = cc.count_batch(dg, [q], [gold["seed"]], [64])
    assert [int(c) for c in counts] == want and not ovf.any()
    plain = cc.count(dg, q, gold["seed"], 64)[0]
    assert np.array_equal(plain, counts)


def test_generated_queries():
    """The C4 shape (20 generated treewidth-2 queries of 4-10 nodes, 16
    colourings each, one batched call) at n = 1000: every colouring of every
    query against the oracle."""
    g = graphs.chung_lu(1000, 8.0, 2.1, None, seed=4)
    dg = cc.Graph.from_csr(g)
    gold = _gold("c4_scaled")["queries"]
    qs = Q.random_queries(204, 20, 4, 10)
    objs = []
    for (k, E, fam), gq in zip(qs, gold):
        assert gq["k"] == k and [tuple(e) for e in gq["edges"]] == [tuple(map(int, e)) for e in E]
        objs.append(cc.Query(k, E))
    print(f"[scale] {len(objs)} generated queries, 16 colourings each, batched", flush=True)
    counts, ovf, est = cc.count_batch(dg, objs, [gq["seed"] for gq in gold], [16] * len(objs))
    for i, gq in enumerate(gold):
        for t in range(16):
            want = int(gq["counts"][t])
            if want >= 2**64:
                assert ovf[16 * i + t], (i, t)
            else:
                assert int(counts[16 * i + t]) == want and not ovf[16 * i + t], (i, gq["family"], t)


@pytest.mark.parametrize("mode", ["dense", "sparse", "dense-ann-per-source"])
def test_generated_queries_one_trial(mode, monkeypatch):
    """The generated queries of 9-10 nodes of the C4 shape at n = 1000, one
    colouring per call (rows up to 70 slots: annotated EdgeJoins whose rows
    are wider than a lane group spread a pair's slots over several steps)."""
    env = {"dense": {"CC_DENSE": "all"}, "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"},
           "dense-ann-per-source": {"CC_DENSE": "all", "CC_EJANNLANES": "0"}}[mode]
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    g = graphs.chung_lu(1000, 8.0, 2.1, None, seed=4)
    dg = cc.Graph.from_csr(g)
    gold = _gold("c4_scaled")["queries"]
    qs = Q.random_queries(204, 20, 4, 10)
    for i, ((k, E, fam), gq) in enumerate(zip(qs, gold)):
        if k < 9:
            continue
        q = cc.Query(k, E)
        print(f"[scale] generated query {i} ({fam}, k={k}), one colouring, mode {mode}", flush=True)
        for t in range(2):
            counts, ovf, exact, est = cc.count(dg, q, gq["seed"] + t, 1)
            want = int(gq["counts"][t])
            assert int(exact[0]) == want, (i, fam, t, int(exact[0]), want)


def _star_forest(hubs, leaves):
    e = []
    n = hubs * (leaves + 1)
    for h in range(hubs):
        c = h * (leaves + 1)
        e += [(c, c + 1 + j) for j in range(leaves)]
    return graphs.from_edges(n, np.array(e, dtype=np.int64))


K8_CYCLE_CHILD = (8, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 5), (5, 6), (6, 7), (7, 0)])


@pytest.mark.parametrize("mode", ["auto", "dense", "sparse"])
def test_k8_cycle_child_every_tree(mode, monkeypatch):
    """A 5-cycle and a 4-cycle sharing a node (k = 8) on a 12500-vertex
    Chung-Lu graph: every tree, two colourings per call and one, repeated
    (equal every time).  NodeJoin terms read split maps whose 16-bit index
    part ends mid-word when (k - 1) * C * ns is odd; a map cut to whole words
    without that last entry gave counts that changed from run to run."""
    env = {"auto": {}, "dense": {"CC_DENSE": "all"}, "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"}}[mode]
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    gold = _gold("k8_cycle_child")
    want = [int(x) for x in gold["counts"]]
    g = graphs.chung_lu(12500, 16.0, 2.4025014618726903, None, seed=50)
    dg = cc.Graph.from_csr(g)
    k, E = K8_CYCLE_CHILD
    for tree in range(cc.Query(k, E).tree_info()["num_trees"]):
        q = cc.Query(k, E, tree=tree)
        print(f"[scale] k8 cycle child, tree {tree}, mode {mode}", flush=True)
        for _ in range(2):
            counts, ovf, exact, est = cc.count(dg, q, gold["seed"], 2)
            assert [int(x) for x in exact] == want and not ovf.any(), (tree, mode, exact, want)
        for t in range(2):
            assert int(cc.count(dg, q, gold["seed"] + t, 1)[2][0]) == want[t], (tree, mode, t)


def test_sum_overflow_reported_exactly():
    """2000 hubs of 500 leaves, 8-node star: every hub's count fits in 64
    bits, their sum does not."""
    g = _star_forest(2000, 500)
    k, E = Q.star(8)
    chi = O.colours(g.n, k, 5, 0)
    want = O.db(g, k, E, chi)
    assert want >= 2**64
    counts, ovf, exact = cc.count_colors(cc.Graph.from_csr(g), cc.Query(k, E), chi)
    assert ovf[0] and int(counts[0]) == 2**64 - 1
    assert exact[0] == want


def test_intermediate_overflow_flagged():
    """One hub of 2000 leaves, 10-node star: the hub's own count leaves 64 bits."""
    g = _star_forest(1, 2000)
    k, E = Q.star(10)
    chi = O.colours(g.n, k, 6, 0)
    want = O.db(g, k, E, chi)
    assert want >= 2**64
    counts, ovf, exact = cc.count_colors(cc.Graph.from_csr(g), cc.Query(k, E), chi)
    assert ovf[0] and int(counts[0]) == 2**64 - 1


@pytest.mark.parametrize("leaves", [500, 2000])
def test_table_overflow_with_small_count(leaves):
    """A star table entry that leaves 64 bits while the count itself is
    small (2 * 11!): flagged, never wrapped; and with fewer leaves (every
    entry below 2^64) the exact count.  Expected values from the oracle with
    its 64-bit table width check."""
    g, chi = graphs.hub_and_clique(leaves)
    k, E = Q.star_triangle(8)
    want, wide = O.db_flagged(g, k, E, chi)
    assert want < 2**64
    counts, ovf, exact = cc.count_colors(cc.Graph.from_csr(g), cc.Query(k, E), chi)
    if wide:
        assert ovf[0] and int(counts[0]) == 2**64 - 1 and exact[0] == 2**128 - 1
    else:
        assert not ovf[0] and exact[0] == want and int(counts[0]) == want
