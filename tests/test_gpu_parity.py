"""Device parity: the HIP path (through the C ABI) against the CPU oracle,
element by element on the same seeded inputs.  Integer counts: bit-exact."""
import numpy as np
import pytest

from cc_inputs import graphs, queries as Q
from oracle import oracle as O

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1602_04478_amd.cc")


def _colours(n, k, trials, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(0, k, size=(trials, n), dtype=np.uint8)


SHAPES = {
    "C3": Q.cycle(3), "C4": Q.cycle(4), "C5": Q.cycle(5), "C6": Q.cycle(6), "C7": Q.cycle(7),
    "C6+pendant": Q.cycle_pendant(6), "C4+pendant": Q.cycle_pendant(4),
    "domino+tail": Q.domino_tail(), "star5": Q.star(5), "path4": Q.path(4), "edge": Q.path(2),
    "chorded6": (6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (0, 3)]),
    "bowtie": (5, [(0, 1), (1, 2), (2, 0), (0, 3), (3, 4), (4, 0)]),
    "tri+tail": (5, [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4)]),
    "C5+chord-tree": (7, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (1, 5), (5, 6)]),
    "two4cycles-node": (7, [(0, 1), (1, 2), (2, 3), (3, 0), (0, 4), (4, 5), (5, 6), (6, 0)]),
}


@pytest.fixture(scope="module")
def small_graphs():
    return [graphs.erdos_renyi(60, 8.0, seed=21), graphs.chung_lu(400, 6.0, 2.2, None, seed=22),
            graphs.erdos_renyi(25, 12.0, seed=23)]


PATH_MODES = {
    "auto": {},
    "dense": {"CC_DENSE": "all"},
    "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"},
    "light": {"CC_DENSE": "none"},
    "light+fallback": {"CC_DENSE": "none", "CC_LIGHT_SCRATCH": "6000"},
    "light+densefallback": {"CC_LIGHT_SCRATCH": "6000", "CC_FALLBACK": "dense"},
    "light-large": {"CC_DENSE": "none", "CC_LIGHT_SCRATCH": "6000", "CC_LIGHT_LARGE": "1"},
    "fused-dense": {"CC_DENSE": "all", "CC_FUSE": "1"},
    "fused-sparse": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_FUSE": "1"},
    "nomap-dense": {"CC_DENSE": "all", "CC_EJMAP": "0", "CC_NJMAP": "0"},
    "nomap-sparse": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_EJMAP": "0", "CC_NJMAP": "0"},
    # hub schedule with tiny chunks: every vertex of degree > 4 runs as chunks of 2 neighbours
    "dense-split": {"CC_DENSE": "all", "CC_SPLIT_CHUNK": "2"},
    "dense-split3": {"CC_DENSE": "all", "CC_SPLIT_CHUNK": "3"},
    # root merges read their AXPY chain as stored rows (the chain not summed inside the merge)
    "nofuseroot-dense": {"CC_DENSE": "all", "CC_FUSE_ROOT": "0"},
    "nofuseroot-sparse": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_FUSE_ROOT": "0"},
    # merges into edge tables one thread per (entry, trial, slot) instead of vertex-major
    "medge-slots-dense": {"CC_DENSE": "all", "CC_MEDGE_V": "0"},
    "medge-slots-sparse": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_MEDGE_V": "0"},
}


@pytest.fixture(params=sorted(PATH_MODES))
def dense_mode(request, monkeypatch):
    """Which execution path the sources take: the library's choice, all in
    dense groups, all in sparse groups, one workgroup per source, or one
    workgroup per source with a scratch so small that many are handed back."""
    for k, v in PATH_MODES[request.param].items():
        monkeypatch.setenv(k, v)
    return request.param


# (mode, shape) pairs not run on the GPU, with the reason
SKIP = {
    ("light+densefallback", "two4cycles-node"):
        "a run of this case with an experimental AXPY-chain kernel (since removed) left the GPU faulted; "
        "the cause was not found by reading the code, so the case stays off the GPU",
}


@pytest.mark.parametrize("name", sorted(SHAPES))
def test_small_shapes_match_oracle(small_graphs, name, dense_mode):
    if (dense_mode, name) in SKIP:
        pytest.skip(SKIP[(dense_mode, name)])
    k, E = SHAPES[name]
    q = cc.Query(k, E)
    for gi, g in enumerate(small_graphs):
        print(f"[parity] {name} graph{gi} n={g.n} m={g.m} mode={dense_mode}", flush=True)
        dg = cc.Graph.from_csr(g)
        col = _colours(g.n, k, 3, seed=100 + gi)
        counts, ovf, exact = cc.count_colors(dg, q, col)
        for t in range(3):
            want = O.db(g, k, E, col[t])
            assert not ovf[t]
            assert exact[t] == want, (name, gi, t, exact[t], want)
            assert int(counts[t]) == want


ONE_TRIAL_MODES = {
    "dense": {"CC_DENSE": "all"},
    "dense-split": {"CC_DENSE": "all", "CC_SPLIT_CHUNK": "2"},
    "dense-split-unpacked": {"CC_DENSE": "all", "CC_SPLIT_CHUNK": "3", "CC_EJPACK": "0"},
    "dense-unpacked": {"CC_DENSE": "all", "CC_EJPACK": "0"},
    "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"},
    "sparse-unpacked": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_EJPACK": "0"},
    # every EdgeJoin launched on its own (no two sharing a neighbour scan)
    "dense-nodual": {"CC_DENSE": "all", "CC_EJDUAL": "0"},
    "sparse-nodual": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_EJDUAL": "0"},
    # the fused root merge with per-slot gathers instead of rows staged in LDS
    "dense-mroot-slots": {"CC_DENSE": "all", "CC_MROOT_ROWS": "0"},
    "sparse-mroot-slots": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_MROOT_ROWS": "0"},
    # the AXPY chains one slot per lane with gathers instead of rows staged in LDS
    "dense-axpy-slots": {"CC_DENSE": "all", "CC_AXPY_ROWS": "0"},
    "sparse-axpy-slots": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_AXPY_ROWS": "0"},
    # annotated EdgeJoins one source per lane (not a pair's slots over the lanes)
    "dense-ann-per-source": {"CC_DENSE": "all", "CC_EJANNLANES": "0"},
    "sparse-ann-per-source": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_EJANNLANES": "0"},
    # the fused EdgeJoin epilogues with one colouring (annotated joins: slots over the lanes, then the epilogue)
    "dense-fused": {"CC_DENSE": "all", "CC_FUSE": "1"},
    "sparse-fused": {"CC_DENSE": "none", "CC_LIGHT": "0", "CC_FUSE": "1"},
}


@pytest.mark.parametrize("mode", sorted(ONE_TRIAL_MODES))
@pytest.mark.parametrize("name", sorted(SHAPES))
def test_one_trial(small_graphs, name, mode, monkeypatch):
    """One colouring per solve: the EdgeJoin packs (neighbour, source) pairs
    over the lanes of a group (unpacked: one source per lane)."""
    for key, val in ONE_TRIAL_MODES[mode].items():
        monkeypatch.setenv(key, val)
    k, E = SHAPES[name]
    q = cc.Query(k, E)
    for gi, g in enumerate(small_graphs):
        print(f"[parity] {name} graph{gi} n={g.n} m={g.m} mode={mode} T=1", flush=True)
        dg = cc.Graph.from_csr(g)
        col = _colours(g.n, k, 2, seed=200 + gi)
        for t in range(2):
            counts, ovf, exact = cc.count_colors(dg, q, col[t:t + 1])
            want = O.db(g, k, E, col[t])
            assert not ovf[0]
            assert exact[0] == want and int(counts[0]) == want, (name, gi, t, exact[0], want)


def test_colour_contract_device_equals_oracle():
    g = graphs.erdos_renyi(500, 6.0, seed=5)
    dg = cc.Graph.from_csr(g)
    for k, seed, t in ((5, 101, 0), (7, 102, 3), (12, 2**64 - 5, 1)):
        assert np.array_equal(dg.colors(k, seed, t), O.colours(g.n, k, seed, t))


def test_config_tiny_er1000_c5():
    """G(n=1000, avg degree 10), 5-cycle, k = 5, colouring seed 101."""
    g = graphs.workload_graph("er1000")
    k, E = Q.cycle(5)
    dg = cc.Graph.from_csr(g)
    q = cc.Query(k, E)
    counts, ovf, exact, est = cc.count(dg, q, 101, 1)
    chi = O.colours(g.n, k, 101, 0)
    want = O.db(g, k, E, chi)
    assert want == O.brute(g, k, E, chi)
    assert exact[0] == want and int(counts[0]) == want and not ovf[0]


def test_reverse_ties_same_total():
    g = graphs.chung_lu(3000, 8.0, 2.1, None, seed=31)
    k, E = Q.cycle_pendant(6)
    q = cc.Query(k, E)
    a = cc.count(cc.Graph.from_csr(g), q, 7, 2)[2]
    b = cc.count(cc.Graph.from_csr(g, cc.CC_GRAPH_REVERSE_TIES), q, 7, 2)[2]
    assert a == b


# queries every decomposition tree of which has a block whose two boundary
# nodes are not adjacent (a table keyed by vertex pairs)
PAIR_SHAPES = {
    "K23": Q.k23(),
    "theta": (6, [(0, 1), (1, 2), (2, 3), (0, 4), (4, 3), (0, 5), (5, 3)]),
    "satellite": Q.satellite(),
    "K23+pendant": (6, Q.k23()[1] + [(2, 5)]),
}

PAIR_MODES = {"auto": {}, "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"}, "light": {"CC_DENSE": "none"}}


@pytest.mark.parametrize("mode", sorted(PAIR_MODES))
@pytest.mark.parametrize("name", sorted(PAIR_SHAPES))
def test_pair_keyed_tables(small_graphs, name, mode, monkeypatch):
    """Pair-keyed blocks (split at their two boundary nodes, the table laid
    out as a graph over the nonzero pairs) and their parents, against the
    oracle's binary tables."""
    for key, val in PAIR_MODES[mode].items():
        monkeypatch.setenv(key, val)
    k, E = PAIR_SHAPES[name]
    q = cc.Query(k, E)
    assert q.tree_info()["pair_keyed_blocks"] >= 1
    for gi, g in enumerate(small_graphs):
        print(f"[parity] pair-keyed {name} graph{gi} n={g.n} m={g.m} mode={mode}", flush=True)
        dg = cc.Graph.from_csr(g)
        col = _colours(g.n, k, 2, seed=300 + gi)
        counts, ovf, exact = cc.count_colors(dg, q, col)
        for t in range(2):
            want = O.db(g, k, E, col[t])
            assert not ovf[t] and exact[t] == want, (name, gi, t, exact[t], want)
        # one colouring per call as well
        c1, o1, e1 = cc.count_colors(dg, q, col[1:2])
        assert e1[0] == exact[1]


PS_MODES = {"auto": {}, "dense": {"CC_DENSE": "all"}, "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"},
            "light": {"CC_DENSE": "none"}, "light+fallback": {"CC_DENSE": "none", "CC_LIGHT_SCRATCH": "6000"}}


@pytest.mark.parametrize("mode", sorted(PS_MODES))
@pytest.mark.parametrize("name", sorted(set(SHAPES) | set(PAIR_SHAPES)))
def test_path_splitting_plans(small_graphs, name, mode, monkeypatch):
    """The path-splitting baseline (every cycle split at its boundary nodes,
    no degree-order filter, one split per cycle) gives the same counts."""
    for key, val in PS_MODES[mode].items():
        monkeypatch.setenv(key, val)
    k, E = SHAPES.get(name) or PAIR_SHAPES[name]
    q = cc.Query(k, E, path_splitting=True)
    for gi, g in enumerate(small_graphs):
        print(f"[parity] path splitting {name} graph{gi} n={g.n} mode={mode}", flush=True)
        dg = cc.Graph.from_csr(g)
        col = _colours(g.n, k, 2, seed=400 + gi)
        counts, ovf, exact = cc.count_colors(dg, q, col)
        for t in range(2):
            want = O.db(g, k, E, col[t])
            assert not ovf[t] and exact[t] == want, (name, gi, t, exact[t], want)


@pytest.mark.parametrize("qseed,count,kmax", [(505, 16, 9), (204, 20, 10)])
def test_maps_equal_subset_walk(qseed, count, kmax, monkeypatch):
    """The EdgeJoin slot maps and NodeJoin split maps (tables built on the host
    once per k) give the counts of the slot arithmetic they replace, on a
    3000-vertex power-law graph for generated queries of 4-10 nodes, with two
    colourings per call and with one."""
    g = graphs.chung_lu(3000, 16.0, 2.3, None, seed=7)
    dg = cc.Graph.from_csr(g)
    for i, (k, E, fam) in enumerate(Q.random_queries(qseed, count, 4, kmax)):
        q = cc.Query(k, E)
        print(f"[parity] maps vs walk: query {i} ({fam}, k={k})", flush=True)
        with_maps = cc.count(dg, q, 900 + i, 2)[2]
        one = [cc.count(dg, q, 900 + i + t, 1)[2][0] for t in range(2)]
        monkeypatch.setenv("CC_NJMAP", "0")
        monkeypatch.setenv("CC_EJMAP", "0")
        walk = cc.count(dg, q, 900 + i, 2)[2]
        monkeypatch.delenv("CC_NJMAP")
        monkeypatch.delenv("CC_EJMAP")
        assert with_maps == walk == one, (qseed, i, k, fam, with_maps, walk, one)


def test_profiling_leaves_counts_and_reports_bytes():
    """Event timing (levels 1 and 3) and the kernels' byte counters (level 2)
    change no count, and every operation but the merges into non-root tables
    reports algorithmic bytes, the one-workgroup tier included."""
    g = graphs.chung_lu(3000, 16.0, 2.3, None, seed=7)
    dg = cc.Graph.from_csr(g)
    q = cc.Query(*Q.cycle_pendant(6))
    base = cc.count(dg, q, 77, 2)[2]
    cc.profile_take()
    for level in (1, 2, 3):
        cc.profile_enable(level)
        got = cc.count(dg, q, 77, 2)[2]
        cc.profile_enable(0)
        stats = cc.profile_take()
        assert got == base, (level, got, base)
        assert stats, level
        if level == 2:
            assert any(name.startswith("light") for name in stats), sorted(stats)
            for name, (launches, secs, byts, work) in stats.items():
                if not name.startswith(("merge_u", "merge_v", "merge_edge", "merge_pair")):
                    assert byts > 0, (name, launches, byts)
        if level == 3:
            assert all(name.startswith("edgejoin") for name in stats), sorted(stats)


def test_every_tree_same_count(small_graphs):
    """Every decomposition tree of a query gives the same count (the choice
    of tree is a cost knob only)."""
    for name, (k, E) in (("domino+tail", Q.domino_tail()), ("C8+chord", (8, Q.cycle(8)[1] + [(0, 4)])),
                         ("satellite", Q.satellite())):
        nt = cc.Query(k, E).tree_info()["num_trees"]
        g = small_graphs[1]
        dg = cc.Graph.from_csr(g)
        col = _colours(g.n, k, 1, seed=500)
        want = O.db(g, k, E, col[0])
        for t in range(min(nt, 12)):
            print(f"[parity] {name} tree {t} of {nt}", flush=True)
            assert cc.count_colors(dg, cc.Query(k, E, tree=t), col)[2][0] == want, (name, t)


def _degenerate_graphs():
    def kbip(a, b):
        return graphs.from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])
    return {
        "edgeless": graphs.from_edges(40, np.zeros((0, 2), dtype=np.int64)),
        "fewer-vertices-than-k": graphs.from_edges(3, [(0, 1), (1, 2), (2, 0)]),
        "bipartite-K66": kbip(6, 6),
        "path30": graphs.from_edges(30, [(i, i + 1) for i in range(29)]),
        "star20": graphs.from_edges(21, [(0, i) for i in range(1, 21)]),
        "clique-and-isolated": graphs.from_edges(20, [(i, j) for i in range(6) for j in range(i + 1, 6)]
                                                 + [(10, 11), (11, 12)]),
        "one-edge": graphs.from_edges(2, [(0, 1)]),
    }


DEGENERATE_SHAPES = ["C3", "C4", "C5", "star5", "path4", "edge", "C6+pendant", "bowtie"]


@pytest.mark.parametrize("mode", ["auto", "dense", "sparse"])
def test_degenerate_graphs(mode, monkeypatch):
    """Graphs with no edges, fewer vertices than query nodes, no odd cycles
    (bipartite), trees, a star, isolated vertices beside a clique and a
    single edge: counts equal the oracle's, zero wherever no match exists
    (an odd cycle in a bipartite graph, any cycle in a tree, anything in an
    edgeless graph), on every execution path and with device colours."""
    env = {"auto": {}, "dense": {"CC_DENSE": "all"}, "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"}}[mode]
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    for gname, g in _degenerate_graphs().items():
        dg = cc.Graph.from_csr(g)
        for name in DEGENERATE_SHAPES:
            k, E = SHAPES[name]
            q = cc.Query(k, E)
            print(f"[parity] degenerate {gname} n={g.n} m={g.m} {name} mode={mode}", flush=True)
            chi = O.colours(g.n, k, 77, 0)
            want = O.db(g, k, E, chi)
            if g.m == 0 or g.n < k or (gname in ("bipartite-K66",) and name in ("C3", "C5", "bowtie")) \
                    or (gname in ("path30", "star20") and name in ("C3", "C4", "C5", "bowtie", "C6+pendant")):
                assert want == 0
            counts, ovf, exact = cc.count_colors(dg, q, chi[None, :])
            assert exact[0] == want and int(counts[0]) == want and not ovf[0], (gname, name, exact[0], want)
            c2, o2, e2, est = cc.count(dg, q, 77, 1)
            assert int(e2[0]) == want, (gname, name, int(e2[0]), want)


LARGEST_QUERIES = {
    "C12": Q.cycle(12),
    "C11+pendant": Q.cycle_pendant(11),
    "C12+chord": (12, [(i, (i + 1) % 12) for i in range(12)] + [(0, 6)]),
    "C6+tree": (12, [(i, (i + 1) % 6) for i in range(6)] + [(5, 6), (6, 7), (7, 8), (6, 9), (9, 10), (10, 11)]),
}


@pytest.mark.parametrize("mode", ["auto", "dense", "sparse"])
def test_largest_queries(mode, monkeypatch):
    """Queries of 12 nodes, the largest the planner takes (rows of up to
    C(10, 5) = 252 slots: the entry-major EdgeJoin and no slot maps), on an
    80-vertex random graph: two colourings per call and one, against the
    oracle."""
    env = {"auto": {}, "dense": {"CC_DENSE": "all"}, "sparse": {"CC_DENSE": "none", "CC_LIGHT": "0"}}[mode]
    for key, val in env.items():
        monkeypatch.setenv(key, val)
    g = graphs.erdos_renyi(80, 6.0, seed=12)
    dg = cc.Graph.from_csr(g)
    for name, (k, E) in LARGEST_QUERIES.items():
        q = cc.Query(k, E)
        chi = np.stack([O.colours(g.n, k, 91, t) for t in range(2)])
        want = [O.db(g, k, E, chi[t]) for t in range(2)]
        print(f"[parity] largest {name} k={k} mode={mode}", flush=True)
        counts, ovf, exact = cc.count_colors(dg, q, chi)
        assert [int(x) for x in exact] == want and not ovf.any(), (name, mode, exact, want)
        one = cc.count_colors(dg, q, chi[1:2])[2]
        assert int(one[0]) == want[1], (name, mode, int(one[0]), want[1])
