"""Batched form (a trial-group launch sequence captured once in a hipGraph and
replayed): every replayed trial group must give exactly the counts of the
plain per-call path and of the oracle, on every execution path."""
import numpy as np
import pytest

from cc_inputs import graphs, queries as Q
from oracle import oracle as O

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1602_04478_amd.cc")

MODES = {
    "auto": {},
    "dense": {"CC_DENSE": "all"},
    "sparse-fallback": {"CC_DENSE": "none", "CC_LIGHT_SCRATCH": "6000"},
}


@pytest.fixture(params=sorted(MODES))
def mode(request, monkeypatch):
    for k, v in MODES[request.param].items():
        monkeypatch.setenv(k, v)
    return request.param


@pytest.fixture(scope="module")
def g_small():
    return graphs.chung_lu(1500, 8.0, 2.1, None, seed=41)


def _plain(dg, q, seed, trials):
    return cc.count(dg, q, seed, trials)[0]


@pytest.mark.parametrize("tg", [1, 2, 3])
def test_replays_equal_plain_and_oracle(g_small, mode, tg):
    """7 trials in groups of tg (ragged tail): the first group runs eagerly,
    the rest replay one captured graph; each replay is checked."""
    dg = cc.Graph.from_csr(g_small)
    k, E = Q.cycle_pendant(5)
    q = cc.Query(k, E)
    seed, trials = 1234, 7
    print(f"[batch] mode={mode} trial_group={tg}", flush=True)
    counts, ovf, est = cc.count_batch(dg, [q], [seed], [trials], tuning={"group_sources": 0, "trial_group": tg,
                                                                          "light_max_keys": 0, "use_graphs": 1})
    rep = cc.last_tune_report()
    assert rep["trial_group"] == tg
    groups = (trials + tg - 1) // tg
    # the first group runs eagerly when the one-workgroup tier has sources to probe
    assert groups - 1 <= rep["graph_replays"] <= groups
    want = [O.db(g_small, k, E, O.colours(g_small.n, k, seed, t)) for t in range(trials)]
    assert [int(c) for c in counts] == want
    assert not ovf.any()
    # the plain path, called between the replays' uses of the same device
    assert [int(c) for c in _plain(dg, q, seed, trials)] == want


def test_replays_interleaved_with_eager_work(g_small):
    """Several batched calls with eager solves and synchronisations between
    them: every replay must match the eager result."""
    dg = cc.Graph.from_csr(g_small)
    k, E = Q.cycle(6)
    q = cc.Query(k, E)
    tun = {"group_sources": 0, "trial_group": 1, "light_max_keys": 0, "use_graphs": 1}
    eager = [int(c) for c in _plain(dg, q, 99, 5)]
    for rep in range(3):
        counts, ovf, _ = cc.count_batch(dg, [q], [99], [5], tuning=tun)
        assert [int(c) for c in counts] == eager, rep
        assert cc.last_tune_report()["graph_replays"] >= 4
        assert [int(c) for c in _plain(dg, q, 99, 2)] == eager[:2]


def test_autotuned_batch_of_uneven_queries(g_small):
    """Several queries of different sizes in one call, trial-group size tuned
    online per query: counts equal the oracle's for every trial."""
    dg = cc.Graph.from_csr(g_small)
    qs = [Q.cycle(4), Q.cycle_pendant(6), Q.domino_tail(), (6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (0, 3)])]
    trials = [9, 6, 4, 5]
    seeds = [11, 12, 13, 14]
    counts, ovf, est = cc.count_batch(dg, [cc.Query(k, E) for k, E in qs], seeds, trials)
    off = 0
    for (k, E), T, sd in zip(qs, trials, seeds):
        for t in range(T):
            want = O.db(g_small, k, E, O.colours(g_small.n, k, sd, t))
            assert int(counts[off + t]) == want, (k, E, t)
        off += T
    assert not ovf.any()
    assert np.all(np.isfinite(est))


def test_estimate_matches_formula(g_small):
    dg = cc.Graph.from_csr(g_small)
    k, E = Q.cycle(5)
    q = cc.Query(k, E)
    counts, ovf, est = cc.count_batch(dg, [q], [5], [8])
    aut = q.info()["aut"]
    import math
    want = sum(int(c) for c in counts) * k ** k / (8 * math.factorial(k) * aut)
    assert est[0] == pytest.approx(want, rel=1e-12)


def test_batched_tunes_the_tree():
    """With 32 or more colourings and several decomposition trees, the
    batched call times up to four trees on colourings of the call and keeps
    the fastest; the counts equal the plain per-colouring counts."""
    from cc_inputs import queries as Q
    from oracle import oracle as O
    g = graphs.chung_lu(2000, 8.0, 2.1, None, seed=61)
    dg = cc.Graph.from_csr(g)
    k, E = Q.domino_tail()
    q = cc.Query(k, E)
    assert q.tree_info()["num_trees"] >= 2
    counts, ovf, est = cc.count_batch(dg, [q], [71], [32])
    rep = cc.last_tune_report()
    assert len(rep["trees"]) >= 2 and rep["tree"] in [t for t, _ in rep["trees"]]
    plain = cc.count(dg, q, 71, 32)[0]
    assert np.array_equal(plain, counts) and not ovf.any()
    for t in (0, 31):
        assert int(counts[t]) == O.db(g, k, E, O.colours(g.n, k, 71, t))
