"""Serving: requests admitted by device footprint onto resident graphs and run
side by side (continuous batching).  Each result must be the same alone and
in the mix -- counts, overflow flags and the estimate, bit for bit -- and the
loop must report a latency for every request."""
import time

import numpy as np
import pytest

from cc_inputs import graphs, queries as Q
from oracle import oracle as O

pytestmark = pytest.mark.gpu

cc = pytest.importorskip("paper_1602_04478_amd.cc")

QUERIES = [Q.cycle(4), Q.cycle(5), Q.cycle_pendant(6), Q.domino_tail(),
           (6, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 5), (5, 0), (0, 3)]), Q.star(4), Q.path(3)]


@pytest.fixture(scope="module")
def pool():
    gs = [graphs.chung_lu(2000, 8.0, 2.2, None, seed=51), graphs.chung_lu(6000, 10.0, 2.4, None, seed=52),
          graphs.erdos_renyi(800, 10.0, seed=53)]
    return gs, [cc.Graph.from_csr(g) for g in gs], [cc.Query(k, E) for k, E in QUERIES]


def _requests(n, seed):
    rng = np.random.default_rng(seed)
    return [(int(rng.integers(0, 3)), int(rng.integers(0, len(QUERIES))), int(rng.integers(0, 2**40)),
             int(rng.integers(1, 5))) for _ in range(n)]


def _serve(srv, ids, qs, reqs, waves=3):
    """Submit in waves while earlier requests are still running; poll all."""
    tickets = {}
    per = (len(reqs) + waves - 1) // waves
    for w in range(waves):
        for i in range(w * per, min(len(reqs), (w + 1) * per)):
            gi, qi, sd, tr = reqs[i]
            tickets[i] = srv.submit(ids[gi], qs[qi], sd, tr)
        time.sleep(0.01)
    out = {}
    t_end = time.time() + 240
    while len(out) < len(reqs):
        assert time.time() < t_end, "server did not finish"
        for i, tk in tickets.items():
            if i in out:
                continue
            r = srv.poll(tk, reqs[i][3])
            if r is not None:
                out[i] = r
        time.sleep(0.002)
    return out


def test_alone_equals_mix(pool):
    gs, dgs, qs = pool
    reqs = _requests(24, seed=7)
    srv = cc.Server(0, max_inflight=4)
    try:
        ids = [srv.add_graph(dg) for dg in dgs]
        mix = _serve(srv, ids, qs, reqs)
    finally:
        srv.close()
    lat = []
    for i, (gi, qi, sd, tr) in enumerate(reqs):
        print(f"[server] request {i}: graph {gi} query {qi} seed {sd} trials {tr}", flush=True)
        counts, ovf, exact, est = cc.count(dgs[gi], qs[qi], sd, tr)
        mc, mo, mest, mlat = mix[i]
        assert np.array_equal(mc, counts) and np.array_equal(mo, ovf), i
        assert (np.isnan(mest) and np.isnan(est)) or mest == est, i
        lat.append(mlat)
    # and the counts themselves are the oracle's (first trial of a few requests)
    for i in range(0, len(reqs), 6):
        gi, qi, sd, tr = reqs[i]
        k, E = QUERIES[qi]
        assert int(mix[i][0][0]) == O.db(gs[gi], k, E, O.colours(gs[gi].n, k, sd, 0)), i
    lat = np.array(lat)
    assert np.all(lat > 0) and np.all(np.isfinite(lat))
    p50, p99 = np.percentile(lat, 50), np.percentile(lat, 99)
    print(f"[server] latency p50 {p50 * 1e3:.1f} ms p99 {p99 * 1e3:.1f} ms", flush=True)
    assert p50 <= p99


def test_budget_admits_one_at_a_time(pool):
    """A budget that holds only the largest request: requests wait for memory,
    and every result is still the one computed alone."""
    gs, dgs, qs = pool
    reqs = _requests(8, seed=8)
    big = max(cc.footprint(dgs[gi], qs[qi], tr) for gi, qi, sd, tr in reqs)
    srv = cc.Server(big, max_inflight=4)
    try:
        ids = [srv.add_graph(dg) for dg in dgs]
        mix = _serve(srv, ids, qs, reqs, waves=1)
    finally:
        srv.close()
    for i, (gi, qi, sd, tr) in enumerate(reqs):
        counts, ovf, exact, est = cc.count(dgs[gi], qs[qi], sd, tr)
        assert np.array_equal(mix[i][0], counts) and np.array_equal(mix[i][1], ovf), i
