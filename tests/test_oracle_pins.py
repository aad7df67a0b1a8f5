"""Pins for the CPU oracle: each checks it against something other than
itself -- the problem definition by enumeration, an independent algebraic
route (inclusion-exclusion over homomorphisms), closed forms, the paper's
worked decomposition, and invariants the method must respect."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from cc_inputs import graphs, queries as Q
from oracle import oracle as O

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_published_value():
    gold = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    assert O.mix64(gold["input"]) == int(gold["output_hex"], 16)
    assert O.lib().orc_mix64(gold["input"]) == int(gold["output_hex"], 16)


def test_colour_contract_c_equals_python():
    for k in (2, 5, 7, 12):
        for seed, t in ((0, 0), (101, 0), (103, 5), (2**63 + 17, 3)):
            assert np.array_equal(O.colours(300, k, seed, t), O.colours_py(300, k, seed, t))


def test_colour_is_the_hash_scaled_to_k():
    """The colour is the hash read as a fraction of 2^64 and scaled to [0, k)
    (its top 32 bits, so the floor may sit below by one when k*h lands within
    k*2^32 above a multiple of 2^64): colours rise with the hash and each takes
    one contiguous k-th of the hash range. A residue (h mod k) or a shift by the
    wrong amount fails this on the first few vertices."""
    n = 2000
    for k, seed, t in ((2, 0, 0), (7, 102, 0), (12, 5, 3), (16, 2**63 + 17, 1)):
        key = O.mix64((seed + t) & O.MASK64)
        h = [O.mix64(key ^ v) for v in range(n)]
        c = O.colours(n, k, seed, t)
        for hv, cv in zip(h, c.tolist()):
            assert cv * 2**64 <= k * hv < (cv + 1) * 2**64 + k * 2**32
        order = np.argsort(np.array(h, dtype=np.uint64), kind="stable")
        assert np.all(np.diff(c[order].astype(int)) >= 0)


def test_colours_uniform_chi_square():
    k, n = 7, 200_000
    c = O.colours(n, k, 102)
    cnt = np.bincount(c, minlength=k)
    exp = n / k
    chi2 = float(((cnt - exp) ** 2 / exp).sum())
    assert chi2 < 30.0  # 6 degrees of freedom; p ~ 4e-5


def _rand_cases(seed, count, nmin, nmax, dmin, dmax, shapes):
    rng = np.random.default_rng(seed)
    for t in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        g = graphs.erdos_renyi(n, float(rng.uniform(dmin, dmax)), seed=int(rng.integers(1 << 30)))
        sh = shapes[t % len(shapes)]
        k, E = sh(rng) if callable(sh) else sh
        chi = O.colours(n, k, seed=int(rng.integers(1 << 40)))
        yield g, k, E, chi


SMALL_SHAPES = [Q.cycle(3), Q.cycle(4), Q.cycle(5), Q.cycle_pendant(4), Q.star(4), Q.path(5),
                Q.k23(), Q.cycle(6), lambda r: Q.random_series_parallel(r, int(r.integers(3, 7))),
                lambda r: Q.random_query(r, 4, 6)[:2]]


def test_brute_equals_inclusion_exclusion():
    nz = 0
    for g, k, E, chi in _rand_cases(11, 40, 8, 12, 4, 9, SMALL_SHAPES):
        a = O.brute(g, k, E, chi)
        b = O.incl_excl(g, k, E, chi)
        assert a == b, (k, E)
        nz += a > 0
    assert nz >= 15


def test_db_equals_brute_both_tie_breaks():
    shapes = SMALL_SHAPES + [Q.domino_tail(), lambda r: Q.random_query(r, 4, 8)[:2]]
    nz = 0
    for g, k, E, chi in _rand_cases(12, 60, 10, 24, 5, 12, shapes):
        a = O.brute(g, k, E, chi)
        assert O.db(g, k, E, chi, reverse_ties=True) == a, (k, E)
        assert O.db(g, k, E, chi, reverse_ties=False) == a, (k, E)
        nz += a > 0
    assert nz >= 30


def test_db_per_source_shares_sum_to_total():
    g = graphs.erdos_renyi(40, 8, seed=3)
    for k, E in (Q.cycle(5), Q.cycle_pendant(6), Q.domino_tail()):
        chi = O.colours(g.n, k, 9)
        tot = O.db(g, k, E, chi, reverse_ties=False)
        t2, per = O.db(g, k, E, chi, reverse_ties=False, sources=np.arange(g.n))
        assert t2 == tot == sum(per) == O.brute(g, k, E, chi)


@pytest.mark.parametrize("shape", [Q.cycle(4), Q.cycle(5), Q.cycle_pendant(5), Q.domino_tail(),
                                   Q.satellite(), Q.k23(), Q.star(6)])
def test_complete_graph_closed_form(shape):
    """In K_n every injective map is a match, so the colourful count is
    k! * prod_c n_c (one vertex per colour, any bijection to the nodes)."""
    k, E = shape
    n = 14 if k <= 8 else 16
    g = graphs.complete(n)
    for seed in (1, 2):
        chi = O.colours(n, k, seed)
        nc = np.bincount(chi, minlength=k)
        expect = math.factorial(k) * math.prod(int(x) for x in nc)
        assert O.db(g, k, E, chi) == expect
        if k <= 8:
            assert O.brute(g, k, E, chi) == expect


def test_cycle_matches_in_complete_graph():
    """Matches of C_k in K_n: n!/(n-k)! (and n!/((n-k)! 2k) copies)."""
    for n, k in ((7, 3), (7, 4), (8, 5)):
        g = graphs.complete(n)
        kk, E = Q.cycle(k)
        m = O.brute(g, kk, E, None)
        assert m == math.factorial(n) // math.factorial(n - k)
        assert m % (2 * k) == 0


def test_estimator_identity_exhaustive():
    """Summed over all k^n colourings, the colourful count equals
    n(G,Q) * k! * k^(n-k): each match is colourful under exactly k! k^(n-k)
    colourings, so the mean times k^k/k! is n(G,Q) (Section 2)."""
    g = graphs.erdos_renyi(6, 3.5, seed=4)
    for k, E in (Q.cycle(3), Q.path(3), Q.cycle(4)):
        matches = O.brute(g, k, E, None)
        total = 0
        for chi in itertools.product(range(k), repeat=g.n):
            c = np.array(chi, dtype=np.uint8)
            total += O.db(g, k, E, c)
        assert total == matches * math.factorial(k) * k ** (g.n - k)


def test_star_closed_form():
    """K_{1,k-1}: (k-1)! * sum_v prod_{c != chi(v)} n_c(v)."""
    g = graphs.chung_lu(3000, 8, 2.3, None, seed=7)
    k, E = Q.star(5)
    chi = O.colours(g.n, k, 5)
    src = np.repeat(np.arange(g.n), g.degrees())
    expect = 0
    cnt = np.zeros((g.n, k), dtype=np.int64)
    np.add.at(cnt, (src, chi[g.col]), 1)
    for v in range(g.n):
        p = 1
        for c in range(k):
            if c != chi[v]:
                p *= int(cnt[v, c])
        expect += p
    expect *= math.factorial(k - 1)
    assert O.db(g, k, E, chi) == expect


def test_triangle_closed_form():
    """C_3: 6 x the number of triangles whose three colours are distinct."""
    g = graphs.chung_lu(4000, 10, 2.2, None, seed=8)
    k, E = Q.cycle(3)
    chi = O.colours(g.n, k, 6)
    nb = [set(g.neighbors(v).tolist()) for v in range(g.n)]
    tri = 0
    for a in range(g.n):
        for b in nb[a]:
            if b <= a:
                continue
            for c in nb[a] & nb[b]:
                if c <= b:
                    continue
                if len({chi[a], chi[b], chi[c]}) == 3:
                    tri += 1
    assert O.db(g, k, E, chi) == 6 * tri


def test_four_cycle_wedge_closed_form():
    """C_4: sum over ordered pairs x != z with distinct colours of
    sum_{c1 != c2, both outside {chi x, chi z}} n_c1(x,z) n_c2(x,z), with
    n_c(x,z) the common neighbours of colour c."""
    g = graphs.erdos_renyi(60, 9, seed=9)
    k, E = Q.cycle(4)
    chi = O.colours(g.n, k, 7)
    nb = [set(g.neighbors(v).tolist()) for v in range(g.n)]
    tot = 0
    for x in range(g.n):
        for z in range(g.n):
            if x == z or chi[x] == chi[z]:
                continue
            cn = np.bincount([chi[y] for y in nb[x] & nb[z]], minlength=k)
            for c1 in range(k):
                for c2 in range(k):
                    if c1 != c2 and c1 not in (chi[x], chi[z]) and c2 not in (chi[x], chi[z]):
                        tot += int(cn[c1]) * int(cn[c2])
    assert O.db(g, k, E, chi) == tot


def test_invariances():
    """Colour permutation, vertex relabelling and disjoint union."""
    g = graphs.erdos_renyi(50, 10, seed=10)
    for k, E in (Q.cycle(5), Q.cycle_pendant(6), Q.domino_tail()):
        chi = O.colours(g.n, k, 3)
        base = O.db(g, k, E, chi)
        perm = np.random.default_rng(1).permutation(k).astype(np.uint8)
        assert O.db(g, k, E, perm[chi]) == base
        vp = np.random.default_rng(2).permutation(g.n)
        g2 = graphs.from_edges(g.n, vp[g.edge_list()])
        chi2 = np.empty_like(chi)
        chi2[vp] = chi
        assert O.db(g2, k, E, chi2) == base
        h = graphs.erdos_renyi(30, 8, seed=11)
        chih = O.colours(h.n, k, 4)
        u = graphs.disjoint_union(g, h)
        assert O.db(u, k, E, np.concatenate([chi, chih])) == base + O.db(h, k, E, chih)


def test_satellite_worked_decomposition():
    gold = json.load(open(os.path.join(GOLD, "satellite_tree.json")))
    p = O.plan(11, gold["edges"], gold["order"])
    names = {}
    for i, (b, want) in enumerate(zip(p["blocks"], gold["blocks"])):
        names[i] = want["name"]
        assert b["kind"] == want["kind"]
        assert sorted(b["nodes"]) == sorted(want["nodes"])
        assert sorted(b["boundary"]) == sorted(want["boundary"])
        assert sorted(names[c] for c in b["children"]) == sorted(want["children"])
    assert p["root_block"] == len(gold["blocks"]) - 1
    # the oracle's own greedy tree is different but counts the same
    g = graphs.erdos_renyi(16, 11, seed=12)
    chi = O.colours(g.n, 11, 1)
    assert O.db(g, 11, gold["edges"], chi) == O.brute(g, 11, gold["edges"], chi)


def test_lemma_41_every_treewidth2_query_decomposes():
    rng = np.random.default_rng(13)
    for _ in range(200):
        k, E = Q.random_series_parallel(rng, int(rng.integers(2, 11)))
        O.plan(k, E)
    for _ in range(100):
        k, E, _f = Q.random_query(rng, 4, 10)
        O.plan(k, E)
    for k, E in (Q.k4(), Q.k33()):
        with pytest.raises(ValueError):
            O.plan(k, E)


@pytest.mark.parametrize("leaves", [500, 2000])
def test_table_width_flag_closed_forms(leaves):
    """The 64-bit width check (tables are 64-bit, overflow flagged): a star
    of 8 leaves with a triangle through its centre (k = 11) on a hub of
    `leaves` leaves (no triangle) beside K_12.  Closed forms: every colourful
    match lies in the clique, where every injective map is a match, so the
    count is 2 * 11! (colour 0 twice, every other colour once); the star
    table at the hub holds 8! * (leaves / 10)^8 for each 8 of its 10 leaf
    colours, the largest entry of any table, and the flag must say whether
    that reaches 2^64."""
    g, chi = graphs.hub_and_clique(leaves)
    k, E = Q.star_triangle(8)
    count, flag = O.db_flagged(g, k, E, chi)
    assert count == 2 * math.factorial(11)
    assert O.db(g, k, E, chi) == count
    per_colour = np.bincount(chi[1:leaves + 1], minlength=k)[1:]
    assert np.all(per_colour == leaves // 10)
    biggest = math.factorial(8) * (leaves // 10) ** 8
    assert flag == (biggest >= 2**64)
