"""Write tests/golden/scale_counts.json: expected colourful counts for the
parity tests at scale, computed by the CPU oracle only (its DB dynamic
program, Sections 4.1-5.2, in 128-bit integers).  Nothing here calls the
device library.

Cases (every input seeded; graphs from cc_inputs, colourings from the
colouring contract, trial t of seed s):
  c2_scaled    the C2 shape scaled down so that one solve runs all three
               execution tiers: Chung-Lu n = 30000, mean degree 16, exponent
               2.1, maximum expected degree scaled with the size
               (1e4 * (n / 1e6)^(1 / (exponent - 1))), seed 2; 6-cycle + pendant,
               k = 7; colourings 102/0 and 102/1.
  c3_scaled    Chung-Lu n = 5000, mean 20, exponent 2.2, structural cutoff,
               seed 3; domino + tail (k = 8); all 64 colourings of seed 103.
  c4_scaled    Chung-Lu n = 1000, mean 8, exponent 2.1, structural cutoff,
               seed 4; the 20 generated queries of query seed 204 (4-10
               nodes), query i with colourings of seed 204 + i, 16 each.
  k8_cycle_child  Chung-Lu n = 12500, mean 16, exponent 2.4025014618726903,
               structural cutoff, seed 50; a 5-cycle and a 4-cycle sharing a
               node (k = 8); colourings 1098605756710/0 and /1.
  c2_sources   the full-size C2 graph (Chung-Lu n = 1e6, seed 2), 6-cycle +
               pendant, colouring 102/0: the share of sampled root sources
               (matches whose highest vertex in the (degree, id) order is the
               source), hubs of the first dense group and low-degree sources.

Usage: python tests/golden/make_scale_golden.py [case ...]   (all by default;
cases already in the file are kept unless named).
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from cc_inputs import graphs, queries as Q  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "scale_counts.json")


def c2_scaled_graph():
    n = 30000
    return graphs.chung_lu(n, 16.0, 2.1, 1e4 * (n / 1e6) ** (1 / 1.1), seed=2)


def c3_scaled_graph():
    return graphs.chung_lu(5000, 20.0, 2.2, None, seed=3)


def c4_scaled_graph():
    return graphs.chung_lu(1000, 8.0, 2.1, None, seed=4)


# ranks counted from the top of the (degree, id) order
C2_HUB_RANKS = list(range(40, 64))
C2_LOW_RANKS = list(range(60000, 60008)) + list(range(400000, 400008))


def sources_by_rank(g, ranks):
    deg = g.degrees()
    order = np.lexsort((np.arange(g.n), deg))[::-1]
    return [int(order[r]) for r in ranks]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def case_c2_scaled():
    g = c2_scaled_graph()
    k, E = Q.cycle_pendant(6)
    counts = []
    for t in range(2):
        t0 = time.time()
        counts.append(str(O.db(g, k, E, O.colours(g.n, k, 102, t))))
        log(f"c2_scaled trial {t}: {time.time() - t0:.1f} s")
    return {"seed": 102, "counts": counts}


def case_c3_scaled():
    g = c3_scaled_graph()
    k, E = Q.domino_tail()
    counts = []
    for t in range(64):
        counts.append(str(O.db(g, k, E, O.colours(g.n, k, 103, t))))
        log(f"c3_scaled trial {t}")
    return {"seed": 103, "counts": counts}


def case_c4_scaled():
    g = c4_scaled_graph()
    out = []
    for i, (k, E, fam) in enumerate(Q.random_queries(204, 20, 4, 10)):
        t0 = time.time()
        cs = [str(O.db(g, k, E, O.colours(g.n, k, 204 + i, t))) for t in range(16)]
        out.append({"k": k, "edges": [list(map(int, e)) for e in E], "family": fam, "seed": 204 + i, "counts": cs})
        log(f"c4_scaled query {i} ({fam}, k={k}): {time.time() - t0:.1f} s")
    return {"queries": out}


def k8_cycle_child_graph():
    return graphs.chung_lu(12500, 16.0, 2.4025014618726903, None, seed=50)


K8_CYCLE_CHILD = (8, [(0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (0, 5), (5, 6), (6, 7), (7, 0)])


def case_k8_cycle_child():
    g = k8_cycle_child_graph()
    k, E = K8_CYCLE_CHILD
    seed = 1098605756710
    return {"seed": seed, "counts": [str(O.db(g, k, E, O.colours(g.n, k, seed, t))) for t in range(2)]}


def case_c2_sources():
    g = graphs.workload_graph("cl1m")
    k, E = Q.cycle_pendant(6)
    chi = O.colours(g.n, k, 102, 0)
    src = sources_by_rank(g, C2_HUB_RANKS + C2_LOW_RANKS)
    t0 = time.time()
    _tot, vals = O.db(g, k, E, chi, reverse_ties=False, sources=src)
    log(f"c2_sources: {len(src)} sources in {time.time() - t0:.1f} s")
    return {"seed": 102, "trial": 0, "ranks": C2_HUB_RANKS + C2_LOW_RANKS, "sources": src,
            "shares": [str(v) for v in vals]}


CASES = {"c2_scaled": case_c2_scaled, "c3_scaled": case_c3_scaled, "c4_scaled": case_c4_scaled,
         "c2_sources": case_c2_sources, "k8_cycle_child": case_k8_cycle_child}


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names or list(CASES):
        data[name] = CASES[name]()
        json.dump(data, open(OUT, "w"), indent=1)
        log(f"wrote {name}")


if __name__ == "__main__":
    main(sys.argv[1:])
