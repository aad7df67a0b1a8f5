"""Benchmark: colourful-match counting throughput on one MI355X.

Workload (one step = one full solve, all blocks, on a resident graph):
  Chung-Lu power-law graph, n = 1,000,000, mean degree 16, exponent 2.1,
  maximum expected degree 1e4 (seed 2); query = 6-cycle with a pendant node
  (7 nodes, treewidth 2); k = 7 colours; 1 colouring per step (colouring seed
  102 + step).  Throughput = colourings x data edges / second.

Prints one JSON line (see the repository's benchmark contract), including a
roofline entry for the dominant kernel (timed with HIP events on the
library's stream) and a CPU baseline from the oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cl1m",
                    help="cl1m (the benchmark), er1000, uneven, serve, ps (degree-based vs path splitting), "
                         "trees (every decomposition tree timed), precision (colour-coding CV vs colourings)")
    ap.add_argument("--ps-n", default="100000,300000",
                    help="sizes of the power-law stand-ins of the DB-vs-PS comparison")
    ap.add_argument("--uneven-n", type=int, default=20_000)
    ap.add_argument("--uneven-trials", type=int, default=16)
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--serve-graphs", type=int, default=4, help="resident graphs of the serving pool")
    ap.add_argument("--serve-max-edges", type=float, default=1e6, help="edges of the largest pool graph (smallest 1e5)")
    ap.add_argument("--serve-max-colourings", type=int, default=8, help="colourings per request: 1 .. this")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--cpu-sample-seconds", type=float, default=20.0)
    ap.add_argument("--batch-trials", type=int, default=8,
                    help="colourings solved plain and in one batched call (0: skip this comparison)")
    ap.add_argument("--legs", default="c3,c4",
                    help="extra legs of the default run (comma-separated; 'none' for none): c3 = domino+tail on the "
                         "Chung-Lu n=2e6 graph, plain against batched; c4 = 20 generated queries batched against plain")
    ap.add_argument("--c3-trials", type=int, default=2)
    ap.add_argument("--c4-n", type=int, default=50_000)
    ap.add_argument("--c4-trials", type=int, default=2)
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run four copies of 1 GiB on the device, so that hardware byte counters "
                         "collected over this run can be scaled against a kernel of known traffic")
    return ap.parse_args()


WORKLOADS = {
    # name: (graph, query, k, trials, seed)
    "cl1m": ("cl1m", "C6+pendant", 7, 1, 102),
    "er1000": ("er1000", "C5", 5, 1, 101),
    "cl2m": ("cl2m", "domino+tail", 8, 1, 103),
}


def query_of(name):
    from cc_inputs import queries as Q
    if name == "C6+pendant":
        return Q.cycle_pendant(6)
    if name == "C5":
        return Q.cycle(5)
    if name == "domino+tail":
        return Q.domino_tail()
    raise KeyError(name)


KERNEL_OF = {  # profiled op name -> the HIP kernel (or the kernels, one per launch, by row width) that runs it
    "edgejoin": "k_ejv", "edgejoin2": "k_ejv", "nodejoin": "k_nj / k_nj_dense",
    "axpy": "k_axpyn_rows / k_axpyn / k_axpyn_dense", "merge_root": "k_mroot_rows / k_mroot", "init": "k_init",
    "merge_u": "k_munary", "merge_v": "k_munary", "merge_edge": "k_medge_v / k_medge", "merge_edge_t": "k_medge_t",
    "level_build": "k_mark_* / k_cmp_*", "light": "k_light", "light_large": "k_light", "leaf": "k_leaf",
    "root_single": "k_root_single", "merge_root_terms": "k_mroot_rows / k_mroot_terms", "merge_pair": "k_mpair",
}


def kernel_of(op_name):
    if "_op" in op_name:  # CC_PROFILE_BY_OP=1: records per program operation
        op_name = op_name[:op_name.index("_op")]
    base = op_name.rsplit("_", 1)[0] if op_name.endswith(("_dense", "_sparse")) else op_name
    return KERNEL_OF.get(base, base)


def traffic_record(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source;
    else None."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    src = os.path.join(ROOT, "paper_1602_04478_amd", "csrc", rec["source"])
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
        return None
    return rec["hbm_bytes_per_launch"]


def roofline(tstats, pstats, cstats, workload):
    """The dominant kernel against the HBM peak.

    tstats: the timed steps, HIP events on the library's stream around the
    EdgeJoin launches only; pstats: one untimed solve with every launch
    event-timed (the split over kernels, and which kernel dominates); cstats:
    one untimed solve of the first step's colouring with the kernels'
    algorithmic-byte counters on.  Bytes per launch of each operation come
    from cstats; the dominant kernel's launch durations from tstats."""
    def per_kernel_of(stats):
        per_kernel, kern = {}, {}
        for op, (launches, secs, _b, _w) in stats.items():
            cl, _cs, cb, cw = cstats.get(op, (0, 0.0, 0.0, (0, 0, 0)))
            bpl = cb / cl if cl else 0.0
            kn = kernel_of(op)
            a = per_kernel.setdefault(kn, [0, 0.0, 0.0, []])
            a[0] += launches
            a[1] += secs
            a[2] += bpl * launches
            a[3].append(op)
            kern[op] = {"kernel": kn, "launches": launches, "ms": 1000.0 * secs, "alg_GB_per_launch": bpl / 1e9,
                        "alg_GBps": bpl * launches / secs / 1e9 if secs > 0 and bpl > 0 else None}
            if op.startswith("edgejoin") and cl:
                # two EdgeJoins on one scan ("edgejoin2") count slots instead of rows
                unit = "slots" if op.startswith("edgejoin2") else "rows"
                kern[op]["per_launch_triples_scanned"] = cw[0] / cl
                kern[op][f"per_launch_{unit}_relaxed"] = cw[1] / cl
                kern[op][f"per_launch_{unit}_written"] = cw[2] / cl
        return per_kernel, kern
    per_kernel, kern = per_kernel_of(pstats)
    name = max(per_kernel, key=lambda x: per_kernel[x][1])
    timed, _ = per_kernel_of(tstats)
    launches, secs, byts, ops = timed.get(name, per_kernel[name])
    ach = byts / secs / 1e9 if secs > 0 else 0.0
    traffic = traffic_record(name, workload)
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": name, "ops": sorted(ops), "launches": launches,
            "avg_launch_ms": 1000.0 * secs / max(1, launches), "alg_bytes_per_launch": byts / max(1, launches),
            "timing": "HIP events around this kernel's launches over the timed steps"}
    tot_s = sum(v[1] for v in per_kernel.values())
    tot_b = sum(v[2] for v in per_kernel.values())
    uncounted = sorted(k for k, v in per_kernel.items() if v[2] == 0)
    roof["all_kernels"] = {"kernel_s": tot_s, "alg_GB": tot_b / 1e9, "alg_GBps": tot_b / tot_s / 1e9 if tot_s else 0,
                           "frac": tot_b / tot_s / 1e9 / HBM_PEAK_GBS if tot_s else 0,
                           "kernels_without_byte_count": uncounted,
                           "timing": "one untimed solve, every launch event-timed"}
    return roof, kern


def cpu_baseline(g, k, E, seed, budget_s):
    """The oracle (as it stands) on a bounded, stratified sample of root
    sources, scaled to the whole solve by a ratio estimator.

    The cost of a root source is concentrated in the hubs, so sources are
    stratified by a work proxy -- W(u), the summed degree of u's lower
    neighbours -- in powers of two.  From the lightest stratum up, each
    stratum's sample (at most 64 sources, systematic) is run as one oracle call
    (its OpenMP threads take the sources in parallel) and its CPU seconds are
    scaled by the stratum's total proxy over the sample's.  Strata beyond the
    time budget are not run: they are priced at the CPU seconds per proxy unit
    of the heaviest stratum that ran.  Wall time on C cores = CPU seconds / C."""
    from oracle import oracle as O
    chi = O.colours(g.n, k, seed, 0)
    deg = g.degrees().astype(np.int64)
    order = np.lexsort((np.arange(g.n), deg))  # ascending (degree, id): the library's order
    rank = np.empty(g.n, dtype=np.int64)
    rank[order] = np.arange(g.n)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    dst = g.col.astype(np.int64)
    low = rank[dst] < rank[src]
    W = np.bincount(src[low], weights=deg[dst[low]], minlength=g.n)
    cand = np.nonzero(W > 0)[0]
    strata = np.floor(np.log2(W[cand])).astype(np.int64)
    cpu_total, spent, used, ran, skipped = 0.0, 0.0, [], 0, 0
    last_rate = None
    cores = O.threads()
    checked = {}  # oracle per-source counts of the sampled sources
    for s_id in np.unique(strata):
        members = cand[strata == s_id]
        members = members[np.argsort(W[members])]
        step = max(1, len(members) // 64)
        sample = members[step // 2::step][:64]
        if spent < budget_s:
            c0, t0 = time.process_time(), time.perf_counter()
            _tot, vals = O.db(g, k, E, chi, reverse_ties=False, sources=sample)
            cpu = time.process_time() - c0
            checked.update({int(s): int(v) for s, v in zip(sample, vals)})
            spent += time.perf_counter() - t0
            last_rate = cpu / W[sample].sum()
            cpu_total += cpu * W[members].sum() / W[sample].sum()
            used.append(f"2^{s_id}:{len(sample)}/{len(members)}")
            ran += len(sample)
        else:
            cpu_total += last_rate * W[members].sum()
            skipped += len(members)
    wall = cpu_total / cores
    return checked, dict(value=g.m / wall, unit="colourings*edges/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(), c1_one_thread_s=c1_one_thread_seconds(),
                sample=(f"DB oracle on {ran} root sources stratified by lower-neighbour degree sum "
                        f"(strata sampled/size: {' '.join(used)}); {skipped} sources in heavier strata priced "
                        f"at the heaviest sampled stratum's CPU s per unit; {spent:.1f} s measured; "
                        f"estimated {cpu_total:.0f} CPU s for the whole solve, / {cores} cores"))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def c1_one_thread_seconds():
    """The oracle's DB count of the tiny configuration (G(1000, 10/999),
    5-cycle, k = 5, colouring seed 101) on one thread, in a child process."""
    import subprocess
    code = ("import time,sys; sys.path.insert(0, %r)\n"
            "from cc_inputs import graphs, queries as Q\nfrom oracle import oracle as O\n"
            "g = graphs.workload_graph('er1000'); k, E = Q.cycle(5); chi = O.colours(g.n, k, 101, 0)\n"
            "O.db(g, k, E, chi)\nt = time.perf_counter(); O.db(g, k, E, chi); print(time.perf_counter() - t)" % ROOT)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120)
    try:
        return float(r.stdout.strip().splitlines()[-1])
    except (ValueError, IndexError):
        return None


def uneven_leg(n, T):
    """Batched uneven queries: 20 generated treewidth-2 queries of 4-10 nodes
    (query seed 204), T colourings each, on a Chung-Lu graph (mean 20,
    exponent 2.1, structural cutoff, seed 4) of n vertices: one cc_count_batch
    call (trial-group size and tree tuned online per query, launch sequences
    replayed from hipGraphs, queries side by side on worker streams) against
    plain per-colouring calls; neither profiled."""
    from cc_inputs import graphs, queries as Q
    from paper_1602_04478_amd import cc
    g = graphs.chung_lu(n, 20.0, 2.1, None, seed=4)
    dg = cc.Graph.from_csr(g)
    qs = [cc.Query(k, E) for k, E, fam in Q.random_queries(204, 20, 4, 10)]
    seeds = [204 + i for i in range(len(qs))]
    cc.count_batch(dg, qs[:1], seeds[:1], [2])  # warm-up
    t0 = time.perf_counter()
    counts, ovf, est = cc.count_batch(dg, qs, seeds, [T] * len(qs))
    t_batch = time.perf_counter() - t0
    print(f"[bench] uneven queries n={n}: batched {t_batch:.2f} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    plain = []
    for q, sd in zip(qs, seeds):
        for t in range(T):
            plain.append(int(cc.count(dg, q, sd + t, 1)[0][0]))
    t_plain = time.perf_counter() - t0
    print(f"[bench] uneven queries n={n}: plain {t_plain:.2f} s", file=sys.stderr, flush=True)
    col = len(qs) * T
    return {"workload": f"uneven queries: Chung-Lu n={g.n} m={g.m} (mean 20, exponent 2.1), 20 generated queries "
                        f"of 4-10 nodes x {T} colourings, one batched call",
            "value": col * g.m / t_batch, "unit": "colourings*edges/s", "seconds": t_batch,
            "plain_value": col * g.m / t_plain, "plain_seconds": t_plain, "speedup_vs_plain": t_plain / t_batch,
            "counts_match_plain": [int(c) for c in counts] == plain, "overflowed": int(ovf.sum())}


def c3_leg(T):
    """The C3 shape at full size (Chung-Lu n = 2e6, mean 20, exponent 2.2,
    structural cutoff, seed 3; domino + tail, k = 8): T colourings as T plain
    calls and as one batched call, neither profiled; counts must agree."""
    from cc_inputs import graphs, queries as Q
    from paper_1602_04478_amd import cc
    t0 = time.perf_counter()
    g = graphs.workload_graph("cl2m")
    print(f"[bench] c3 graph: n={g.n} m={g.m} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    k, E = Q.domino_tail()
    dg, q = cc.Graph.from_csr(g), cc.Query(k, E)
    pl, tp = [], []
    for t in range(T):
        t1 = time.perf_counter()
        pl.append(cc.count(dg, q, 103 + t, 1))
        tp.append(time.perf_counter() - t1)
        print(f"[bench] c3 plain colouring {t}: {tp[-1]:.2f} s", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    bc, bo, be = cc.count_batch(dg, [q], [103], [T])
    dt = time.perf_counter() - t1
    print(f"[bench] c3 batched ({T} colourings): {dt:.2f} s", file=sys.stderr, flush=True)
    rep = cc.last_tune_report()
    return {"workload": f"cl2m: n={g.n} m={g.m} maxdeg={int(g.degrees().max())}; query domino+tail; k=8; "
                        f"{T} colourings (seed 103)",
            "value": T * g.m / dt, "unit": "colourings*edges/s", "seconds": dt, "trial_group": rep["trial_group"],
            "plain_value": T * g.m / sum(tp), "plain_seconds_per_colouring": tp, "speedup_vs_plain": sum(tp) / dt,
            "counts": [[int(bc[t]), int(bo[t])] for t in range(T)],
            "counts_match_plain": all(int(bc[t]) == int(pl[t][0][0]) and int(bo[t]) == int(pl[t][1][0])
                                      for t in range(T))}


def run_uneven(a):
    leg = uneven_leg(a.uneven_n, a.uneven_trials)
    out = {"metric": "colourings*data-edges/sec (exact uint64 colourful counts)",
           "value": leg["value"], "unit": "colourings*edges/s", "n_gpus": 1, "steps": 1, "warmup": 1,
           "ms_per_step": 1000 * leg["seconds"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64", "data": "synthetic", "config": {"workload": leg["workload"]},
           **{k: v for k, v in leg.items() if k not in ("workload", "value", "unit", "seconds")}}
    print(json.dumps(out))


def run_serve(a):
    """Serving: a pool of --serve-graphs resident Chung-Lu graphs (mean degree
    16, edges log-spaced from 1e5 to --serve-max-edges, exponent uniform in
    [2.0, 2.5], seed 5); --serve-requests requests (graph uniform, a generated
    query of 4-9 nodes, 1 .. --serve-max-colourings colourings) arriving as a
    Poisson stream at 0.8 x the measured one-at-a-time capacity; latency =
    completion - arrival.  Afterwards up to 16 distinct (graph, query) pairs
    are solved again alone (plain calls): their counts must equal the served
    ones."""
    from cc_inputs import graphs, queries as Q
    from paper_1602_04478_amd import cc
    rng = np.random.default_rng(5)
    pool = []
    G = a.serve_graphs
    for i in range(G):
        m = 1e5 * (a.serve_max_edges / 1e5) ** (i / max(1, G - 1))
        pool.append(graphs.chung_lu(int(m / 8), 16.0, float(rng.uniform(2.0, 2.5)), None, seed=50 + i))
        print(f"[bench] serve graph {i}: n={pool[-1].n} m={pool[-1].m}", file=sys.stderr, flush=True)
    dgs = [cc.Graph.from_csr(g) for g in pool]
    qlist = [cc.Query(k, E) for k, E, fam in Q.random_queries(505, 16, 4, 9)]
    reqs = [(int(rng.integers(0, len(pool))), int(rng.integers(0, len(qlist))), int(rng.integers(0, 2**40)),
             int(rng.integers(1, a.serve_max_colourings + 1))) for _ in range(a.serve_requests)]
    # capacity: the first 8 requests one at a time
    t0 = time.perf_counter()
    for j, (gi, qi, sd, tr) in enumerate(reqs[:8]):
        cc.count(dgs[gi], qlist[qi], sd, tr)
        print(f"[bench] serve capacity: request {j} (graph {gi}, {tr} colourings) done at "
              f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    svc = (time.perf_counter() - t0) / 8
    print(f"[bench] serve: {1000 * svc:.0f} ms per request one at a time", file=sys.stderr, flush=True)
    lam = 0.8 / svc
    arrivals = np.cumsum(rng.exponential(1.0 / lam, size=len(reqs)))
    srv = cc.Server(0, max_inflight=4)
    ids = [srv.add_graph(dg) for dg in dgs]
    pending, lat, done_edges, served, failed = {}, [], 0, {}, []
    t0 = time.perf_counter()
    i = 0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and arrivals[i] <= now:
            gi, qi, sd, tr = reqs[i]
            pending[srv.submit(ids[gi], qlist[qi], sd, tr)] = i
            i += 1
        for tk, ri in list(pending.items()):
            try:
                r = srv.poll(tk, reqs[ri][3])
            except cc.CCError as e:  # the request failed (reported, not retried)
                failed.append((ri, str(e)))
                del pending[tk]
                continue
            if r is not None:
                lat.append(r[3])
                served[ri] = [int(x) for x in r[0]]
                done_edges += reqs[ri][3] * pool[reqs[ri][0]].m
                del pending[tk]
                print(f"[bench] serve: {len(lat)} of {len(reqs)} done at {now:.1f} s", file=sys.stderr, flush=True)
        time.sleep(0.0005)
    wall = time.perf_counter() - t0
    srv.close()
    # alone == served on up to 16 distinct (graph, query) pairs of the smaller half of the pool
    seen, checked, equal = set(), 0, 0
    for ri, (gi, qi, sd, tr) in enumerate(reqs):
        if (gi, qi) in seen or checked >= 16 or gi >= max(1, G // 2) or ri not in served:
            continue
        seen.add((gi, qi))
        alone = [int(x) for x in cc.count(dgs[gi], qlist[qi], sd, tr)[0]]
        checked += 1
        equal += alone == served[ri]
        print(f"[bench] serve check {checked}: alone == served {alone == served[ri]}", file=sys.stderr, flush=True)
    lat = np.array(lat)
    out = {"metric": "colourings*data-edges/sec (exact uint64 colourful counts), served",
           "value": done_edges / wall, "unit": "colourings*edges/s", "n_gpus": 1, "steps": 1, "warmup": 0,
           "ms_per_step": 1000 * wall, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "u64", "data": "synthetic",
           "config": {"workload": f"serving: {len(reqs)} requests, Poisson arrivals at {lam:.2f}/s "
                                  f"(0.8 x one-at-a-time capacity), pool of {len(pool)} graphs "
                                  f"(m = {', '.join(str(g.m) for g in pool)}), queries of 4-9 nodes, "
                                  f"1-{a.serve_max_colourings} colourings"},
           "p50_ms": 1000 * float(np.percentile(lat, 50)), "p99_ms": 1000 * float(np.percentile(lat, 99)),
           "requests_per_s": len(reqs) / wall, "one_at_a_time_ms": 1000 * svc,
           "alone_equals_served": f"{equal}/{checked}", "failed_requests": failed}
    print(json.dumps(out))


def _timed_count(dg, q, seed, trials=1):
    t0 = time.perf_counter()
    r = __import__("paper_1602_04478_amd.cc", fromlist=["cc"]).count(dg, q, seed, trials)
    return time.perf_counter() - t0, r


def run_ps(a):
    """The paper's headline comparison (Section 8: DB against its path-
    splitting baseline PS) on the same kernels: PS splits every cycle at its
    boundary nodes (the root at a node and the one opposite) and lets paths
    take any vertex; DB starts them at the highest vertex.  Power-law
    stand-ins of the C2 and C3 shapes at the sizes given; one colouring per
    solve after a warm-up; counts must agree."""
    from cc_inputs import graphs, queries as Q
    from paper_1602_04478_amd import cc
    rows = []
    for n in [int(x) for x in a.ps_n.split(",") if x]:
        for shape, (k, E), gen in (("C2 shape: 6-cycle + pendant, exponent 2.1", Q.cycle_pendant(6),
                                    lambda n: graphs.chung_lu(n, 16.0, 2.1, 1e4 * (n / 1e6) ** (1 / 1.1), seed=2)),
                                   ("C3 shape: domino + tail, exponent 2.2", Q.domino_tail(),
                                    lambda n: graphs.chung_lu(n, 20.0, 2.2, None, seed=3))):
            g = gen(n)
            dg = cc.Graph.from_csr(g)
            qdb, qps = cc.Query(k, E), cc.Query(k, E, path_splitting=True)
            cc.count(dg, qdb, 7, 1)  # warm-up
            t_db, r_db = _timed_count(dg, qdb, 11)
            t_db2, _ = _timed_count(dg, qdb, 12)
            cc.count(dg, qps, 7, 1) if t_db < 5 else None
            t_ps, r_ps = _timed_count(dg, qps, 11)
            row = {"shape": shape, "n": g.n, "m": g.m, "max_degree": int(g.degrees().max()),
                   "db_s": min(t_db, t_db2), "ps_s": t_ps, "improvement_ps_over_db": t_ps / min(t_db, t_db2),
                   "counts_equal": r_db[2] == r_ps[2] and bool(r_db[1][0] == r_ps[1][0]), "count": int(r_db[2][0])}
            rows.append(row)
            print(f"[bench] ps {shape} n={g.n}: DB {row['db_s']:.3f} s, PS {t_ps:.3f} s", file=sys.stderr, flush=True)
    f = [r["improvement_ps_over_db"] for r in rows]
    out = {"metric": "DB-vs-PS improvement factor (t_PS / t_DB, same kernels, one colouring)",
           "value": float(np.exp(np.mean(np.log(f)))), "unit": "x (geometric mean)", "n_gpus": 1, "steps": 1,
           "warmup": 1, "higher_is_better": True, "dtype": "u64", "data": "synthetic",
           "config": {"workload": "degree-based vs path splitting on power-law stand-ins"},
           "max": max(f), "all_counts_equal": all(r["counts_equal"] for r in rows), "rows": rows}
    print(json.dumps(out))


def run_trees(a):
    """Every decomposition tree of a query timed (Section 8: the choice of
    tree changes the time by up to an order of magnitude; the heuristic of
    Section 6 picks a good one): per query, each tree's solve of one
    colouring after a warm-up, the heuristic's tree, the fastest, and whether
    the counts agree.  Power-law stand-in (Chung-Lu n = 1e5, mean 16,
    exponent 2.1) and queries with several trees (the 20 generated ones that
    have more than one, plus domino + tail, the chorded 8-cycle and the
    worked example of Section 4.1)."""
    from cc_inputs import graphs, queries as Q
    from paper_1602_04478_amd import cc
    g = graphs.chung_lu(100_000, 16.0, 2.1, None, seed=12)
    dg = cc.Graph.from_csr(g)
    qs = [("domino+tail", *Q.domino_tail()), ("C8+chord(0,4)", 8, Q.cycle(8)[1] + [(0, 4)]),
          ("satellite", *Q.satellite())]
    for i, (k, E, fam) in enumerate(Q.random_queries(204, 20, 4, 10)):
        qs.append((f"generated {i} ({fam}, k={k})", k, E))
    rows = []
    for name, k, E in qs:
        h = cc.Query(k, E)
        ti = h.tree_info()
        nt = min(ti["num_trees"], 12)
        if nt < 2:
            continue
        times, counts, failed = [], [], []
        print(f"[bench] trees {name}: timing {nt} trees", file=sys.stderr, flush=True)
        for t in range(nt):
            q = cc.Query(k, E, tree=t)
            try:
                cc.count(dg, q, 5, 1)
                dt, r = _timed_count(dg, q, 6)
            except cc.CCError as e:  # e.g. a pair-keyed table larger than the device memory
                failed.append((t, e.name))
                times.append(float("inf"))
                continue
            times.append(dt)
            counts.append(r[2][0])
        if len(failed) == nt:
            rows.append({"query": name, "trees": ti["num_trees"], "timed": 0, "failed": failed})
            continue
        best = int(np.argmin(times))
        heur = ti["tree"] if ti["tree"] < nt else None
        # the batched call's own choice (tree tuned online on 32 of its
        # colourings), where a colouring takes well under a second
        tuned = None
        if max(times) < 1.0:
            try:
                cc.count_batch(dg, [h], [77], [32])
                tuned = cc.last_tune_report()["tree"]
            except cc.CCError:
                pass
        fin = [x for x in times if x != float("inf")]
        rows.append({"query": name, "trees": ti["num_trees"], "timed": nt,
                     "seconds": [x if x != float("inf") else None for x in times], "failed": failed,
                     "heuristic": heur, "fastest": best, "batched_tuned": tuned,
                     "tuned_over_best": (times[tuned] / times[best]) if tuned is not None and tuned < nt else None,
                     "spread_max_over_min": max(fin) / min(fin),
                     "heuristic_over_best": (times[heur] / times[best]) if heur is not None else None,
                     "counts_equal": len(set(counts)) == 1})
        print(f"[bench] trees {name}: {nt} trees, spread {max(fin) / min(fin):.2f}x", file=sys.stderr,
              flush=True)
    ho = [r["heuristic_over_best"] for r in rows if r.get("heuristic_over_best") is not None]
    out = {"metric": "decomposition trees: heuristic time / best time", "value": float(np.mean(ho)) if ho else None,
           "unit": "x (mean)", "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": False, "dtype": "u64",
           "data": "synthetic",
           "config": {"workload": f"every tree (up to 12) of queries with several trees, Chung-Lu n={g.n} m={g.m}"},
           "heuristic_optimal_fraction": float(np.mean([h <= 1.05 for h in ho])) if ho else None,
           "batched_tuned_over_best": float(np.mean([r["tuned_over_best"] for r in rows
                                                     if r.get("tuned_over_best") is not None] or [float("nan")])),
           "max_spread": max((r["spread_max_over_min"] for r in rows if "spread_max_over_min" in r), default=None),
           "all_counts_equal": all(r.get("counts_equal", True) for r in rows), "rows": rows}
    print(json.dumps(out))


def run_precision(a):
    """Colour-coding precision (Section 8): the coefficient of variation
    (standard deviation / mean) of the estimate made from T colourings, for
    T = 3 and T = 10, over disjoint groups of 60 colourings solved in one
    batched call; per (graph, query) pair, and the fraction of pairs with
    CV <= 0.1.  Power-law and Erdos-Renyi stand-ins, cycle and generated
    queries."""
    from cc_inputs import graphs, queries as Q
    from paper_1602_04478_amd import cc
    gl = [("Chung-Lu n=1e5 mean 16 exp 2.1", graphs.chung_lu(100_000, 16.0, 2.1, None, seed=21)),
          ("Chung-Lu n=1e5 mean 20 exp 2.5", graphs.chung_lu(100_000, 20.0, 2.5, None, seed=22)),
          ("near-regular Chung-Lu n=2e4 mean 10 exp 8", graphs.chung_lu(20_000, 10.0, 8.0, None, seed=23))]
    ql = [("C5", *Q.cycle(5)), ("C6+pendant", *Q.cycle_pendant(6)), ("domino+tail", *Q.domino_tail())]
    for i, (k, E, fam) in enumerate(Q.random_queries(606, 5, 4, 8)):
        ql.append((f"generated {i} ({fam}, k={k})", k, E))
    T = 60
    rows = []
    for gname, g in gl:
        dg = cc.Graph.from_csr(g)
        for qname, k, E in ql:
            q = cc.Query(k, E)
            counts, ovf, _ = cc.count_batch(dg, [q], [1000 + len(rows)], [T])
            if ovf.any():
                continue
            scale = k ** k / math.factorial(k) / q.info()["aut"]
            est = counts.astype(np.float64) * scale
            row = {"graph": gname, "query": qname, "mean_estimate": float(est.mean())}
            for tt in (3, 10):
                grp = est[: (T // tt) * tt].reshape(-1, tt).mean(axis=1)
                row[f"cv_{tt}"] = float(grp.std(ddof=1) / grp.mean()) if grp.mean() > 0 else None
            rows.append(row)
    ok = [r for r in rows if r["cv_3"] is not None]
    out = {"metric": "colour-coding precision: pairs with CV <= 0.1", "value": float(np.mean([r["cv_3"] <= 0.1 for r in ok])),
           "unit": "fraction of (graph, query) pairs at 3 colourings", "n_gpus": 1, "steps": 1, "warmup": 0,
           "higher_is_better": True, "dtype": "u64", "data": "synthetic",
           "config": {"workload": f"{len(gl)} stand-in graphs x {len(ql)} queries, {T} colourings each, CV over "
                                  "disjoint groups of 3 and of 10"},
           "fraction_cv_le_0.1_at_10": float(np.mean([r["cv_10"] <= 0.1 for r in ok if r["cv_10"] is not None])),
           "rows": rows}
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if a.workload == "uneven":
        return run_uneven(a)
    if a.workload == "serve":
        return run_serve(a)
    if a.workload == "ps":
        return run_ps(a)
    if a.workload == "trees":
        return run_trees(a)
    if a.workload == "precision":
        return run_precision(a)
    from cc_inputs import graphs
    from paper_1602_04478_amd import cc
    gname, qname, k, trials, seed0 = WORKLOADS[a.workload]
    t0 = time.perf_counter()
    g = graphs.workload_graph(gname)
    t_gen = time.perf_counter() - t0
    k, E = query_of(qname)
    dg = cc.Graph.from_csr(g)
    q = cc.Query(k, E)
    if a.copy_probe:
        cc.probe_copy(1 << 30, 4)  # 4 copies of 1 GiB: 8 GiB read + written
    for i in range(a.warmup):
        cc.count(dg, q, seed0 + 1000 + i, trials)
    times, results = [], []
    prof = not a.no_profile
    # timed steps: HIP events on the library's stream around the EdgeJoin launches (no counters)
    cc.profile_take()
    cc.profile_enable(3 if prof else 0)  # events around the EdgeJoin launches only
    t_all = time.perf_counter()
    for i in range(a.steps):
        t1 = time.perf_counter()
        counts, ovf, exact, est = cc.count(dg, q, seed0 + i, trials)
        times.append(time.perf_counter() - t1)
        results.append((int(counts[0]), int(ovf[0])))
        print(f"[bench] step {i}: {times[-1]:.3f} s", file=sys.stderr, flush=True)
    total = time.perf_counter() - t_all
    cc.profile_enable(0)
    tstats = cc.profile_take()
    ms = 1000.0 * total / a.steps
    value = trials * g.m / (total / a.steps)
    out = {
        "metric": "colourings*data-edges/sec (exact uint64 colourful counts)",
        "value": value,
        "unit": "colourings*edges/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"{gname}: n={g.n} m={g.m} maxdeg={int(g.degrees().max())}; query {qname}; "
                               f"k={k}; {trials} colouring(s) per step", "graph": gname, "query": qname,
                   "k": k, "trials": trials},
        "counts": results,
    }
    if prof:
        # untimed: the first step's colouring again, with the kernels' byte counters
        # untimed: one solve with every launch event-timed (the split over kernels)
        cc.profile_enable(1)
        cc.count(dg, q, seed0, trials)
        cc.profile_enable(0)
        pstats = cc.profile_take()
        cc.profile_enable(2)
        c2 = cc.count(dg, q, seed0, trials)
        cc.profile_enable(0)
        cstats = cc.profile_take()
        assert (int(c2[0][0]), int(c2[1][0])) == results[0], "counting pass disagrees with the timed step"
        out["roofline"], out["kernels"] = roofline(tstats, pstats, cstats, a.workload)
        # the rate of a plain streaming copy on this device: what an HBM-bound kernel can reach
        out["roofline"]["copy_probe_GBps"] = cc.probe_copy(1 << 30, 10)
    if a.batch_trials > 0:
        # plain vs batched on the same colourings, neither with profiling:
        # plain = one cc_count call per colouring; batched = one call of all,
        # trial groups replaying a captured hipGraph (group size tuned online)
        B = a.batch_trials
        print(f"[bench] plain vs batched: {B} colourings each", file=sys.stderr, flush=True)
        t1 = time.perf_counter()
        pl = [cc.count(dg, q, seed0 + 500 + t, 1) for t in range(B)]
        dt_plain = time.perf_counter() - t1
        t1 = time.perf_counter()
        bc, bo, be = cc.count_batch(dg, [q], [seed0 + 500], [B])
        dt = time.perf_counter() - t1
        rep = cc.last_tune_report()
        out["batched"] = {"value": B * g.m / dt, "unit": "colourings*edges/s", "colourings": B, "seconds": dt,
                          "trial_group": rep["trial_group"], "graph_replays": rep["graph_replays"],
                          "tuning": rep["tried"], "plain_value": B * g.m / dt_plain, "plain_seconds": dt_plain,
                          "speedup_vs_plain": dt_plain / dt,
                          "counts_match_plain": all(int(bc[t]) == int(pl[t][0][0]) and int(bo[t]) == int(pl[t][1][0])
                                                    for t in range(B))}
    if a.batch_trials > 0 and a.workload == "cl1m":
        # the tiny configuration (G(1000, 10/999), 5-cycle, k = 5), where a
        # solve is a handful of short launches: 64 colourings as 64 plain
        # calls and as one batched call (trial groups, graph replays)
        from cc_inputs import queries as Q
        g1 = graphs.workload_graph("er1000")
        d1, q1 = cc.Graph.from_csr(g1), cc.Query(*Q.cycle(5))
        cc.count(d1, q1, 101, 1)
        cc.count_batch(d1, [q1], [101], [8])
        t1 = time.perf_counter()
        p1 = [cc.count(d1, q1, 101 + t, 1) for t in range(64)]
        dt_p = time.perf_counter() - t1
        t1 = time.perf_counter()
        b1 = cc.count_batch(d1, [q1], [101], [64])
        dt_b = time.perf_counter() - t1
        rep = cc.last_tune_report()
        out["batched_tiny"] = {"workload": f"er1000: n={g1.n} m={g1.m}; query C5; k=5; 64 colourings",
                               "value": 64 * g1.m / dt_b, "plain_value": 64 * g1.m / dt_p,
                               "unit": "colourings*edges/s", "seconds": dt_b, "plain_seconds": dt_p,
                               "speedup_vs_plain": dt_p / dt_b, "trial_group": rep["trial_group"],
                               "graph_replays": rep["graph_replays"],
                               "counts_match_plain": all(int(b1[0][t]) == int(p1[t][0][0]) for t in range(64))}
    if not a.no_cpu_baseline:
        checked, out["cpu_baseline"] = cpu_baseline(g, k, E, seed0, a.cpu_sample_seconds)
        # the same colouring on the device with per-source shares: the sampled
        # sources' shares must equal the oracle's, and they sum to the step's count
        from oracle import oracle as O
        chi = O.colours(g.n, k, seed0, 0)
        _c, _o, ex, per = cc.count_colors(dg, q, chi, per_source=True)
        bad = [s for s, v in checked.items() if int(per[0][s]) != v]
        out["oracle_check"] = {"colouring": f"seed {seed0}, trial 0 (step 0)", "sources_checked": len(checked),
                               "sources_with_matches": sum(1 for v in checked.values() if v),
                               "mismatches": len(bad), "device_total_equals_step0": int(ex[0]) == results[0][0],
                               "shares_sum_to_total": sum(int(x) for x in per[0]) == int(ex[0])}
    out["graph_gen_s"] = t_gen
    legs = [] if a.legs == "none" or a.workload != "cl1m" else a.legs.split(",")
    if "c3" in legs:
        out["c3_leg"] = c3_leg(a.c3_trials)
    if "c4" in legs:
        out["c4_leg"] = uneven_leg(a.c4_n, a.c4_trials)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
