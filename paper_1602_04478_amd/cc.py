"""Thin ctypes binding of libcc.so (include/cc.h).  Argument marshalling only:
every step of the counting runs in the library's HIP kernels.  There is no
fallback: if the library cannot be loaded, every call raises."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcc.so")

CC_GRAPH_CLEAN = 1
CC_GRAPH_REVERSE_TIES = 2
CC_QUERY_PATH_SPLITTING = 1

STATUS = {0: "CC_OK", 1: "CC_E_ARG", 2: "CC_E_GRAPH", 3: "CC_E_QUERY_TW", 4: "CC_E_QUERY_DISCONNECTED",
          5: "CC_E_K_RANGE", 6: "CC_E_UNSUPPORTED", 7: "CC_E_NOMEM", 8: "CC_E_DEVICE", 9: "CC_E_BUSY"}

# every entry point declared in include/cc.h
EXPORTS = ["cc_graph_create", "cc_graph_destroy", "cc_graph_info", "cc_query_create", "cc_query_create_ex",
           "cc_query_tree_info", "cc_query_destroy",
           "cc_query_info", "cc_query_plan", "cc_footprint", "cc_colors", "cc_count", "cc_count_static", "cc_count_colors",
           "cc_count_batch", "cc_server_create", "cc_server_add_graph", "cc_server_submit", "cc_server_poll",
           "cc_server_drain", "cc_server_destroy", "cc_last_tune_report", "cc_last_solve_stats", "cc_profile_enable", "cc_profile_read", "cc_probe_copy",
           "cc_status_str", "cc_last_error"]


class CCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]


class KernelStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("seconds", ctypes.c_double),
                ("bytes", ctypes.c_double), ("work", ctypes.c_uint64 * 3)]


class Tuning(ctypes.Structure):
    _fields_ = [("group_sources", ctypes.c_int32), ("trial_group", ctypes.c_int32),
                ("light_max_keys", ctypes.c_int32), ("use_graphs", ctypes.c_int32),
                ("dense_sources", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1602_04478_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    sig = {
        "cc_graph_create": [i64, vp, vp, ctypes.c_uint32, vp, P(vp)],
        "cc_graph_destroy": [vp],
        "cc_graph_info": [vp, P(i64), P(i64), P(i64)],
        "cc_query_create": [i32, i32, vp, P(vp)],
        "cc_query_create_ex": [i32, i32, vp, ctypes.c_uint32, i32, P(vp)],
        "cc_query_tree_info": [vp, P(i32), P(i32), P(i32)],
        "cc_query_destroy": [vp],
        "cc_query_info": [vp, P(u64), P(i32), P(i32)],
        "cc_query_plan": [vp, vp, i32, P(i32)],
        "cc_footprint": [vp, vp, i32, P(u64)],
        "cc_colors": [vp, i32, u64, i32, vp],
        "cc_count": [vp, vp, u64, i32, vp, vp, vp, vp, vp],
        "cc_count_static": [vp, vp, u64, i32, vp, vp, vp, vp, vp],
        "cc_count_colors": [vp, vp, i32, vp, vp, vp, vp, vp, vp],
        "cc_count_batch": [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp],
        "cc_server_create": [u64, i32, P(vp)],
        "cc_server_add_graph": [vp, vp, P(i32)],
        "cc_server_submit": [vp, i32, vp, u64, i32, P(u64)],
        "cc_server_poll": [vp, u64, P(i32), vp, vp, vp, vp],
        "cc_server_drain": [vp],
        "cc_server_destroy": [vp],
        "cc_profile_enable": [i32],
        "cc_profile_read": [vp, i32, P(i32)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.cc_status_str.argtypes = [ctypes.c_int]
    L.cc_status_str.restype = ctypes.c_char_p
    L.cc_last_error.argtypes = []
    L.cc_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(st: int):
    if st != 0:
        raise CCError(st, lib().cc_last_error().decode())


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


class Graph:
    """A data graph resident on the current device (cc_graph_create)."""

    def __init__(self, n: int, row_ptr, col, flags: int = 0, stream=None):
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        h = ctypes.c_void_p()
        _check(lib().cc_graph_create(n, _ptr(rp), _ptr(cl), flags, stream, ctypes.byref(h)))
        self.h = h
        self.n = n

    @classmethod
    def from_csr(cls, g, flags: int = 0):
        return cls(g.n, g.row_ptr, g.col, flags)

    def info(self):
        n, m, d = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().cc_graph_info(self.h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d)))
        return n.value, m.value, d.value

    def colors(self, k: int, seed: int, trial: int = 0) -> np.ndarray:
        out = np.empty(self.n, dtype=np.uint8)
        _check(lib().cc_colors(self.h, k, seed & (2**64 - 1), trial, _ptr(out)))
        return out

    def close(self):
        if self.h:
            _check(lib().cc_graph_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Query:
    """A planned query (cc_query_create)."""

    def __init__(self, k: int, edges, path_splitting: bool = False, tree: int = -1):
        """path_splitting: the PS baseline for every cycle block
        (cc_query_create_ex); tree: a tree index of the planner's
        enumeration (-1: the heuristic's choice)."""
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        h = ctypes.c_void_p()
        flags = CC_QUERY_PATH_SPLITTING if path_splitting else 0
        _check(lib().cc_query_create_ex(k, e.shape[0], _ptr(e), flags, tree, ctypes.byref(h)))
        self.h = h
        self.k = k

    def tree_info(self):
        t, nt, npk = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().cc_query_tree_info(self.h, ctypes.byref(t), ctypes.byref(nt), ctypes.byref(npk)))
        return dict(tree=t.value, num_trees=nt.value, pair_keyed_blocks=npk.value)

    def info(self):
        a, nb, lc = ctypes.c_uint64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().cc_query_info(self.h, ctypes.byref(a), ctypes.byref(nb), ctypes.byref(lc)))
        return dict(aut=a.value, num_blocks=nb.value, longest_cycle=lc.value)

    def plan(self):
        ln = ctypes.c_int32()
        _check(lib().cc_query_plan(self.h, None, 0, ctypes.byref(ln)))
        buf = np.zeros(ln.value, dtype=np.int32)
        _check(lib().cc_query_plan(self.h, _ptr(buf), ln.value, ctypes.byref(ln)))
        v = buf.tolist()
        nb = v[0]
        i = 1
        out = []
        kinds = {0: "leaf", 1: "cycle", 2: "root_cycle", 3: "root_single"}
        for _ in range(nb):
            kind, size, L = v[i:i + 3]
            i += 3
            nodes = v[i:i + L]
            i += L
            nbd = v[i]
            i += 1
            bd = v[i:i + nbd]
            i += nbd
            nch = v[i]
            i += 1
            ch = v[i:i + nch]
            i += nch
            out.append(dict(kind=kinds[kind], size=size, nodes=nodes, boundary=bd, children=ch))
        return out

    def close(self):
        if self.h:
            _check(lib().cc_query_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(g: Graph, q: Query, trials: int) -> int:
    b = ctypes.c_uint64()
    _check(lib().cc_footprint(g.h, q.h, trials, ctypes.byref(b)))
    return b.value


def count(g: Graph, q: Query, seed: int, trials: int = 1, stream=None):
    """cc_count: returns (counts u64[trials], overflow u8[trials], exact [int], estimate)."""
    counts = np.zeros(trials, dtype=np.uint64)
    ovf = np.zeros(trials, dtype=np.uint8)
    ex = (U128 * trials)()
    est = ctypes.c_double()
    _check(lib().cc_count(g.h, q.h, seed & (2**64 - 1), trials, _ptr(counts), _ptr(ovf), ex,
                          ctypes.byref(est), stream))
    exact = [e.lo | (e.hi << 64) for e in ex]
    return counts, ovf, exact, est.value


def count_static(g: Graph, q: Query, seed: int, trials: int = 1, stream=None):
    """cc_count_static: as count, with every device buffer carved from the
    library's static scratch (no device allocation)."""
    counts = np.zeros(trials, dtype=np.uint64)
    ovf = np.zeros(trials, dtype=np.uint8)
    ex = (U128 * trials)()
    est = ctypes.c_double()
    _check(lib().cc_count_static(g.h, q.h, seed & (2**64 - 1), trials, _ptr(counts), _ptr(ovf), ex,
                                 ctypes.byref(est), stream))
    exact = [e.lo | (e.hi << 64) for e in ex]
    return counts, ovf, exact, est.value


def count_colors(g: Graph, q: Query, colors: np.ndarray, per_source: bool = False, stream=None):
    """cc_count_colors: colours given (trials x n, original ids)."""
    c = np.ascontiguousarray(colors, dtype=np.uint8)
    if c.ndim == 1:
        c = c.reshape(1, -1)
    trials = c.shape[0]
    counts = np.zeros(trials, dtype=np.uint64)
    ovf = np.zeros(trials, dtype=np.uint8)
    ex = (U128 * trials)()
    per = (U128 * (trials * g.n))() if per_source else None
    _check(lib().cc_count_colors(g.h, q.h, trials, _ptr(c), _ptr(counts), _ptr(ovf), ex, per, stream))
    exact = [e.lo | (e.hi << 64) for e in ex]
    if per_source:
        ps = [[per[t * g.n + v].lo | (per[t * g.n + v].hi << 64) for v in range(g.n)] for t in range(trials)]
        return counts, ovf, exact, ps
    return counts, ovf, exact


def count_batch(g: Graph, queries, seeds, trials, tuning: dict | None = None, stream=None):
    nq = len(queries)
    qs = (ctypes.c_void_p * nq)(*[q.h.value for q in queries])
    sd = np.ascontiguousarray(np.asarray(seeds, dtype=np.uint64))
    tr = np.ascontiguousarray(np.asarray(trials, dtype=np.int32))
    tot = int(tr.sum())
    counts = np.zeros(tot, dtype=np.uint64)
    ovf = np.zeros(tot, dtype=np.uint8)
    est = np.zeros(nq, dtype=np.float64)
    tun = None
    if tuning:
        tun = Tuning(**{"group_sources": 0, "trial_group": 0, "light_max_keys": 0, "use_graphs": 1,
                        "dense_sources": -1, **tuning})
    _check(lib().cc_count_batch(g.h, nq, qs, _ptr(sd), _ptr(tr), _ptr(counts), _ptr(ovf), _ptr(est),
                                ctypes.byref(tun) if tun else None, stream))
    return counts, ovf, est


class TuneReport(ctypes.Structure):
    _fields_ = [("trial_group", ctypes.c_int32), ("candidates", ctypes.c_int32),
                ("tried_trial_group", ctypes.c_int32 * 8), ("tried_seconds_per_colouring", ctypes.c_double * 8),
                ("graph_replays", ctypes.c_uint64), ("dense_sources", ctypes.c_int32),
                ("tried_dense_sources", ctypes.c_int32 * 8), ("tree", ctypes.c_int32),
                ("trees_tried", ctypes.c_int32), ("tried_tree", ctypes.c_int32 * 8),
                ("tried_tree_seconds", ctypes.c_double * 8)]


def last_tune_report() -> dict:
    """What the calling thread's last count_batch chose (cc_last_tune_report)."""
    r = TuneReport()
    _check(lib().cc_last_tune_report(ctypes.byref(r)))
    n = min(r.candidates, 8)
    nt = min(r.trees_tried, 8)
    return {"trial_group": r.trial_group, "dense_sources": r.dense_sources, "graph_replays": int(r.graph_replays),
            "tree": r.tree, "trees": [(r.tried_tree[i], r.tried_tree_seconds[i]) for i in range(nt)],
            "tried": [(r.tried_trial_group[i], r.tried_dense_sources[i], r.tried_seconds_per_colouring[i])
                      for i in range(n)]}


class SolveStats(ctypes.Structure):
    _fields_ = [("sources", ctypes.c_int64), ("dense_sources", ctypes.c_int64), ("light_sources", ctypes.c_int64),
                ("handed_back", ctypes.c_int64), ("trial_group", ctypes.c_int32), ("group_sources", ctypes.c_int32)]


def last_solve_stats() -> dict:
    """How the calling thread's last counting call split the root block's
    sources over the tiers (cc_last_solve_stats)."""
    r = SolveStats()
    _check(lib().cc_last_solve_stats(ctypes.byref(r)))
    return {f: int(getattr(r, f)) for f, _ in SolveStats._fields_}


class Server:
    """The serving loop (cc_server_*)."""

    def __init__(self, hbm_budget_bytes: int = 0, max_inflight: int = 4):
        h = ctypes.c_void_p()
        _check(lib().cc_server_create(hbm_budget_bytes, max_inflight, ctypes.byref(h)))
        self.h = h

    def add_graph(self, g: Graph) -> int:
        gid = ctypes.c_int32()
        _check(lib().cc_server_add_graph(self.h, g.h, ctypes.byref(gid)))
        return gid.value

    def submit(self, graph_id: int, q: Query, seed: int, trials: int) -> int:
        t = ctypes.c_uint64()
        _check(lib().cc_server_submit(self.h, graph_id, q.h, seed & (2**64 - 1), trials, ctypes.byref(t)))
        return t.value

    def poll(self, ticket: int, trials: int):
        done = ctypes.c_int32()
        counts = np.zeros(trials, dtype=np.uint64)
        ovf = np.zeros(trials, dtype=np.uint8)
        est = ctypes.c_double()
        lat = ctypes.c_double()
        _check(lib().cc_server_poll(self.h, ticket, ctypes.byref(done), _ptr(counts), _ptr(ovf),
                                    ctypes.byref(est), ctypes.byref(lat)))
        if not done.value:
            return None
        return counts, ovf, est.value, lat.value

    def drain(self):
        _check(lib().cc_server_drain(self.h))

    def close(self):
        if self.h:
            _check(lib().cc_server_destroy(self.h))
            self.h = None


def probe_copy(nbytes: int, reps: int = 10) -> float:
    """GB/s (read + write) of a plain device copy of nbytes (cc_probe_copy)."""
    r = ctypes.c_double()
    _check(lib().cc_probe_copy(nbytes, reps, ctypes.byref(r)))
    return r.value


def profile_enable(level: int = 1):
    """0: off; 1: per-launch HIP-event timing; 2: timing and the kernels'
    algorithmic-byte counters; 3: event timing of the EdgeJoin launches only."""
    _check(lib().cc_profile_enable(int(level)))


def profile_take():
    """Read and reset per-kernel statistics:
    {name: (launches, seconds, algorithmic bytes, (scanned pairs, rows read, rows written))}."""
    cap = 256
    buf = (KernelStat * cap)()
    n = ctypes.c_int32()
    _check(lib().cc_profile_read(buf, cap, ctypes.byref(n)))
    return {buf[i].name.decode(): (int(buf[i].launches), float(buf[i].seconds), float(buf[i].bytes),
                                   tuple(int(x) for x in buf[i].work))
            for i in range(min(n.value, cap))}

