"""CPU oracle for colourful subgraph counting -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares nothing with the device library.

Three independent ways to the same exact number (Preliminaries: the number
of colourful matches of a query Q with k nodes in a data graph G under a
colouring chi with k colours):

* ``brute``          -- enumeration of matches (the definition), in C.
* ``incl_excl``      -- inclusion-exclusion over colour subsets of
                        homomorphism counts, pure Python integers.  A map that
                        uses all k colours with k query nodes is a bijection
                        onto the colours, hence injective, so
                        N = sum_{S subset K} (-1)^(k-|S|) hom(Q, G[chi^-1(S)]).
                        hom is computed by eliminating query nodes of degree
                        <= 2 (every treewidth-2 graph has one), each
                        elimination being a sum over one data vertex of a
                        product of vector/matrix factors.
* ``db``             -- the paper's degree-based dynamic program (Sections
                        4.1-5.2), in C, with 128-bit counts.

``colours`` implements the colouring contract: for trial t,
chi_t(v) = ((mix(mix(seed + t) XOR v) >> 32) * k) >> 32, mix = splitmix64's
output function.  ``mix64`` is written again here, in Python, so that the C
and Python versions check each other.
"""
from __future__ import annotations

import ctypes
import itertools
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "cc_oracle.cpp")
_lib = None


def build() -> str:
    """Compile the C part of the oracle (g++, OpenMP)."""
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", "-o", _LIB_PATH, _SRC]
    subprocess.run(cmd, check=True)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(ctypes.c_int32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.orc_mix64.restype = ctypes.c_uint64
        L.orc_mix64.argtypes = [ctypes.c_uint64]
        L.orc_colours.restype = None
        L.orc_colours.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, u8p]
        L.orc_brute.restype = ctypes.c_int
        L.orc_brute.argtypes = [ctypes.c_int64, i64p, i32p, u8p, ctypes.c_int, ctypes.c_int, i32p, u64p]
        L.orc_plan.restype = ctypes.c_int
        L.orc_plan.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int, i32p, ctypes.c_int]
        L.orc_db.restype = ctypes.c_int
        L.orc_db.argtypes = [ctypes.c_int64, i64p, i32p, u8p, ctypes.c_int, ctypes.c_int, i32p,
                             ctypes.c_int, i64p, ctypes.c_int64, u64p, u64p]
        L.orc_db_flagged.restype = ctypes.c_int
        L.orc_db_flagged.argtypes = [ctypes.c_int64, i64p, i32p, u8p, ctypes.c_int, ctypes.c_int, i32p,
                                     ctypes.c_int, u64p]
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _u128(out) -> int:
    return int(out[0]) | (int(out[1]) << 64)


MASK64 = (1 << 64) - 1


def mix64(x: int) -> int:
    """splitmix64 output function (Vigna): add the golden-ratio increment,
    then two xor-shift-multiply rounds and a final xor-shift."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def colours(n: int, k: int, seed: int, trial: int = 0) -> np.ndarray:
    """Colouring contract, evaluated in C (vector) -- see module docstring."""
    out = np.empty(n, dtype=np.uint8)
    lib().orc_colours(n, k, seed & MASK64, trial, _p(out, ctypes.c_uint8))
    return out


def colours_py(n: int, k: int, seed: int, trial: int = 0) -> np.ndarray:
    key = mix64((seed + trial) & MASK64)
    return np.array([((mix64(key ^ v) >> 32) * k) >> 32 for v in range(n)], dtype=np.uint8)


def _qe(edges) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))


def brute(g, k: int, edges, chi: np.ndarray | None) -> int:
    """Number of colourful matches (chi given) or of all matches (chi None)."""
    qe = _qe(edges)
    out = np.zeros(2, dtype=np.uint64)
    rc = lib().orc_brute(g.n, _p(g.row_ptr, ctypes.c_int64), _p(g.col, ctypes.c_int32),
                         _p(chi, ctypes.c_uint8) if chi is not None else None,
                         k, qe.shape[0], _p(qe, ctypes.c_int32), _p(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("oracle brute force rejected the query")
    return _u128(out)


def db(g, k: int, edges, chi: np.ndarray, reverse_ties: bool = True, sources=None):
    """The paper's DB dynamic program.  Returns the exact colourful count, or
    (count over the given root sources, per-source counts) when ``sources``
    is given."""
    qe = _qe(edges)
    out = np.zeros(2, dtype=np.uint64)
    if sources is None:
        rc = lib().orc_db(g.n, _p(g.row_ptr, ctypes.c_int64), _p(g.col, ctypes.c_int32),
                          _p(chi, ctypes.c_uint8), k, qe.shape[0], _p(qe, ctypes.c_int32),
                          int(reverse_ties), None, 0, None, _p(out, ctypes.c_uint64))
        if rc != 0:
            raise ValueError("oracle DB rejected the query")
        return _u128(out)
    src = np.ascontiguousarray(np.asarray(sources, dtype=np.int64))
    per = np.zeros(2 * src.size, dtype=np.uint64)
    rc = lib().orc_db(g.n, _p(g.row_ptr, ctypes.c_int64), _p(g.col, ctypes.c_int32),
                      _p(chi, ctypes.c_uint8), k, qe.shape[0], _p(qe, ctypes.c_int32),
                      int(reverse_ties), _p(src, ctypes.c_int64), src.size,
                      _p(per, ctypes.c_uint64), _p(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("oracle DB rejected the query")
    vals = [int(per[2 * i]) | (int(per[2 * i + 1]) << 64) for i in range(src.size)]
    return _u128(out), vals


def db_flagged(g, k: int, edges, chi: np.ndarray, reverse_ties: bool = True):
    """The DB count with the 64-bit width check of the tables: returns
    (exact count, flag), flag = some entry of a child block's table (colourful
    matches of the block's subquery keyed by its boundary images) does not fit
    in 64 bits."""
    qe = _qe(edges)
    out = np.zeros(3, dtype=np.uint64)
    rc = lib().orc_db_flagged(g.n, _p(g.row_ptr, ctypes.c_int64), _p(g.col, ctypes.c_int32),
                              _p(chi, ctypes.c_uint8), k, qe.shape[0], _p(qe, ctypes.c_int32),
                              int(reverse_ties), _p(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError("oracle DB rejected the query")
    return _u128(out), bool(out[2])


def plan(k: int, edges, order=None):
    """The oracle's own decomposition tree, as a list of dicts.  ``order``
    optionally forces the sequence of node sets to contract."""
    qe = _qe(edges)
    buf = np.zeros(4096, dtype=np.int32)
    flat = []
    for s in (order or []):
        flat.append(len(s))
        flat.extend(int(x) for x in s)
    fo = np.ascontiguousarray(np.asarray(flat, dtype=np.int32))
    r = lib().orc_plan(k, qe.shape[0], _p(qe, ctypes.c_int32),
                       _p(fo, ctypes.c_int32) if flat else None, len(flat),
                       _p(buf, ctypes.c_int32), buf.size)
    if r < 0:
        raise ValueError("query has treewidth > 2 or is malformed")
    v = buf[:r].tolist()
    nb, root, single = v[0], v[1], v[2]
    i = 3
    blocks = []
    for _ in range(nb):
        kind, isroot, size, L = v[i:i + 4]
        i += 4
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
        blocks.append(dict(kind="leaf" if kind == 0 else "cycle", root=bool(isroot), size=size,
                           nodes=nodes, boundary=bd, children=ch))
    return dict(blocks=blocks, root_block=root, root_single_child=single)


# ------------------------------------------------------------------ O2
def _hom(k: int, edges, adj_sets) -> int:
    """hom(Q, H) for a treewidth <= 2 query Q by node elimination.

    ``adj_sets[x]`` is the neighbour set of data vertex x in H (vertices are
    0..n-1).  Factors are dicts: () -> int, (a,) -> vector, (a, b) -> matrix
    (lists of Python ints).  Eliminating query node x multiplies every factor
    that mentions x and sums over x's image; with at most two other query
    nodes left in those factors the result is again a scalar, vector or
    matrix."""
    n = len(adj_sets)
    A = [[1 if j in adj_sets[i] else 0 for j in range(n)] for i in range(n)]
    factors = []  # (scope tuple, table)
    for a, b in edges:
        factors.append(((a, b), A))
    remaining = set(range(k))
    while remaining:
        # pick a node whose elimination touches <= 2 other nodes
        best = None
        for x in sorted(remaining):
            nb = set()
            for sc, _ in factors:
                if x in sc:
                    nb.update(s for s in sc if s != x)
            if len(nb) <= 2:
                best = (x, sorted(nb))
                break
        if best is None:
            raise ValueError("query treewidth > 2")
        x, nb = best
        mine = [(sc, t) for sc, t in factors if x in sc]
        factors = [(sc, t) for sc, t in factors if x not in sc]

        def val(sc, t, asg):
            if len(sc) == 0:
                return t
            if len(sc) == 1:
                return t[asg[sc[0]]]
            return t[asg[sc[0]]][asg[sc[1]]]

        if len(nb) == 0:
            out = 0
            for vx in range(n):
                p = 1
                for sc, t in mine:
                    p *= val(sc, t, {x: vx})
                out += p
            factors.append(((), out))
        elif len(nb) == 1:
            y = nb[0]
            out = [0] * n
            for vy in range(n):
                s = 0
                for vx in range(n):
                    p = 1
                    for sc, t in mine:
                        p *= val(sc, t, {x: vx, y: vy})
                        if p == 0:
                            break
                    s += p
                out[vy] = s
            factors.append(((y,), out))
        else:
            y, z = nb
            out = [[0] * n for _ in range(n)]
            for vx in range(n):
                for vy in range(n):
                    for vz in range(n):
                        p = 1
                        for sc, t in mine:
                            p *= val(sc, t, {x: vx, y: vy, z: vz})
                            if p == 0:
                                break
                        out[vy][vz] += p
            factors.append(((y, z), out))
        remaining.discard(x)
    total = 1
    for sc, t in factors:
        assert sc == ()
        total *= t
    return total


def incl_excl(g, k: int, edges, chi: np.ndarray) -> int:
    """Colourful matches by inclusion-exclusion over colour subsets (small n)."""
    n = g.n
    nbrs = [set(int(x) for x in g.neighbors(v)) for v in range(n)]
    total = 0
    for r in range(k + 1):
        for S in itertools.combinations(range(k), r):
            keep = [v for v in range(n) if int(chi[v]) in S]
            idx = {v: i for i, v in enumerate(keep)}
            sub = [set(idx[w] for w in nbrs[v] if w in idx) for v in keep]
            h = _hom(k, edges, sub) if keep else 0
            total += (-1) ** (k - r) * h
    return total


def threads() -> int:
    return int(lib().orc_threads())
