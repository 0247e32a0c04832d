"""ORACLE -- TEST INFRASTRUCTURE ONLY.

Plain CPU implementation of exact induced 4- and 5-vertex subgraph counting,
following Pinar, Seshadhri and Vishal, "ESCAPE: Efficiently Counting All
5-Vertex Subgraphs" (arXiv 1610.09411).  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import this package.  It shares no code
with the GPU library.

* ``escape_oracle.c`` -- the paper's enumeration and cut-formula sums (Secs. 4-6),
  integer exact (uint64 per item, 128-bit sums).
* ``brute.c``         -- the plain definition: classify every k-subset.
* ``patterns.py``     -- pattern drawings, isomorphism classes, the matrix A
  (Appendix B) and the disconnected-pattern inclusion-exclusion (Appendix A).

Functions that no test pins to something other than themselves are marked
"parity unpinned"; at present every exported count is pinned (brute force on
small graphs, textbook closed forms, the paper's printed matrices).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import patterns as pat

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, "escape_oracle.c"), os.path.join(_HERE, "brute.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

# Names of the 128-bit sums exported by escape_oracle.c, in order.
SUM_NAMES = [
    "n", "m", "W", "T", "TT", "D", "C4", "K4", "sum_C(d,3)", "sum_e(d-1)(d-1)",
    "N1", "N2", "N3", "N4", "N5", "N6", "N7", "N8", "N9", "N10",
    "N11", "N12", "N13", "N14", "N15", "N16", "N17", "N18", "N19", "N20", "N21",
    "DP", "DBP",
]


def build(force: bool = False) -> str:
    newest = max(os.path.getmtime(s) for s in _SRCS)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp] + _SRCS)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.oracle_run.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int, vp, ctypes.c_int, vp,
                                   vp, vp, vp, vp, vp, vp, ctypes.c_int, vp]
        lib.oracle_run.restype = ctypes.c_int
        lib.oracle_num_sums.restype = ctypes.c_int
        lib.oracle_set_sample_offset.argtypes = [ctypes.c_int]
        lib.oracle_set_sample_offset.restype = None
        lib.brute_count.argtypes = [ctypes.c_int32, vp, vp, ctypes.c_int, vp, ctypes.c_int,
                                    ctypes.c_int, vp]
        lib.brute_count.restype = ctypes.c_int
        assert lib.oracle_num_sums() == len(SUM_NAMES)
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _csr(graph):
    rp = np.ascontiguousarray(graph.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(graph.col, dtype=np.int32)
    return rp, ci


def sums(graph, k=5, order_rank=None, threads=0, per_item=False):
    """Run the enumeration stage.  Returns {name: int} and, with per_item, the
    per-vertex arrays t, C4, K4 and per-arc (input CSR order) arrays t(e),
    C4(e), K4(e)."""
    lib = _load()
    rp, ci = _csr(graph)
    n = graph.n
    out = np.zeros(2 * len(SUM_NAMES), dtype=np.uint64)
    rank = None if order_rank is None else np.ascontiguousarray(order_rank, dtype=np.int64)
    items = None
    if per_item:
        items = [np.zeros(n, np.uint64) for _ in range(3)] + [np.zeros(len(ci), np.uint64) for _ in range(3)]
    args = [_ptr(x) for x in items] if items else [None] * 6
    rc = lib.oracle_run(n, _ptr(rp), _ptr(ci), k, _ptr(rank), threads, _ptr(out), *args, 1, None)
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    S = {name: int(out[2 * i]) | (int(out[2 * i + 1]) << 64) for i, name in enumerate(SUM_NAMES)}
    if per_item:
        keys = ["t_v", "c4_v", "k4_v", "t_e", "c4_e", "k4_e"]
        return S, dict(zip(keys, items))
    return S


def _connected_counter(S, N4):
    """Unlabeled non-induced counts of connected patterns with <= 4 vertices,
    keyed by (k, canonical mask)."""
    table = {
        (1, 0): S["n"],
        (2, pat.canon(2, 1)): S["m"],
        (3, pat.canon(3, pat.mask_of(3, [(1, 2), (1, 3)]))): S["W"],
        (3, pat.canon(3, pat.mask_of(3, [(1, 2), (1, 3), (2, 3)]))): S["T"],
    }
    for i, (_, edges) in enumerate(pat.FOUR_CONNECTED):
        table[(4, pat.canon(4, pat.mask_of(4, edges)))] = N4[i]

    def count(k, cmask):
        return table[(k, cmask)]
    return count


def noninduced_from_sums(S, k):
    """Non-induced counts of all k-vertex patterns, in output order.
    Connected 4-vertex (Thm 4vertex-easy, Thm 4cycle, Thm 4clique):
      3-stars = sum C(d,3); 3-paths = sum_e (d(u)-1)(d(v)-1) - 3T;
      tailed triangles = TT; 4-cycles = C4; diamonds = D; 4-cliques = K4.
    Connected 5-vertex: N1..N21 as summed by escape_oracle.c.
    Disconnected: Appendix A inclusion-exclusion."""
    N4 = [S["sum_C(d,3)"], S["sum_e(d-1)(d-1)"] - 3 * S["T"], S["TT"], S["C4"], S["D"], S["K4"]]
    count = _connected_counter(S, N4)
    if k == 4:
        N = list(N4)
        for idx in range(len(pat.FOUR_CONNECTED), len(pat.FOUR)):
            N.append(pat.noninduced_disconnected(4, idx, count))
        return N
    N = [S["N%d" % i] for i in range(1, 22)]
    for idx in range(len(pat.FIVE_CONNECTED), len(pat.FIVE)):
        N.append(pat.noninduced_disconnected(5, idx, count))
    return N


def count(graph, k=5, order_rank=None, threads=0):
    """Induced counts: 11 values for k=4, 45 values (11 four-vertex followed by
    34 five-vertex) for k=5, as Python ints."""
    S = sums(graph, k, order_rank, threads)
    C4 = pat.induced_from_noninduced(4, noninduced_from_sums(S, 4))
    if k == 4:
        return C4
    C5 = pat.induced_from_noninduced(5, noninduced_from_sums(S, 5))
    return C4 + C5


def timed_sample(graph, k=5, sample=64, threads=0, offset=0):
    """Time the oracle on a sample of its own work: the degree order, triangle
    stage and triangle lists run in full; every later loop visits only sources
    and edges whose id plus `offset` is a multiple of `sample` (ids are a
    seeded shuffle, so this is a uniform sample).  Returns (setup_seconds,
    sampled_seconds); the counts of such a run are not meaningful and are not
    returned."""
    lib = _load()
    lib.oracle_set_sample_offset(int(offset) % max(1, int(sample)))
    rp, ci = _csr(graph)
    out = np.zeros(2 * len(SUM_NAMES), dtype=np.uint64)
    secs = np.zeros(2, dtype=np.float64)
    rc = lib.oracle_run(graph.n, _ptr(rp), _ptr(ci), k, None, threads, _ptr(out), *([None] * 6),
                        int(sample), _ptr(secs))
    lib.oracle_set_sample_offset(0)
    if rc != 0:
        raise MemoryError("oracle allocation failed")
    return float(secs[0]), float(secs[1])


def brute(graph, k, threads=0):
    """Induced counts of all k-vertex patterns by classifying every k-subset
    (k = 3: [empty, one edge, wedge, triangle])."""
    lib = _load()
    rp, ci = _csr(graph)
    lut = np.array(pat.class_lut(k), dtype=np.int32)
    ncls = 4 if k == 3 else len(pat.patterns(k))
    out = np.zeros(ncls, dtype=np.uint64)
    rc = lib.brute_count(graph.n, _ptr(rp), _ptr(ci), k, _ptr(lut), ncls, threads, _ptr(out))
    if rc != 0:
        raise ValueError("brute force supports n <= 4096")
    return [int(x) for x in out]


# ------------------------------------------------------------------ one by one
# Single-item fragment counts written out from their definitions; used to
# check sampled outputs on graphs too large for the full oracle in a test.

def _row(graph, v):
    return graph.col[graph.row_ptr[v]:graph.row_ptr[v + 1]]


def edge_fragments(graph, u, v):
    """For edge {u,v}: t = triangles on it (common neighbours), k4 = 4-cliques
    on it (edges inside the common neighbourhood), c4 = 4-cycles through it
    (sum over j in N(v)-u of |N(u) & N(j)| - 1)."""
    nu, nv = _row(graph, u), _row(graph, v)
    common = np.intersect1d(nu, nv, assume_unique=True)
    k4 = 0
    for x in common:
        k4 += len(np.intersect1d(_row(graph, int(x)), common, assume_unique=True))
    c4 = 0
    for j in nv:
        j = int(j)
        if j == u:
            continue
        c4 += len(np.intersect1d(nu, _row(graph, j), assume_unique=True)) - 1
    return {"t": len(common), "k4": k4 // 2, "c4": c4}


def vertex_triangles(graph, v):
    """Triangles through v = edges inside N(v)."""
    nv = _row(graph, v)
    s = 0
    for x in nv:
        s += len(np.intersect1d(_row(graph, int(x)), nv, assume_unique=True))
    return s // 2


def three_vertex_brute(graph):
    """Induced 3-vertex counts by definition: classify every 3-subset by its
    number of edges.  [no edge, one edge, path, triangle].  Small graphs only."""
    n = graph.n
    adj = [set(int(x) for x in graph.col[graph.row_ptr[v]:graph.row_ptr[v + 1]]) for v in range(n)]
    out = [0, 0, 0, 0]
    for a in range(n):
        for b in range(a + 1, n):
            ab = b in adj[a]
            for c in range(b + 1, n):
                out[int(ab) + int(c in adj[a]) + int(c in adj[b])] += 1
    return out


def three_vertex(graph):
    """Induced 3-vertex counts from the oracle's triangle and wedge totals
    (the method's 3-vertex by-products): triangles T, paths W - 3T, one-edge
    sets m (n-2) - 2 (W - 3T) - 3T, and the rest of the C(n,3) sets.  Pinned
    to three_vertex_brute in the CPU tests."""
    S = sums(graph, 4)
    n, m, W, T = S["n"], S["m"], S["W"], S["T"]
    P3 = W - 3 * T
    E1 = m * (n - 2) - 2 * P3 - 3 * T if n >= 2 else 0
    from math import comb
    return [comb(n, 3) - E1 - P3 - T, E1, P3, T]
