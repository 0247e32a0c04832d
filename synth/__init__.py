"""Seeded synthetic graph inputs shared by the tests, the benchmark and the
oracle's golden-value script.

Nothing here computes any part of the subgraph-counting method: the module only
draws simple undirected graphs (Erdos-Renyi, Chung-Lu power-law) and returns them
as symmetric CSR with rows sorted by vertex id.  The heavy lifting is in
``synth.c`` (splitmix64 streams keyed by seed and stream index, so the same
seed gives the same graph on every machine running this image).

Workload recipes (they stand in for the paper's Network-Repository/SNAP graphs,
which are power-law-like web, social and technology networks):

* ``er_small``          G(200, 0.05)
* ``chung_lu_1m``       n=1e6, gamma=2.1, mean degree 20, max expected degree 1e4
* ``chung_lu_4m``       n=4e6, gamma=1.9, mean degree 40, max expected degree 5e4
* ``batch_specs``       10,000 graphs, n log-uniform in [20, 2000], half ER
                        (mean degree U[4,30]), half Chung-Lu (gamma U[2.0,2.8],
                        mean degree U[4,30], d_max = min(n-1, floor(sqrt(d_bar n))))
* ``request_specs``     n log-uniform in [50, 5e4], Chung-Lu gamma U[2.0,2.5],
                        mean degree U[8,32], same d_max rule
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``synth.c`` into ``libsynth.so`` (plain gcc, host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P64 = ctypes.POINTER(ctypes.POINTER(ctypes.c_int64))
        P32 = ctypes.POINTER(ctypes.POINTER(ctypes.c_int32))
        lib.synth_er.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, P64, P32]
        lib.synth_er.restype = ctypes.c_int64
        lib.synth_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_uint64, P64, P32]
        lib.synth_chung_lu.restype = ctypes.c_int64
        lib.synth_mix.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.synth_mix.restype = ctypes.c_uint64
        lib.synth_free.argtypes = [ctypes.c_void_p]
        lib.synth_free.restype = None
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Simple undirected graph as symmetric CSR (int32 offsets and ids)."""
    n: int
    row_ptr: np.ndarray   # int32, n+1
    col: np.ndarray       # int32, 2m, each row sorted ascending
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)


def _take(n, m, rp, col, name):
    if m < 0:
        raise MemoryError("synthetic graph generation failed")
    row_ptr = np.ctypeslib.as_array(rp, shape=(n + 1,)).astype(np.int64)
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("graph too large for int32 CSR offsets")
    out_rp = row_ptr.astype(np.int32)
    if m > 0:
        out_col = np.ctypeslib.as_array(col, shape=(2 * m,)).astype(np.int32)
    else:
        out_col = np.zeros(0, dtype=np.int32)
    lib = _load()
    lib.synth_free(ctypes.cast(rp, ctypes.c_void_p))
    lib.synth_free(ctypes.cast(col, ctypes.c_void_p))
    return Graph(n, out_rp, out_col, name)


def mix(seed: int, index: int) -> int:
    """splitmix64-derived child seed for item ``index`` of stream ``seed``."""
    return int(_load().synth_mix(ctypes.c_uint64(seed & (2**64 - 1)), ctypes.c_uint64(index)))


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    lib = _load()
    rp = ctypes.POINTER(ctypes.c_int64)()
    col = ctypes.POINTER(ctypes.c_int32)()
    m = lib.synth_er(n, p, seed & (2**64 - 1), ctypes.byref(rp), ctypes.byref(col))
    return _take(n, m, rp, col, f"er(n={n},p={p},seed={seed})")


def chung_lu(n: int, gamma: float, dbar: float, dmax: float, seed: int) -> Graph:
    lib = _load()
    rp = ctypes.POINTER(ctypes.c_int64)()
    col = ctypes.POINTER(ctypes.c_int32)()
    m = lib.synth_chung_lu(n, gamma, dbar, dmax, seed & (2**64 - 1), ctypes.byref(rp), ctypes.byref(col))
    return _take(n, m, rp, col, f"chung_lu(n={n},gamma={gamma},dbar={dbar},dmax={dmax},seed={seed})")


def from_edges(n: int, edges, name: str = "") -> Graph:
    """Symmetric sorted CSR from an iterable of undirected (u, v) pairs.
    Self-loops and duplicates are dropped (used for hand-built special graphs)."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        u, v = int(u), int(v)
        if u == v:
            continue
        adj[u].add(v)
        adj[v].add(u)
    rp = np.zeros(n + 1, dtype=np.int64)
    for i in range(n):
        rp[i + 1] = rp[i] + len(adj[i])
    col = np.zeros(int(rp[-1]), dtype=np.int32)
    for i in range(n):
        col[rp[i]:rp[i + 1]] = sorted(adj[i])
    return Graph(n, rp.astype(np.int32), col, name)


# ---- named workloads -------------------------------------------------------

def er_small(seed: int = 0) -> Graph:
    """G(n=200, p=0.05)."""
    return erdos_renyi(200, 0.05, seed)


def chung_lu_1m(seed: int = 0) -> Graph:
    """Chung-Lu, n=1e6, gamma=2.1, mean degree 20, max expected degree 1e4."""
    return chung_lu(1_000_000, 2.1, 20.0, 10_000.0, seed)


def chung_lu_4m(seed: int = 0) -> Graph:
    """Chung-Lu, n=4e6, gamma=1.9, mean degree 40, max expected degree 5e4."""
    return chung_lu(4_000_000, 1.9, 40.0, 50_000.0, seed)


def _u(seed: int, idx: int, k: int) -> float:
    """k-th uniform in [0,1) for item idx, from the splitmix64 stream."""
    return (mix(mix(seed, idx), k) >> 11) * (1.0 / 9007199254740992.0)


def batch_specs(count: int = 10_000, seed: int = 0):
    """Per-graph recipes for the batched workload (see module docstring)."""
    specs = []
    for g in range(count):
        n = int(round(math.exp(math.log(20) + _u(seed, g, 0) * (math.log(2000) - math.log(20)))))
        dbar = 4.0 + 26.0 * _u(seed, g, 1)
        gseed = mix(seed, g)
        if g % 2 == 0:
            p = min(1.0, dbar / max(1, n - 1))
            specs.append(("er", n, p, gseed))
        else:
            gamma = 2.0 + 0.8 * _u(seed, g, 2)
            dmax = float(min(n - 1, math.floor(math.sqrt(dbar * n))))
            specs.append(("cl", n, gamma, min(dbar, dmax), dmax, gseed))
    return specs


def request_specs(count: int, seed: int = 0):
    """Per-request recipes for the serving workload (see module docstring)."""
    specs = []
    for r in range(count):
        n = int(round(math.exp(math.log(50) + _u(seed, r, 0) * (math.log(50_000) - math.log(50)))))
        dbar = 8.0 + 24.0 * _u(seed, r, 1)
        gamma = 2.0 + 0.5 * _u(seed, r, 2)
        dmax = float(min(n - 1, math.floor(math.sqrt(dbar * n))))
        specs.append(("cl", n, gamma, min(dbar, dmax), dmax, mix(seed, r)))
    return specs


def from_spec(spec) -> Graph:
    if spec[0] == "er":
        _, n, p, s = spec
        return erdos_renyi(n, p, s)
    _, n, gamma, dbar, dmax, s = spec
    return chung_lu(n, gamma, dbar, dmax, s)
