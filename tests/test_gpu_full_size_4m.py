"""The 4M-vertex Chung-Lu graph (exponent 1.9, mean degree 40, max expected
degree 5e4, seed 0: 7.65e7 edges, 9.2e9 triangles) at full size, 4-vertex
counts: the 11 counts sum to C(n,4), and per-vertex / per-edge fragment
counts on sampled vertices and edges (hubs included) equal their definitions
recomputed one by one.  Its per-arc triangle lists hold 5.5e10 entries, so
they are kept in the compact layout (arc positions only).
"""
import random
from math import comb

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

SMALL = 300   # k4 / c4 / vertex triangles are recomputed only around vertices below this degree


def test_chung_lu_4m_four_vertex_full_size():
    import paper_1610_09411_amd as esc
    g = synth.chung_lu_4m(0)
    print("chung_lu_4m", g.n, g.m, flush=True)
    ctx = esc.Context(0)
    try:
        counts, fr = ctx.fragments(g, 4)
        work = ctx.last_work()
    finally:
        ctx.close()
    print("counted; checking samples", flush=True)
    assert sum(counts) == comb(g.n, 4)
    assert work["m"] == g.m
    deg = g.degrees()
    assert int(fr["tri_v"].sum()) == 3 * work["T"]
    rng = random.Random(4)
    hubs = [int(v) for v in np.argsort(-deg)[:4]]
    verts = hubs + [rng.randrange(g.n) for _ in range(24)]
    checked = 0
    for v in verts:
        s, t = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
        if t == s:
            continue
        for p in [s, t - 1] + [rng.randrange(s, t) for _ in range(2)]:
            u = int(g.col[p])
            nu, nv = g.col[g.row_ptr[u]:g.row_ptr[u + 1]], g.col[s:t]
            assert fr["tri_e"][p] == len(np.intersect1d(nu, nv, assume_unique=True)), (v, u)
            if deg[v] < SMALL and deg[u] < SMALL:
                exp = oracle.edge_fragments(g, v, u)
                assert fr["k4_e"][p] == exp["k4"], (v, u)
                assert fr["c4_e"][p] == exp["c4"], (v, u)
                checked += 1
        if deg[v] < SMALL:
            assert fr["tri_v"][v] == oracle.vertex_triangles(g, v)
        print("vertex", v, "degree", int(deg[v]), "ok", flush=True)
    assert checked > 20
