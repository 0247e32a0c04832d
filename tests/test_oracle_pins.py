"""Pins for the CPU oracle (no GPU).

The oracle (oracle/) is checked against things that do not come from itself:
the paper's printed matrices, the plain definition (classify every k-subset),
textbook closed forms, trace formulas for cycle counts, per-item counts written
out from their definitions with numpy, and invariants (sums over items, sum of
all induced counts = C(n,k), independence of the vertex order).
"""
import os
import random
from math import comb

import numpy as np
import pytest

import oracle
import synth
from oracle import patterns as pat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_matrix(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            rows.append([int(x) for x in line.split()])
    return rows


# ------------------------------------------------------------ pattern library

def test_number_of_isomorphism_classes():
    # there are 11 graphs on 4 vertices and 34 on 5 (up to isomorphism)
    assert len(set(pat.canon(4, m) for m in range(1 << 6))) == 11
    assert len(set(pat.canon(5, m) for m in range(1 << 10))) == 34
    assert sorted(set(pat.class_lut(4))) == list(range(11))
    assert sorted(set(pat.class_lut(5))) == list(range(34))


def test_connectivity_of_drawings():
    for _, e in pat.FOUR_CONNECTED:
        assert pat.is_connected(4, e)
    for _, e in pat.FOUR_DISCONNECTED:
        assert not pat.is_connected(4, e)
    for _, e in pat.FIVE_CONNECTED:
        assert pat.is_connected(5, e)
    for _, e in pat.FIVE_DISCONNECTED:
        assert not pat.is_connected(5, e)


def test_matrix_A_equals_paper_fig_A():
    paper = _read_matrix("paper_fig_A.txt")
    A = pat.a_matrix(5)
    assert [list(r[:21]) for r in A[:21]] == paper


def test_matrix_Ainv_equals_paper_fig_Ainv():
    paper = _read_matrix("paper_fig_Ainv.txt")
    Ai = pat.a_inverse(5)
    assert [list(r[:21]) for r in Ai[:21]] == paper


@pytest.mark.parametrize("k", [4, 5])
def test_inverse_sign_rule(k):
    A = pat.a_matrix(k)
    Ai = pat.a_inverse(k)
    n = len(A)
    for i in range(n):
        for j in range(n):
            s = (-1) ** (pat.edge_count(k, j) - pat.edge_count(k, i))
            assert Ai[i][j] == s * A[i][j]


def test_clique_columns_are_textbook_copy_counts():
    A4 = pat.a_matrix(4)
    # copies inside K4: 3-stars 4, 3-paths 4!/2, tailed triangles 12, 4-cycles 3, diamonds 6
    assert [A4[i][5] for i in range(6)] == [4, 12, 12, 3, 6, 1]
    A5 = pat.a_matrix(5)
    # inside K5: 4-stars 5, 5-cycles 4!/2, K_{2,3} C(5,2), wheels 5*3, K4+pendant 5*4
    assert A5[0][20] == 5 and A5[7][20] == 12 and A5[12][20] == 10
    assert A5[17][20] == 15 and A5[14][20] == 20 and A5[20][20] == 1


# ---------------------------------------------------- brute force vs closed forms

def _induced(g, k):
    return oracle.brute(g, k)


def test_brute_empty_and_complete():
    for n in (4, 7, 10):
        empty = synth.from_edges(n, [])
        full = synth.from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
        b4, b5 = _induced(empty, 4), _induced(empty, 5)
        assert b4[6] == comb(n, 4) and sum(b4) == comb(n, 4)
        assert b5[21] == comb(n, 5) and sum(b5) == comb(n, 5)
        c4, c5 = _induced(full, 4), _induced(full, 5)
        assert c4[5] == comb(n, 4) and sum(c4) == comb(n, 4)
        assert c5[20] == comb(n, 5) and sum(c5) == comb(n, 5)


def test_brute_star_cycle_bipartite():
    n = 9
    star = synth.from_edges(n, [(0, v) for v in range(1, n)])
    b4, b5 = _induced(star, 4), _induced(star, 5)
    assert b4[0] == comb(n - 1, 3) and b4[6] == comb(n - 1, 4)
    assert b5[0] == comb(n - 1, 4) and b5[21] == comb(n - 1, 5)
    for n in (5, 11):
        cyc = synth.from_edges(n, [(i, (i + 1) % n) for i in range(n)])
        b5 = _induced(cyc, 5)
        if n == 5:
            assert b5[7] == 1
        else:
            assert b5[2] == n            # induced paths on 5 vertices
        b4 = _induced(cyc, 4)
        if n > 5:
            assert b4[1] == n            # induced 3-paths
    for a, b in ((3, 4), (4, 5), (2, 6)):
        kab = synth.from_edges(a + b, [(u, a + v) for u in range(a) for v in range(b)])
        b4, b5 = _induced(kab, 4), _induced(kab, 5)
        assert b4[3] == comb(a, 2) * comb(b, 2)
        assert b4[0] == a * comb(b, 3) + b * comb(a, 3)
        assert b5[12] == comb(a, 2) * comb(b, 3) + comb(a, 3) * comb(b, 2)
        assert b5[0] == a * comb(b, 4) + b * comb(a, 4)


def test_brute_three_vertex_matches_adjacency_powers():
    g = synth.erdos_renyi(25, 0.3, 7)
    A = _dense(g)
    tri = int(np.trace(A @ A @ A)) // 6
    d = A.sum(1)
    wedges = int(sum(x * (x - 1) // 2 for x in d))
    b3 = oracle.brute(g, 3)
    assert b3[3] == tri
    assert b3[2] == wedges - 3 * tri
    assert sum(b3) == comb(25, 3)


# --------------------------------------------------------- oracle vs definition

def _dense(g):
    A = np.zeros((g.n, g.n), dtype=np.int64)
    for u in range(g.n):
        A[u, g.col[g.row_ptr[u]:g.row_ptr[u + 1]]] = 1
    return A


def _random_graphs():
    out = []
    for s in range(24):
        out.append(synth.erdos_renyi(10 + s % 9, 0.15 + 0.04 * (s % 12), 100 + s))
    for s in range(16):
        out.append(synth.chung_lu(16 + s % 8, 2.0 + 0.1 * (s % 5), 4.0 + (s % 4), 12.0, 200 + s))
    # dense and hub-heavy shapes
    out.append(synth.erdos_renyi(14, 0.85, 5))
    out.append(synth.from_edges(13, [(0, v) for v in range(1, 13)] + [(v, v + 1) for v in range(1, 12)]))  # wheel-like fan
    out.append(synth.from_edges(10, [(u, v) for u in range(5) for v in range(u + 1, 10)]))  # split graph
    return out


@pytest.mark.parametrize("g", _random_graphs(), ids=lambda g: g.name or "special")
def test_oracle_equals_brute_force(g):
    got = oracle.count(g, 5)
    assert got[:11] == _induced(g, 4)
    assert got[11:] == _induced(g, 5)


def test_each_noninduced_formula_against_brute_force():
    """N = A . C with C from brute force pins each cut formula on its own."""
    for g in _random_graphs()[:30]:
        S = oracle.sums(g, 5)
        for k in (4, 5):
            C = _induced(g, k)
            A = pat.a_matrix(k)
            N_brute = [sum(A[i][j] * C[j] for j in range(len(C))) for i in range(len(C))]
            assert oracle.noninduced_from_sums(S, k) == N_brute, (g.name, k)


def test_small_n_and_degenerate():
    for n in range(0, 6):
        for g in (synth.from_edges(n, []), synth.from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n)])):
            got = oracle.count(g, 5)
            assert sum(got[:11]) == comb(n, 4)
            assert sum(got[11:]) == comb(n, 5)
            if n >= 4:
                assert got[:11] == _induced(g, 4)
            if n >= 5:
                assert got[11:] == _induced(g, 5)


def test_order_independence():
    rng = random.Random(3)
    for g in _random_graphs()[::3]:
        base = oracle.count(g, 5)
        perm = list(range(g.n))
        rng.shuffle(perm)
        assert oracle.count(g, 5, order_rank=np.array(perm, dtype=np.int64)) == base


def test_relabel_invariance():
    rng = random.Random(11)
    g = synth.chung_lu(60, 2.1, 8.0, 30.0, 9)
    perm = list(range(g.n))
    rng.shuffle(perm)
    edges = [(perm[u], perm[int(v)]) for u in range(g.n) for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]] if u < v]
    h = synth.from_edges(g.n, edges)
    assert oracle.count(g, 5) == oracle.count(h, 5)


@pytest.mark.parametrize("seed", range(5))
def test_er200_equals_brute_force(seed):
    """G(200, 0.05): 2.5e9 five-subsets classified one by one."""
    g = synth.er_small(seed)
    got = oracle.count(g, 5)
    assert got[11:] == _induced(g, 5)
    assert got[:11] == _induced(g, 4)
    assert sum(got[11:]) == comb(200, 5)


# ------------------------------------------------------- per-item definitions

def test_per_item_counts_match_definitions():
    g = synth.chung_lu(120, 2.0, 10.0, 60.0, 4)
    S, it = oracle.sums(g, 5, per_item=True)
    A = _dense(g)
    A2 = A @ A
    n = g.n
    T = int(np.trace(A2 @ A)) // 6
    assert S["T"] == T
    for u in range(n):
        nbrs = g.col[g.row_ptr[u]:g.row_ptr[u + 1]]
        sub = A[np.ix_(nbrs, nbrs)]
        # t(v) = edges inside N(v); K4(v) = triangles inside N(v)
        assert it["t_v"][u] == sub.sum() // 2
        assert it["k4_v"][u] == int(np.trace(sub @ sub @ sub)) // 6
        for p in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[p])
            common = np.nonzero(A[u] & A[v])[0]
            assert it["t_e"][p] == len(common)
            assert it["k4_e"][p] == A[np.ix_(common, common)].sum() // 2
            # 4-cycles through edge uv: u - v - j - x - u with x != v
            c4 = sum(int(A2[u, j]) - 1 for j in np.nonzero(A[v])[0] if j != u)
            assert it["c4_e"][p] == c4
    assert int(it["t_v"].sum()) == 3 * S["T"]
    assert int(it["t_e"].sum()) == 2 * 3 * S["T"]
    assert int(it["c4_e"].sum()) == 2 * 4 * S["C4"]
    assert int(it["c4_v"].sum()) == 4 * S["C4"]
    assert int(it["k4_v"].sum()) == 4 * S["K4"]
    assert int(it["k4_e"].sum()) == 2 * 6 * S["K4"]


@pytest.mark.parametrize("n,p,seed", [(300, 0.08, 1), (400, 0.03, 2), (250, 0.3, 3)])
def test_cycle_counts_match_trace_formulas(n, p, seed):
    """C4 = (tr A^4 - 4 W - 2 m)/8;
    C5 = (tr A^5 - 5 tr A^3 - 5 sum_i (d_i - 2) (A^3)_ii) / 10."""
    g = synth.erdos_renyi(n, p, seed)
    A = _dense(g)
    d = A.sum(1)
    A2 = A @ A
    A3 = A2 @ A
    m = int(d.sum()) // 2
    W = int(sum(x * (x - 1) // 2 for x in d))
    c4 = (int(np.trace(A2 @ A2)) - 4 * W - 2 * m) // 8
    c5 = (int(np.trace(A3 @ A2)) - 5 * int(np.trace(A3)) - 5 * int(((d - 2) * np.diag(A3)).sum())) // 10
    S = oracle.sums(g, 5)
    assert S["C4"] == c4
    assert S["N8"] == c5


def test_sum_of_induced_counts_is_binomial():
    g = synth.chung_lu(3000, 2.1, 10.0, 300.0, 5)
    got = oracle.count(g, 5)
    assert sum(got[:11]) == comb(g.n, 4)
    assert sum(got[11:]) == comb(g.n, 5)
    assert min(got) >= 0


@pytest.mark.parametrize("seed", range(4))
def test_three_vertex_closed_form_equals_definition(seed):
    """3-vertex by-products (triangles, paths, one edge, none) against the
    classification of every 3-subset."""
    for g in (synth.erdos_renyi(40 + 10 * seed, 0.15, 900 + seed),
              synth.chung_lu(60, 2.1, 6.0, 20.0, 910 + seed)):
        assert oracle.three_vertex(g) == oracle.three_vertex_brute(g)


def test_three_vertex_special_graphs():
    from math import comb
    k6 = synth.from_edges(6, [(u, v) for u in range(6) for v in range(u + 1, 6)])
    assert oracle.three_vertex_brute(k6) == [0, 0, 0, comb(6, 3)]
    star = synth.from_edges(7, [(0, v) for v in range(1, 7)])
    assert oracle.three_vertex_brute(star) == [comb(6, 3), 0, comb(6, 2), 0]
    path = synth.from_edges(4, [(0, 1), (1, 2), (2, 3)])
    # {0,1,2},{1,2,3} paths; {0,1,3},{0,2,3} one edge
    assert oracle.three_vertex_brute(path) == [0, 2, 2, 0]
    assert oracle.three_vertex(path) == [0, 2, 2, 0]


# ------------------------------------------- one-by-one checkers (sampled tests)

def _fragment_graphs():
    out = [synth.erdos_renyi(18 + s, 0.2 + 0.05 * s, 700 + s) for s in range(5)]
    out += [synth.chung_lu(30 + 5 * s, 2.0 + 0.15 * s, 6.0 + s, 20.0, 720 + s) for s in range(5)]
    out.append(synth.erdos_renyi(16, 0.8, 731))                                              # dense
    out.append(synth.from_edges(12, [(0, v) for v in range(1, 12)] + [(v, v % 11 + 1) for v in range(1, 12)]))  # wheel W11
    out.append(synth.from_edges(11, [(u, v) for u in range(4) for v in range(u + 1, 11)]))    # split graph, 4-clique core
    return out


def _brute_edge(A, u, v):
    """Triangles, 4-cliques and 4-cycles through edge uv by enumerating the
    vertex sets that contain u and v."""
    n = len(A)
    rest = [x for x in range(n) if x != u and x != v]
    t = sum(1 for x in rest if A[u, x] and A[v, x])
    k4 = sum(1 for i, x in enumerate(rest) for y in rest[i + 1:]
             if A[u, x] and A[v, x] and A[u, y] and A[v, y] and A[x, y])
    # a 4-cycle u-v-x-y-u for each ordered pair (x, y) of distinct other vertices
    c4 = sum(1 for x in rest for y in rest if x != y and A[v, x] and A[x, y] and A[y, u])
    return t, k4, c4


@pytest.mark.parametrize("g", _fragment_graphs(), ids=lambda g: g.name or "special")
def test_edge_fragments_and_vertex_triangles_brute_force(g):
    """The one-by-one checkers against subset enumeration and against the
    oracle's per-item arrays (a separate code path, escape_oracle.c)."""
    A = _dense(g)
    _, it = oracle.sums(g, 4, per_item=True)
    for u in range(g.n):
        tv = sum(1 for x in range(g.n) for y in range(x + 1, g.n)
                 if A[u, x] and A[u, y] and A[x, y])
        assert oracle.vertex_triangles(g, u) == tv == int(it["t_v"][u])
        for p in range(g.row_ptr[u], g.row_ptr[u + 1]):
            v = int(g.col[p])
            t, k4, c4 = _brute_edge(A, u, v)
            got = oracle.edge_fragments(g, u, v)
            assert (got["t"], got["k4"], got["c4"]) == (t, k4, c4), (u, v)
            assert (int(it["t_e"][p]), int(it["k4_e"][p]), int(it["c4_e"][p])) == (t, k4, c4)


def test_edge_fragments_closed_forms():
    for n in (5, 8):
        kn = synth.from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
        # K_n: every other vertex closes a triangle, every other pair a 4-clique,
        # every ordered pair of other vertices a 4-cycle through the edge
        assert oracle.edge_fragments(kn, 0, 1) == {"t": n - 2, "k4": comb(n - 2, 2), "c4": (n - 2) * (n - 3)}
        assert oracle.vertex_triangles(kn, 0) == comb(n - 1, 2)
    for a, b in ((2, 5), (3, 4)):
        kab = synth.from_edges(a + b, [(u, a + v) for u in range(a) for v in range(b)])
        assert oracle.edge_fragments(kab, 0, a) == {"t": 0, "k4": 0, "c4": (a - 1) * (b - 1)}
        assert oracle.vertex_triangles(kab, 0) == 0
    c4g = synth.from_edges(4, [(0, 1), (1, 2), (2, 3), (3, 0)])
    assert oracle.edge_fragments(c4g, 0, 1) == {"t": 0, "k4": 0, "c4": 1}
    wheel = synth.from_edges(7, [(0, v) for v in range(1, 7)] + [(v, v % 6 + 1) for v in range(1, 7)])
    # spoke 0-1: triangles 0-1-2 and 0-1-6; rim vertex 1 lies on its two rim
    # triangles only; no 4-clique in a wheel with a 6-rim
    assert oracle.edge_fragments(wheel, 0, 1)["t"] == 2
    assert oracle.edge_fragments(wheel, 0, 1)["k4"] == 0
    assert oracle.vertex_triangles(wheel, 0) == 6
    assert oracle.vertex_triangles(wheel, 1) == 2


def _complement(g):
    A = _dense(g)
    return synth.from_edges(g.n, [(u, v) for u in range(g.n) for v in range(u + 1, g.n) if not A[u, v]])


@pytest.mark.parametrize("seed", range(6))
def test_clique_count_through_the_complement(seed):
    """The 4-cliques of a dense graph H are the 4-sets spanning no edge of its
    complement Hc: with the sign rule of the inverse of A (App. B) on the
    empty pattern's row, K4(H) = sum over the 11 four-vertex patterns j of
    (-1)^e(j) N_j(Hc), N_j the non-induced counts of Hc (the 5-clique pass
    counts dense out-neighbourhoods this way).  Checked against the
    classification of every 4-subset of H."""
    n = 14 + 3 * seed
    h = synth.erdos_renyi(n, 0.55 + 0.07 * seed, 800 + seed)
    hc = _complement(h)
    N = oracle.noninduced_from_sums(oracle.sums(hc, 4), 4)
    signed = sum((-1) ** pat.edge_count(4, j) * N[j] for j in range(11))
    assert signed == _induced(h, 4)[5]
    assert list(pat.a_inverse(4)[6]) == [(-1) ** pat.edge_count(4, j) for j in range(11)]


@pytest.mark.parametrize("seed", range(5))
def test_work_counts_directed_paths_and_bipyramids(seed):
    """The work counts of Thm fivevertex that Fig. predict fits the running
    time with, by their definitions in the degree-ordered DAG (arcs from the
    earlier to the later vertex): DP = ordered 4-tuples (i, a, b, j) of
    distinct vertices with arcs a->i, a->b, b->j (the directed 3-path);
    DBP = 5-subsets whose three earliest vertices form a triangle and whose
    two latest vertices are each adjacent to all three (the bipyramid from the
    triangle of its three earliest vertices)."""
    from itertools import combinations
    g = synth.erdos_renyi(14 + seed, 0.45 + 0.08 * seed, 940 + seed)
    A = _dense(g).astype(bool)
    n = g.n
    d = A.sum(1)
    order = sorted(range(n), key=lambda v: (d[v], v))
    rank = np.empty(n, np.int64)
    rank[order] = np.arange(n)
    arc = A & (rank[:, None] < rank[None, :])
    dp = 0
    for a in range(n):
        for i in range(n):
            if not arc[a, i]:
                continue
            for b in range(n):
                if b == i or not arc[a, b]:
                    continue
                dp += int(sum(1 for j in range(n) if j != i and arc[b, j]))
    dbp = 0
    for sub in combinations(order, 5):
        x, y, z, p, q = sub   # in rank order
        if A[x, y] and A[x, z] and A[y, z] and all(A[w, t] for w in (p, q) for t in (x, y, z)):
            dbp += 1
    S = oracle.sums(g, 5)
    assert S["DP"] == dp and S["DBP"] == dbp, (dp, dbp, S["DP"], S["DBP"])
    # closed form of DP: sum over arcs a->b of (d+(a) - 1) d+(b), less T
    dplus = arc.sum(1)
    assert dp == int(sum((dplus[a] - 1) * dplus[b] for a in range(n) for b in range(n) if arc[a, b])) - S["T"]
