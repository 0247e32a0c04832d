"""ORACLE -- TEST INFRASTRUCTURE ONLY.

Pattern library for the oracle: the 11 four-vertex and 34 five-vertex graphs,
their isomorphism classes, the induced/non-induced transform (Appendix B) and
the inclusion-exclusion for disconnected patterns (Appendix A).

Edge lists use the vertex labels of the paper's pattern drawings (Fig. 5vertex
for the connected patterns, Figs. 4vertex-disc and 5vertex-disc for the
disconnected ones), 1-based as drawn.  The drawings of the disconnected
5-vertex patterns stop at eleven; the two missing ones (a wedge plus a disjoint
edge, a triangle plus a disjoint edge) are appended at the end.

Output order (45 slots):
  [0..5]   connected 4-vertex: 3-star, 3-path, tailed triangle, 4-cycle,
           diamond, 4-clique (Fig. 5vertex, top row)
  [6..10]  disconnected 4-vertex: independent set, only edge, matching,
           only wedge, only triangle (Fig. 4vertex-disc)
  [11..31] connected 5-vertex patterns 1..21 (Fig. 5vertex)
  [32..42] disconnected 5-vertex patterns (1)..(11) (Fig. 5vertex-disc)
  [43]     wedge + disjoint edge,  [44] triangle + disjoint edge
"""
from __future__ import annotations

import itertools
from functools import lru_cache
from math import comb

FOUR_CONNECTED = [
    ("3-star", [(1, 2), (1, 3), (1, 4)]),
    ("3-path", [(1, 2), (1, 3), (2, 4)]),
    ("tailed-triangle", [(1, 2), (1, 3), (1, 4), (2, 4)]),
    ("4-cycle", [(1, 2), (1, 3), (2, 4), (3, 4)]),
    ("diamond", [(1, 2), (1, 3), (1, 4), (2, 4), (3, 4)]),
    ("4-clique", [(1, 2), (1, 3), (1, 4), (2, 3), (2, 4), (3, 4)]),
]
FOUR_DISCONNECTED = [
    ("4-ind-set", []),
    ("4-only-edge", [(1, 2)]),
    ("4-matching", [(1, 2), (3, 4)]),
    ("4-only-wedge", [(1, 2), (2, 3)]),
    ("4-only-triangle", [(1, 2), (1, 3), (2, 3)]),
]
FIVE_CONNECTED = [
    ("P1", [(1, 2), (1, 3), (1, 4), (1, 5)]),
    ("P2", [(1, 2), (1, 3), (1, 4), (2, 5)]),
    ("P3", [(1, 2), (1, 3), (2, 4), (3, 5)]),
    ("P4", [(1, 2), (1, 3), (2, 3), (3, 4), (3, 5)]),
    ("P5", [(1, 2), (1, 3), (2, 3), (2, 4), (4, 5)]),
    ("P6", [(1, 2), (1, 3), (2, 3), (2, 4), (3, 5)]),
    ("P7", [(1, 2), (2, 4), (3, 4), (3, 1), (3, 5)]),
    ("P8", [(1, 2), (1, 3), (4, 2), (3, 5), (5, 4)]),
    ("P9", [(1, 2), (1, 3), (2, 3), (3, 4), (3, 5), (4, 5)]),
    ("P10", [(1, 2), (2, 4), (3, 4), (3, 1), (3, 5), (1, 4)]),
    ("P11", [(1, 2), (2, 4), (3, 4), (3, 1), (3, 5), (3, 2)]),
    ("P12", [(1, 2), (2, 4), (3, 4), (3, 1), (3, 5), (4, 5)]),
    ("P13", [(1, 2), (2, 5), (1, 3), (3, 5), (1, 4), (4, 5)]),
    ("P14", [(1, 2), (2, 5), (1, 3), (3, 5), (1, 4), (4, 5), (1, 5)]),
    ("P15", [(1, 2), (2, 4), (3, 4), (3, 1), (3, 5), (1, 4), (3, 2)]),
    ("P16", [(1, 2), (2, 4), (3, 4), (3, 1), (3, 5), (3, 2), (4, 5)]),
    ("P17", [(1, 2), (1, 3), (1, 4), (3, 2), (4, 2), (3, 5), (5, 4)]),
    ("P18", [(1, 2), (1, 3), (1, 4), (1, 5), (3, 2), (5, 3), (5, 4), (2, 4)]),
    ("P19", [(1, 2), (2, 4), (3, 4), (3, 1), (3, 5), (3, 2), (4, 5), (1, 4)]),
    ("P20", [(1, 3), (1, 4), (1, 5), (3, 2), (4, 2), (2, 5), (3, 4), (3, 5), (4, 5)]),
    ("P21", [(1, 2), (1, 3), (1, 4), (1, 5), (3, 2), (4, 2), (2, 5), (3, 4), (3, 5), (5, 4)]),
]
FIVE_DISCONNECTED = [
    ("5-ind-set", []),
    ("5-only-edge", [(1, 2)]),
    ("5-matching", [(1, 2), (3, 4)]),
    ("5-only-wedge", [(1, 2), (1, 3)]),
    ("5-only-triangle", [(1, 2), (1, 3), (2, 3)]),
    ("5-only-3-star", [(1, 2), (1, 3), (1, 4)]),
    ("5-only-3-path", [(1, 2), (1, 3), (3, 4)]),
    ("5-only-tailed-triangle", [(1, 2), (2, 3), (1, 3), (3, 4)]),
    ("5-only-4-cycle", [(1, 2), (2, 4), (3, 4), (1, 3)]),
    ("5-only-diamond", [(1, 2), (2, 4), (3, 4), (1, 4), (1, 3)]),
    ("5-only-4-clique", [(1, 2), (2, 3), (3, 4), (1, 4), (2, 4), (1, 3)]),
    ("5-wedge+edge", [(1, 2), (1, 3), (4, 5)]),
    ("5-triangle+edge", [(1, 2), (1, 3), (2, 3), (4, 5)]),
]

FOUR = FOUR_CONNECTED + FOUR_DISCONNECTED          # 11, slots 0..10
FIVE = FIVE_CONNECTED + FIVE_DISCONNECTED          # 34, slots 11..44
ALL_NAMES = [name for name, _ in FOUR + FIVE]


def pairs(k):
    """Vertex pairs of a k-set in bitmask order (0,1),(0,2),...,(k-2,k-1)."""
    return [(a, b) for a in range(k) for b in range(a + 1, k)]


def mask_of(k, edges):
    """Bitmask over `pairs(k)` for 1-based edge list."""
    idx = {p: i for i, p in enumerate(pairs(k))}
    m = 0
    for u, v in edges:
        a, b = sorted((u - 1, v - 1))
        m |= 1 << idx[(a, b)]
    return m


@lru_cache(maxsize=None)
def _perm_tables(k):
    """For every vertex permutation, the image of each pair index."""
    ps = pairs(k)
    idx = {p: i for i, p in enumerate(ps)}
    tables = []
    for perm in itertools.permutations(range(k)):
        tables.append([idx[tuple(sorted((perm[a], perm[b])))] for a, b in ps])
    return tables


def canon(k, m):
    """Canonical form: least mask over all relabellings."""
    best = None
    npairs = k * (k - 1) // 2
    for tab in _perm_tables(k):
        x = 0
        for i in range(npairs):
            if m >> i & 1:
                x |= 1 << tab[i]
        if best is None or x < best:
            best = x
    return best


def automorphisms(k, m):
    count = 0
    npairs = k * (k - 1) // 2
    for tab in _perm_tables(k):
        x = 0
        for i in range(npairs):
            if m >> i & 1:
                x |= 1 << tab[i]
        if x == m:
            count += 1
    return count


def patterns(k):
    return FOUR if k == 4 else FIVE


@lru_cache(maxsize=None)
def class_lut(k):
    """Table mask -> pattern index (within the k-vertex list) for all 2^C(k,2) masks.
    For k=3 the classes are: 0 empty, 1 one edge, 2 wedge, 3 triangle."""
    npairs = k * (k - 1) // 2
    if k == 3:
        return tuple(bin(m).count("1") for m in range(1 << npairs))
    canon_to_idx = {}
    for i, (_, edges) in enumerate(patterns(k)):
        c = canon(k, mask_of(k, edges))
        assert c not in canon_to_idx, "two patterns drawn isomorphic"
        canon_to_idx[c] = i
    return tuple(canon_to_idx[canon(k, m)] for m in range(1 << npairs))


@lru_cache(maxsize=None)
def a_matrix(k):
    """A[i][j] = number of edge subsets of pattern j (same vertex set) that form
    pattern i.  Non-induced = A . induced (Appendix B)."""
    lut = class_lut(k)
    pats = patterns(k)
    npat = len(pats)
    A = [[0] * npat for _ in range(npat)]
    for j, (_, edges) in enumerate(pats):
        m = mask_of(k, edges)
        bits = [b for b in range(k * (k - 1) // 2) if m >> b & 1]
        for r in range(len(bits) + 1):
            for sub in itertools.combinations(bits, r):
                x = 0
                for b in sub:
                    x |= 1 << b
                A[lut[x]][j] += 1
    return tuple(tuple(row) for row in A)


def edge_count(k, i):
    return len(patterns(k)[i][1])


def induced_from_noninduced(k, N):
    """Solve A C = N exactly.  A is unit upper-triangular once patterns are
    ordered by edge count, so back-substitution in integers suffices."""
    A = a_matrix(k)
    npat = len(N)
    order = sorted(range(npat), key=lambda i: -edge_count(k, i))
    C = [0] * npat
    for i in order:
        s = N[i]
        for j in range(npat):
            if j != i and A[i][j]:
                s -= A[i][j] * C[j]
        C[i] = s
    return C


def a_inverse(k):
    """A^{-1} computed exactly by solving A X = I column by column."""
    npat = len(patterns(k))
    cols = []
    for j in range(npat):
        e = [0] * npat
        e[j] = 1
        cols.append(induced_from_noninduced(k, e))
    return tuple(tuple(cols[j][i] for j in range(npat)) for i in range(npat))


# ---------------------------------------------------------------- Appendix A

def _components(k, edges):
    parent = list(range(k))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for u, v in edges:
        parent[find(u)] = find(v)
    comps = {}
    for v in range(k):
        comps.setdefault(find(v), []).append(v)
    return list(comps.values())


def _set_partitions(items):
    if not items:
        yield []
        return
    first, rest = items[0], items[1:]
    for part in _set_partitions(rest):
        for i in range(len(part)):
            yield part[:i] + [[first] + part[i]] + part[i + 1:]
        yield [[first]] + part


def labeled_matches(k, edges, connected_count):
    """match(H) of Appendix A: injective maps V(H) -> V(G) sending edges to
    edges.  `edges` are 0-based pairs on vertices 0..k-1.  For connected H the
    count is connected_count(k, canonical mask) * |Aut(H)|; for disconnected H
    the appendix's inclusion-exclusion over vertex merges applies:
        match(H) = prod_i match(H_i) - sum_S match(H_S)
    where S runs over the non-trivial partitions of V(H) whose blocks take at
    most one vertex from each component, and H_S merges every block."""
    edges = sorted({tuple(sorted(e)) for e in edges})
    comps = _components(k, edges)
    if len(comps) == 1:
        m = 0
        idx = {p: i for i, p in enumerate(pairs(k))}
        for e in edges:
            m |= 1 << idx[e]
        return connected_count(k, canon(k, m)) * automorphisms(k, m)
    comp_of = {}
    for ci, comp in enumerate(comps):
        for v in comp:
            comp_of[v] = ci
    prod = 1
    for comp in comps:
        relabel = {v: i for i, v in enumerate(comp)}
        sub = [(relabel[u], relabel[v]) for u, v in edges if u in relabel]
        prod *= labeled_matches(len(comp), sub, connected_count)
    total = 0
    for part in _set_partitions(list(range(k))):
        if len(part) == k:
            continue
        if any(len({comp_of[v] for v in block}) < len(block) for block in part):
            continue
        block_of = {}
        for bi, block in enumerate(part):
            for v in block:
                block_of[v] = bi
        merged = {tuple(sorted((block_of[u], block_of[v]))) for u, v in edges}
        total += labeled_matches(len(part), sorted(merged), connected_count)
    return prod - total


def noninduced_disconnected(k, idx, connected_count):
    """Non-induced (unlabeled) count of disconnected pattern idx of size k."""
    _, edges = patterns(k)[idx]
    e0 = [(u - 1, v - 1) for u, v in edges]
    m = mask_of(k, edges)
    return labeled_matches(k, e0, connected_count) // automorphisms(k, m)


def is_connected(k, edges):
    return len(_components(k, [(u - 1, v - 1) for u, v in edges])) == 1


def binom(n, r):
    return comb(n, r) if n >= r >= 0 else 0
