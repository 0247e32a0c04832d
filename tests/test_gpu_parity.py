"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Exact integer counts: the bar is equality of every one of the 45 counts
(and of every per-item fragment count).
"""
import json
import os
import random
from math import comb

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def ctx():
    import paper_1610_09411_amd as esc
    c = esc.Context(0)
    yield c
    c.close()


def _cases_small():
    out = []
    for s in range(12):
        out.append(synth.erdos_renyi(10 + 3 * s, 0.1 + 0.05 * (s % 8), 500 + s))
    for s in range(10):
        out.append(synth.chung_lu(40 + 17 * s, 2.0 + 0.08 * s, 5.0 + s, 30.0, 600 + s))
    out.append(synth.from_edges(9, [(u, v) for u in range(9) for v in range(u + 1, 9)]))          # K9
    out.append(synth.from_edges(12, [(u, 6 + v) for u in range(6) for v in range(6)]))            # K6,6
    out.append(synth.from_edges(15, [(i, (i + 1) % 15) for i in range(15)]))                      # C15
    out.append(synth.from_edges(20, [(0, v) for v in range(1, 20)]))                              # star
    out.append(synth.from_edges(30, [(0, v) for v in range(1, 30)] + [(v, v + 1) for v in range(1, 29)]))  # fan
    return out


def test_library_is_native_and_loaded(ctx):
    import paper_1610_09411_amd as esc
    assert os.path.exists(esc.LIB_PATH)
    assert esc._lib is not None


def _check_equal(ctx, g, k=5, **kw):
    """GPU counts == oracle counts; on a mismatch name the non-induced counts
    that differ (they map one-to-one onto the device sums)."""
    from oracle import patterns as pat
    got = ctx.count(g, k, **kw)
    want = oracle.count(g, k, threads=8)
    if got != want:
        S = oracle.sums(g, k)
        nonind = oracle.noninduced_from_sums(S, 4) + (oracle.noninduced_from_sums(S, 5) if k == 5 else [])
        gpu_non = ctx.last_noninduced(k)
        diff = [(pat.ALL_NAMES[i], gpu_non[i], nonind[i]) for i in range(len(nonind)) if gpu_non[i] != nonind[i]]
        raise AssertionError("%s: non-induced (name, gpu, oracle) differing: %s" % (g.name, diff))
    return got


@pytest.mark.parametrize("idx", range(len(_cases_small())))
def test_small_graphs_equal_oracle(ctx, idx):
    g = _cases_small()[idx]
    print("case", idx, g.name, g.n, g.m, flush=True)
    _check_equal(ctx, g, 5)
    _check_equal(ctx, g, 4)


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6])
def test_tiny_and_degenerate(ctx, n):
    empty = synth.from_edges(n, [])
    full = synth.from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
    for g in (empty, full):
        got = ctx.count(g, 5)
        assert got == oracle.count(g, 5)
        assert sum(got[:11]) == comb(n, 4) and sum(got[11:]) == comb(n, 5)


@pytest.mark.parametrize("seed", range(5))
def test_er200_equals_brute_force(ctx, seed):
    g = synth.er_small(seed)
    got = ctx.count(g, 5)
    assert got[:11] == oracle.brute(g, 4)
    assert got[11:] == oracle.brute(g, 5)


@pytest.mark.parametrize("n,gamma,dbar,dmax,seed", [
    (3000, 2.1, 12.0, 400.0, 1),
    (20000, 2.1, 20.0, 1500.0, 2),
    (12000, 1.9, 30.0, 3000.0, 3),
])
def test_power_law_graphs_equal_oracle(ctx, n, gamma, dbar, dmax, seed):
    """Several thousand vertices: many workgroups, hubs, ragged lists."""
    g = synth.chung_lu(n, gamma, dbar, dmax, seed)
    print("chung_lu", n, g.m, flush=True)
    _check_equal(ctx, g, 5)


def test_three_vertex_counts(ctx):
    """The 3-vertex by-products of a call equal the oracle's, and the
    classification of every 3-subset on a 200-vertex graph."""
    g = synth.er_small(0)
    ctx.count(g, 5)
    assert ctx.last_three() == oracle.three_vertex_brute(g)
    for g in _cases_small()[:8] + [synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2), synth.from_edges(2, [(0, 1)])]:
        ctx.count(g, 4)
        got = ctx.last_three()
        assert got == oracle.three_vertex(g), g.name
        assert sum(got) == comb(g.n, 3)


def test_random_order_gives_same_counts(ctx):
    import paper_1610_09411_amd as esc
    g = synth.chung_lu(5000, 2.1, 15.0, 600.0, 9)
    assert ctx.count(g, 5, flags=esc.ESC_F_RANDOM_ORDER) == ctx.count(g, 5)


def test_compact_lists_give_same_counts(ctx):
    """Triangle lists without apex ids (read through the adjacency), the
    layout chosen when device memory is short."""
    import paper_1610_09411_amd as esc
    for g in (synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2), synth.chung_lu(12000, 1.9, 30.0, 3000.0, 3)):
        assert ctx.count(g, 5, flags=esc.ESC_F_COMPACT_LISTS) == ctx.count(g, 5)
    g = synth.chung_lu(3000, 2.1, 12.0, 400.0, 1)
    assert ctx.count(g, 5, flags=esc.ESC_F_COMPACT_LISTS) == oracle.count(g, 5, threads=8)
    counts, fr = ctx.fragments(g, 4, flags=esc.ESC_F_COMPACT_LISTS)
    S, it = oracle.sums(g, 4, per_item=True)
    assert np.array_equal(fr["k4_e"], it["k4_e"])


def _messy_csr(g, seed):
    """The same graph written carelessly: each edge in one row or both,
    some entries repeated, self-loops added, rows unsorted."""
    rng = np.random.default_rng(seed)
    rows = [[] for _ in range(g.n)]
    for u in range(g.n):
        for v in g.col[g.row_ptr[u]:g.row_ptr[u + 1]]:
            v = int(v)
            if u < v:
                r = rng.integers(3)
                if r == 0:
                    rows[u].append(v)
                elif r == 1:
                    rows[v].append(u)
                else:
                    rows[u].append(v)
                    rows[v].append(u)
                if rng.integers(5) == 0:
                    rows[u].append(v)
        if rng.integers(7) == 0:
            rows[u].append(u)
    for r in rows:
        rng.shuffle(r)
    rp = np.zeros(g.n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([x for r in rows for x in r], np.int32)
    return synth.Graph(g.n, rp, col)


def test_canonicalize_counts_the_described_graph(ctx):
    import paper_1610_09411_amd as esc
    for g in (synth.chung_lu(3000, 2.1, 12.0, 400.0, 1), synth.er_small(2), synth.from_edges(6, [])):
        messy = _messy_csr(g, 7)
        got = ctx.count(messy, 5, flags=esc.ESC_F_CANONICALIZE)
        assert got == oracle.count(g, 5, threads=8), g.name
        assert ctx.last_work()["m"] == g.m
    # rows above 1024 entries with repeated neighbours: the long-segment sort
    # meets repeated keys and takes its sorting network
    g = synth.chung_lu(8000, 2.0, 12.0, 4000.0, 4)
    messy = _messy_csr(g, 8)
    assert int(np.diff(messy.row_ptr).max()) > 1024
    assert ctx.count(messy, 4, flags=esc.ESC_F_CANONICALIZE) == oracle.count(g, 4, threads=8)
    assert ctx.count(messy, 5, flags=esc.ESC_F_CANONICALIZE) == ctx.count(g, 5)
    bad = synth.Graph(3, np.array([0, 1, 2, 3], np.int32), np.array([1, 2, 5], np.int32))
    with pytest.raises(esc.EscapeError) as e:
        ctx.count(bad, 5, flags=esc.ESC_F_CANONICALIZE)
    assert e.value.status == esc.ESC_ERANGE
    with pytest.raises(esc.EscapeError) as e:
        ctx.fragments(synth.er_small(2), 5, flags=esc.ESC_F_CANONICALIZE)
    assert e.value.status == esc.ESC_EINVAL


def test_tuned_and_forced_parameters_give_same_counts(ctx):
    """The autotuner picks launch parameters per degree-statistics key; any
    parameters give the same counts."""
    import paper_1610_09411_amd as esc
    g = synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2)
    want = oracle.count(g, 5, threads=8)
    best, ms = ctx.tune(g, 5)
    assert ms > 0 and 1 <= best["wg_per_cu"] <= 3 and best["task_chunk"] in (1, 4, 16)
    assert ctx.count(g, 5) == want
    assert ctx.last_params() == best             # the table entry is used for this graph
    assert best["five_order"] == 0
    # five_order 1: the 5-cycle sum in the Wnt-table order (else taken only
    # by graphs whose largest degree reaches 2^16, and by batches)
    # the split thresholds at their extremes: every 4-cycle top above 16
    # neighbours in key-range tasks, every wheel hub split into rim tasks,
    # 5-clique vertices above 8 out-neighbours through the complement (or
    # never), rows of one word in the per-b wave path or none of them
    for p in ({"task_chunk": 64, "wg_per_cu": 1, "k5_work_log2": 16, "five_order": 1},
              {"task_chunk": 3, "wg_per_cu": 3, "k5_work_log2": 30, "five_order": 0},
              {"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20, "five_order": 1},
              {"task_chunk": 1, "wg_per_cu": 2, "k5_work_log2": 20, "k5_light": 8, "k5_wave_words": 1,
               "k5_dense_pct": 0, "wheel_split_deg": 32, "four_range_deg": 16},
              {"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20, "k5_light": 3, "k5_wave_words": 8,
               "k5_dense_pct": 101, "wheel_split_deg": 1 << 30, "four_range_deg": 1 << 30}):
        ctx.set_params(p)
        assert ctx.count(g, 5) == want, p
        assert ctx.last_params() == dict(esc.PARAM_DEFAULTS, **p)
    for bad in ({"task_chunk": 0, "wg_per_cu": 1, "k5_work_log2": 24},
                {"task_chunk": 1, "wg_per_cu": 1, "k5_work_log2": 24, "five_order": 2},
                {"task_chunk": 1, "wg_per_cu": 1, "k5_work_log2": 24, "k5_light": 65},
                {"task_chunk": 1, "wg_per_cu": 1, "k5_work_log2": 24, "k5_wave_words": 9},
                {"task_chunk": 1, "wg_per_cu": 1, "k5_work_log2": 24, "k5_dense_pct": 102},
                {"task_chunk": 1, "wg_per_cu": 1, "k5_work_log2": 24, "wheel_split_deg": 31},
                {"task_chunk": 1, "wg_per_cu": 1, "k5_work_log2": 24, "four_range_deg": 15}):
        with pytest.raises(esc.EscapeError) as e:
            ctx.set_params(bad)
        assert e.value.status == esc.ESC_EINVAL, bad
    ctx.set_params(None)
    graphs = [synth.from_spec(s) for s in synth.batch_specs(40, 3)]
    bbest, _ = ctx.tune_batched(graphs, 5)
    rows, _ = ctx.count_batched(graphs, 5)
    assert ctx.last_params() == bbest
    for i in (0, 7, 39):
        assert [int(x) for x in rows[i]] == oracle.count(graphs[i], 5), i


def test_dense_graphs_closed_forms(ctx):
    """Dense graphs with closed-form counts.  K_600: every k-subset is a
    clique (its out-degrees run from 0 to 599, so the 5-clique pass takes
    its light, wave and block paths).  K_{300,300}: only stars, 4-cycles,
    4-stars and K_{2,3} are induced (Thm 5clique and the bipartite cases of
    the brute-force pins)."""
    from math import comb
    n = 600
    kn = synth.from_edges(n, [(u, v) for u in range(n) for v in range(u + 1, n)])
    got5 = ctx.count(kn, 5)
    want5 = [0] * 45
    want5[5] = comb(n, 4)
    want5[31] = comb(n, 5)
    assert got5 == want5
    got4 = ctx.count(kn, 4)
    assert got4 == want5[:11]
    a = b = 300
    kab = synth.from_edges(a + b, [(u, a + v) for u in range(a) for v in range(b)])
    got = ctx.count(kab, 5)
    want = [0] * 45
    want[0] = a * comb(b, 3) + b * comb(a, 3)          # 3-stars
    want[3] = comb(a, 2) * comb(b, 2)                  # 4-cycles
    want[6] = comb(a, 4) + comb(b, 4)                  # 4 independent vertices
    want[11] = a * comb(b, 4) + b * comb(a, 4)         # 4-stars
    want[11 + 12] = comb(a, 2) * comb(b, 3) + comb(a, 3) * comb(b, 2)   # K_{2,3}
    want[32] = comb(a, 5) + comb(b, 5)                 # 5 independent vertices
    assert got == want


def test_repeat_calls_are_identical(ctx):
    g = synth.chung_lu(8000, 2.0, 16.0, 900.0, 4)
    a = ctx.count(g, 5)
    small = synth.er_small(1)
    ctx.count(small, 5)
    assert ctx.count(g, 5) == a


def test_fragments_equal_oracle(ctx):
    g = synth.chung_lu(4000, 2.1, 14.0, 500.0, 5)
    counts, fr = ctx.fragments(g, 5)
    S, it = oracle.sums(g, 5, per_item=True)
    assert counts == oracle.count(g, 5)
    assert np.array_equal(fr["tri_v"], it["t_v"])
    assert np.array_equal(fr["c4_v"], it["c4_v"])
    assert np.array_equal(fr["k4_v"], it["k4_v"])
    assert np.array_equal(fr["tri_e"], it["t_e"])
    assert np.array_equal(fr["c4_e"], it["c4_e"])
    assert np.array_equal(fr["k4_e"], it["k4_e"])


def test_device_input(ctx):
    import torch
    g = synth.chung_lu(2000, 2.2, 10.0, 300.0, 6)
    rp = torch.from_numpy(g.row_ptr).cuda()
    ci = torch.from_numpy(g.col).cuda()
    import paper_1610_09411_amd as esc
    got = esc.esc_count_subgraphs(ctx.ptr, g.n, rp, ci, 5)
    assert got == oracle.count(g, 5)


def test_invalid_input_is_rejected(ctx):
    import paper_1610_09411_amd as esc
    bad_range = synth.Graph(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 7], np.int32))
    with pytest.raises(esc.EscapeError) as e:
        ctx.count(bad_range, 5, flags=esc.ESC_F_VALIDATE)
    assert e.value.status == esc.ESC_ERANGE
    loop = synth.Graph(2, np.array([0, 2, 3], np.int32), np.array([0, 1, 0], np.int32))
    with pytest.raises(esc.EscapeError) as e:
        ctx.count(loop, 5, flags=esc.ESC_F_VALIDATE)
    assert e.value.status in (esc.ESC_ENOTSIMPLE, esc.ESC_ERANGE)
    asym = synth.Graph(3, np.array([0, 1, 2, 2], np.int32), np.array([1, 2], np.int32))
    with pytest.raises(esc.EscapeError) as e:
        ctx.count(asym, 5, flags=esc.ESC_F_VALIDATE)
    assert e.value.status == esc.ESC_ENOTSIMPLE
    with pytest.raises(esc.EscapeError) as e:
        esc.esc_count_subgraphs(ctx.ptr, 3, np.array([0, 1, 2, 2], np.int32), np.array([1, 0], np.int32), k=6)
    assert e.value.status == esc.ESC_EINVAL
    # the context still works afterwards
    g = synth.er_small(2)
    assert ctx.count(g, 5) == oracle.count(g, 5)


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip("golden file %s not generated" % name)
    with open(path) as f:
        return json.load(f)


def test_chung_lu_1m_full_size(ctx):
    """n=1e6, gamma=2.1, mean degree 20, max expected degree 1e4: the benchmark
    workload, checked against the oracle's stored counts and by properties
    that hold at any size."""
    gold = _golden("chung_lu_1m_seed0.json")
    g = synth.chung_lu_1m(0)
    assert g.m == gold["m"]
    got = ctx.count(g, 5)
    assert sum(got[:11]) == comb(g.n, 4)
    assert sum(got[11:]) == comb(g.n, 5)
    assert [int(x) for x in gold["counts"]] == got
    # the 5-cycle sum in the Wnt-table order gives the same counts
    ctx.set_params({"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20, "five_order": 1})
    try:
        assert ctx.count(g, 5) == got
    finally:
        ctx.set_params(None)


def test_chung_lu_1m_sampled_fragments(ctx):
    """Per-vertex and per-edge fragment counts at full size, sampled and
    recomputed one by one from their definitions."""
    g = synth.chung_lu_1m(0)
    _, fr = ctx.fragments(g, 4)
    rng = random.Random(0)
    deg = g.degrees()
    hubs = list(np.argsort(-deg)[:5])
    verts = hubs + [rng.randrange(g.n) for _ in range(20)]
    for v in verts:
        v = int(v)
        s, t = g.row_ptr[v], g.row_ptr[v + 1]
        if t == s:
            continue
        arcs = [s, t - 1] + [rng.randrange(s, t) for _ in range(2)]
        for p in arcs:
            u = int(g.col[p])
            exp = oracle.edge_fragments(g, v, u)
            assert fr["tri_e"][p] == exp["t"], (v, u)
            assert fr["k4_e"][p] == exp["k4"], (v, u)
            if deg[v] < 3000 and deg[u] < 3000:
                assert fr["c4_e"][p] == exp["c4"], (v, u)
        assert fr["tri_v"][v] == oracle.vertex_triangles(g, v)


def test_binomials_at_the_vertex_bound(ctx):
    """Edgeless graph with n at the k = 5 bound (1e8): every 4- and 5-subset
    is independent, so the empty-pattern slots must be C(n,4) and C(n,5)
    exactly (a multiply-before-divide binomial passes 2^128 from n near
    9.6e7).  One vertex more is refused."""
    import paper_1610_09411_amd as esc
    n = 100_000_000
    g = synth.Graph(n, np.zeros(n + 1, np.int32), np.zeros(0, np.int32), "edgeless 1e8")
    got = ctx.count(g, 5)
    want = [0] * 45
    want[6] = comb(n, 4)
    want[32] = comb(n, 5)
    assert got == want
    g1 = synth.Graph(n + 1, np.zeros(n + 2, np.int32), np.zeros(0, np.int32), "edgeless 1e8+1")
    with pytest.raises(esc.EscapeError) as e:
        ctx.count(g1, 5)
    assert e.value.status == esc.ESC_EOVERFLOW


def _dense_core_graph(seed, core=130, per=250):
    """A near-clique core (each core pair missing with probability 0.04) and
    periphery vertices tied to random fractions of it and sparsely to each
    other: out-neighbourhoods of every density, many above 64 vertices."""
    rng = random.Random(seed)
    edges = [(u, v) for u in range(core) for v in range(u + 1, core) if rng.random() > 0.04]
    for x in range(core, core + per):
        q = rng.random() * 0.6
        edges += [(x, u) for u in range(core) if rng.random() < q]
        edges += [(x, y) for y in range(core, x) if rng.random() < 0.02]
    return synth.from_edges(core + per, edges, "dense core %d" % seed)


def test_five_cliques_through_the_complement(ctx):
    """Thm 5clique with dense out-neighbourhoods counted through their
    complement (every vertex above 64 out-neighbours: pct 0; the default
    density cut: 50; never: 101): the same 45 counts as the oracle."""
    for g in (_dense_core_graph(1), synth.erdos_renyi(160, 0.6, 11), synth.erdos_renyi(200, 0.45, 12)):
        print(g.name, g.n, g.m, flush=True)
        want = oracle.count(g, 5, threads=8)
        for pct in (0, 50, 101):
            ctx.set_params({"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20, "k5_dense_pct": pct})
            try:
                got = ctx.count(g, 5)
            finally:
                ctx.set_params(None)
            assert got == want, (g.name, pct)


def test_hub_pair_product(ctx):
    """Pattern 17 with the diamonds of two hub tips over a dense edge summed
    as the matrix-core product of the hub / dense-edge incidence (Thm 5cutwed):
    hubs of one 256-rank tile up to 39 tiles, every edge with a hub apex
    dense (several chunks of dense edges) or only the heaviest, the lists
    with and without apex ids.  Same counts as the oracle."""
    import paper_1610_09411_amd as esc
    base = {"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20}
    g = synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2)
    want = oracle.count(g, 5, threads=8)
    try:
        for r, q, flags in ((256, 1, 0), (512, 1, 0), (1024, 4, esc.ESC_F_COMPACT_LISTS), (8192, 1, 0),
                            (8192, 64, 0), (9984, 2, esc.ESC_F_COMPACT_LISTS), (0, 1, 0)):
            ctx.set_params(dict(base, pairs_hub_ranks=r, pairs_hub_q=q))
            print("hubs", r, "q", q, "flags", flags, flush=True)
            assert ctx.count(g, 5, flags=flags) == want, (r, q, flags)
            assert ctx.count(g, 4, flags=flags) == want[:11], (r, q, flags)
        # a near-clique core: edges with hundreds of hub apexes
        gc = _dense_core_graph(2, core=300, per=400)
        wc = oracle.count(gc, 5, threads=8)
        for r, q in ((256, 1), (256, 100), (256, 1 << 30)):
            ctx.set_params(dict(base, pairs_hub_ranks=r, pairs_hub_q=q))
            print("dense core hubs", r, "q", q, flush=True)
            assert ctx.count(gc, 5) == wc, (r, q)
        for bad in ({"pairs_hub_ranks": 100}, {"pairs_hub_ranks": 384}, {"pairs_hub_ranks": 65536 + 256}, {"pairs_hub_ranks": -128},
                    {"pairs_hub_q": 0}):
            with pytest.raises(esc.EscapeError) as e:
                ctx.set_params(dict(base, **bad))
            assert e.value.status == esc.ESC_EINVAL, bad
    finally:
        ctx.set_params(None)


def test_dense_hub_wheels(ctx):
    """Pattern 18 with the rim 4-cycles of chosen hubs counted as
    (1/2) sum over rim pairs of C(c,2), c = (A A)(i,j) over the adjacency of
    the hub's neighbourhood on the matrix cores: every hub from 4, 64 or
    512 neighbours (matrices of one to six 256-tiles a side, several per
    launch), the default choice, never; lists with and without apex ids.
    Same counts as the oracle."""
    import paper_1610_09411_amd as esc
    base = {"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20}
    g = synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2)
    want = oracle.count(g, 5, threads=8)
    gc = _dense_core_graph(3)
    wc = oracle.count(gc, 5, threads=8)
    try:
        for deg, ratio, flags in ((4, 1 << 20, 0), (64, 1 << 20, esc.ESC_F_COMPACT_LISTS), (512, 1 << 20, 0),
                                  (1024, 256, 0), (0, 1, 0)):
            ctx.set_params(dict(base, wheel_dense_deg=deg, wheel_dense_ratio=ratio))
            print("dense wheels from", deg, "ratio", ratio, "flags", flags, flush=True)
            assert ctx.count(g, 5, flags=flags) == want, (deg, ratio, flags)
            assert ctx.count(gc, 5, flags=flags) == wc, (deg, ratio, flags)
        for bad in ({"wheel_dense_deg": 3}, {"wheel_dense_deg": -1}, {"wheel_dense_ratio": 0},
                    {"wheel_dense_ratio": (1 << 20) + 1}):
            with pytest.raises(esc.EscapeError) as e:
                ctx.set_params(dict(base, **bad))
            assert e.value.status == esc.ESC_EINVAL, bad
    finally:
        ctx.set_params(None)


def test_dense_row_four_cliques(ctx):
    """Thm 4clique with K4 of the triangles (a,b,c), a earliest, read from
    C = B B^T on the matrix cores for vertices a with many
    out-neighbours (B: out-neighbours by neighbours of a): from 16, 64, 256
    out-neighbours or never, lists with and without apex ids.  Same 45
    counts and the same per-edge and per-vertex K4 as the oracle."""
    import paper_1610_09411_amd as esc
    base = {"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20}
    g = synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2)
    want = oracle.count(g, 5, threads=8)
    gf = synth.chung_lu(4000, 1.9, 20.0, 900.0, 6)
    S, it = oracle.sums(gf, 4, per_item=True)
    gc = _dense_core_graph(4)
    wc = oracle.count(gc, 5, threads=8)
    try:
        for dmin, flags in ((16, 0), (64, esc.ESC_F_COMPACT_LISTS), (256, 0), (0, 0)):
            ctx.set_params(dict(base, k4_dense_dplus=dmin))
            print("dense K4 rows from", dmin, "flags", flags, flush=True)
            assert ctx.count(g, 5, flags=flags) == want, (dmin, flags)
            assert ctx.count(gc, 5, flags=flags) == wc, (dmin, flags)
            counts, fr = ctx.fragments(gf, 4, flags=flags)
            assert np.array_equal(fr["k4_e"], it["k4_e"]), (dmin, flags)
            assert np.array_equal(fr["k4_v"], it["k4_v"]), (dmin, flags)
        for bad in ({"k4_dense_dplus": 15}, {"k4_dense_dplus": -1}):
            with pytest.raises(esc.EscapeError) as e:
                ctx.set_params(dict(base, **bad))
            assert e.value.status == esc.ESC_EINVAL, bad
    finally:
        ctx.set_params(None)


def test_stage_split_into_walk_and_product(ctx):
    """esc_last_products: with every product forced on, the three stages that
    have one report a walk no longer than the stage, a product taking the
    rest and the multiply-adds of their 256 x 256 tiles; the other stages and
    a call with the products off report no product."""
    base = {"task_chunk": 1, "wg_per_cu": 3, "k5_work_log2": 20}
    g = synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2)
    try:
        ctx.set_params(dict(base, pairs_hub_ranks=512, pairs_hub_q=1, wheel_dense_deg=64,
                            wheel_dense_ratio=1 << 20, k4_dense_dplus=16))
        ctx.count(g, 5)
        prof, prods = ctx.last_profile(), ctx.last_products()
        for st in ("k4_triangles", "pairs_13_17", "wheels"):
            walk, prod, macs = prods[st]
            assert macs > 0 and macs % (256 * 256 * 128) == 0, (st, macs)
            assert 0 <= walk <= prof[st][0] + 1e-3 and abs(walk + prod - prof[st][0]) < 1e-2, (st, prods[st])
        for st in ("orient", "triangles", "four_cycles", "five_cliques", "reduce", "five_cycles", "combine"):
            assert prods[st][2] == 0 and abs(prods[st][0] - prof[st][0]) < 1e-3, st
        ctx.set_params(dict(base, pairs_hub_ranks=0, wheel_dense_deg=0, k4_dense_dplus=0))
        ctx.count(g, 5)
        assert all(v[2] == 0 for v in ctx.last_products().values())
    finally:
        ctx.set_params(None)


def test_time_sliced_launches_give_same_counts():
    """Per-source kernels launched in 2 ms slices (ESC_SLICE_MS, read when
    the context is created): each stage is relaunched from its task counter
    until every task is taken; counts equal the oracle's."""
    import paper_1610_09411_amd as esc
    g = synth.chung_lu(20000, 2.1, 20.0, 1500.0, 2)
    want = oracle.count(g, 5, threads=8)
    os.environ["ESC_SLICE_MS"] = "2"
    try:
        c = esc.Context(0)
    finally:
        del os.environ["ESC_SLICE_MS"]
    try:
        assert c.count(g, 5) == want
        assert c.count(g, 4) == want[:11]
        batch = [synth.from_spec(s) for s in synth.batch_specs(30, 5)]
        rows, _ = c.count_batched(batch, 5)
        for i in (0, 11, 29):
            assert [int(x) for x in rows[i]] == oracle.count(batch[i], 5), i
    finally:
        c.close()


@pytest.mark.parametrize("a", [2, 3])
def test_degrees_above_2_16(ctx, a):
    """K_{a,70000}: hubs of degree 70000 >= 2^16, so the per-source tables
    keep 32-bit counts, the wheel pass its 32-bit key ranges and the 5-cycle
    pass the Wnt order; induced counts in closed form (4-subsets with x
    vertices on the small side: an independent set, a 3-star, a 4-cycle;
    5-subsets: an independent set, a 4-star, K_{2,3})."""
    b = 70000
    g = synth.from_edges(a + b, [(u, a + v) for u in range(a) for v in range(b)], "K_%d,%d" % (a, b))
    want = [0] * 45
    want[0] = a * comb(b, 3) + b * comb(a, 3)
    want[3] = comb(a, 2) * comb(b, 2)
    want[6] = comb(a, 4) + comb(b, 4)
    want[11] = a * comb(b, 4) + b * comb(a, 4)
    want[11 + 12] = comb(a, 2) * comb(b, 3) + comb(a, 3) * comb(b, 2)
    want[32] = comb(a, 5) + comb(b, 5)
    assert ctx.count(g, 5) == want
    assert ctx.count(g, 4) == want[:11]
    # and a hub of degree >= 2^16 that also has triangles and wheels: the
    # hub joined to a path and a clique
    h = synth.from_edges(b + 1, [(0, v) for v in range(1, b + 1)] + [(v, v + 1) for v in range(1, b)] +
                         [(u, v) for u in range(1, 40) for v in range(u + 1, 40)], "hub 70000")
    assert ctx.count(h, 5) == oracle.count(h, 5, threads=8)


def _degree_order_work(g):
    d = g.degrees()
    order = np.lexsort((np.arange(g.n), d))            # by degree, ties by id
    rank = np.empty(g.n, np.int64)
    rank[order] = np.arange(g.n)
    dp = np.zeros(g.n, np.int64)
    for u in range(g.n):
        nb = g.col[g.row_ptr[u]:g.row_ptr[u + 1]]
        dp[u] = int((rank[nb] > rank[u]).sum())
    dm = d - dp
    return {"W++": int((dp * (dp - 1) // 2).sum()), "W+-": int((dp * dm).sum()),
            "W": int((d * (d - 1) // 2).sum()), "max_dplus": int(dp.max()) if g.n else 0}


def test_noninduced_and_work_counters(ctx):
    """esc_last_noninduced against the oracle's non-induced counts (App. B:
    N = A C), and esc_last_work against the definitions of its counters
    (out-wedges and in-out wedges of the degree-ordered DAG, wedges, the
    largest out-degree) and the oracle's triangle and diamond totals."""
    for g in _cases_small()[::3] + [synth.chung_lu(3000, 2.1, 12.0, 400.0, 1), synth.er_small(4),
                                    synth.erdos_renyi(160, 0.6, 11), _dense_core_graph(2, core=90, per=120)]:
        S = oracle.sums(g, 5)
        want_non = oracle.noninduced_from_sums(S, 4) + oracle.noninduced_from_sums(S, 5)
        for k in (4, 5):
            ctx.count(g, k)
            assert ctx.last_noninduced(k) == want_non[:11 if k == 4 else 45], (g.name, k)
            w = ctx.last_work()
            dw = _degree_order_work(g)
            for key in ("W++", "W+-", "W", "max_dplus"):
                assert w[key] == dw[key], (g.name, k, key)
            assert (w["T"], w["D"], w["n"], w["m"]) == (S["T"], S["D"], g.n, g.m), (g.name, k)
            # directed 3-paths and directed bipyramids (the oracle enumerates
            # them; the 5-clique pass, and so DBP, runs for k = 5 only)
            assert w["DP"] == S["DP"], (g.name, k)
            assert w["DBP"] == (S["DBP"] if k == 5 else 0), (g.name, k)


def _big_core_graph(seed, core=2300, per=1500):
    """A near-clique core (pairs missing with probability 0.03) and periphery
    vertices tied to random fractions (up to 0.3) of it and sparsely to each
    other; returns the graph and its dense 0/1 adjacency."""
    rng = np.random.default_rng(seed)
    n = core + per
    p = np.full((n, n), 0.01)
    p[:core, :core] = 0.97
    p[:core, core:] = (rng.random(per) * 0.3)[None, :]
    a = np.triu(rng.random((n, n)) < p, 1)
    a = a | a.T
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(a.sum(1))
    col = np.nonzero(a)[1].astype(np.int32)
    return synth.Graph(n, rp, col, "big core %d" % seed), a


def test_triangles_of_large_out_neighbourhoods(ctx):
    """Thm 4vertex-tri on out-neighbourhoods too large for one wave's hash set
    (d+ above 1024, up to beyond 2048: a workgroup's set of 2^12 or 2^13
    slots): t of every arc equals (A^2)(u,v) and t of every vertex half the
    diagonal of A^3, the definitions over the dense adjacency; sampled
    per-edge K4 and C4 equal the oracle's; the 11 counts sum to C(n,4)."""
    g, a = _big_core_graph(3)
    deg = g.degrees()
    rank = np.empty(g.n, np.int64)
    rank[np.lexsort((np.arange(g.n), deg))] = np.arange(g.n)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    dplus = np.bincount(rows[rank[g.col] > rank[rows]], minlength=g.n)
    assert dplus.max() > 2048 and ((dplus > 1024) & (dplus <= 2048)).any()
    counts, fr = ctx.fragments(g, 4)
    assert sum(counts) == comb(g.n, 4)
    af = a.astype(np.float64)
    a2 = af @ af
    assert np.array_equal(fr["tri_e"], a2[rows, g.col].astype(np.uint64))
    assert np.array_equal(fr["tri_v"], np.rint((a2 * af).sum(1) / 2).astype(np.uint64))
    rng = random.Random(3)
    big = [int(v) for v in np.argsort(-dplus)[:4]]
    for v in big + [rng.randrange(g.n) for _ in range(8)]:
        s, t = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
        for p in [s, t - 1, rng.randrange(s, t)]:
            u = int(g.col[p])
            exp = oracle.edge_fragments(g, v, u)
            assert fr["k4_e"][p] == exp["k4"], (v, u)
            assert fr["c4_e"][p] == exp["c4"], (v, u)
