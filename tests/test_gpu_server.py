"""The request server (esc_server_*): results are the same alone and in the
mix, requests overlap and share launches, admission respects the budget.

Exact integer counts: each served result must equal the single-graph call
on the same graph (and the oracle where it is quick).
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1610_09411_amd as esc
    c = esc.Context(0)
    yield c
    c.close()


def _requests(count, seed, nmax=None):
    specs = synth.request_specs(count, seed)
    if nmax:
        specs = [s for s in specs if s[1] <= nmax]
    return [synth.from_spec(s) for s in specs]


def test_served_results_equal_alone(ctx):
    import paper_1610_09411_amd as esc
    graphs = _requests(96, 1)
    graphs += [synth.from_edges(0, []), synth.from_edges(3, [(0, 1)]), synth.er_small(3)]
    print("requests", len(graphs), "max n", max(g.n for g in graphs), flush=True)
    alone = [ctx.count(g, 5) for g in graphs]
    with esc.Server(ctx, max_inflight=4) as srv:
        tickets = [srv.submit(g, 5) for g in graphs]      # a burst: queued while others run
        served = [srv.wait(t)[0] for t in tickets]
        st = srv.stats()
    print("server stats", st, flush=True)
    for i, (a, b) in enumerate(zip(alone, served)):
        assert a == b, (i, graphs[i].name)
    for i, g in enumerate(graphs):
        if g.n <= 3000:
            assert served[i] == oracle.count(g, 5, threads=8), (i, g.name)
    assert st["completed"] == len(graphs)
    assert st["launches"] < len(graphs)          # small requests shared launches
    assert st["batched_requests"] > 0
    assert st["peak_inflight"] >= 2              # launches overlapped on the device


def test_mixed_k_and_polling(ctx):
    import paper_1610_09411_amd as esc
    graphs = _requests(40, 2, nmax=5000)
    with esc.Server(ctx, max_inflight=3) as srv:
        tickets = [srv.submit(g, 4 if i % 3 == 0 else 5) for i, g in enumerate(graphs)]
        results = {}
        while len(results) < len(tickets):
            for i, t in enumerate(tickets):
                if i not in results:
                    r = srv.poll(t)
                    if r is not None:
                        results[i] = r
    for i, g in enumerate(graphs):
        k = 4 if i % 3 == 0 else 5
        counts, seconds = results[i]
        assert counts == ctx.count(g, k), (i, k)
        assert seconds >= 0.0


def test_invalid_request_does_not_poison_its_batch(ctx):
    import paper_1610_09411_amd as esc
    good = _requests(12, 3, nmax=3000)
    bad = synth.Graph(4, np.array([0, 1, 2, 3, 4], np.int32), np.array([1, 0, 3, 7], np.int32))   # id 7 out of range
    asym = synth.Graph(3, np.array([0, 1, 1, 2], np.int32), np.array([1, 1], np.int32))          # not symmetric
    with esc.Server(ctx, max_inflight=1) as srv:
        with pytest.raises(esc.EscapeError) as e:
            srv.submit(synth.Graph(2, np.array([0, 2, 1], np.int32), np.array([1, 0], np.int32)))  # offsets decrease
        assert e.value.status == esc.ESC_ERANGE
        order = good[:6] + [bad] + good[6:] + [asym]
        tickets = [srv.submit(g, 5) for g in order]
        for g, t in zip(order, tickets):
            if g is bad or g is asym:
                with pytest.raises(esc.EscapeError) as e:
                    srv.wait(t)
                assert e.value.status in (esc.ESC_ERANGE, esc.ESC_ENOTSIMPLE)
            else:
                assert srv.wait(t)[0] == ctx.count(g, 5)


def test_admission_budget(ctx):
    """A small device budget: requests run within it (peak estimated
    footprint in flight <= budget) and a request that cannot fit alone fails
    with ESC_ENOMEM instead of blocking the queue."""
    import paper_1610_09411_amd as esc
    budget = 400 << 20
    small_ctx = esc.Context(0, hbm_budget_bytes=budget)
    try:
        graphs = _requests(24, 4, nmax=4000)
        too_big = synth.chung_lu(45000, 2.2, 10.0, 600.0, 5)      # tables alone exceed the budget
        with esc.Server(small_ctx, max_inflight=4) as srv:
            tickets = [srv.submit(g, 5) for g in graphs[:12]]
            tb = srv.submit(too_big, 5)
            tickets += [srv.submit(g, 5) for g in graphs[12:]]
            served = [srv.wait(t)[0] for t in tickets]
            with pytest.raises(esc.EscapeError) as e:
                srv.wait(tb)
            assert e.value.status == esc.ESC_ENOMEM
            st = srv.stats()
        assert st["budget_bytes"] == budget
        assert st["peak_reserved_bytes"] <= budget
        for g, r in zip(graphs, served):
            assert r == ctx.count(g, 5)
    finally:
        small_ctx.close()
