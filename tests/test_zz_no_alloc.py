"""The no-allocation entry point (every device buffer of the call taken from
the library's fixed per-GPU region) against esc_count_subgraphs, through the
C ABI: the same counts on two calls in a row, the second on a smaller
graph, and a graph too large for the region refused with ESC_ENOMEM."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def test_noalloc_equals_allocating_entry_point():
    import torch
    import paper_1610_09411_amd as esc
    with esc.Context(0) as ctx:
        big = synth.chung_lu(6000, 2.1, 14.0, 600.0, 31)
        small = synth.er_small(3)
        for g, k in ((big, 5), (small, 5), (big, 4)):
            print(g.name, g.n, g.m, k, flush=True)
            want = esc.esc_count_subgraphs(ctx.ptr, g.n, g.row_ptr, g.col, k)
            got = esc.esc_count_subgraphs_noalloc(ctx.ptr, g.n, g.row_ptr, g.col, k)
            assert got == want, g.name
        # device input, and the allocating call still works afterwards
        rp = torch.from_numpy(small.row_ptr).cuda()
        ci = torch.from_numpy(small.col).cuda()
        got = esc.esc_count_subgraphs_noalloc(ctx.ptr, small.n, rp, ci, 5)
        assert got == esc.esc_count_subgraphs(ctx.ptr, small.n, small.row_ptr, small.col, 5)
        # too large for the region: refused, the context keeps working
        huge = synth.chung_lu(300000, 2.1, 20.0, 2000.0, 32)
        with pytest.raises(esc.EscapeError) as e:
            esc.esc_count_subgraphs_noalloc(ctx.ptr, huge.n, huge.row_ptr, huge.col, 5)
        assert e.value.status == esc.ESC_ENOMEM
        assert esc.esc_count_subgraphs_noalloc(ctx.ptr, small.n, small.row_ptr, small.col, 5) == \
            esc.esc_count_subgraphs(ctx.ptr, small.n, small.row_ptr, small.col, 5)
