"""bbc_count_noalloc: the allocation-free variant of bbc_count, called through
the C ABI and compared with bbc_count on the same inputs (bit-exact: the
counts are integers).  Two calls in a row, the second on a smaller graph, so
the fixed scratch is reused with stale contents from the first; per-vertex
counts, the min-wedge side, an oversized graph and dense blocks are covered
too.  No call here may leave the device's fixed scratch in use: the file also
runs after every other GPU test."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2601_17707_amd import bbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import __graft_entry__

    __graft_entry__._ensure_built()
    c = bbc.Context(0)
    yield c
    c.close()


def say(*a):
    print(*a, flush=True)


def both(ctx, g, per_vertex=False, **kw):
    """(bbc_count, bbc_count_noalloc) results on the same device tensors."""
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    o = bbc.options(**kw)
    if per_vertex:
        pv_a = torch.full((g.n_u + g.n_v,), -1, dtype=torch.int64, device="cuda:0")
        pv_b = torch.full((g.n_u + g.n_v,), -7, dtype=torch.int64, device="cuda:0")
        a = ctx.count(off, adj, sg, g.n_v, per_vertex=pv_a, opts=o)
        b = ctx.count_noalloc(off, adj, sg, g.n_v, per_vertex=pv_b, opts=o)
        return (a, pv_a.cpu().numpy()), (b, pv_b.cpu().numpy())
    a = ctx.count(off, adj, sg, g.n_v, opts=o)
    b = ctx.count_noalloc(off, adj, sg, g.n_v, opts=o)
    return a, b


def test_two_calls_second_smaller(ctx):
    big = synth.chung_lu_graph(60_000, 30_000, 900_000, 2.1, 2.1, 5_000, 5_000, seed=11, p_neg=0.3)
    small = synth.uniform_graph(2_000, 1_000, 20_000, 0.3, seed=12)
    say(f"noalloc: big graph m={big.m}, then small m={small.m}")
    a1, b1 = both(ctx, big)
    a2, b2 = both(ctx, small)
    say(f"noalloc: {a1} == {b1}, {a2} == {b2}")
    assert a1 == b1 and a1 > 0
    assert a2 == b2 and a2 > 0
    # and back again, then the small one once more (stale scratch from a larger graph)
    assert both(ctx, big) == (a1, a1)
    assert both(ctx, small) == (a2, a2)


def test_per_vertex_and_sides(ctx):
    g = synth.chung_lu_graph(5_000, 8_000, 120_000, 2.2, 2.0, 900, 1_500, seed=21, p_neg=0.25)
    (a, pa), (b, pb) = both(ctx, g, per_vertex=True)
    say(f"noalloc per-vertex: totals {a} {b}")
    assert a == b
    np.testing.assert_array_equal(pa, pb)
    for side in ("u", "v", "min_wedges"):
        a, b = both(ctx, g, side=side)
        assert a == b, side
    g2 = synth.uniform_graph(300, 500, 4_000, 0.5, seed=22)
    (a, pa), (b, pb) = both(ctx, g2, per_vertex=True)
    assert a == b
    np.testing.assert_array_equal(pa, pb)


def test_degenerate_graphs(ctx):
    empty = synth.from_edges(5, 7, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int64))
    assert both(ctx, empty) == (0, 0)
    one_side = synth.complete_graph(1, 9)
    assert both(ctx, one_side) == (0, 0)
    k = synth.complete_graph(4, 6)
    a, b = both(ctx, k)
    assert a == b == 6 * 15


def test_oversized_graph_is_rejected_untouched(ctx):
    g = synth.uniform_graph(400_000, 300_000, 2_000_000, 0.3, seed=31)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    lib = bbc.load_library()
    out = ctypes.c_uint64(12345)
    o = bbc.options()
    st = lib.bbc_count_noalloc(ctx._h, g.n_u, g.n_v, g.m, off.data_ptr(), adj.data_ptr(), sg.data_ptr(),
                               ctypes.byref(out), None, ctypes.byref(o), None)
    say(f"noalloc oversized: status {st}: {ctx.last_error()}")
    assert st == bbc.ETOOBIG
    assert out.value == 12345
    assert "bytes of scratch" in ctx.last_error()
    # the context still works afterwards, through both entry points
    small = synth.uniform_graph(2_000, 1_000, 20_000, 0.3, seed=12)
    a, b = both(ctx, small)
    assert a == b


def test_dense_blocks_and_bad_input_rejected(ctx):
    g = synth.uniform_graph(200, 100, 2_000, 0.3, seed=41)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    ids = torch.arange(4, dtype=torch.int32, device="cuda:0")
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_noalloc(off, adj, sg, g.n_v, opts=bbc.options(blocks=[(ids, ids)]))
    assert e.value.status == bbc.EINVAL
    bad = sg.clone()
    bad[3] = 2
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_noalloc(off, adj, bad, g.n_v)
    assert e.value.status == bbc.ESIGN
    a, b = both(ctx, g)
    assert a == b
