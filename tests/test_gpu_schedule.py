"""The static schedule (BBC_SCHED_STATIC: workgroup b takes positions b,
b + G, ... of the descending-work anchor list) must give the same results
as the dynamic queue and the oracle on every entry point that runs the
wedge kernel, at every instantiated shape and grid."""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_17707_amd import bbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import __graft_entry__

    __graft_entry__._ensure_built()
    c = bbc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("seed", range(1, 4))
def test_static_matches_oracle_every_shape(ctx, seed):
    g = synth.chung_lu_graph(20000, 8000, 150000, 2.1, 2.1, 3000, 3000, seed, p_neg=0.3)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    want = oracle.count(g)
    for bw, wg in bbc.WEDGE_SHAPES:
        for wpc in (1, 2):
            o = bbc.options(band_words=bw, wg_size=wg, wg_per_cu=wpc, schedule="static")
            assert ctx.count(off, adj, sg, g.n_v, opts=o) == want, (bw, wg, wpc)
            assert ctx.stats()["schedule"] == bbc.SCHED_STATIC
    # grid far larger than the anchor list: most workgroups take nothing
    small = synth.small_random_graph(np.random.default_rng(seed), max_n=20)
    so, sa, ss = bbc.graph_tensors(small, "cuda:0")
    assert ctx.count(so, sa, ss, small.n_v, opts=bbc.options(schedule="static")) == oracle.count(small)


def test_static_other_entry_points(ctx):
    g = synth.chung_lu_graph(6000, 2500, 50000, 2.1, 2.2, 900, 700, 11, p_neg=0.35)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    st = bbc.options(schedule="static")
    pv = torch.zeros(g.n_u + g.n_v, dtype=torch.int64, device="cuda:0")
    assert ctx.count(off, adj, sg, g.n_v, per_vertex=pv, opts=st) == oracle.count(g)
    assert np.array_equal(pv.cpu().numpy().astype(np.uint64), oracle.per_vertex(g))
    assert ctx.count_classes(off, adj, sg, g.n_v, opts=bbc.options(side="u", schedule="static")) == \
        oracle.count_classes(g, oracle.SIDE_U)
    assert ctx.count_bicliques(off, adj, sg, g.n_v, 3, opts=bbc.options(side="v", schedule="static")) == \
        oracle.count_bicliques(g, 3, oracle.SIDE_V)
    graphs = [synth.chung_lu_graph(500 + 40 * i, 300 + 25 * i, 3000 + 300 * i, 2.1, 2.1, 200, 200, 20 + i)
              for i in range(12)]
    batch = bbc.Batch(graphs)
    got = ctx.count_batched(batch, opts=st).cpu().numpy()[: len(graphs)]
    assert list(got) == [oracle.count(h) for h in graphs]


def test_bad_schedule_rejected(ctx):
    g = synth.uniform_graph(100, 80, 800, 0.3, 2)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    o = bbc.options()
    o.schedule = 2
    with pytest.raises(bbc.BbcError) as e:
        ctx.count(off, adj, sg, g.n_v, opts=o)
    assert e.value.status == bbc.EINVAL
