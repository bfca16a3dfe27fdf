"""The min-wedge anchor side (BBC_SIDE_MIN_WEDGES): the side whose walk has
fewer wedges, sum of C(deg, 2) over the other side, with the default rule
(smaller side, tie -> V) breaking ties.  The count must not depend on it;
the side it reports is checked against the wedge sums computed here."""
import numpy as np
import pytest

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


def expected_side(g):
    du = np.diff(g.offsets).astype(np.int64)
    dv = np.bincount(g.adj, minlength=g.n_v).astype(np.int64)
    w_anchor_v = int((du * (du - 1) // 2).sum())  # centres U
    w_anchor_u = int((dv * (dv - 1) // 2).sum())
    if w_anchor_u != w_anchor_v:
        return bbc.SIDE_U if w_anchor_u < w_anchor_v else bbc.SIDE_V
    return bbc.SIDE_U if g.n_u < g.n_v else bbc.SIDE_V


def check(ctx, g):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    got = ctx.count(off, adj, sg, g.n_v, opts=bbc.options(side="min_wedges"))
    assert got == oracle.count(g)
    assert ctx.stats()["side"] == expected_side(g)
    return ctx.stats()["side"]


def hubs_on_v(seed, n_u=1000, n_v=5000, hubs=20):
    """U is the smaller side, but a few V hubs adjacent to all of U make the
    walk from U (centres V) far longer than the walk from V."""
    rng = np.random.default_rng(seed)
    u = [np.tile(np.arange(n_u), hubs), rng.integers(0, n_u, n_v - hubs)]
    v = [np.repeat(np.arange(hubs), n_u), np.arange(hubs, n_v)]
    u, v = np.concatenate(u), np.concatenate(v)
    s = np.where(rng.random(u.size) < 0.3, -1, 1)
    return synth.from_edges(n_u, n_v, u, v, s)


def test_min_wedges_picks_the_larger_side_when_cheaper(ctx):
    g = hubs_on_v(1)
    assert g.n_u < g.n_v
    assert check(ctx, g) == bbc.SIDE_V
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    ctx.count(off, adj, sg, g.n_v)
    assert ctx.stats()["side"] == bbc.SIDE_U  # the paper's rule: the smaller side


@pytest.mark.parametrize("seed", range(1, 6))
def test_min_wedges_random(ctx, seed):
    rng = np.random.default_rng(seed)
    check(ctx, synth.chung_lu_graph(4000, 2500, 30000, 2.1, 2.6, 800, 300, seed, p_neg=0.3))
    check(ctx, synth.small_random_graph(rng, max_n=30))


def test_min_wedges_degenerate_and_per_vertex(ctx):
    for n_u, n_v in [(0, 0), (3, 0), (0, 4), (5, 5)]:
        e = synth.from_edges(n_u, n_v, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int8))
        check(ctx, e)
    g = hubs_on_v(2, 300, 900, 6)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    import torch

    pv = torch.zeros(g.n_u + g.n_v, dtype=torch.int64, device="cuda:0")
    ctx.count(off, adj, sg, g.n_v, per_vertex=pv, opts=bbc.options(side="min_wedges"))
    assert np.array_equal(pv.cpu().numpy().astype(np.uint64), oracle.per_vertex(g))


def test_min_wedges_rejected_where_it_does_not_apply(ctx):
    g = hubs_on_v(3, 200, 600, 4)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_classes(off, adj, sg, g.n_v, opts=bbc.options(side="min_wedges"))
    assert e.value.status == bbc.EINVAL
    batch = bbc.Batch([g, g])
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_batched(batch, opts=bbc.options(side="min_wedges"))
    assert e.value.status == bbc.EINVAL
