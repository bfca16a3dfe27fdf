"""GPU parity of the wedge kernel's regimes and queue chunks.

Light anchors (few wedges, at most 63 centres, fewer than 2^20 vertices
ranked above them in their graph) are counted by one wavefront in a hashed
LDS table; every other anchor by a whole workgroup, queue_chunk anchors per
pop.  Which anchor goes where never changes the count, so every setting is
compared bit for bit with the CPU oracle: the wave regime off
(wave_max_work = -1), on at several thresholds, and with chunked pops.
"""
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


def say(*a):
    print(*a, flush=True)


def gpu_count(ctx, g, side="auto", **kw):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    return ctx.count(off, adj, sg, g.n_v, opts=bbc.options(side=side, **kw))


SETTINGS = [dict(wave_max_work=-1), dict(), dict(wave_max_work=1), dict(wave_max_work=16),
            dict(wave_max_work=200), dict(queue_chunk=3), dict(queue_chunk=64, wave_max_work=300),
            dict(schedule="static", queue_chunk=5), dict(wave_max_work=100000)]


@pytest.mark.parametrize("kw", SETTINGS, ids=[str(k) for k in SETTINGS])
def test_random_graphs_every_setting(ctx, kw):
    rng = np.random.default_rng(5)
    for i in range(60):
        g = synth.small_random_graph(rng, max_n=40)
        side = ("auto", "u", "v")[i % 3]
        want = oracle.count(g, {"auto": oracle.SIDE_AUTO, "u": oracle.SIDE_U, "v": oracle.SIDE_V}[side])
        assert gpu_count(ctx, g, side, **kw) == want, (i, side, kw)


@pytest.mark.parametrize("kw", SETTINGS, ids=[str(k) for k in SETTINGS])
def test_power_law_every_setting(ctx, kw):
    """Anchors of every kind: light ones, workgroup ones with few and many
    bands, hubs."""
    g = synth.chung_lu_graph(60_000, 25_000, 400_000, 2.1, 2.0, 3_000, 900, seed=77, p_neg=0.35)
    want = oracle.count(g)
    say("power law", kw, want)
    assert gpu_count(ctx, g, **kw) == want
    assert gpu_count(ctx, g, "u", **kw) == want


def test_high_degree_light_work_anchor(ctx):
    """An anchor with 100 centres but only 70 wedges above it (the one
    higher-degree anchor shares 70 of its centres) exceeds the wave regime's
    63 centres and must take the workgroup path; its neighbours are light."""
    rng = np.random.default_rng(3)
    us, vs, ss = [], [], []
    # anchors on V: 0 (degree 100), 1 (degree 150), 2..40 small
    for c in range(100):
        us.append(c), vs.append(0), ss.append(1 if rng.random() < 0.7 else -1)
    for c in list(range(30, 100)) + list(range(100, 180)):
        us.append(c), vs.append(1), ss.append(1 if rng.random() < 0.6 else -1)
    for v in range(2, 41):
        for c in rng.choice(180, size=int(rng.integers(2, 9)), replace=False):
            us.append(int(c)), vs.append(v), ss.append(1 if rng.random() < 0.5 else -1)
    g = synth.from_edges(180, 41, us, vs, ss)
    want = oracle.count(g, oracle.SIDE_V)
    for kw in SETTINGS:
        assert gpu_count(ctx, g, "v", **kw) == want, kw


def test_anchor_side_wider_than_the_light_key(ctx):
    """More than 2^20 anchors: the lowest-ranked ones have more than 2^20
    vertices above them and must stay out of the wave regime."""
    g = synth.uniform_graph(2_300_000, 1_100_000, 3_500_000, 0.4, seed=9)
    assert g.n_v > (1 << 20)
    want = oracle.count(g, oracle.SIDE_V)
    say("wide anchor side", g.m, want)
    for kw in (dict(), dict(wave_max_work=-1), dict(queue_chunk=16)):
        assert gpu_count(ctx, g, "v", **kw) == want, kw


def test_batch_every_setting(ctx):
    graphs = [synth.chung_lu_graph(int(n_u), int(n_v), int(m), 2.0, 2.2, 200, 300, seed=int(i), p_neg=0.3)
              for i, (n_u, n_v, m) in enumerate([(300, 500, 3000), (2000, 800, 15000), (50, 60, 900),
                                                 (4000, 4000, 30000), (900, 150, 4000), (10, 10, 40)])]
    want = [oracle.count(g) for g in graphs]
    batch = bbc.Batch(graphs, "cuda:0")
    for kw in SETTINGS:
        got = ctx.count_batched(batch, opts=bbc.options(**kw)).cpu().tolist()
        assert got == want, kw
        plan = ctx.plan(batch, opts=bbc.options(**kw))
        for _ in range(2):
            plan.launch()
            assert plan.wait().cpu().tolist()[:len(graphs)] == want, kw
        plan.close()


def test_hybrid_with_light_background(ctx):
    """Dense-block anchors always take the workgroup path (their cross
    term); light background anchors around them use the wave regime."""
    g = synth.hybrid_graph(20_000, 10_000, 60_000, 2, 160, 0.5, 0.1, seed=5)
    want = oracle.count(g)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    blocks = [(torch.from_numpy(c).to("cuda:0"), torch.from_numpy(r).to("cuda:0")) for r, c in g.meta["blocks"]]
    for kw in (dict(), dict(wave_max_work=-1), dict(queue_chunk=4)):
        assert ctx.count(off, adj, sg, g.n_v, opts=bbc.options(blocks=blocks, **kw)) == want, kw


def test_rejected_regime_options(ctx):
    g = synth.uniform_graph(100, 50, 500, 0.3, seed=1)
    for kw in (dict(queue_chunk=-1), dict(queue_chunk=65537), dict(wave_max_work=-2)):
        with pytest.raises(bbc.BbcError) as e:
            gpu_count(ctx, g, **kw)
        assert e.value.status == bbc.EINVAL
