"""GPU parity of balanced (2,k)-bicliques (bbc_count_bicliques) with the
oracle's general-k walk, exact to 128 bits: random graphs on both pair
sides, k = 1..6, k = 2 against the balanced count, every counter width with
terms past 64 bits, overflow, degenerate inputs and rejected arguments."""
from math import comb

import numpy as np
import pytest

import oracle
from paper_2601_17707_amd import bbc, synth

pytestmark = pytest.mark.gpu

SIDES = {"auto": oracle.SIDE_AUTO, "u": oracle.SIDE_U, "v": oracle.SIDE_V}


@pytest.fixture(scope="module")
def ctx():
    import __graft_entry__

    __graft_entry__._ensure_built()
    c = bbc.Context(0)
    yield c
    c.close()


def gpu(ctx, g, k, side="auto"):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    return ctx.count_bicliques(off, adj, sg, g.n_v, k, opts=bbc.options(side=side))


def check(ctx, g, k, side="auto"):
    want = oracle.count_bicliques(g, k, SIDES[side])
    got = gpu(ctx, g, k, side)
    assert got == want, (k, side)
    return got


@pytest.mark.parametrize("seed", range(1, 4))
@pytest.mark.parametrize("side", ["auto", "u", "v"])
def test_random_graphs(ctx, seed, side):
    rng = np.random.default_rng(seed)
    g = synth.chung_lu_graph(3000, 1500, 40000, 2.1, 2.1, 600, 600, seed, p_neg=0.35)
    small = synth.small_random_graph(rng, max_n=40)
    for k in (1, 2, 3, 4, 6):
        check(ctx, g, k, side)
        check(ctx, small, k, side)


def test_k2_is_the_balanced_count(ctx):
    g = synth.chung_lu_graph(5000, 2000, 60000, 2.1, 2.3, 900, 500, 9, p_neg=0.25)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    t = ctx.count(off, adj, sg, g.n_v)
    for side in ("u", "v"):
        assert gpu(ctx, g, 2, side) == t == oracle.count(g)


def wide_graph(seed=7):
    """V anchors of degree 3 .. 9,000 plus two adjacent to all 200,000 U
    vertices and one to 150,000: pairs sharing up to 200,000 centres fill
    32-bit counter fields."""
    rng = np.random.default_rng(seed)
    n_u, n_v = 200000, 40
    us, vs = [np.arange(n_u), np.arange(n_u), rng.choice(n_u, 150000, replace=False)], \
        [np.zeros(n_u, np.int64), np.ones(n_u, np.int64), np.full(150000, 2)]
    for v in range(3, n_v):
        d = int(rng.choice([3, 12, 90, 200, 1500, 9000]))
        us.append(rng.choice(n_u, d, replace=False))
        vs.append(np.full(d, v))
    u, v = np.concatenate(us), np.concatenate(vs)
    s = np.where(rng.random(u.size) < 0.4, -1, 1)
    return synth.from_edges(n_u, n_v, u, v, s)


def test_every_counter_width_past_64_bits(ctx):
    g = wide_graph()
    for k in (3, 5, 8):
        got = check(ctx, g, k, "v")
        if k == 8:
            assert got >= 1 << 100
    with pytest.raises(OverflowError):
        oracle.count_bicliques(g, 16, oracle.SIDE_V)
    with pytest.raises(bbc.BbcError) as e:
        gpu(ctx, g, 16, "v")
    assert e.value.status == bbc.EOVERFLOW


def test_one_pair_exact_and_overflow(ctx):
    for n, k in ((1000, 9), (3000, 12), (255, 16), (256, 16)):
        g = synth.complete_graph(2, n)
        assert gpu(ctx, g, k, "u") == comb(n, k)
        assert gpu(ctx, g, k, "v") == comb(n, 2) * comb(2, k)
    g = synth.complete_graph(2, 20000)
    with pytest.raises(bbc.BbcError) as e:
        gpu(ctx, g, 16, "u")
    assert e.value.status == bbc.EOVERFLOW


@pytest.mark.parametrize("k", [3, 4])
@pytest.mark.parametrize("side", ["auto", "u", "v"])
def test_band_crossing(ctx, k, side):
    """70,000 V and 200,000 U vertices, 1.2M edges, hubs of about 3,000 on
    both sides: anchors of either side fall in the 4-, 8- and 16-bit
    layouts, whose bands (32,768, 16,384 and 8,192 endpoint ranks) the rank
    ranges cross several times; the automatic side puts the pair on U."""
    g = synth.chung_lu_graph(200_000, 70_000, 1_200_000, 2.1, 2.1, 4000, 4000, 11, p_neg=0.35)
    got = check(ctx, g, k, side)
    assert got > 0
    if side == "auto":
        assert got == oracle.count_bicliques(g, k, oracle.SIDE_U)


def test_degenerate(ctx):
    for n_u, n_v, edges in [(1, 1, [(0, 0, 1)]), (3, 2, []), (2, 1, [(0, 0, 1), (1, 0, -1)]),
                            (2, 2, [(0, 0, 1), (0, 1, -1), (1, 0, -1), (1, 1, -1)])]:
        e = np.array(edges, np.int64).reshape(-1, 3)
        g = synth.from_edges(n_u, n_v, e[:, 0], e[:, 1], e[:, 2])
        for side in ("auto", "u", "v"):
            for k in (1, 2, 3, 16):
                check(ctx, g, k, side)


def test_rejected_arguments(ctx):
    import torch

    g = synth.uniform_graph(200, 100, 2000, 0.3, 3)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    for k in (0, -1, 17):
        with pytest.raises(bbc.BbcError) as e:
            ctx.count_bicliques(off, adj, sg, g.n_v, k)
        assert e.value.status == bbc.EINVAL
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_bicliques(off, adj, sg, g.n_v, 3, opts=bbc.options(side="min_wedges"))
    assert e.value.status == bbc.EINVAL
    blk = [(torch.arange(5, dtype=torch.int32, device="cuda:0"), torch.arange(5, dtype=torch.int32, device="cuda:0"))]
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_bicliques(off, adj, sg, g.n_v, 3, opts=bbc.options(blocks=blk))
    assert e.value.status == bbc.EINVAL
    bad = adj.clone()
    bad[0] = g.n_v
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_bicliques(off, bad, sg, g.n_v, 3)
    assert e.value.status == bbc.ERANGE
