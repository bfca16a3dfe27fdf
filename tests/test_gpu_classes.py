"""GPU parity of the six sign-pattern classes (bbc_count_classes) with the
oracle's three-bucket walk, bit-exact, on the case study's sample network,
random graphs whose anchors fall in every counter width (4, 8, 16 and
32-bit fields), both pair sides, ragged and degenerate inputs."""
import numpy as np
import pytest

import oracle
from paper_2601_17707_amd import bbc, synth
from tests.fixtures import load_graphs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import __graft_entry__

    __graft_entry__._ensure_built()
    c = bbc.Context(0)
    yield c
    c.close()


SIDES = {"auto": oracle.SIDE_AUTO, "u": oracle.SIDE_U, "v": oracle.SIDE_V}


def check(ctx, g, side="auto"):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    got = ctx.count_classes(off, adj, sg, g.n_v, opts=bbc.options(side=side))
    want = oracle.count_classes(g, SIDES[side])
    assert got == want
    assert sum(got[:4]) == ctx.count(off, adj, sg, g.n_v, opts=bbc.options(side=side))
    return got


def test_case_study_sample(ctx):
    g, exp = load_graphs("drug_target_sample.txt")["drug_target"]
    got = check(ctx, g, "u")
    assert got == [exp["class_" + n] for n in oracle.CLASS_NAMES]
    check(ctx, g, "v")


@pytest.mark.parametrize("seed", range(1, 5))
@pytest.mark.parametrize("side", ["auto", "u", "v"])
def test_random_graphs(ctx, seed, side):
    rng = np.random.default_rng(seed)
    g = synth.chung_lu_graph(3000, 1500, 40000, 2.1, 2.1, 600, 600, seed, p_neg=0.35)
    check(ctx, g, side)
    g = synth.small_random_graph(rng, max_n=40)
    check(ctx, g, side)


def test_every_counter_width(ctx):
    """Anchors on V (the smaller side) of degree <= 15, <= 255, <= 65,535 and
    above; the anchor with the lower (degree, id) rank picks the field width,
    so two anchors adjacent to every U vertex share 200,000 centres and fill
    32-bit fields (each class above 65,535), and every lower-degree anchor
    shares all its centres with them."""
    rng = np.random.default_rng(7)
    n_u, n_v = 200000, 40
    us, vs = [np.arange(n_u), np.arange(n_u), rng.choice(n_u, 150000, replace=False)], \
        [np.zeros(n_u, np.int64), np.ones(n_u, np.int64), np.full(150000, 2)]
    for v in range(3, n_v):
        d = int(rng.choice([3, 12, 90, 200, 1500, 9000]))
        us.append(rng.choice(n_u, d, replace=False))
        vs.append(np.full(d, v))
    u, v = np.concatenate(us), np.concatenate(vs)
    s = np.where(rng.random(u.size) < 0.4, -1, 1)
    g = synth.from_edges(n_u, n_v, u, v, s)
    got = check(ctx, g, "v")
    assert min(got) > 65535


def band_graph():
    """70,000 V and 200,000 U vertices, 1.2M edges, hubs of about 3,000 on
    both sides: anchors on either side fall in the 4-, 8- and 16-bit class
    layouts, and their rank ranges (70,000 or 200,000) span several bands of
    every layout (16,384 slots at 4 bits, 8,192 at 8 bits, 4,096 at 16
    bits), so band edges are crossed in an element-wise comparison."""
    return synth.chung_lu_graph(200_000, 70_000, 1_200_000, 2.1, 2.1, 4000, 4000, 11, p_neg=0.35)


@pytest.mark.parametrize("side", ["u", "v"])
def test_band_crossing(ctx, side):
    g = band_graph()
    du = np.diff(g.offsets.astype(np.int64))
    dv = np.bincount(g.adj, minlength=g.n_v)
    d = du if side == "u" else dv
    # anchors in every narrow layout, rank ranges of several bands
    assert (d[d > 1] <= 15).sum() > 1000 and ((d > 15) & (d <= 255)).sum() > 1000 and (d > 255).sum() > 100
    assert len(d) > 4 * 16384
    got = check(ctx, g, side)
    assert min(got) > 0


def test_degenerate(ctx):
    for n_u, n_v, edges in [(1, 1, [(0, 0, 1)]), (3, 2, []), (2, 2, [(0, 0, 1), (0, 1, -1), (1, 0, -1), (1, 1, -1)])]:
        e = np.array(edges, np.int64).reshape(-1, 3)
        g = synth.from_edges(n_u, n_v, e[:, 0], e[:, 1], e[:, 2])
        for side in ("auto", "u", "v"):
            check(ctx, g, side)


def test_rejects_blocks(ctx):
    import torch

    g = synth.uniform_graph(200, 100, 2000, 0.3, 3)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    blk = [(torch.arange(5, dtype=torch.int32, device="cuda:0"), torch.arange(5, dtype=torch.int32, device="cuda:0"))]
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_classes(off, adj, sg, g.n_v, opts=bbc.options(blocks=blk))
    assert e.value.status == bbc.EINVAL
