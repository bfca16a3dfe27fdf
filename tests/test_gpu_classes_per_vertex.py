"""GPU parity of the per-vertex sign-pattern classes
(bbc_count_classes_per_vertex) with the oracle, element by element: the
case study's sample, random graphs on both pair sides, anchors in every
counter width (4, 8, 16 and 32-bit class fields), graphs whose class bands
cross band edges, degenerate inputs; and the sums every per-vertex table
must meet."""
import numpy as np
import pytest
import torch

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


def say(*a):
    print(*a, flush=True)


def check(ctx, g, side="auto"):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    pv = torch.full(((g.n_u + g.n_v) * 6,), -3, dtype=torch.int64, device="cuda:0")
    tot = ctx.count_classes_per_vertex(off, adj, sg, g.n_v, pv, opts=bbc.options(side=side))
    got = pv.cpu().numpy().astype(np.uint64).reshape(-1, 6)
    want = oracle.per_vertex_classes(g, SIDES[side])
    np.testing.assert_array_equal(got, want)
    assert tot == oracle.count_classes(g, SIDES[side])
    assert tot == ctx.count_classes(off, adj, sg, g.n_v, opts=bbc.options(side=side))
    return got


def test_case_study_sample(ctx):
    g, exp = load_graphs("drug_target_sample.txt")["drug_target"]
    got = check(ctx, g, "u")
    assert list(got[: g.n_u].sum(axis=0)) == [2 * exp["class_" + n] for n in oracle.CLASS_NAMES]
    check(ctx, g, "v")


def test_tiny_random_graphs(ctx):
    rng = np.random.default_rng(61)
    for i in range(120):
        g = synth.small_random_graph(rng, max_n=12)
        check(ctx, g, ("auto", "u", "v")[i % 3])


@pytest.mark.parametrize("side", ["auto", "u", "v"])
def test_power_law_graphs(ctx, side):
    g = synth.chung_lu_graph(4000, 2000, 50000, 2.1, 2.1, 700, 700, seed=62, p_neg=0.35)
    check(ctx, g, side)


def test_every_counter_width(ctx):
    """Anchors on V of degree <= 15, <= 255, <= 65,535 and above (4, 8, 16
    and 32-bit class fields), all sharing centres with the two widest."""
    rng = np.random.default_rng(63)
    n_c = 70_000
    us, vs = [], []
    for a, d in enumerate([3, 15, 16, 200, 255, 256, 1_000, 66_000, 67_000]):
        us.append(rng.choice(n_c, size=d, replace=False))
        vs.append(np.full(d, a))
    u, v = np.concatenate(us), np.concatenate(vs)
    s = np.where(rng.random(u.size) < 0.4, -1, 1)
    g = synth.from_edges(n_c, 9, u, v, s)
    got = check(ctx, g, "v")
    say("widths: max per-vertex class count", int(got.max()))


def test_band_edges(ctx):
    """More anchors than one band of the 4-bit class layout holds (16,384
    slots), with hub centres, so the per-vertex walk crosses band edges."""
    g = synth.chung_lu_graph(120_000, 40_000, 300_000, 2.1, 2.0, 2_000, 300, seed=64, p_neg=0.3)
    got = check(ctx, g)
    tot = oracle.count_classes(g)
    assert list(got[: g.n_u].sum(axis=0).astype(np.int64)) == [2 * t for t in tot]
    assert list(got[g.n_u:].sum(axis=0).astype(np.int64)) == [2 * t for t in tot]


def test_degenerate_and_rejected(ctx):
    for n_u, n_v in [(0, 0), (0, 4), (3, 0), (1, 5), (5, 1)]:
        g = synth.from_edges(n_u, n_v, [], [], [])
        check(ctx, g)
    check(ctx, synth.complete_graph(1, 6))
    check(ctx, synth.complete_graph(3, 4))
    g = synth.complete_graph(3, 4)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    with pytest.raises(ValueError):
        ctx.count_classes_per_vertex(off, adj, sg, g.n_v, torch.zeros(5, dtype=torch.int64, device="cuda:0"))
    lib = bbc.load_library()
    import ctypes

    out = (ctypes.c_uint64 * 6)()
    o = bbc.options()
    st = lib.bbc_count_classes_per_vertex(ctx._h, g.n_u, g.n_v, g.m, off.data_ptr(), adj.data_ptr(), sg.data_ptr(),
                                          out, None, ctypes.byref(o), None)
    assert st == bbc.EINVAL
