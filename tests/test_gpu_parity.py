"""GPU parity: libbbc.so through the C ABI against the CPU oracle.

Counts are integers, so the bar is bit-exact equality.  Inputs are seeded
and synthetic (paper_2601_17707_amd.synth); expected values come from the
oracle on the same inputs (or, for the paper's drawn examples, from the
fixtures under tests/golden/).
"""
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


def gpu_count(ctx, g, side="auto", checks=bbc.CHECK_ALL, **kw):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    return ctx.count(off, adj, sg, g.n_v, opts=bbc.options(side=side, checks=checks, **kw))


def say(*a):
    print(*a, flush=True)


FIXTURES = {}
for _f in ("fig2_butterflies.txt", "fig1b_signed_k44.txt", "drug_target_sample.txt"):
    FIXTURES.update(load_graphs(_f))


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_paper_examples(ctx, name):
    g, exp = FIXTURES[name]
    for side in ("auto", "u", "v"):
        assert gpu_count(ctx, g, side) == exp["balanced"]


def test_tiny_random_graphs(ctx):
    rng = np.random.default_rng(101)
    for i in range(400):
        g = synth.small_random_graph(rng, max_n=12)
        want = oracle.count(g)
        side = ("auto", "u", "v")[i % 3]
        got = gpu_count(ctx, g, side)
        assert got == want, (i, side, g.n_u, g.n_v, g.m)


def test_degenerate_inputs(ctx):
    for n_u, n_v in [(0, 0), (0, 4), (4, 0), (1, 1), (1, 7), (7, 1), (2, 2)]:
        g = synth.from_edges(n_u, n_v, [], [], [])
        assert gpu_count(ctx, g) == 0
    for n_u, n_v in [(1, 9), (9, 1), (2, 1)]:
        assert gpu_count(ctx, synth.complete_graph(n_u, n_v)) == 0


@pytest.mark.parametrize("m,n", [(2, 2), (5, 7), (16, 16), (17, 40), (64, 300)])
def test_complete_bipartite(ctx, m, n):
    rng = np.random.default_rng(m * 100 + n)
    s = rng.choice([-1, 1], (m, n)).astype(np.int8)
    g = synth.complete_graph(m, n, s)
    want = oracle.count(g)
    for side in ("auto", "u", "v"):
        assert gpu_count(ctx, g, side) == want


def _degree_graph(anchor_degrees, n_centre, seed, p_neg=0.3):
    """Anchors (U) with the given degrees over n_centre centres (V); every
    anchor also shares a few hub centres so many pairs close butterflies."""
    rng = np.random.default_rng(seed)
    us, vs = [], []
    for a, d in enumerate(anchor_degrees):
        cs = rng.choice(n_centre, size=d, replace=False)
        us.append(np.full(d, a))
        vs.append(cs)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    s = np.where(rng.random(u.size) < p_neg, -1, 1)
    return synth.from_edges(len(anchor_degrees), n_centre, u, v, s)


@pytest.mark.parametrize("degs", [[15] * 6 + [16] * 6, [255] * 4 + [256] * 4, [2, 3, 15, 16, 255, 256, 300]])
def test_counter_width_boundaries(ctx, degs):
    """Anchor degrees at the 4/8/16-bit counter limits (15|16, 255|256)."""
    g = _degree_graph(degs, 400, seed=sum(degs))
    want = oracle.count(g, oracle.SIDE_U)
    assert gpu_count(ctx, g, "u") == want
    assert gpu_count(ctx, g, "v") == want


def test_wide_counters(ctx):
    """Anchors of degree >= 65536 use 32-bit counters."""
    n_c = 70000
    rng = np.random.default_rng(7)
    degs = [65535, 65536, 69000]
    us, vs = [], []
    for a, d in enumerate(degs):
        us.append(np.full(d, a))
        vs.append(rng.choice(n_c, size=d, replace=False))
    u, v = np.concatenate(us), np.concatenate(vs)
    s = np.where(rng.random(u.size) < 0.4, -1, 1)
    g = synth.from_edges(3, n_c, u, v, s)
    want = oracle.count(g)
    say("wide counters: want", want)
    assert gpu_count(ctx, g, "u") == want


@pytest.mark.parametrize("n_s", [65535, 65536, 65537, 131073, 200000])
def test_band_boundaries(ctx, n_s):
    """Anchor sides wider than one LDS band (64K 4-bit slots, 32K 8-bit,
    16K 16-bit), with hub centres so suffixes cross band edges."""
    g = synth.chung_lu_graph(n_s * 3, n_s, n_s * 8, 2.1, 2.0, 3000, 400, seed=n_s)
    assert g.n_v < g.n_u
    want = oracle.count(g)
    say("band", n_s, "m", g.m, "want", want)
    assert gpu_count(ctx, g) == want
    assert gpu_count(ctx, g, "v") == want


SHAPES = bbc.WEDGE_SHAPES


@pytest.mark.parametrize("bw,wg", SHAPES)
def test_kernel_shapes(ctx, bw, wg):
    """Every instantiated (band words, workgroup) shape on graphs that cross
    band edges in all four counter widths."""
    say("shape", bw, wg)
    cases = [synth.chung_lu_graph(140_000, 70_000, 700_000, 2.1, 2.0, 3000, 600, seed=21),
             _degree_graph([3, 15, 16, 200, 255, 256, 900], 40_000, seed=22)]
    for g in cases:
        want = oracle.count(g)
        for side in ("auto", "u", "v"):
            assert gpu_count(ctx, g, side, band_words=bw, wg_size=wg) == want, (bw, wg, side)
    g = cases[0]
    assert gpu_count(ctx, g, band_words=bw, wg_size=wg, wg_per_cu=1) == oracle.count(g)


def test_unknown_shape_rejected(ctx):
    g = synth.complete_graph(3, 3)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    with pytest.raises(bbc.BbcError) as e:
        ctx.count(off, adj, sg, g.n_v, opts=bbc.options(band_words=1000))
    assert e.value.status == bbc.EINVAL


def test_mid_degree_band_split(ctx):
    """Anchors of degree 16..300 over an anchor side wider than a band."""
    g = synth.chung_lu_graph(60000, 50000, 1_500_000, 2.3, 2.3, 2000, 2000, seed=9, p_neg=0.35)
    want = oracle.count(g)
    assert gpu_count(ctx, g) == want


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_uniform_workload(ctx, seed):
    g = synth.workload("uniform-2k-1k-20k", seed)
    want = oracle.count(g)
    for side in ("auto", "u", "v"):
        assert gpu_count(ctx, g, side) == want


def test_powerlaw_small(ctx):
    """Power-law graph with the shape of the 20M-edge workload at 1/20 size."""
    g = synth.chung_lu_graph(50_000, 25_000, 1_000_000, 2.1, 2.1, 2500, 2500, seed=3, p_neg=0.2)
    want = oracle.count(g)
    say("powerlaw small want", want)
    assert gpu_count(ctx, g) == want
    assert gpu_count(ctx, g, "u") == want


def test_skewed_small(ctx):
    """Skewed graph (hub anchors) with the shape of the 200M-edge workload, scaled down."""
    g = synth.chung_lu_graph(250_000, 10_000, 2_000_000, 2.5, 1.8, 1400, 25_000, seed=4, beta_bias=(2, 5, 0.7))
    want = oracle.count(g)
    say("skewed small want", want)
    assert gpu_count(ctx, g) == want


def test_invariants_on_gpu(ctx):
    """Switching, global flip and unsigned = balanced + unbalanced, on the GPU path."""
    g = synth.chung_lu_graph(3000, 2000, 40_000, 2.1, 2.1, 400, 400, seed=8, p_neg=0.3)
    t = gpu_count(ctx, g)
    u, v, s = g.edges()
    rng = np.random.default_rng(5)
    fu = rng.choice([-1, 1], g.n_u)
    fv = rng.choice([-1, 1], g.n_v)
    g2 = synth.Graph(g.n_u, g.n_v, g.offsets, g.adj, (s * fu[u] * fv[v]).astype(np.int8), {})
    assert gpu_count(ctx, g2) == t
    g3 = synth.Graph(g.n_u, g.n_v, g.offsets, g.adj, (-s).astype(np.int8), {})
    assert gpu_count(ctx, g3) == t
    b, n, all_ = oracle.count_kinds(g)
    g4 = synth.Graph(g.n_u, g.n_v, g.offsets, g.adj, np.ones_like(g.signs), {})
    assert gpu_count(ctx, g4) == all_ == t + n


def test_unsorted_rows(ctx):
    g = synth.chung_lu_graph(5000, 3000, 60_000, 2.1, 2.1, 500, 500, seed=10)
    want = oracle.count(g)
    g2 = synth.shuffle_rows(g, np.random.default_rng(3))
    assert gpu_count(ctx, g2) == want


def test_repeatable(ctx):
    g = synth.chung_lu_graph(20000, 10000, 300_000, 2.1, 2.1, 2000, 2000, seed=12)
    vals = {gpu_count(ctx, g) for _ in range(6)}
    assert len(vals) == 1
    assert vals.pop() == oracle.count(g)


# ------------------------------------------------------------------- errors


def _expect_error(ctx, g, status, **kw):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    with pytest.raises(bbc.BbcError) as e:
        ctx.count(off, adj, sg, g.n_v, opts=bbc.options(**kw))
    assert e.value.status == status, e.value


def test_error_codes(ctx):
    g = synth.complete_graph(4, 5)
    bad = synth.Graph(4, 5, g.offsets, g.adj.copy(), g.signs, {})
    bad.adj[3] = 5
    _expect_error(ctx, bad, bbc.ERANGE)
    bad.adj[3] = -1
    _expect_error(ctx, bad, bbc.ERANGE)
    bad = synth.Graph(4, 5, g.offsets, g.adj, g.signs.copy(), {})
    bad.signs[2] = 0
    _expect_error(ctx, bad, bbc.ESIGN)
    off = g.offsets.copy()
    off[2] = off[1] - 1
    _expect_error(ctx, synth.Graph(4, 5, off, g.adj, g.signs, {}), bbc.EOFFSETS)
    off = g.offsets.copy()
    off[0] = 1
    _expect_error(ctx, synth.Graph(4, 5, off, g.adj, g.signs, {}), bbc.EOFFSETS)
    dup = synth.Graph(4, 5, g.offsets, g.adj.copy(), g.signs, {})
    dup.adj[1] = dup.adj[0]
    _expect_error(ctx, dup, bbc.EDUP)
    # the duplicate check can be switched off; the count is then defined by the
    # multigraph but the call must stay memory-safe
    off_t, adj_t, sg_t = bbc.graph_tensors(dup, "cuda:0")
    ctx.count(off_t, adj_t, sg_t, dup.n_v, opts=bbc.options(checks=bbc.CHECK_SIGNS))
    # a good call after errors still works
    assert gpu_count(ctx, g) == oracle.count(g)


def test_output_untouched_on_error(ctx):
    import ctypes

    lib = bbc.load_library()
    g = synth.complete_graph(3, 3)
    bad = synth.Graph(3, 3, g.offsets, g.adj.copy(), g.signs, {})
    bad.adj[0] = 9
    off, adj, sg = bbc.graph_tensors(bad, "cuda:0")
    out = ctypes.c_uint64(12345)
    o = bbc.options()
    st = lib.bbc_count(ctx._h, 3, 3, adj.numel(), bbc._ptr(off), bbc._ptr(adj), bbc._ptr(sg), ctypes.byref(out),
                       None, ctypes.byref(o), None)
    assert st == bbc.ERANGE and out.value == 12345
    assert lib.bbc_count(ctx._h, 3, 3, 2**31, bbc._ptr(off), bbc._ptr(adj), bbc._ptr(sg), ctypes.byref(out),
                         None, ctypes.byref(o), None) == bbc.ETOOBIG
    assert lib.bbc_count(ctx._h, -1, 3, 0, bbc._ptr(off), None, None, ctypes.byref(out), None,
                         ctypes.byref(o), None) == bbc.EINVAL


def test_stream_ordering(ctx):
    """The count runs on the caller's stream."""
    g = synth.workload("uniform-2k-1k-20k", 2)
    want = oracle.count(g)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        off, adj, sg = bbc.graph_tensors(g, "cuda:0")
        got = ctx.count(off, adj, sg, g.n_v, stream=s)
    assert got == want


# --------------------------------------------------------------- per vertex


def gpu_per_vertex(ctx, g, side="auto"):
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    pv = torch.full((g.n_u + g.n_v,), 7, dtype=torch.int64, device="cuda:0")  # overwritten, not accumulated
    t = ctx.count(off, adj, sg, g.n_v, per_vertex=pv, opts=bbc.options(side=side))
    return t, pv.cpu().numpy().astype(np.uint64)


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_per_vertex_paper_examples(ctx, name):
    g, exp = FIXTURES[name]
    _, _, want = oracle.brute(g, per_vertex=True)
    for side in ("auto", "u", "v"):
        t, pv = gpu_per_vertex(ctx, g, side)
        assert t == exp["balanced"]
        assert np.array_equal(pv, want)


def test_per_vertex_tiny_random(ctx):
    rng = np.random.default_rng(202)
    for i in range(150):
        g = synth.small_random_graph(rng, max_n=10)
        want = oracle.per_vertex(g)
        side = ("auto", "u", "v")[i % 3]
        t, pv = gpu_per_vertex(ctx, g, side)
        assert t == oracle.count(g), i
        assert np.array_equal(pv, want), i


@pytest.mark.parametrize("case", ["bands", "widths", "wide", "skewed"])
def test_per_vertex_structured(ctx, case):
    """Band crossings (above and below the anchor), every counter width, and
    anchors wider than one workgroup (chunked centre lists)."""
    if case == "bands":
        g = synth.chung_lu_graph(200_000, 70_000, 600_000, 2.1, 2.0, 3000, 600, seed=31)
    elif case == "widths":
        g = _degree_graph([2, 3, 15, 16, 200, 255, 256, 257, 900, 2000], 30_000, seed=32)
    elif case == "wide":
        rng = np.random.default_rng(33)
        us, vs = [], []
        for a, d in enumerate([65535, 65536, 66000]):
            us.append(np.full(d, a))
            vs.append(rng.choice(70_000, size=d, replace=False))
        u, v = np.concatenate(us), np.concatenate(vs)
        g = synth.from_edges(3, 70_000, u, v, np.where(rng.random(u.size) < 0.4, -1, 1))
    else:
        g = synth.chung_lu_graph(120_000, 6_000, 800_000, 2.5, 1.8, 900, 12_000, seed=34, beta_bias=(2, 5, 0.7))
    want = oracle.per_vertex(g)
    t_want = oracle.count(g)
    say("per-vertex", case, "m", g.m, "total", t_want)
    for side in ("auto", "u", "v"):
        t, pv = gpu_per_vertex(ctx, g, side)
        assert t == t_want, side
        assert np.array_equal(pv, want), side
        assert int(pv[: g.n_u].sum()) == 2 * t == int(pv[g.n_u:].sum())


@pytest.mark.parametrize("side", ["auto", "u", "v"])
def test_stats_wedge_counts(ctx, side):
    """The wedge count the benchmark divides by: sum over centres of
    C(deg, 2), computed here from the degrees, for every kernel shape."""
    g = synth.chung_lu_graph(50_000, 20_000, 400_000, 2.1, 2.0, 2_000, 800, seed=77)
    u, v, _ = g.edges()
    s_is_u = side == "u" or (side == "auto" and g.n_u < g.n_v)
    d = np.bincount(v if s_is_u else u, minlength=g.n_v if s_is_u else g.n_u).astype(np.int64)
    want_w = int((d * (d - 1) // 2).sum())
    for bw, wg in SHAPES:
        gpu_count(ctx, g, side, band_words=bw, wg_size=wg)
        st = ctx.stats()
        assert st["wedges"] == want_w and st["wedges_all"] == want_w, (bw, wg)
        assert st["n_anchor"] == (g.n_u if s_is_u else g.n_v)
        assert st["n_edges"] == g.m
