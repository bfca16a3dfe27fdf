"""GPU parity at the full workload sizes (20M and 200M edges).

Expected values are the oracle's, stored by tests/golden/make_expected.py
(minutes of single-core work per graph).  The generator's SHA-256 confirms
the regenerated input is the one the oracle saw.  Totals are compared
exactly; per-vertex counts are compared on the stored sample of vertices
(the highest-degree vertex of each side plus uniform picks), in the launch
configuration the benchmark uses.
"""
import json
import os

import numpy as np
import pytest
import torch

from paper_2601_17707_amd import bbc, synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
EXPECTED = json.load(open(os.path.join(HERE, "golden", "expected_counts.json")))
BIG = sorted(k for k in EXPECTED if not k.startswith("uniform"))


@pytest.fixture(scope="module")
def ctx():
    import __graft_entry__

    __graft_entry__._ensure_built()
    c = bbc.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("key", sorted(EXPECTED))
def test_full_size(ctx, key):
    e = EXPECTED[key]
    print("full size", key, flush=True)
    g = synth.workload(e["workload"], e["seed"])
    assert g.sha256() == e["sha256"], "generator output changed"
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    t = ctx.count(off, adj, sg, g.n_v)
    assert t == int(e["total"])
    pv = torch.empty(g.n_u + g.n_v, dtype=torch.int64, device="cuda:0")
    t2 = ctx.count(off, adj, sg, g.n_v, per_vertex=pv)
    assert t2 == t
    got = pv.cpu().numpy().astype(np.uint64)
    ids = np.asarray(e["vertex_ids"], np.int64)
    want = np.asarray([int(x) for x in e["vertex_counts"]], np.uint64)
    assert np.array_equal(got[ids], want)
    # each butterfly holds two vertices of each side
    assert int(got[: g.n_u].sum()) == 2 * t == int(got[g.n_u:].sum())


@pytest.mark.parametrize("key", [k for k in sorted(EXPECTED) if k.startswith("hybrid")])
def test_full_size_dense_blocks(ctx, key):
    """The planted-block workload at full size with its 16 blocks on the
    matrix cores: the oracle's total, in the launch the benchmark times."""
    e = EXPECTED[key]
    print("full size with blocks", key, flush=True)
    g = synth.workload(e["workload"], e["seed"])
    assert g.sha256() == e["sha256"], "generator output changed"
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    blocks = [(torch.from_numpy(c).cuda(), torch.from_numpy(r).cuda()) for r, c in g.meta["blocks"]]
    assert ctx.count(off, adj, sg, g.n_v, opts=bbc.options(blocks=blocks)) == int(e["total"])
    st = ctx.stats()
    assert st["n_blocks"] == 16 and st["wedges"] < st["wedges_all"]


@pytest.mark.parametrize("key", [k for k in sorted(EXPECTED) if k.startswith("hybrid")])
def test_full_size_planned_blocks(ctx, key):
    """The planner on the planted-block workload: it finds the 16 planted
    blocks (Jaccard >= 0.9 on both sides) among 3M vertices (it may add
    blocks of the background's densely linked hubs), and the count with its
    blocks is the oracle's total."""
    e = EXPECTED[key]
    print("full size, planned blocks", key, flush=True)
    g = synth.workload(e["workload"], e["seed"])
    assert g.sha256() == e["sha256"], "generator output changed"
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    found = ctx.plan_blocks(off, adj, g.n_v)
    print("planned", [(int(u.numel()), int(v.numel())) for u, v in found], flush=True)
    assert len(found) >= 16
    got = [(set(u.cpu().numpy().tolist()), set(v.cpu().numpy().tolist())) for u, v in found]
    for r, c in g.meta["blocks"]:
        rs, cs = set(r.tolist()), set(c.tolist())
        best = max(got, key=lambda f: len(f[1] & rs))
        assert len(best[1] & rs) / len(best[1] | rs) >= 0.9
        assert len(best[0] & cs) / len(best[0] | cs) >= 0.9
    assert ctx.count(off, adj, sg, g.n_v, opts=bbc.options(blocks=found)) == int(e["total"])


BENCH_KEY = "powerlaw-1m-500k-20m:1"


@pytest.fixture(scope="module")
def bench_graph():
    e = EXPECTED[BENCH_KEY]
    g = synth.workload(e["workload"], e["seed"])
    assert g.sha256() == e["sha256"], "generator output changed"
    return g, int(e["total"])


def test_full_size_classes(ctx, bench_graph):
    """The six classes at full size: the balanced four sum to the oracle's
    total, and all six to the unsigned butterfly count (the same graph with
    every sign +1, where every butterfly is balanced)."""
    g, total = bench_graph
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    cls = ctx.count_classes(off, adj, sg, g.n_v)
    assert sum(cls[:4]) == total
    ones = torch.ones_like(sg)
    assert sum(cls) == ctx.count(off, adj, ones, g.n_v)


@pytest.mark.parametrize("side", ["u", "v"])
def test_full_size_classes_elementwise(ctx, bench_graph, side):
    """Each of the six classes at full size, pairs on U and on V, against
    the oracle's stored class totals."""
    g, total = bench_graph
    e = EXPECTED[BENCH_KEY]
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    got = ctx.count_classes(off, adj, sg, g.n_v, opts=bbc.options(side=side))
    assert got == [int(x) for x in e[f"classes_{side}"]]


@pytest.mark.parametrize("k", [3, 4])
@pytest.mark.parametrize("side", ["u", "v"])
def test_full_size_bicliques_k(ctx, bench_graph, k, side):
    """(2,3) and (2,4)-bicliques at full size, pairs on U and on V, against
    the oracle's stored counts."""
    g, total = bench_graph
    e = EXPECTED[BENCH_KEY]
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    assert ctx.count_bicliques(off, adj, sg, g.n_v, k, opts=bbc.options(side=side)) == int(e[f"bicliques_k{k}_{side}"])


def test_full_size_bicliques(ctx, bench_graph):
    """k = 2 is the oracle's total on both pair sides; k = 1 counts the
    wedges, sum of C(deg, 2) over the other side."""
    g, total = bench_graph
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    du = np.diff(g.offsets.astype(np.int64))
    dv = np.bincount(g.adj, minlength=g.n_v).astype(np.int64)
    for side, dc in (("u", dv), ("v", du)):
        assert ctx.count_bicliques(off, adj, sg, g.n_v, 2, opts=bbc.options(side=side)) == total
        assert ctx.count_bicliques(off, adj, sg, g.n_v, 1, opts=bbc.options(side=side)) == int((dc * (dc - 1) // 2).sum())


def test_full_size_updates(ctx, bench_graph):
    """1,000 updates on the full graph (half on existing edges): the count
    of the updated graph equals the oracle's total plus the change, the
    inverse batch on the updated graph gives the opposite change, and the
    shares add up."""
    g, total = bench_graph
    rng = np.random.default_rng(77)
    q = 1000
    eu = np.repeat(np.arange(g.n_u, dtype=np.int64), np.diff(g.offsets.astype(np.int64)))
    keys_g = eu * g.n_v + g.adj
    pick = rng.choice(g.m, q // 2, replace=False)
    keys = set(keys_g[pick].tolist())
    while len(keys) < q:
        keys.add(int(rng.integers(0, g.n_u)) * g.n_v + int(rng.integers(0, g.n_v)))
    k = np.array(sorted(keys), np.int64)
    rng.shuffle(k)
    new = rng.choice([-1, 0, 1], size=q).astype(np.int8)
    # states before: sign of the existing edge, else 0 (rows come sorted by
    # V id, so the keys are sorted)
    assert np.all(keys_g[1:] > keys_g[:-1])
    pos = np.searchsorted(keys_g, k)
    hit = (pos < g.m) & (keys_g[np.minimum(pos, g.m - 1)] == k)
    old = np.zeros(q, np.int8)
    old[hit] = g.signs[pos[hit]]
    # the updated graph, built on the host
    keep = np.ones(g.m, bool)
    keep[pos[hit]] = False
    add = new != 0
    ku = np.concatenate([keys_g[keep], k[add]])
    su = np.concatenate([g.signs[keep], new[add]])
    g2 = synth.from_edges(g.n_u, g.n_v, ku // g.n_v, ku % g.n_v, su)

    def delta(h, states):
        off, adj, sg = bbc.graph_tensors(h, "cuda:0")
        tu = torch.as_tensor((k // g.n_v).astype(np.int32), device="cuda:0")
        tv = torch.as_tensor((k % g.n_v).astype(np.int32), device="cuda:0")
        ts = torch.as_tensor(states, device="cuda:0")
        shares = torch.empty(q, dtype=torch.int64, device="cuda:0")
        d = ctx.update_delta(off, adj, sg, h.n_v, tu, tv, ts, per_update=shares)
        assert int(shares.sum()) == d
        return d

    d = delta(g, new)
    off2, adj2, sg2 = bbc.graph_tensors(g2, "cuda:0")
    assert ctx.count(off2, adj2, sg2, g2.n_v) == total + d
    assert delta(g2, old) == -d
