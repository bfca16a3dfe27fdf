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
