"""BBC_ENOMEM through the scratch_limit option: a call whose scratch would
exceed the limit fails before any work with its outputs untouched, and the
context keeps working afterwards (the error path of device allocation,
forced from the host without exhausting the device)."""
import ctypes

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


def test_count_over_the_limit(ctx):
    g = synth.chung_lu_graph(20_000, 9_000, 150_000, 2.1, 2.1, 800, 800, seed=3, p_neg=0.3)
    want = oracle.count(g)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    lib = bbc.load_library()
    # a fresh context, so its arena has never grown
    with bbc.Context(0) as c2:
        out = ctypes.c_uint64(4242)
        pv = torch.full((g.n_u + g.n_v,), 7, dtype=torch.int64, device="cuda:0")
        o = bbc.options(scratch_limit=4096)
        st = lib.bbc_count(c2._h, g.n_u, g.n_v, g.m, off.data_ptr(), adj.data_ptr(), sg.data_ptr(),
                           ctypes.byref(out), pv.data_ptr(), ctypes.byref(o), None)
        assert st == bbc.ENOMEM
        assert "scratch_limit" in c2.last_error()
        assert out.value == 4242
        assert bool((pv == 7).all())
        # the context recovers: no limit, then a limit the call fits in
        assert c2.count(off, adj, sg, g.n_v) == want
        assert c2.count(off, adj, sg, g.n_v, opts=bbc.options(scratch_limit=1 << 34)) == want
        # and the limit is checked against the need, not against the arena already held
        with pytest.raises(bbc.BbcError) as e:
            c2.count(off, adj, sg, g.n_v, opts=bbc.options(scratch_limit=4096))
        assert e.value.status == bbc.ENOMEM
        assert c2.count(off, adj, sg, g.n_v) == want
        for fn in (lambda o: c2.count_classes(off, adj, sg, g.n_v, opts=o),
                   lambda o: c2.count_bicliques(off, adj, sg, g.n_v, 3, opts=o),
                   lambda o: c2.count_noalloc(off, adj, sg, g.n_v, opts=o)):
            with pytest.raises(bbc.BbcError) as e:
                fn(bbc.options(scratch_limit=4096))
            assert e.value.status == bbc.ENOMEM
        assert c2.count(off, adj, sg, g.n_v) == want


def test_batch_and_plan_over_the_limit(ctx):
    graphs = [synth.uniform_graph(300, 200, 3000, 0.3, seed=s) for s in range(4)]
    want = [oracle.count(g) for g in graphs]
    batch = bbc.Batch(graphs, "cuda:0")
    batch.totals.fill_(-1)
    with pytest.raises(bbc.BbcError) as e:
        ctx.count_batched(batch, opts=bbc.options(scratch_limit=1024))
    assert e.value.status == bbc.ENOMEM
    with pytest.raises(bbc.BbcError) as e:
        ctx.plan(batch, opts=bbc.options(scratch_limit=1024))
    assert e.value.status == bbc.ENOMEM
    assert ctx.count_batched(batch).cpu().tolist() == want
    plan = ctx.plan(batch, opts=bbc.options(scratch_limit=1 << 32))
    plan.launch()
    assert plan.wait().cpu().tolist()[:4] == want
    plan.close()


def test_negative_limit_rejected(ctx):
    g = synth.uniform_graph(30, 20, 100, 0.3, seed=1)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    with pytest.raises(bbc.BbcError) as e:
        ctx.count(off, adj, sg, g.n_v, opts=bbc.options(scratch_limit=-5))
    assert e.value.status == bbc.EINVAL
