"""GPU tests of the autotuner: the tuned shape never changes the count, the
table is keyed by size class, and it survives a save / load round trip."""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_17707_amd import bbc, synth

pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    import __graft_entry__

    __graft_entry__._ensure_built()
    c = bbc.Context(0)
    yield c
    c.close()


def test_autotune_picks_an_instantiated_shape_and_keeps_the_count(ctx, tmp_path):
    g = synth.chung_lu_graph(60_000, 30_000, 600_000, 2.1, 2.1, 3_000, 3_000, seed=5, p_neg=0.2)
    want = oracle.count(g)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    chosen = ctx.autotune(off, adj, sg, g.n_v, reps=1)
    assert (chosen["band_words"], chosen["wg_size"]) in bbc.WEDGE_SHAPES
    assert chosen["wg_per_cu"] >= 1
    assert chosen["queue_chunk"] in (1, 2, 4, 8, 16) and chosen["wave_max_work"] in (0, 256, -1)
    # a default call of the same class now uses the entry
    assert ctx.count(off, adj, sg, g.n_v) == want
    st = ctx.stats()
    assert st["tuned"] == 1
    assert st["band_words"] == chosen["band_words"] and st["block"] == chosen["wg_size"]
    assert st["schedule"] == chosen["schedule"] in (bbc.SCHED_DYNAMIC, bbc.SCHED_STATIC)
    # options that fix the shape, no_tuning, or per-vertex output bypass it
    assert ctx.count(off, adj, sg, g.n_v, opts=bbc.options(no_tuning=True)) == want
    assert ctx.stats()["tuned"] == 0
    assert ctx.count(off, adj, sg, g.n_v, opts=bbc.options(band_words=8192, wg_size=256)) == want
    assert ctx.stats()["tuned"] == 0
    pv = torch.empty(g.n_u + g.n_v, dtype=torch.int64, device="cuda:0")
    assert ctx.count(off, adj, sg, g.n_v, per_vertex=pv) == want
    assert ctx.stats()["tuned"] == 0
    # another size class is not affected
    h = synth.chung_lu_graph(3_000, 1_000, 20_000, 2.1, 2.1, 300, 300, seed=6, p_neg=0.3)
    o2, a2, s2 = bbc.graph_tensors(h, "cuda:0")
    assert ctx.count(o2, a2, s2, h.n_v) == oracle.count(h)
    assert ctx.stats()["tuned"] == 0

    # save / load round trip into a fresh context
    path = str(tmp_path / "tune.txt")
    ctx.tune_save(path)
    text = open(path).read().splitlines()
    assert text[0] == "bbc-tune 3 gfx950" and len(text) == 2
    f = text[1].split()
    assert len(f) == 11 and int(f[6]) == chosen["queue_chunk"] and int(f[7]) == chosen["wave_max_work"]
    c2 = bbc.Context(0)
    try:
        c2.tune_load(path)
        assert c2.count(off, adj, sg, g.n_v) == want
        st2 = c2.stats()
        assert st2["tuned"] == 1 and st2["band_words"] == chosen["band_words"]
        p2 = str(tmp_path / "tune2.txt")
        c2.tune_save(p2)
        assert open(p2).read() == open(path).read()
    finally:
        c2.close()


def test_batched_calls_use_the_table(ctx):
    graphs = synth.batch_graphs(40, seed=3)
    b = bbc.Batch(graphs, "cuda:0")
    want = [oracle.count(g) for g in graphs]
    assert list(ctx.count_batched(b).cpu().numpy()[: len(graphs)]) == want
    assert ctx.stats()["tuned"] == 0
    # tune on the union of the batch (same size class as the batch)
    us, vs, ss = [], [], []
    bu = bv = 0
    for g in graphs:
        u, v, s = g.edges()
        if g.n_u < g.n_v:  # keep each member's anchor side on V in the union
            u, v = v, u
            nu, nv = g.n_v, g.n_u
        else:
            nu, nv = g.n_u, g.n_v
        us.append(u + bu)
        vs.append(v + bv)
        ss.append(s)
        bu += nu
        bv += nv
    union = synth.from_edges(bu, bv, np.concatenate(us), np.concatenate(vs), np.concatenate(ss))
    off, adj, sg = bbc.graph_tensors(union, "cuda:0")
    ctx.autotune(off, adj, sg, union.n_v, reps=1)
    got = ctx.count_batched(b).cpu().numpy()[: len(graphs)]
    assert list(got) == want
    assert ctx.stats()["tuned"] == 1


def test_tune_load_rejects_bad_files(ctx, tmp_path):
    cases = {
        "header": "bbc-tune 3 gfx950\n1 2 16384 512 2 1.0\n",
        "v2 fields": "bbc-tune 2 gfx950\n19 6 16384 512 2 1.0\n",
        "v2 schedule": "bbc-tune 2 gfx950\n19 6 16384 512 2 2 1.0\n",
        "arch": "bbc-tune 1 gfx942\n",
        "shape": "bbc-tune 1 gfx950\n19 6 12345 512 2 1.0\n",
        "fields": "bbc-tune 1 gfx950\n19 6 16384 512\n",
        "trailing": "bbc-tune 1 gfx950\n19 6 16384 512 2 1.0 x\n",
        "negative": "bbc-tune 1 gfx950\n19 6 16384 512 -1 1.0\n",
        "v3 fields": "bbc-tune 3 gfx950\n19 6 16384 512 2 1 1 0 0 1.0\n",
        "v3 tile": "bbc-tune 3 gfx950\n19 6 16384 512 2 1 1 0 0 96 1.0\n",
        "v3 chunk": "bbc-tune 3 gfx950\n19 6 16384 512 2 1 -3 0 0 0 1.0\n",
        "v3 wave": "bbc-tune 3 gfx950\n19 6 16384 512 2 1 1 -2 0 0 1.0\n",
        "v3 empty shape": "bbc-tune 3 gfx950\n19 6 0 512 2 1 1 0 0 0 1.0\n",
        "empty": "",
    }
    for name, text in cases.items():
        p = str(tmp_path / f"{name}.txt")
        with open(p, "w") as f:
            f.write(text)
        with pytest.raises(bbc.BbcError) as e:
            ctx.tune_load(p)
        assert e.value.status == bbc.EINVAL, name
    with pytest.raises(bbc.BbcError):
        ctx.tune_load(str(tmp_path / "missing.txt"))
    # a valid file after the failures: entries merge, later lines replace earlier ones
    p = str(tmp_path / "ok.txt")
    with open(p, "w") as f:
        f.write("bbc-tune 1 gfx950\n3 4 8192 256 1 0.5\n3 4 16384 256 2 0.4\n")
    ctx.tune_load(p)
    out = str(tmp_path / "out.txt")
    ctx.tune_save(out)
    lines = open(out).read().splitlines()
    assert lines == ["bbc-tune 3 gfx950", "3 4 16384 256 2 0 0 0 0 0 0.4000"]
    # version 2 entries carry the schedule
    with open(p, "w") as f:
        f.write("bbc-tune 2 gfx950\n3 4 8192 256 1 1 0.3\n")
    ctx.tune_load(p)
    ctx.tune_save(out)
    assert open(out).read().splitlines() == ["bbc-tune 3 gfx950", "3 4 8192 256 1 1 0 0 0 0 0.3000"]
    # version 3: regime and dense-block columns; an entry may hold only the latter
    with open(p, "w") as f:
        f.write("bbc-tune 3 gfx950\n3 4 8192 256 1 0 4 -1 512 64 0.2\n5 6 0 0 0 0 0 0 1024 128 0.1\n")
    ctx.tune_load(p)
    ctx.tune_save(out)
    assert open(out).read().splitlines() == ["bbc-tune 3 gfx950", "3 4 8192 256 1 0 4 -1 512 64 0.2000",
                                              "5 6 0 0 0 0 0 0 1024 128 0.1000"]


def test_autotune_batched_records_the_batch_class(ctx):
    graphs = synth.batch_graphs(60, seed=4)
    b = bbc.Batch(graphs, "cuda:0")
    want = [oracle.count(g) for g in graphs]
    chosen = ctx.autotune_batched(b, reps=1)
    assert (chosen["band_words"], chosen["wg_size"]) in bbc.WEDGE_SHAPES
    assert chosen["queue_chunk"] in (1, 2, 4, 8, 16) and chosen["wave_max_work"] in (0, 256, -1)
    assert list(b.totals.cpu().numpy()[: len(graphs)]) == want
    assert list(ctx.count_batched(b).cpu().numpy()[: len(graphs)]) == want
    st = ctx.stats()
    assert st["tuned"] == 1 and st["band_words"] == chosen["band_words"]
    plan = ctx.plan(b)
    for _ in range(2):
        plan.launch()
        assert list(plan.wait().cpu().numpy()[: len(graphs)]) == want
    plan.close()


def test_autotune_blocks_and_the_int8_tiles(ctx):
    g = synth.hybrid_graph(12_000, 6_000, 40_000, 3, 200, 0.5, 0.1, seed=8)
    want = oracle.count(g)
    off, adj, sg = bbc.graph_tensors(g, "cuda:0")
    blocks = [(torch.from_numpy(c).to("cuda:0"), torch.from_numpy(r).to("cuda:0")) for r, c in g.meta["blocks"]]
    # both tiles on the planted blocks (200 rows: not a multiple of either tile)
    for tile in (64, 128, 0):
        assert ctx.count(off, adj, sg, g.n_v, opts=bbc.options(blocks=blocks, dense_tile=tile)) == want
    with pytest.raises(bbc.BbcError) as e:
        ctx.count(off, adj, sg, g.n_v, opts=bbc.options(blocks=blocks, dense_tile=96))
    assert e.value.status == bbc.EINVAL
    chosen = ctx.autotune_blocks(off, adj, sg, g.n_v, reps=1)
    assert chosen["min_degree"] in (128, 256, 512, 1024) and chosen["dense_tile"] in (64, 128)
    # planner calls with min_degree 0 and counts with dense_tile 0 of the class use the entry
    found = ctx.plan_blocks(off, adj, g.n_v)
    assert ctx.count(off, adj, sg, g.n_v, opts=bbc.options(blocks=found)) == want
    path_blocks = ctx.plan_blocks(off, adj, g.n_v, opts=bbc.plan_options(min_degree=chosen["min_degree"]))
    assert len(path_blocks) == len(found)
