"""GPU parity of dynamic updates (bbc_update_delta): the change of the
balanced count under a batch of edge insertions, removals and sign changes
against the oracle's difference of two full counts, exact; per-update
shares sum to it; rows in any order; batches whose updates share
butterflies; rejected inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2601_17707_amd import bbc, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def ctx():
    import __graft_entry__

    __graft_entry__._ensure_built()
    c = bbc.Context(0)
    yield c
    c.close()


def gpu_delta(ctx, g, uu, vv, ss, shares=False):
    off, adj, sg = bbc.graph_tensors(g, DEV)
    tu = torch.as_tensor(np.asarray(uu, np.int32), device=DEV)
    tv = torch.as_tensor(np.asarray(vv, np.int32), device=DEV)
    ts = torch.as_tensor(np.asarray(ss, np.int8), device=DEV)
    pu = torch.full((len(uu),), 7, dtype=torch.int64, device=DEV) if shares else None
    d = ctx.update_delta(off, adj, sg, g.n_v, tu, tv, ts, per_update=pu)
    if shares:
        assert int(pu.sum()) == d
    return d


def random_batch(rng, g, q, p_existing=0.5):
    """q distinct pairs, about p_existing of them existing edges; states
    drawn from {-1, 0, +1}."""
    deg = np.diff(g.offsets.astype(np.int64))
    eu = np.repeat(np.arange(g.n_u), deg)
    n_old = min(int(q * p_existing), g.m)
    pick = rng.choice(g.m, n_old, replace=False) if n_old else np.zeros(0, np.int64)
    keys = set((eu[pick].astype(np.int64) * g.n_v + g.adj[pick]).tolist())
    while len(keys) < q:
        keys.add(int(rng.integers(0, g.n_u)) * g.n_v + int(rng.integers(0, g.n_v)))
    k = np.array(sorted(keys), np.int64)
    rng.shuffle(k)
    return k // g.n_v, k % g.n_v, rng.choice([-1, 0, 1], size=k.size)


@pytest.mark.parametrize("seed", range(1, 5))
def test_random_batches(ctx, seed):
    rng = np.random.default_rng(seed)
    g = synth.shuffle_rows(synth.chung_lu_graph(3000, 1500, 30000, 2.1, 2.1, 500, 500, seed, p_neg=0.3), rng)
    for q in (1, 17, 600):
        uu, vv, ss = random_batch(rng, g, q)
        assert gpu_delta(ctx, g, uu, vv, ss, shares=True) == oracle.update_delta(g, uu, vv, ss)


def test_interacting_updates(ctx):
    """Every pair of a small dense graph updated at once: most butterflies
    hold several updated pairs."""
    rng = np.random.default_rng(9)
    for _ in range(10):
        g = synth.random_graph(rng, 7, 6, 0.6, 0.4)
        k = np.arange(g.n_u * g.n_v)
        rng.shuffle(k)
        uu, vv = k // g.n_v, k % g.n_v
        ss = rng.choice([-1, 0, 1], size=k.size)
        assert gpu_delta(ctx, g, uu, vv, ss, shares=True) == oracle.update_delta(g, uu, vv, ss)


@pytest.mark.parametrize("m,n", [(2, 2), (4, 5)])
def test_closed_forms(ctx, m, n):
    g = synth.complete_graph(m, n)
    k = (m - 1) * (n - 1)
    assert gpu_delta(ctx, g, [0], [0], [-1]) == -k
    assert gpu_delta(ctx, g, [0], [0], [0]) == -k
    assert gpu_delta(ctx, g, [0], [0], [1]) == 0
    assert gpu_delta(ctx, g, [0, 0], [0, 1], [-1, -1]) == -2 * (m - 1) * (n - 2)
    h = oracle.apply_updates(g, [0], [0], [0])
    h = synth.from_edges(h.n_u, h.n_v, np.repeat(np.arange(h.n_u), np.diff(h.offsets)), h.adj, h.signs)
    assert gpu_delta(ctx, h, [0], [0], [1]) == k
    assert gpu_delta(ctx, h, [0], [0], [-1]) == 0
    assert gpu_delta(ctx, h, [0], [0], [0]) == 0


def test_larger_graph(ctx):
    rng = np.random.default_rng(3)
    g = synth.chung_lu_graph(40000, 20000, 300000, 2.1, 2.1, 4000, 4000, 3, p_neg=0.25)
    uu, vv, ss = random_batch(rng, g, 20000)
    assert gpu_delta(ctx, g, uu, vv, ss, shares=True) == oracle.update_delta(g, uu, vv, ss)


def test_empty_graph_and_batch(ctx):
    e = synth.from_edges(4, 3, np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0, np.int8))
    assert gpu_delta(ctx, e, [], [], []) == 0
    uu, vv = np.array([0, 0, 1, 1]), np.array([0, 1, 0, 1])
    for ss in ([1, 1, 1, 1], [1, -1, -1, 1], [1, -1, 1, 1], [0, 1, 1, 1]):
        assert gpu_delta(ctx, e, uu, vv, ss) == oracle.update_delta(e, uu, vv, ss)


def test_rejected_inputs(ctx):
    g = synth.complete_graph(3, 3)
    cases = [(([0, 0], [1, 1], [1, -1]), bbc.EINVAL), (([0], [3], [1]), bbc.ERANGE), (([3], [0], [1]), bbc.ERANGE),
             (([0], [0], [2]), bbc.ESIGN), (([-1], [0], [1]), bbc.ERANGE)]
    for (uu, vv, ss), code in cases:
        with pytest.raises(bbc.BbcError) as e:
            gpu_delta(ctx, g, uu, vv, ss)
        assert e.value.status == code, (uu, vv, ss)
    bad = synth.Graph(2, 2, np.array([0, 2, 3], np.int32), np.array([1, 1, 0], np.int32),
                      np.array([1, 1, 1], np.int8), {})
    with pytest.raises(bbc.BbcError) as e:
        gpu_delta(ctx, bad, [0], [0], [1])
    assert e.value.status == bbc.EDUP


def test_rejected_inputs_leave_shares(ctx):
    """A rejected batch (repeated pair, repeated edge, bad id or state)
    leaves the per-update shares untouched."""
    g = synth.complete_graph(3, 3)
    bad = synth.Graph(2, 2, np.array([0, 2, 3], np.int32), np.array([1, 1, 0], np.int32),
                      np.array([1, 1, 1], np.int8), {})
    for h, (uu, vv, ss) in ((g, ([0, 0], [1, 1], [1, -1])), (bad, ([0], [0], [1])), (g, ([0], [3], [1])),
                            (g, ([0], [0], [2]))):
        off, adj, sg = bbc.graph_tensors(h, DEV)
        pu = torch.full((len(uu),), 7, dtype=torch.int64, device=DEV)
        with pytest.raises(bbc.BbcError):
            ctx.update_delta(off, adj, sg, h.n_v, torch.as_tensor(np.asarray(uu, np.int32), device=DEV),
                             torch.as_tensor(np.asarray(vv, np.int32), device=DEV),
                             torch.as_tensor(np.asarray(ss, np.int8), device=DEV), per_update=pu)
        assert torch.all(pu == 7)


@pytest.mark.parametrize("cap", [1, 2, 3, 0])
def test_task_caps(ctx, cap):
    """Updates whose pairs mode outgrows the task cap: the w list (about
    1,100 entries, two 1,024-entry chunks) is cut into spans of whole chunks
    against every x chunk, one span per task when the cap allows; cap 0 is
    the default tiling.  Rows of u are sparser than the average U row, so
    the pairs mode is the cheaper one."""
    rng = np.random.default_rng(21)
    n_u, n_v = 1500, 1300
    dens = np.where(np.arange(n_u) < 40, 0.3, 0.75)
    present = rng.random((n_u, n_v)) < dens[:, None]
    uu, vv = np.nonzero(present)
    g = synth.from_edges(n_u, n_v, uu, vv, np.where(rng.random(uu.size) < 0.3, -1, 1))
    q = 40
    bu = np.arange(q)
    bv = rng.choice(n_v, q, replace=False)
    bs = rng.choice([-1, 0, 1], size=q)
    want = oracle.update_delta(g, bu, bv, bs)
    ctx.set_update_task_cap(cap)
    try:
        assert gpu_delta(ctx, g, bu, bv, bs, shares=True) == want
    finally:
        ctx.set_update_task_cap(0)


def test_task_cap_rejects_negative(ctx):
    with pytest.raises(bbc.BbcError) as e:
        ctx.set_update_task_cap(-1)
    assert e.value.status == bbc.EINVAL
