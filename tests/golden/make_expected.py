"""Writes tests/golden/expected_counts.json: oracle results on the full-size
synthetic workloads, for the GPU parity tests at those sizes.

Calls only the CPU oracle (oracle/) and the seeded generator; no value here
comes from the GPU library.  Each entry records the generator's SHA-256 of
the graph so a test can tell that it regenerated the same input.

    python tests/golden/make_expected.py [--procs N] [workload:seed ...]
    python tests/golden/make_expected.py [--procs N] batch-10k:1
    python tests/golden/make_expected.py [--procs N] --extensions workload:seed

--extensions adds, to an existing entry, the oracle's six class totals
and its (2,3) and (2,4)-biclique counts, each with the pairs on U and on V.

The batch workload goes to its own file (batch10k_totals.json): the
oracle's total of every member graph, in batch order, with the SHA-256 of
the whole batch (each member's digest, hashed in order).

The full-size oracle runs take minutes (the 20M-edge graph) to tens of
minutes (the 200M-edge graphs) on one core.  With --procs N the total is
the sum of the oracle's counts over N x 4 anchor-id ranges run in N forked
processes (the ranges partition the anchors, so the sum is the total).
"""
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2601_17707_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "expected_counts.json")
BATCH_OUT = os.path.join(HERE, "batch10k_totals.json")
DEFAULT = ["uniform-2k-1k-20k:1", "uniform-2k-1k-20k:2", "uniform-2k-1k-20k:3", "powerlaw-1m-500k-20m:1",
           "skewed-5m-200k-200m:1", "hybrid-2m-1m-50m-16x4096:1"]
_G = None  # the graph shared with forked workers


def _range_count(bounds):
    lo, hi = bounds
    return oracle.count_anchors(_G, lo, hi)[0]


def parallel_total(g, procs):
    """Sum of the oracle's anchor-range counts over a partition of the anchors."""
    global _G
    _G = g
    n_s = g.n_u if g.n_u < g.n_v else g.n_v
    cuts = np.linspace(0, n_s, procs * 4 + 1).astype(np.int64)
    with mp.get_context("fork").Pool(procs) as pool:
        parts = pool.map(_range_count, list(zip(cuts[:-1].tolist(), cuts[1:].tolist())), chunksize=1)
    _G = None
    return int(sum(parts))
N_VERTEX_SAMPLES = 48


def vertex_sample(g, seed):
    """Seeded vertex ids: the largest-degree vertex of each side plus uniform picks."""
    rng = np.random.default_rng(seed + 7919)
    deg_u = np.diff(g.offsets.astype(np.int64))
    deg_v = np.bincount(g.adj, minlength=g.n_v)
    picks = {int(np.argmax(deg_u)), g.n_u + int(np.argmax(deg_v))}
    picks.update(int(x) for x in rng.choice(g.n_u + g.n_v, N_VERTEX_SAMPLES, replace=False))
    return sorted(picks)


def batch_sha256(graphs):
    """Digest of a batch: the members' SHA-256 digests hashed in order."""
    import hashlib

    h = hashlib.sha256()
    for g in graphs:
        h.update(bytes.fromhex(g.sha256()))
    return h.hexdigest()


def _member_count(g):
    return oracle.count(g)


def batch_main(name, seed, procs):
    t0 = time.time()
    graphs = synth.workload(name, seed)
    sha = batch_sha256(graphs)
    t1 = time.time()
    if procs <= 1:
        totals = [oracle.count(g) for g in graphs]
    else:
        with mp.get_context("fork").Pool(procs) as pool:
            totals = pool.map(_member_count, graphs, chunksize=16)
    t2 = time.time()
    data = json.load(open(BATCH_OUT)) if os.path.exists(BATCH_OUT) else {}
    data[f"{name}:{seed}"] = dict(workload=name, seed=seed, sha256=sha, n_graphs=len(graphs),
                                  edges=int(sum(g.m for g in graphs)), totals=[str(int(t)) for t in totals],
                                  oracle_seconds=round(t2 - t1, 1))
    with open(BATCH_OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=0, sort_keys=True)
    os.replace(BATCH_OUT + ".tmp", BATCH_OUT)
    print(f"{name}:{seed}: {len(graphs)} totals, sum {sum(totals)} (gen {t1 - t0:.1f}s, count {t2 - t1:.1f}s)",
          flush=True)


def _extension(job):
    kind, side, k = job
    sides = {"u": oracle.SIDE_U, "v": oracle.SIDE_V}
    if kind == "classes":
        return job, [str(int(x)) for x in oracle.count_classes(_G, sides[side])]
    return job, str(int(oracle.count_bicliques(_G, k, sides[side])))


def extensions_main(key, procs):
    """Class totals (pairs on U and on V) and (2,3) / (2,4)-biclique counts
    (pairs on U and on V) of a full-size workload, one oracle walk per
    process, stored under the workload's entry."""
    global _G
    data = json.load(open(OUT))
    name, seed = key.split(":")
    e = data[key]
    t0 = time.time()
    _G = synth.workload(name, int(seed))
    assert _G.sha256() == e["sha256"], "generator output changed"
    jobs = [("classes", "u", 0), ("classes", "v", 0)] + [("bicliques", sd, k) for k in (3, 4) for sd in ("u", "v")]
    with mp.get_context("fork").Pool(max(1, min(procs, len(jobs)))) as pool:
        res = pool.map(_extension, jobs, chunksize=1)
    _G = None
    for (kind, side, k), val in res:
        e[f"{kind}_{side}" if kind == "classes" else f"bicliques_k{k}_{side}"] = val
    e["extensions_seconds"] = round(time.time() - t0, 1)
    with open(OUT + ".tmp", "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(OUT + ".tmp", OUT)
    print(f"{key}: extensions {dict(res)} ({time.time() - t0:.1f}s)", flush=True)


def main(keys, procs=1):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for key in keys:
        name, seed = key.split(":")
        seed = int(seed)
        if name == "batch-10k":
            batch_main(name, seed, procs)
            continue
        t0 = time.time()
        g = synth.workload(name, seed)
        sha = g.sha256()
        t1 = time.time()
        total = oracle.count(g) if procs <= 1 else parallel_total(g, procs)
        t2 = time.time()
        xs = vertex_sample(g, seed)
        vc = oracle.vertices(g, xs)
        t3 = time.time()
        data[key] = dict(workload=name, seed=seed, sha256=sha, n_u=g.n_u, n_v=g.n_v, m=g.m, total=str(total),
                         vertex_ids=xs, vertex_counts=[str(int(v)) for v in vc],
                         oracle_seconds=round(t2 - t1, 1))
        print(f"{key}: total {total} (gen {t1 - t0:.1f}s, count {t2 - t1:.1f}s, vertices {t3 - t2:.1f}s)",
              flush=True)
        with open(OUT + ".tmp", "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)


if __name__ == "__main__":
    args = sys.argv[1:]
    procs = 1
    if args[:1] == ["--procs"]:
        procs, args = int(args[1]), args[2:]
    if args[:1] == ["--extensions"]:
        for key in args[1:]:
            extensions_main(key, procs)
    else:
        main(args or DEFAULT, procs)
