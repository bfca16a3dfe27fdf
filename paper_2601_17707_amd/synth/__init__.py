"""Seeded synthetic signed bipartite graphs.

This package only draws inputs: it holds none of the counting arithmetic and
imports neither the oracle nor the HIP binding, so the CPU oracle and the GPU
path are both fed from it.

The paper measures on fifteen public rating and interaction datasets
(Sec. "Datasets Description", Table 2).  None of them is available here, so
the named workloads are synthetic stand-ins with the shapes of the paper's
graphs: a uniform graph, power-law (Chung-Lu) graphs with heavy tails on both
sides, a highly skewed graph whose smaller side has huge hubs, a power-law
background with planted dense signed blocks, and a batch of many small graphs
of uneven size.  Signs follow the paper's convention for unsigned datasets
(each edge negative with a fixed probability) or a per-vertex bias model.

The large workloads are drawn by ``synth.c`` (SplitMix64 streams, batch-wise
rejection of repeated pairs); tiny exhaustive-test graphs use numpy.  Graphs
are a CSR over U: ``offsets`` (int32, n_u+1), ``adj`` (int32 V ids, rows
sorted by V id), ``signs`` (int8, +1/-1).
"""
from __future__ import annotations

import ctypes
import hashlib
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libsynth.so")
_SRC = os.path.join(_HERE, "synth.c")


def build() -> str:
    """Compile the generator (plain C, host only)."""
    subprocess.check_call(["gcc", "-O2", "-Wall", "-fopenmp", "-shared", "-fPIC", "-o", _SO, _SRC, "-lm"])
    return _SO


class _CGraph(ctypes.Structure):
    _fields_ = [
        ("n_u", ctypes.c_int32),
        ("n_v", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("offsets", ctypes.POINTER(ctypes.c_int32)),
        ("adj", ctypes.POINTER(ctypes.c_int32)),
        ("signs", ctypes.POINTER(ctypes.c_int8)),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        G = ctypes.POINTER(_CGraph)
        i32, i64, u64, f64, ci = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_double, ctypes.c_int)
        lib.synth_uniform.argtypes = [i32, i32, i64, f64, u64, G]
        lib.synth_uniform.restype = ci
        lib.synth_chung_lu.argtypes = [i32, i32, i64, f64, f64, f64, f64, ci, f64, ci, ci, f64, u64, G]
        lib.synth_chung_lu.restype = ci
        lib.synth_hybrid.argtypes = [i32, i32, i64, f64, f64, f64, i32, i32, f64, f64, u64, G,
                                     ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.synth_hybrid.restype = ci
        lib.synth_batch_params.argtypes = [u64, i32, f64, f64, ctypes.POINTER(i64), ctypes.POINTER(i32),
                                           ctypes.POINTER(i32), ctypes.POINTER(f64), ctypes.POINTER(f64),
                                           ctypes.POINTER(u64)]
        lib.synth_batch_params.restype = None
        lib.synth_free.argtypes = [G]
        lib.synth_free.restype = None
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Signed bipartite graph as a CSR over U (rows) with V ids as columns."""

    n_u: int
    n_v: int
    offsets: np.ndarray  # int32 [n_u + 1]
    adj: np.ndarray  # int32 [m]
    signs: np.ndarray  # int8 [m], +1 / -1
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.adj.shape[0])

    def edges(self):
        """(u, v, s) int64 arrays in CSR order."""
        deg = np.diff(self.offsets.astype(np.int64))
        u = np.repeat(np.arange(self.n_u, dtype=np.int64), deg)
        return u, self.adj.astype(np.int64), self.signs.astype(np.int64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.asarray([self.n_u, self.n_v, self.m], np.int64).tobytes())
        h.update(np.ascontiguousarray(self.offsets, np.int32).tobytes())
        h.update(np.ascontiguousarray(self.adj, np.int32).tobytes())
        h.update(np.ascontiguousarray(self.signs, np.int8).tobytes())
        return h.hexdigest()


def from_edges(n_u: int, n_v: int, u, v, s, meta=None) -> Graph:
    """CSR over U from an edge list; rows are sorted by V id."""
    u = np.asarray(u, np.int64).ravel()
    v = np.asarray(v, np.int64).ravel()
    s = np.asarray(s, np.int8).ravel()
    if u.size:
        if u.min() < 0 or u.max() >= n_u or v.min() < 0 or v.max() >= n_v:
            raise ValueError("edge endpoint out of range")
    order = np.lexsort((v, u))
    u, v, s = u[order], v[order], s[order]
    counts = np.bincount(u, minlength=n_u) if u.size else np.zeros(n_u, np.int64)
    offsets = np.zeros(n_u + 1, np.int64)
    np.cumsum(counts, out=offsets[1:])
    return Graph(n_u, n_v, offsets.astype(np.int32), v.astype(np.int32), s.astype(np.int8),
                 dict(meta or {}))


def _take(cg: _CGraph, meta: dict) -> Graph:
    lib = _load()
    try:
        m = int(cg.m)
        off = np.ctypeslib.as_array(cg.offsets, shape=(cg.n_u + 1,)).copy()
        adj = np.ctypeslib.as_array(cg.adj, shape=(max(m, 1),))[:m].copy()
        sg = np.ctypeslib.as_array(cg.signs, shape=(max(m, 1),))[:m].copy()
    finally:
        lib.synth_free(ctypes.byref(cg))
    return Graph(int(cg.n_u), int(cg.n_v), off, adj, sg, meta)


def uniform_graph(n_u: int, n_v: int, m: int, p_neg: float, seed: int) -> Graph:
    """m distinct edges with both endpoints uniform; each sign is -1 w.p. p_neg."""
    cg = _CGraph()
    rc = _load().synth_uniform(n_u, n_v, m, p_neg, seed, ctypes.byref(cg))
    if rc:
        raise ValueError("bad uniform graph parameters")
    return _take(cg, dict(kind="uniform", n_u=n_u, n_v=n_v, m=m, p_neg=p_neg, seed=seed))


def chung_lu_graph(n_u: int, n_v: int, m: int, gamma_u: float, gamma_v: float, dmax_u: float,
                   dmax_v: float, seed: int, p_neg: float = 0.2, beta_bias=None) -> Graph:
    """Chung-Lu bipartite graph with m distinct edges.

    Vertex i of a side with n vertices is drawn with probability
    (H(i+1) - H(i)) / H(n), H(x) = integral_0^x (t + i0)^(-1/(gamma-1)) dt, a
    power law of exponent gamma whose head shift i0 makes the largest expected
    degree dmax.  Ids are shuffled so id order is unrelated to degree.  Signs
    are i.i.d. with P(-) = p_neg, or with ``beta_bias=(a, b, scale)`` every
    vertex draws beta_x ~ Beta(a, b) and uv is negative with probability
    clip(scale * (beta_u + beta_v), 0, 1).
    """
    cg = _CGraph()
    if beta_bias is None:
        mode, a, b, sc = 0, 0, 0, 0.0
    else:
        mode, (a, b, sc) = 1, beta_bias
    rc = _load().synth_chung_lu(n_u, n_v, m, gamma_u, gamma_v, dmax_u, dmax_v, mode, p_neg,
                                int(a), int(b), float(sc), seed, ctypes.byref(cg))
    if rc:
        raise ValueError("bad Chung-Lu parameters")
    return _take(cg, dict(kind="chung_lu", n_u=n_u, n_v=n_v, m=m, gamma_u=gamma_u, gamma_v=gamma_v,
                          dmax_u=dmax_u, dmax_v=dmax_v, p_neg=p_neg, beta_bias=beta_bias, seed=seed))


def hybrid_graph(n_u: int, n_v: int, m_bg: int, n_blocks: int, block: int, density: float,
                 flip: float, seed: int, gamma: float = 2.1, dmax: float = 50_000,
                 p_neg: float = 0.2) -> Graph:
    """Power-law background plus planted dense signed blocks.

    Blocks use pairwise-disjoint rows R_i (V side) and columns C_i (U side) of
    ``block`` vertices each.  Inside R_i x C_i each pair is an edge with
    probability ``density``; every vertex has a faction f_x in {+1, -1}; the
    sign of rc is f_r f_c, flipped with probability ``flip``.  Block draws
    replace the background inside the blocks.  ``meta['blocks']`` lists
    (V ids, U ids) per block.
    """
    cg = _CGraph()
    rows = np.zeros(max(n_blocks * block, 1), np.int32)
    cols = np.zeros(max(n_blocks * block, 1), np.int32)
    P = ctypes.POINTER(ctypes.c_int32)
    rc = _load().synth_hybrid(n_u, n_v, m_bg, gamma, dmax, p_neg, n_blocks, block, density, flip,
                              seed, ctypes.byref(cg), rows.ctypes.data_as(P), cols.ctypes.data_as(P))
    if rc:
        raise ValueError("bad hybrid parameters")
    blocks = [(rows[i * block:(i + 1) * block].copy(), cols[i * block:(i + 1) * block].copy())
              for i in range(n_blocks)]
    return _take(cg, dict(kind="hybrid", n_u=n_u, n_v=n_v, m_bg=m_bg, n_blocks=n_blocks,
                          block=block, density=density, flip=flip, seed=seed, gamma=gamma,
                          dmax=dmax, p_neg=p_neg, blocks=blocks))


def batch_member_params(seed: int, i: int, m_lo: float = 100, m_hi: float = 200_000):
    lib = _load()
    m = ctypes.c_int64()
    nu = ctypes.c_int32()
    nv = ctypes.c_int32()
    g = ctypes.c_double()
    p = ctypes.c_double()
    s = ctypes.c_uint64()
    lib.synth_batch_params(seed, i, m_lo, m_hi, ctypes.byref(m), ctypes.byref(nu), ctypes.byref(nv),
                           ctypes.byref(g), ctypes.byref(p), ctypes.byref(s))
    return dict(m=m.value, n_u=nu.value, n_v=nv.value, gamma=g.value, p_neg=p.value,
                seed=s.value)


def batch_graphs(n_graphs: int, seed: int, m_lo: float = 100, m_hi: float = 200_000):
    """Independent Chung-Lu graphs of uneven size.

    Edge counts are log-uniform in [m_lo, m_hi]; |U|/|V| is uniform in
    [0.2, 5]; one exponent uniform in [1.8, 2.8] serves both sides; P(-) is
    uniform in [0.1, 0.5]; |U|+|V| keeps the mean total degree at most 8 and
    the density at most 0.25; the largest expected degree is
    min(sqrt(m), other side).
    """
    out = []
    for i in range(n_graphs):
        q = batch_member_params(seed, i, m_lo, m_hi)
        d = float(np.sqrt(q["m"]))
        out.append(chung_lu_graph(q["n_u"], q["n_v"], q["m"], q["gamma"], q["gamma"],
                                  min(d, q["n_v"]), min(d, q["n_u"]), q["seed"], p_neg=q["p_neg"]))
    return out


def small_random_graph(rng: np.random.Generator, max_n: int = 12, density=None, p_neg=None) -> Graph:
    """Tiny random graph for exhaustive checks (0..max_n vertices per side)."""
    n_u = int(rng.integers(0, max_n + 1))
    n_v = int(rng.integers(0, max_n + 1))
    d = rng.uniform(0.1, 0.9) if density is None else density
    p = rng.uniform(0.0, 1.0) if p_neg is None else p_neg
    present = rng.random((n_u, n_v)) < d
    uu, vv = np.nonzero(present)
    s = np.where(rng.random(uu.size) < p, -1, 1).astype(np.int8)
    return from_edges(n_u, n_v, uu, vv, s, dict(kind="small", density=d, p_neg=p))


def random_graph(rng: np.random.Generator, n_u: int, n_v: int, density: float, p_neg: float) -> Graph:
    """Erdos-Renyi bipartite graph of a given size (numpy stream)."""
    present = rng.random((n_u, n_v)) < density
    uu, vv = np.nonzero(present)
    s = np.where(rng.random(uu.size) < p_neg, -1, 1).astype(np.int8)
    return from_edges(n_u, n_v, uu, vv, s, dict(kind="er", density=density, p_neg=p_neg))


def complete_graph(n_u: int, n_v: int, signs=None) -> Graph:
    """K_{n_u,n_v}; ``signs`` is an optional (n_u, n_v) array of +1/-1."""
    uu, vv = np.meshgrid(np.arange(n_u), np.arange(n_v), indexing="ij")
    s = np.ones((n_u, n_v), np.int8) if signs is None else np.asarray(signs, np.int8)
    return from_edges(n_u, n_v, uu.ravel(), vv.ravel(), s.ravel(), dict(kind="complete"))


def shuffle_rows(g: Graph, rng: np.random.Generator) -> Graph:
    """Same graph with every row's entries in a random order."""
    adj = g.adj.copy()
    sg = g.signs.copy()
    for u in range(g.n_u):
        a, b = int(g.offsets[u]), int(g.offsets[u + 1])
        if b - a > 1:
            p = rng.permutation(b - a) + a
            adj[a:b] = g.adj[p]
            sg[a:b] = g.signs[p]
    return Graph(g.n_u, g.n_v, g.offsets.copy(), adj, sg, dict(g.meta, shuffled=True))


# ---------------------------------------------------------------------------
# named workloads (seed selects the instance)

WORKLOADS = {
    "uniform-2k-1k-20k": "uniform 2,000 x 1,000, 20,000 distinct edges, P(-)=0.3",
    "powerlaw-1m-500k-20m": "Chung-Lu 1,000,000 x 500,000, 20M edges, gamma 2.1 both sides, "
                            "max expected degree 50,000, P(-)=0.2",
    "skewed-5m-200k-200m": "Chung-Lu 5,000,000 x 200,000, 200M edges, gamma_U 2.5 (max 14,142), "
                           "gamma_V 1.8 (max 500,000), Beta(2,5) vertex sign bias, mean P(-)=0.4",
    "hybrid-2m-1m-50m-16x4096": "Chung-Lu 2,000,000 x 1,000,000, 50M edges (gamma 2.1, max 50,000, "
                                "P(-)=0.2) + 16 planted 4,096 x 4,096 blocks at density 0.5, "
                                "two factions, 10% sign flips",
    "batch-10k": "10,000 Chung-Lu graphs, m log-uniform in [100, 200,000]",
}


def workload(name: str, seed: int = 1):
    """Build a named workload; ``batch-10k`` returns a list of graphs."""
    if name == "uniform-2k-1k-20k":
        return uniform_graph(2_000, 1_000, 20_000, 0.3, seed)
    if name == "powerlaw-1m-500k-20m":
        return chung_lu_graph(1_000_000, 500_000, 20_000_000, 2.1, 2.1, 50_000, 50_000, seed,
                              p_neg=0.2)
    if name == "skewed-5m-200k-200m":
        return chung_lu_graph(5_000_000, 200_000, 200_000_000, 2.5, 1.8,
                              float(np.sqrt(200_000_000)), 500_000, seed, beta_bias=(2, 5, 0.7))
    if name == "hybrid-2m-1m-50m-16x4096":
        return hybrid_graph(2_000_000, 1_000_000, 50_000_000, 16, 4096, 0.5, 0.1, seed)
    if name == "batch-10k":
        return batch_graphs(10_000, seed)
    raise KeyError(name)
