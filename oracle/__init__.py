"""Serial CPU oracle for balanced butterfly counting.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  The product path never imports
this package; it shares no code with the GPU library.

``bbc_oracle.c`` holds the arithmetic (plain C, compiled with gcc):

* :func:`count` - Algorithm 1 (BB2K) with k = 2, per-anchor symmetric /
  asymmetric wedge buckets (Definitions 7-9, Lemma 1), plain id order;
* :func:`count_anchors` - the same over a range of anchors (timing samples);
* :func:`brute` - Definitions 1 and 2 applied to every 2x2 vertex choice;
* :func:`count_kinds` - balanced / unbalanced / all butterflies per pair;
* :func:`count_classes` and :func:`brute_classes` - the six sign-pattern
  classes of the case study (Table 8), by the walk and by brute force;
* :func:`per_vertex`, :func:`vertex` and :func:`vertices` - balanced butterflies containing
  each vertex (the paper reports totals only; see the C header);
* :func:`count_bicliques` and :func:`brute_bicliques` - balanced
  (2,k)-bicliques (Definition 5), by the general-k walk and by enumeration;
* :func:`apply_updates` and :func:`update_delta` - dynamic graphs (Sec.
  "Future Directions": edges added, removed or re-signed): the graph after
  a batch of updates, and the change of the count as the difference of two
  full counts.

``mbbc.c`` is a separate multicore timing baseline (OpenMP, in the manner of
Algorithm 2), checked against the serial walk: :func:`mbbc_count`.

Graphs are passed as any object with ``n_u, n_v, offsets, adj, signs``
(CSR over U, int32 / int32 / int8).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "bbc_oracle.c")

SIDE_AUTO, SIDE_U, SIDE_V = 0, 1, 2


_MBBC_SO = os.path.join(_HERE, "libmbbc.so")
_MBBC_SRC = os.path.join(_HERE, "mbbc.c")


def build() -> str:
    subprocess.check_call(["gcc", "-O2", "-Wall", "-Wextra", "-shared", "-fPIC", "-o", _SO, _SRC])
    subprocess.check_call(["gcc", "-O3", "-Wall", "-Wextra", "-fopenmp", "-shared", "-fPIC", "-o", _MBBC_SO,
                           _MBBC_SRC])
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        P32 = ctypes.POINTER(ctypes.c_int32)
        P8 = ctypes.POINTER(ctypes.c_int8)
        PU = ctypes.POINTER(ctypes.c_uint64)
        head = [i32, i32, i64, P32, P32, P8]
        lib.oracle_count.argtypes = head + [ctypes.c_int, PU]
        lib.oracle_count_kinds.argtypes = head + [ctypes.c_int, PU, PU, PU]
        lib.oracle_per_vertex.argtypes = head + [ctypes.c_int, PU]
        lib.oracle_vertex.argtypes = head + [i64, PU]
        lib.oracle_brute.argtypes = head + [PU, PU, PU]
        lib.oracle_count_classes.argtypes = head + [ctypes.c_int, PU]
        lib.oracle_brute_classes.argtypes = head + [ctypes.c_int, PU]
        lib.oracle_per_vertex_classes.argtypes = head + [ctypes.c_int, PU]
        lib.oracle_brute_per_vertex_classes.argtypes = head + [ctypes.c_int, PU]
        lib.oracle_count_bicliques.argtypes = head + [ctypes.c_int, ctypes.c_int, PU]
        lib.oracle_brute_bicliques.argtypes = head + [ctypes.c_int, ctypes.c_int, PU]
        lib.oracle_count_anchors.argtypes = head + [ctypes.c_int, i32, i32, PU, PU]
        lib.oracle_vertices.argtypes = head + [ctypes.POINTER(ctypes.c_int64), i64, PU]
        lib.oracle_vertices.restype = ctypes.c_int
        for f in (lib.oracle_count_anchors, lib.oracle_count, lib.oracle_count_kinds, lib.oracle_per_vertex, lib.oracle_vertex,
                  lib.oracle_brute, lib.oracle_count_classes, lib.oracle_brute_classes, lib.oracle_count_bicliques,
                  lib.oracle_brute_bicliques):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def _args(g):
    off = np.ascontiguousarray(g.offsets, np.int32)
    adj = np.ascontiguousarray(g.adj, np.int32)
    sg = np.ascontiguousarray(g.signs, np.int8)
    keep = (off, adj, sg)
    P32 = ctypes.POINTER(ctypes.c_int32)
    P8 = ctypes.POINTER(ctypes.c_int8)
    return keep, [int(g.n_u), int(g.n_v), int(adj.shape[0]), off.ctypes.data_as(P32),
                  adj.ctypes.data_as(P32), sg.ctypes.data_as(P8)]


def _u64():
    return ctypes.c_uint64(0)


def _check(rc):
    if rc != 0:
        raise ValueError("oracle: malformed graph (offsets, ids or signs)")


def count(g, side: int = SIDE_AUTO) -> int:
    """Number of balanced butterflies (Algorithm 1, k = 2)."""
    keep, a = _args(g)
    out = _u64()
    _check(_load().oracle_count(*a, side, ctypes.byref(out)))
    del keep
    return int(out.value)


_mbbc = None


def mbbc_count(g):
    """Multicore CPU baseline in the manner of Algorithm 2 (M-BBC): OpenMP
    over anchors of the smaller side, heaviest first, thread-local buckets,
    priority-ordered pair filter.  Returns (total, threads used); the
    thread count follows OMP_NUM_THREADS (default: every host core)."""
    global _mbbc
    if _mbbc is None:
        if not os.path.exists(_MBBC_SO):
            build()
        lib = ctypes.CDLL(_MBBC_SO)
        P32 = ctypes.POINTER(ctypes.c_int32)
        lib.mbbc_count.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P32, P32,
                                   ctypes.POINTER(ctypes.c_int8), ctypes.POINTER(ctypes.c_uint64), P32]
        lib.mbbc_count.restype = ctypes.c_int
        _mbbc = lib
    keep, a = _args(g)
    out = _u64()
    th = ctypes.c_int32(0)
    if _mbbc.mbbc_count(*a, ctypes.byref(out), ctypes.byref(th)) != 0:
        raise MemoryError("mbbc: out of host memory")
    del keep
    return int(out.value), int(th.value)


def count_anchors(g, a_lo: int, a_hi: int, side: int = SIDE_AUTO):
    """(partial count, wedges bucketed) of Algorithm 1 over anchors a_lo <= u < a_hi."""
    keep, a = _args(g)
    p, w = _u64(), _u64()
    _check(_load().oracle_count_anchors(*a, side, int(a_lo), int(a_hi), ctypes.byref(p), ctypes.byref(w)))
    del keep
    return int(p.value), int(w.value)


def count_kinds(g, side: int = SIDE_AUTO):
    """(balanced, unbalanced, all butterflies) from per-pair wedge counts."""
    keep, a = _args(g)
    b, u, t = _u64(), _u64(), _u64()
    _check(_load().oracle_count_kinds(*a, side, ctypes.byref(b), ctypes.byref(u), ctypes.byref(t)))
    del keep
    return int(b.value), int(u.value), int(t.value)


def per_vertex(g, side: int = SIDE_AUTO) -> np.ndarray:
    """uint64 [n_u + n_v]: balanced butterflies containing each vertex (U first)."""
    keep, a = _args(g)
    out = np.zeros(int(g.n_u) + int(g.n_v), np.uint64)
    _check(_load().oracle_per_vertex(*a, side, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    del keep
    return out


def vertex(g, x: int) -> int:
    """Balanced butterflies containing vertex x (global index, U first)."""
    keep, a = _args(g)
    out = _u64()
    _check(_load().oracle_vertex(*a, int(x), ctypes.byref(out)))
    del keep
    return int(out.value)


def vertices(g, xs) -> np.ndarray:
    """uint64 counts of the vertices xs (global indices, U first)."""
    keep, a = _args(g)
    xs = np.ascontiguousarray(xs, np.int64)
    out = np.zeros(xs.size, np.uint64)
    _check(_load().oracle_vertices(*a, xs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), xs.size,
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    del keep
    return out


def brute(g, per_vertex: bool = False):
    """(balanced, unbalanced[, per-vertex]) by enumerating every 2x2 choice."""
    keep, a = _args(g)
    b, u = _u64(), _u64()
    pv = np.zeros(int(g.n_u) + int(g.n_v), np.uint64) if per_vertex else None
    ptr = pv.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)) if per_vertex else None
    _check(_load().oracle_brute(*a, ctypes.byref(b), ctypes.byref(u), ptr))
    del keep
    if per_vertex:
        return int(b.value), int(u.value), pv
    return int(b.value), int(u.value)


CLASS_NAMES = ("pp_pp", "pp_mm", "mm_mm", "pm_pm", "pp_pm", "pm_mm")


def count_classes(g, side: int = SIDE_AUTO) -> list:
    """Six sign-pattern classes [++/++, ++/--, --/--, +-/+-, ++/+-, +-/--]
    over pairs of the anchor side (see the C header)."""
    keep, a = _args(g)
    out = (ctypes.c_uint64 * 6)()
    _check(_load().oracle_count_classes(*a, side, out))
    return [int(x) for x in out]


def brute_classes(g, side: int = SIDE_AUTO) -> list:
    """The same classes by brute force over all 2 x 2 vertex choices."""
    keep, a = _args(g)
    out = (ctypes.c_uint64 * 6)()
    _check(_load().oracle_brute_classes(*a, side, out))
    return [int(x) for x in out]


def per_vertex_classes(g, side: int = SIDE_AUTO) -> np.ndarray:
    """uint64 [n_u + n_v, 6]: class-k butterflies containing each vertex
    (U first), classes in the order of count_classes."""
    keep, a = _args(g)
    out = np.zeros((int(g.n_u) + int(g.n_v), 6), np.uint64)
    _check(_load().oracle_per_vertex_classes(*a, side, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    del keep
    return out


def brute_per_vertex_classes(g, side: int = SIDE_AUTO) -> np.ndarray:
    """The same by brute force over every 2 x 2 vertex choice (tiny graphs)."""
    keep, a = _args(g)
    out = np.zeros((int(g.n_u) + int(g.n_v), 6), np.uint64)
    _check(_load().oracle_brute_per_vertex_classes(*a, side, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))))
    del keep
    return out


def count_bicliques(g, k: int, side: int = SIDE_AUTO) -> int:
    """Balanced (2,k)-bicliques with the two vertices on `side` (Definition
    5; Algorithm 1 with general k), exact in 128 bits.  The BB2K section
    fixes the size-two side as U, so SIDE_AUTO means U here.  OverflowError
    when a term or the total does not fit 128 bits."""
    keep, a = _args(g)
    out = (ctypes.c_uint64 * 2)()
    rc = _load().oracle_count_bicliques(*a, side, int(k), out)
    if rc == 2:
        raise OverflowError("(2,k)-biclique count does not fit 128 bits")
    _check(rc)
    return int(out[0]) | (int(out[1]) << 64)


def brute_bicliques(g, k: int, side: int = SIDE_AUTO) -> int:
    """The same by enumerating every pair and every k-subset of its common
    neighbours (tiny graphs, at most 24 common neighbours per pair)."""
    keep, a = _args(g)
    out = _u64()
    _check(_load().oracle_brute_bicliques(*a, side, int(k), ctypes.byref(out)))
    return int(out.value)


class _G:
    """Minimal CSR graph (the attributes the oracle reads)."""

    def __init__(self, n_u, n_v, offsets, adj, signs):
        self.n_u, self.n_v, self.offsets, self.adj, self.signs = n_u, n_v, offsets, adj, signs


def apply_updates(g, uu, vv, ss):
    """The graph after a batch of edge updates: pair (uu[i], vv[i]) takes
    sign ss[i] (+1 / -1), or is removed when ss[i] == 0.  Pairs are
    distinct; removing an absent pair does nothing."""
    deg = np.diff(np.asarray(g.offsets, np.int64))
    state = {}
    for u, v, s in zip(np.repeat(np.arange(g.n_u), deg).tolist(), np.asarray(g.adj).tolist(),
                       np.asarray(g.signs).tolist()):
        state[(u, v)] = s
    seen = set()
    for u, v, s in zip(np.asarray(uu).tolist(), np.asarray(vv).tolist(), np.asarray(ss).tolist()):
        if (u, v) in seen:
            raise ValueError("repeated pair in one update batch")
        seen.add((u, v))
        if s == 0:
            state.pop((u, v), None)
        else:
            state[(u, v)] = s
    keys = sorted(state)
    u = np.array([k[0] for k in keys], np.int64)
    v = np.array([k[1] for k in keys], np.int64)
    s = np.array([state[k] for k in keys], np.int8)
    off = np.zeros(g.n_u + 1, np.int64)
    if u.size:
        np.cumsum(np.bincount(u, minlength=g.n_u), out=off[1:])
    return _G(g.n_u, g.n_v, off.astype(np.int32), v.astype(np.int32), s)


def update_delta(g, uu, vv, ss) -> int:
    """T(after) - T(before) for a batch of updates, from two full counts."""
    return count(apply_updates(g, uu, vv, ss)) - count(g)
