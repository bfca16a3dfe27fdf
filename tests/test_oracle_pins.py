"""Pins of the CPU oracle to facts the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check is a value printed
(or drawn) in the paper, a closed form, an invariant of the definition, or an
exhaustive enumeration written independently below.
"""
import itertools
import os
import shutil
import subprocess
from math import comb

import numpy as np
import pytest

import oracle
from paper_2601_17707_amd import synth
from tests.fixtures import load_graphs, load_table8

pytestmark = pytest.mark.filterwarnings("ignore")


def py_brute(g):
    """Definitions 1 and 2 in pure Python: (balanced, unbalanced, per-vertex)."""
    sign = {}
    for u in range(g.n_u):
        for e in range(g.offsets[u], g.offsets[u + 1]):
            sign[(u, int(g.adj[e]))] = int(g.signs[e])
    bal = unb = 0
    pv = [0] * (g.n_u + g.n_v)
    for u1, u2 in itertools.combinations(range(g.n_u), 2):
        for v1, v2 in itertools.combinations(range(g.n_v), 2):
            quad = [(u1, v1), (u1, v2), (u2, v1), (u2, v2)]
            if all(q in sign for q in quad):
                negs = sum(sign[q] < 0 for q in quad)
                if negs % 2 == 0:
                    bal += 1
                    for x in (u1, u2, g.n_u + v1, g.n_u + v2):
                        pv[x] += 1
                else:
                    unb += 1
    return bal, unb, pv


FIXTURES = {}
for fname in ("fig2_butterflies.txt", "fig1b_signed_k44.txt", "drug_target_sample.txt"):
    FIXTURES.update(load_graphs(fname))


# --------------------------------------------------------------- paper examples


@pytest.mark.parametrize("name", sorted(FIXTURES))
def test_paper_examples(name):
    """Fig. 1(b), Fig. 2 panels and the case-study sample graph."""
    g, exp = FIXTURES[name]
    for side in (oracle.SIDE_AUTO, oracle.SIDE_U, oracle.SIDE_V):
        assert oracle.count(g, side) == exp["balanced"]
    b, u = oracle.brute(g)
    assert b == exp["balanced"]
    if "unbalanced" in exp:
        assert u == exp["unbalanced"]
        kb, ku, kt = oracle.count_kinds(g)
        assert (kb, ku) == (exp["balanced"], exp["unbalanced"])
        assert kt == exp["balanced"] + exp["unbalanced"]
    if "butterflies" in exp:
        assert b + u == exp["butterflies"]
    pb, pu, _ = py_brute(g)
    assert pb == exp["balanced"]


def test_table8_identity():
    """Table 8: the six classes sum to the stated 69,537 butterflies; balanced
    (coherent + incoherent) and mixed split 65,741 / 3,796."""
    total, classes = load_table8()
    assert sum(c for _, c, _ in classes) == total == 69537
    assert sum(c for _, c, k in classes if k == "balanced") == 65741
    assert sum(c for _, c, k in classes if k == "unbalanced") == 3796
    # the percentages quoted in the text: about 81 %, 13.5 % and 5.5 %
    coh = sum(c for n, c, _ in classes if n.startswith("coherent"))
    inc = sum(c for n, c, _ in classes if n.startswith("incoherent"))
    assert round(100 * coh / total) == 81
    assert round(100 * inc / total, 1) == 13.5
    assert round(100 * 3796 / total, 1) == 5.5


# ----------------------------------------------------------------- brute force


def py_classes(g, side):
    """The six sign-pattern classes in pure Python, from the definition: a
    butterfly is two anchor-side vertices and two centres; each centre's
    pattern is ++, -- or +- (the two edges differ); its class is the
    unordered pair of the two patterns."""
    sign = {}
    for u in range(g.n_u):
        for e in range(g.offsets[u], g.offsets[u + 1]):
            sign[(u, int(g.adj[e]))] = int(g.signs[e])
    su = side == oracle.SIDE_U or (side == oracle.SIDE_AUTO and g.n_u < g.n_v)
    n_s, n_c = (g.n_u, g.n_v) if su else (g.n_v, g.n_u)
    key = (lambda a, c: (a, c)) if su else (lambda a, c: (c, a))
    order = {("pp", "pp"): 0, ("mm", "pp"): 1, ("mm", "mm"): 2, ("pm", "pm"): 3, ("pm", "pp"): 4, ("mm", "pm"): 5}
    out = [0] * 6
    for a1, a2 in itertools.combinations(range(n_s), 2):
        for c1, c2 in itertools.combinations(range(n_c), 2):
            s = [sign.get(key(a, c)) for a in (a1, a2) for c in (c1, c2)]
            if None in s:
                continue
            x1, x2, y1, y2 = s  # a1c1, a1c2, a2c1, a2c2
            pat = sorted("pm" if x != y else ("pp" if x > 0 else "mm") for x, y in ((x1, y1), (x2, y2)))
            out[order[tuple(pat)]] += 1
    return out


def test_classes_of_the_case_study_sample():
    """The sample drug-target network (drugs on U, the case study's pair
    side): the class split derived by hand from the figure, 5 coherent
    (1 ++/++, 3 ++/--, 1 --/--), 1 incoherent, 2 mixed (one of each)."""
    g, exp = load_graphs("drug_target_sample.txt")["drug_target"]
    got = oracle.count_classes(g, oracle.SIDE_U)
    assert got == [exp["class_" + n] for n in oracle.CLASS_NAMES]
    assert got == oracle.brute_classes(g, oracle.SIDE_U) == py_classes(g, oracle.SIDE_U)
    assert sum(got[:4]) == exp["balanced"] and sum(got[4:]) == exp["unbalanced"]
    # pairs of targets instead: the same butterflies, other classes
    assert oracle.count_classes(g, oracle.SIDE_V) == py_classes(g, oracle.SIDE_V)


def test_class_order_matches_table8():
    """The class order and kinds follow Table 8: coherent ++/++, ++/--,
    --/--, incoherent +-/+- balanced; mixed ++/+- and +-/-- unbalanced."""
    _, classes = load_table8()
    assert [n.split("_", 1)[1] for n, _, _ in classes] == list(oracle.CLASS_NAMES)
    assert [k for _, _, k in classes] == ["balanced"] * 4 + ["unbalanced"] * 2


@pytest.mark.parametrize("seed", range(6))
def test_classes_walk_matches_definitions(seed):
    rng = np.random.default_rng(100 + seed)
    for _ in range(25):
        n_u, n_v = int(rng.integers(1, 9)), int(rng.integers(1, 9))
        A = rng.random((n_u, n_v)) < rng.random()
        u, v = np.nonzero(A)
        sg = np.where(rng.random(u.size) < rng.random(), -1, 1)
        g = synth.from_edges(n_u, n_v, u, v, sg)
        for side in (oracle.SIDE_AUTO, oracle.SIDE_U, oracle.SIDE_V):
            got = oracle.count_classes(g, side)
            assert got == oracle.brute_classes(g, side) == py_classes(g, side)
            bal, unb, allb = oracle.count_kinds(g, side)
            assert sum(got[:4]) == bal and sum(got[4:]) == unb and sum(got) == allb


@pytest.mark.parametrize("s,c", [(2, 2), (3, 5), (6, 4)])
def test_classes_closed_forms(s, c):
    """K_{s,c} with the s vertices of U as the pair side: all positive ->
    C(s,2) C(c,2) of ++/++; one negative edge at (u0, c0) -> the s - 1 pairs
    holding u0 keep C(c-1,2) ++/++ and gain c - 1 ++/+- each."""
    u, v = np.divmod(np.arange(s * c), c)
    g = synth.from_edges(s, c, u, v, np.ones(s * c, np.int8))
    assert oracle.count_classes(g, oracle.SIDE_U) == [comb(s, 2) * comb(c, 2), 0, 0, 0, 0, 0]
    sg = np.ones(s * c, np.int8)
    sg[0] = -1
    g = synth.from_edges(s, c, u, v, sg)
    pp = (s - 1) * comb(c - 1, 2) + comb(s - 1, 2) * comb(c, 2)
    assert oracle.count_classes(g, oracle.SIDE_U) == [pp, 0, 0, 0, (s - 1) * (c - 1), 0]
    # every sign negative: the mirror image
    g = synth.from_edges(s, c, u, v, -np.ones(s * c, np.int8))
    assert oracle.count_classes(g, oracle.SIDE_U) == [0, 0, comb(s, 2) * comb(c, 2), 0, 0, 0]


def test_brute_matches_python_definition():
    rng = np.random.default_rng(11)
    for _ in range(150):
        g = synth.small_random_graph(rng, max_n=7)
        b, u, pv = oracle.brute(g, per_vertex=True)
        pb, pu, ppv = py_brute(g)
        assert (b, u) == (pb, pu)
        assert list(pv) == ppv


def test_bucket_method_equals_enumeration():
    """Algorithm 1 (k = 2) on 1,500 random tiny graphs, every anchor side."""
    rng = np.random.default_rng(12)
    for i in range(1500):
        g = synth.small_random_graph(rng, max_n=12)
        b, u = oracle.brute(g)
        for side in (oracle.SIDE_AUTO, oracle.SIDE_U, oracle.SIDE_V):
            assert oracle.count(g, side) == b, (i, side)
        kb, ku, kt = oracle.count_kinds(g)
        assert (kb, ku, kt) == (b, u, b + u)


def test_bucket_method_equals_enumeration_medium():
    rng = np.random.default_rng(13)
    for n_u, n_v, d in [(40, 25, 0.3), (25, 60, 0.5), (64, 64, 0.15), (30, 30, 0.9)]:
        g = synth.random_graph(rng, n_u, n_v, d, 0.35)
        b, u = oracle.brute(g)
        assert oracle.count(g, oracle.SIDE_U) == b
        assert oracle.count(g, oracle.SIDE_V) == b


# ----------------------------------------------------------------- closed forms


@pytest.mark.parametrize("m,n", [(2, 2), (2, 7), (5, 7), (6, 3), (9, 11)])
def test_complete_bipartite_closed_forms(m, n):
    base = comb(m, 2) * comb(n, 2)
    g = synth.complete_graph(m, n)
    assert oracle.count(g) == base
    # signs s_uv = x_u y_v: every butterfly has an even number of negatives
    rng = np.random.default_rng(m * 31 + n)
    x = rng.choice([-1, 1], m)
    y = rng.choice([-1, 1], n)
    assert oracle.count(synth.complete_graph(m, n, np.outer(x, y))) == base
    # one negative edge: it lies in (m-1)(n-1) butterflies, all unbalanced
    s = np.ones((m, n), np.int8)
    s[0, 0] = -1
    assert oracle.count(synth.complete_graph(m, n, s)) == base - (m - 1) * (n - 1)
    if n >= 2:  # two negatives sharing a U vertex: unbalanced 2(m-1)(n-1) - 2(m-1)
        s = np.ones((m, n), np.int8)
        s[0, 0] = s[0, 1] = -1
        assert oracle.count(synth.complete_graph(m, n, s)) == base - (2 * (m - 1) * (n - 1) - 2 * (m - 1))
    if m >= 2:  # sharing a V vertex
        s = np.ones((m, n), np.int8)
        s[0, 0] = s[1, 0] = -1
        assert oracle.count(synth.complete_graph(m, n, s)) == base - (2 * (m - 1) * (n - 1) - 2 * (n - 1))
    if m >= 2 and n >= 2:  # disjoint: only the butterfly holding both is balanced
        s = np.ones((m, n), np.int8)
        s[0, 0] = s[1, 1] = -1
        assert oracle.count(synth.complete_graph(m, n, s)) == base - (2 * (m - 1) * (n - 1) - 2)


def test_k57_values():
    """K_{5,7} with one negative, two sharing u, two disjoint: 186 / 170 / 164."""
    vals = []
    for neg in ([(0, 0)], [(0, 0), (0, 1)], [(0, 0), (1, 1)]):
        s = np.ones((5, 7), np.int8)
        for a, b in neg:
            s[a, b] = -1
        vals.append(oracle.count(synth.complete_graph(5, 7, s)))
    assert vals == [186, 170, 164]


def test_k2n_closed_form():
    """Two anchors: T = C(a,2) + C(b,2) over their agree / disagree columns."""
    rng = np.random.default_rng(14)
    for n in range(1, 30):
        s = rng.choice([-1, 1], (2, n)).astype(np.int8)
        a = int((s[0] == s[1]).sum())
        assert oracle.count(synth.complete_graph(2, n, s)) == comb(a, 2) + comb(n - a, 2)


def test_degenerate_graphs():
    for n_u, n_v in [(0, 0), (0, 5), (5, 0), (1, 9), (9, 1)]:
        g = synth.complete_graph(n_u, n_v)
        assert oracle.count(g) == 0
    g = synth.from_edges(10, 10, [], [], [])
    assert oracle.count(g) == 0
    assert oracle.per_vertex(g).sum() == 0


# ------------------------------------------------------------------- invariants


def _mid_graphs():
    rng = np.random.default_rng(21)
    out = [synth.random_graph(rng, 60, 40, 0.25, 0.3), synth.random_graph(rng, 35, 80, 0.2, 0.5)]
    out.append(synth.chung_lu_graph(300, 200, 2500, 2.1, 2.1, 80, 80, seed=5, p_neg=0.25))
    out.append(synth.chung_lu_graph(150, 400, 3000, 2.5, 1.8, 60, 200, seed=6, beta_bias=(2, 5, 0.7)))
    return out


def _with_signs(g, s):
    return synth.Graph(g.n_u, g.n_v, g.offsets, g.adj, np.asarray(s, np.int8), {})


def test_balanced_plus_unbalanced_is_unsigned_count():
    for g in _mid_graphs():
        t = oracle.count(g)
        b, n, all_ = oracle.count_kinds(g)
        assert b == t and b + n == all_
        assert oracle.count(_with_signs(g, np.ones_like(g.signs))) == all_


def test_switching_and_global_flip():
    """Negating every edge at one vertex keeps each butterfly's parity (it has
    0 or 2 edges at that vertex); a global flip negates all four edges."""
    rng = np.random.default_rng(22)
    for g in _mid_graphs():
        t = oracle.count(g)
        pv = oracle.per_vertex(g)
        u, v, s = g.edges()
        assert oracle.count(_with_signs(g, -s)) == t
        for _ in range(5):
            x = int(rng.integers(0, g.n_u + g.n_v))
            s2 = s.copy()
            if x < g.n_u:
                s2[u == x] *= -1
            else:
                s2[v == x - g.n_u] *= -1
            g2 = _with_signs(g, s2)
            assert oracle.count(g2) == t
            assert np.array_equal(oracle.per_vertex(g2), pv)
        # switching a random vertex subset on both sides at once
        fu = rng.choice([-1, 1], g.n_u)
        fv = rng.choice([-1, 1], g.n_v)
        assert oracle.count(_with_signs(g, s * fu[u] * fv[v])) == t


def test_side_and_relabelling_invariance():
    rng = np.random.default_rng(23)
    for g in _mid_graphs():
        t = oracle.count(g)
        assert oracle.count(g, oracle.SIDE_U) == t == oracle.count(g, oracle.SIDE_V)
        u, v, s = g.edges()
        pu = rng.permutation(g.n_u)
        pv = rng.permutation(g.n_v)
        g2 = synth.from_edges(g.n_u, g.n_v, pu[u], pv[v], s)
        assert oracle.count(g2) == t
        assert oracle.count(synth.shuffle_rows(g, rng)) == t
        # swapping the roles of U and V
        assert oracle.count(synth.from_edges(g.n_v, g.n_u, v, u, s)) == t


def test_disjoint_union_is_additive():
    gs = _mid_graphs()
    a, b = gs[0], gs[2]
    ua, va, sa = a.edges()
    ub, vb, sb = b.edges()
    g = synth.from_edges(a.n_u + b.n_u, a.n_v + b.n_v, np.concatenate([ua, ub + a.n_u]),
                         np.concatenate([va, vb + a.n_v]), np.concatenate([sa, sb]))
    assert oracle.count(g) == oracle.count(a) + oracle.count(b)


def test_pendant_and_isolated_vertices_add_nothing():
    g = _mid_graphs()[1]
    t = oracle.count(g)
    u, v, s = g.edges()
    # one isolated vertex per side, one degree-1 vertex per side
    u2 = np.concatenate([u, [g.n_u + 1], [0]])
    v2 = np.concatenate([v, [0], [g.n_v + 1]])
    s2 = np.concatenate([s, [-1], [1]])
    assert oracle.count(synth.from_edges(g.n_u + 2, g.n_v + 2, u2, v2, s2)) == t


def test_per_vertex_definition_and_sums():
    rng = np.random.default_rng(24)
    for _ in range(300):
        g = synth.small_random_graph(rng, max_n=9)
        b, _, pv = oracle.brute(g, per_vertex=True)
        for side in (oracle.SIDE_AUTO, oracle.SIDE_U, oracle.SIDE_V):
            assert np.array_equal(oracle.per_vertex(g, side), pv)
    for g in _mid_graphs():
        t = oracle.count(g)
        pv = oracle.per_vertex(g)
        assert int(pv[: g.n_u].sum()) == 2 * t == int(pv[g.n_u:].sum())
        xs = rng.choice(g.n_u + g.n_v, 12, replace=False)
        for x in xs:
            assert oracle.vertex(g, int(x)) == int(pv[x])
        assert np.array_equal(oracle.vertices(g, xs), pv[xs])
        assert np.array_equal(oracle.per_vertex(g, oracle.SIDE_U), oracle.per_vertex(g, oracle.SIDE_V))


def test_anchor_ranges_partition_the_count():
    for g in _mid_graphs():
        t = oracle.count(g)
        n_s = g.n_u if g.n_u < g.n_v else g.n_v
        cuts = [0, n_s // 3, n_s // 2, n_s]
        parts = [oracle.count_anchors(g, a, b) for a, b in zip(cuts, cuts[1:])]
        assert sum(p for p, _ in parts) == t
        # wedges bucketed over all anchors = sum over centres of C(d, 2)
        deg_c = np.diff(g.offsets) if n_s == g.n_v else np.bincount(g.adj, minlength=g.n_v)
        assert sum(w for _, w in parts) == int((deg_c.astype(np.int64) * (deg_c - 1) // 2).sum())


def _signed_matrix(g):
    A = np.zeros((g.n_u, g.n_v), np.int64)
    u, v, s = g.edges()
    A[u, v] = s
    return A


def _pair_terms(a, b):
    """sum over unordered anchor pairs of C(a,2) + C(b,2) (upper triangle)."""
    iu = np.triu_indices(a.shape[0], 1)
    a, b = a[iu], b[iu]
    return int((a * (a - 1) // 2 + b * (b - 1) // 2).sum())


def test_lemma1_matrix_form():
    """Lemma 1 as matrix products: with S the signed adjacency seen from the
    anchor side, S S^T = a - b and |S| |S|^T = a + b for every anchor pair;
    the pair terms sum to the oracle's count, on either side."""
    rng = np.random.default_rng(31)
    for _ in range(40):
        g = synth.random_graph(rng, int(rng.integers(2, 30)), int(rng.integers(2, 30)), 0.5, 0.4)
        A = _signed_matrix(g)
        for M in (A.T, A):  # anchors on V, then on U
            D, P = M @ M.T, np.abs(M) @ np.abs(M).T
            assert np.all((P + D) % 2 == 0)
            assert _pair_terms((P + D) // 2, (P - D) // 2) == oracle.count(g)


def test_dense_block_split_identity():
    """The split the dense-block path relies on: with the edges between a
    block's anchors R and centres C called dense, a wedge is dense when both
    its edges are; a_D (from the dense part's matrix products) vanishes unless
    both anchors lie in the same block (blocks disjoint on both sides), and
    C(a,2) = C(a_D,2) + C(a_S,2) + a_D a_S with a_S = a - a_D.  Summed, the
    three parts give the oracle's count; leaving out the cross term does not."""
    rng = np.random.default_rng(32)
    for trial in range(30):
        n_u, n_v = int(rng.integers(20, 60)), int(rng.integers(15, 50))
        g = synth.random_graph(rng, n_u, n_v, float(rng.uniform(0.2, 0.7)), 0.35)
        A = _signed_matrix(g).T  # anchors on V
        pu, pv = rng.permutation(n_u), rng.permutation(n_v)
        mask = np.zeros_like(A)
        blocks, ou, ov = [], 0, 0
        for _ in range(int(rng.integers(1, 4))):
            nr, nc = int(rng.integers(1, n_v // 3 + 1)), int(rng.integers(1, n_u // 3 + 1))
            R, C = pv[ov:ov + nr], pu[ou:ou + nc]
            ov, ou = ov + nr, ou + nc
            mask[np.ix_(R, C)] = 1
            blocks.append(R)
        Dm = A * mask
        aD, bD = (np.abs(Dm) @ np.abs(Dm).T + Dm @ Dm.T) // 2, (np.abs(Dm) @ np.abs(Dm).T - Dm @ Dm.T) // 2
        a, b = (np.abs(A) @ np.abs(A).T + A @ A.T) // 2, (np.abs(A) @ np.abs(A).T - A @ A.T) // 2
        # every other wedge (both edges outside the blocks, or one edge in) is sparse
        aS, bS = a - aD, b - bD
        assert aS.min() >= 0 and bS.min() >= 0
        same = np.zeros((n_v, n_v), bool)
        for R in blocks:
            same[np.ix_(R, R)] = True
        assert not np.any((aD + bD)[~same & ~np.eye(n_v, dtype=bool)])
        iu = np.triu_indices(n_v, 1)
        cross = int((aD * aS + bD * bS)[iu].sum())
        want = oracle.count(g)
        assert _pair_terms(aD, bD) + _pair_terms(aS, bS) + cross == want
        if cross:
            assert _pair_terms(aD, bD) + _pair_terms(aS, bS) != want


def test_malformed_input_rejected():
    g = synth.complete_graph(3, 3)
    bad = synth.Graph(3, 3, g.offsets, g.adj.copy(), g.signs, {})
    bad.adj[0] = 7
    with pytest.raises(ValueError):
        oracle.count(bad)
    bad = synth.Graph(3, 3, g.offsets, g.adj, g.signs.copy(), {})
    bad.signs[0] = 0
    with pytest.raises(ValueError):
        oracle.count(bad)


# ------------------------------------------------------- planted oracle mistakes

MUTANTS = {
    "pair filter admits w == u": ("if (w <= u) continue; /* each endpoint pair once */",
                                  "if (w < u) continue; /* each endpoint pair once */"),
    "no pair filter": ("if (w <= u) continue; /* each endpoint pair once */", ""),
    "asymmetric term dropped": ("total += choose2(B1[w]) + choose2(B2[w]);", "total += choose2(B1[w]);"),
    "C(x,2) off by one": ("return x * (x - 1) / 2;", "return x * (x + 1) / 2;"),
    "sign of centre edge ignored": ("if (g->c_sgn[j] == s1) B1[w]++;", "if (s1 > 0) B1[w]++;"),
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_oracle_mistakes(name, tmp_path):
    """Each plausible slip in the bucket method makes a pin fail."""
    import ctypes

    src = open(os.path.join(os.path.dirname(oracle.__file__), "bbc_oracle.c")).read()
    old, new = MUTANTS[name]
    assert old in src
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-o", str(so), str(mut)])
    lib = ctypes.CDLL(str(so))
    P32, P8 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8)
    lib.oracle_count.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P32, P32, P8,
                                 ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]

    def mcount(g):
        off = np.ascontiguousarray(g.offsets, np.int32)
        adj = np.ascontiguousarray(g.adj, np.int32)
        sg = np.ascontiguousarray(g.signs, np.int8)
        out = ctypes.c_uint64()
        lib.oracle_count(g.n_u, g.n_v, adj.size, off.ctypes.data_as(P32), adj.ctypes.data_as(P32),
                         sg.ctypes.data_as(P8), 0, ctypes.byref(out))
        return int(out.value)

    failures = 0
    for g, exp in FIXTURES.values():
        failures += mcount(g) != exp["balanced"]
    rng = np.random.default_rng(31)
    for _ in range(50):
        g = synth.small_random_graph(rng, max_n=8)
        failures += mcount(g) != py_brute(g)[0]
    assert failures > 0, f"mutant '{name}' passed every pin"


CLASS_MUTANTS = {
    "patterns p and n swapped": ("else if (g.s_sgn[i] > 0) P[w]++;", "else if (g.s_sgn[i] < 0) P[w]++;"),
    "mixed ++/+- dropped": ("            c[4] += p * b;\n", ""),
    "incoherent as a product": ("            c[3] += choose2(b);", "            c[3] += b * b;"),
    "pair filter dropped": ("                if (w <= u) continue;\n                if (P[w] == 0", "                if (w == u) continue;\n                if (P[w] == 0"),
}


@pytest.mark.parametrize("name", sorted(CLASS_MUTANTS))
def test_class_pins_catch_planted_mistakes(name, tmp_path):
    """Each plausible slip in the three-bucket class walk makes a pin fail."""
    import ctypes

    src = open(os.path.join(os.path.dirname(oracle.__file__), "bbc_oracle.c")).read()
    old, new = CLASS_MUTANTS[name]
    assert src.count(old) >= 1
    i = src.index("int oracle_count_classes(")
    j = src.index("int oracle_brute_classes(")
    body = src[i:j]
    assert old in body
    mut = tmp_path / "mut.c"
    mut.write_text(src[:i] + body.replace(old, new) + src[j:])
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-o", str(so), str(mut)])
    lib = ctypes.CDLL(str(so))
    P32, P8 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8)
    lib.oracle_count_classes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P32, P32, P8,
                                         ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]

    def mclasses(g, side):
        off = np.ascontiguousarray(g.offsets, np.int32)
        adj = np.ascontiguousarray(g.adj, np.int32)
        sg = np.ascontiguousarray(g.signs, np.int8)
        out = (ctypes.c_uint64 * 6)()
        lib.oracle_count_classes(g.n_u, g.n_v, adj.size, off.ctypes.data_as(P32), adj.ctypes.data_as(P32),
                                 sg.ctypes.data_as(P8), side, out)
        return [int(x) for x in out]

    g, exp = load_graphs("drug_target_sample.txt")["drug_target"]
    failures = int(mclasses(g, oracle.SIDE_U) != [exp["class_" + n] for n in oracle.CLASS_NAMES])
    rng = np.random.default_rng(32)
    for _ in range(40):
        g = synth.small_random_graph(rng, max_n=7)
        failures += mclasses(g, oracle.SIDE_U) != py_classes(g, oracle.SIDE_U)
    assert failures > 0, f"mutant '{name}' passed every pin"


# --------------------------------------------- balanced (2,k)-bicliques

def py_bicliques(g, k, side):
    """Definition 5 by enumeration (pure Python, tiny graphs): pairs of the
    side, k-subsets of their common neighbours with every butterfly inside
    balanced (an even number of negative edges)."""
    import itertools

    su = side != oracle.SIDE_V  # the size-two side is U unless V is named (BB2K)
    nbr = {}
    for u in range(g.n_u):
        for e in range(g.offsets[u], g.offsets[u + 1]):
            a, c = (u, int(g.adj[e])) if su else (int(g.adj[e]), u)
            nbr.setdefault(a, {})[c] = int(g.signs[e])
    keys = sorted(nbr)
    n = 0
    for i, a1 in enumerate(keys):
        for a2 in keys[i + 1:]:
            common = sorted(set(nbr[a1]) & set(nbr[a2]))
            for sub in itertools.combinations(common, k):
                n += all(nbr[a1][c1] * nbr[a2][c1] * nbr[a1][c2] * nbr[a2][c2] > 0
                         for c1, c2 in itertools.combinations(sub, 2))
    return n


def test_bicliques_walk_matches_definition():
    """Algorithm 1 with general k against the definition, enumerated in C
    and in Python, k = 1..5, both sides."""
    rng = np.random.default_rng(41)
    for t in range(150):
        g = synth.small_random_graph(rng, max_n=8)
        for side in (oracle.SIDE_U, oracle.SIDE_V):
            for k in (1, 2, 3, 4, 5):
                want = oracle.brute_bicliques(g, k, side)
                assert oracle.count_bicliques(g, k, side) == want
                if t < 40:
                    assert py_bicliques(g, k, side) == want


def test_bicliques_auto_side_is_u():
    """The BB2K section fixes U as the size-two side: the automatic choice
    pairs U vertices even when U is the larger side.  On K_{2,5} (U smaller)
    and K_{5,2} (U larger) the (2,3) count is C(|U|,2) C(|V|,3) (pairs on U),
    never C(|V|,2) C(|U|,3)."""
    from math import comb

    for m, n in ((2, 5), (5, 2), (4, 6), (6, 4)):
        g = synth.complete_graph(m, n)
        want = comb(m, 2) * comb(n, 3)
        assert oracle.count_bicliques(g, 3, oracle.SIDE_AUTO) == want
        assert oracle.count_bicliques(g, 3, oracle.SIDE_U) == want
        assert oracle.brute_bicliques(g, 3, oracle.SIDE_AUTO) == want
        assert py_bicliques(g, 3, oracle.SIDE_AUTO) == want
        assert oracle.count_bicliques(g, 3, oracle.SIDE_V) == comb(n, 2) * comb(m, 3)


def test_bicliques_special_cases():
    """k = 2 is the balanced butterfly count (either side); k = 1 counts the
    wedges with both ends on the side, sum of C(deg, 2) over the other side;
    k above every degree gives 0."""
    rng = np.random.default_rng(42)
    for _ in range(40):
        g = synth.random_graph(rng, int(rng.integers(2, 30)), int(rng.integers(2, 30)), 0.4, 0.4)
        t = oracle.count(g)
        du = np.diff(g.offsets).astype(np.int64)
        dv = np.bincount(g.adj, minlength=g.n_v).astype(np.int64)
        for side, dc in ((oracle.SIDE_U, dv), (oracle.SIDE_V, du)):
            assert oracle.count_bicliques(g, 2, side) == t
            assert oracle.count_bicliques(g, 1, side) == int((dc * (dc - 1) // 2).sum())
            dmax = int(max(du.max(initial=0), dv.max(initial=0)))
            assert oracle.count_bicliques(g, dmax + 1, side) == 0


@pytest.mark.parametrize("m,n", [(2, 3), (3, 5), (5, 7), (4, 12)])
def test_bicliques_closed_forms(m, n):
    """K_{m,n}: all positive, C(m,2) C(n,k) with pairs on U; one negative
    edge (u0, v0): pairs with u0 have n-1 symmetric and 1 asymmetric wedge,
    (m-1) (C(n-1,k) + C(1,k)) + C(m-1,2) C(n,k); pairs on V swap m and n."""
    from math import comb

    for k in range(1, n + 2):
        g = synth.complete_graph(m, n)
        assert oracle.count_bicliques(g, k, oracle.SIDE_U) == comb(m, 2) * comb(n, k)
        assert oracle.count_bicliques(g, k, oracle.SIDE_V) == comb(n, 2) * comb(m, k)
        s = np.ones(m * n, np.int8)
        s[0] = -1  # edge (u0, v0): CSR row 0, first entry
        g1 = synth.complete_graph(m, n, signs=s)
        assert int(g1.adj[0]) == 0
        assert oracle.count_bicliques(g1, k, oracle.SIDE_U) == \
            (m - 1) * (comb(n - 1, k) + comb(1, k)) + comb(m - 1, 2) * comb(n, k)
        assert oracle.count_bicliques(g1, k, oracle.SIDE_V) == \
            (n - 1) * (comb(m - 1, k) + comb(1, k)) + comb(n - 1, 2) * comb(m, k)


def test_bicliques_128_bit_range():
    """One pair sharing n centres: C(n,k) exactly past 64 bits, and an
    error once the count leaves 128 bits."""
    from math import comb

    for n, k in ((1000, 9), (1000, 16), (3000, 12)):
        g = synth.complete_graph(2, n)
        want = comb(n, k)
        assert want >= 1 << 64
        assert oracle.count_bicliques(g, k, oracle.SIDE_U) == want
    g = synth.complete_graph(2, 20000)
    assert comb(20000, 16) >= 1 << 128
    with pytest.raises(OverflowError):
        oracle.count_bicliques(g, 16, oracle.SIDE_U)


BICLIQUE_MUTANTS = {
    "buckets merged": ("const u128 x = tab[(size_t)B1[w] * (k + 1) + k], y = tab[(size_t)B2[w] * (k + 1) + k];",
                       "const u128 x = tab[(size_t)(B1[w] + B2[w]) * (k + 1) + k], y = 0;"),
    "k ignored (k = 2)": ("const u128 x = tab[(size_t)B1[w] * (k + 1) + k], y = tab[(size_t)B2[w] * (k + 1) + k];",
                          "const u128 x = tab[(size_t)B1[w] * (k + 1) + 2], y = tab[(size_t)B2[w] * (k + 1) + 2];"),
    "Pascal rule off by one": ("const u128 p = tab[(size_t)(x - 1) * w + j - 1], q = tab[(size_t)(x - 1) * w + j];",
                               "const u128 p = tab[(size_t)(x - 1) * w + j - 1], q = tab[(size_t)(x - 1) * w + j - 1];"),
    "pair filter dropped": ("                if (w <= u) continue;\n                if (B1[w] == 0 && B2[w] == 0)",
                            "                if (w == u) continue;\n                if (B1[w] == 0 && B2[w] == 0)"),
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name", sorted(BICLIQUE_MUTANTS))
def test_biclique_pins_catch_planted_mistakes(name, tmp_path):
    """Each plausible slip in the general-k walk makes a pin fail."""
    import ctypes

    src = open(os.path.join(os.path.dirname(oracle.__file__), "bbc_oracle.c")).read()
    old, new = BICLIQUE_MUTANTS[name]
    i = src.index("static int pascal_table(")
    j = src.index("int oracle_brute_bicliques(")
    body = src[i:j]
    assert body.count(old) == 1
    mut = tmp_path / "mut.c"
    mut.write_text(src[:i] + body.replace(old, new) + src[j:])
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-o", str(so), str(mut)])
    lib = ctypes.CDLL(str(so))
    P32, P8 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8)
    lib.oracle_count_bicliques.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P32, P32, P8,
                                           ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]

    def mcount(g, k, side):
        off = np.ascontiguousarray(g.offsets, np.int32)
        adj = np.ascontiguousarray(g.adj, np.int32)
        sg = np.ascontiguousarray(g.signs, np.int8)
        out = (ctypes.c_uint64 * 2)()
        lib.oracle_count_bicliques(g.n_u, g.n_v, adj.size, off.ctypes.data_as(P32), adj.ctypes.data_as(P32),
                                   sg.ctypes.data_as(P8), side, k, out)
        return int(out[0]) | (int(out[1]) << 64)

    failures = 0
    rng = np.random.default_rng(43)
    for _ in range(30):
        g = synth.small_random_graph(rng, max_n=7)
        for k in (1, 3):
            failures += mcount(g, k, oracle.SIDE_U) != py_bicliques(g, k, oracle.SIDE_U)
    assert failures > 0, f"mutant '{name}' passed every pin"


# ------------------------------------------------------------ dynamic updates

@pytest.mark.parametrize("m,n", [(2, 2), (3, 4), (5, 7)])
def test_update_delta_closed_forms(m, n):
    """K_{m,n}, all positive: re-signing or removing one edge unbalances or
    removes its (m-1)(n-1) butterflies; adding it back with + restores them
    and with - adds only unbalanced ones; re-signing two edges of one U
    vertex keeps the (m-1) butterflies holding both balanced."""
    g = synth.complete_graph(m, n)
    k = (m - 1) * (n - 1)
    assert oracle.update_delta(g, [0], [0], [-1]) == -k
    assert oracle.update_delta(g, [0], [0], [0]) == -k
    assert oracle.update_delta(g, [0], [0], [1]) == 0  # same sign: nothing changes
    h = oracle.apply_updates(g, [0], [0], [0])
    assert oracle.count(h) == comb2(m) * comb2(n) - k
    assert oracle.update_delta(h, [0], [0], [1]) == k
    assert oracle.update_delta(h, [0], [0], [-1]) == 0
    assert oracle.update_delta(h, [0], [0], [0]) == 0  # removing an absent pair
    if n >= 2:
        assert oracle.update_delta(g, [0, 0], [0, 1], [-1, -1]) == -2 * (m - 1) * (n - 2)


def comb2(x):
    return x * (x - 1) // 2


def test_update_batch_equals_sequence():
    """A batch equals its updates applied one after another, in any order,
    including updates that share butterflies."""
    rng = np.random.default_rng(51)
    for _ in range(40):
        g = synth.random_graph(rng, int(rng.integers(3, 12)), int(rng.integers(3, 12)), 0.5, 0.4)
        q = int(rng.integers(1, 8))
        pairs = rng.choice(g.n_u * g.n_v, size=min(q, g.n_u * g.n_v), replace=False)
        uu, vv = pairs // g.n_v, pairs % g.n_v
        ss = rng.choice([-1, 0, 1], size=uu.size)
        batch = oracle.update_delta(g, uu, vv, ss)
        for order in (np.arange(uu.size), rng.permutation(uu.size)):
            h, total = g, 0
            for i in order:
                total += oracle.update_delta(h, uu[i:i + 1], vv[i:i + 1], ss[i:i + 1])
                h = oracle.apply_updates(h, uu[i:i + 1], vv[i:i + 1], ss[i:i + 1])
            assert total == batch
        assert oracle.count(oracle.apply_updates(g, uu, vv, ss)) == py_brute(oracle.apply_updates(g, uu, vv, ss))[0]
    with pytest.raises(ValueError):
        oracle.apply_updates(synth.complete_graph(2, 2), [0, 0], [1, 1], [1, -1])


# ------------------------------------------- per-vertex sign-pattern classes

def py_per_vertex_classes(g, side):
    """Definition-level per-vertex classes (pure Python, tiny graphs): every
    butterfly, classified by the patterns at its two centres, adds one to
    its class at each of its four vertices (U first, then V)."""
    import itertools

    su = oracle.SIDE_U == side or (side == oracle.SIDE_AUTO and g.n_u < g.n_v)
    sign = {}
    for u in range(g.n_u):
        for e in range(g.offsets[u], g.offsets[u + 1]):
            sign[(u, int(g.adj[e]))] = int(g.signs[e])
    n_s, n_c = (g.n_u, g.n_v) if su else (g.n_v, g.n_u)
    key = (lambda a, c: (a, c)) if su else (lambda a, c: (c, a))
    gid_a = (lambda a: a) if su else (lambda a: g.n_u + a)
    gid_c = (lambda c: g.n_u + c) if su else (lambda c: c)
    order = {("pp", "pp"): 0, ("mm", "pp"): 1, ("mm", "mm"): 2, ("pm", "pm"): 3, ("pm", "pp"): 4, ("mm", "pm"): 5}
    out = np.zeros((g.n_u + g.n_v, 6), np.uint64)
    for a1, a2 in itertools.combinations(range(n_s), 2):
        for c1, c2 in itertools.combinations(range(n_c), 2):
            s = [sign.get(key(a, c)) for a in (a1, a2) for c in (c1, c2)]
            if None in s:
                continue
            x1, x2, y1, y2 = s
            pat = sorted("pm" if x != y else ("pp" if x > 0 else "mm") for x, y in ((x1, y1), (x2, y2)))
            k = order[tuple(pat)]
            for x in (gid_a(a1), gid_a(a2), gid_c(c1), gid_c(c2)):
                out[x, k] += 1
    return out


def test_per_vertex_classes_match_definitions():
    """The walk equals the brute force and a pure-Python enumeration."""
    rng = np.random.default_rng(41)
    for i in range(60):
        g = synth.small_random_graph(rng, max_n=8)
        for side in (oracle.SIDE_AUTO, oracle.SIDE_U, oracle.SIDE_V):
            got = oracle.per_vertex_classes(g, side)
            np.testing.assert_array_equal(got, oracle.brute_per_vertex_classes(g, side))
            if i < 25:
                np.testing.assert_array_equal(got, py_per_vertex_classes(g, side))


def test_per_vertex_classes_sums():
    """Each butterfly holds two vertices of each side: per class the U
    column and the V column sum to twice the class total; the four balanced
    classes add up to the balanced per-vertex count."""
    for g in _mid_graphs():
        for side in (oracle.SIDE_U, oracle.SIDE_V):
            pv = oracle.per_vertex_classes(g, side).astype(np.int64)
            tot = oracle.count_classes(g, side)
            assert list(pv[: g.n_u].sum(axis=0)) == [2 * t for t in tot]
            assert list(pv[g.n_u:].sum(axis=0)) == [2 * t for t in tot]
            np.testing.assert_array_equal(pv[:, :4].sum(axis=1), oracle.per_vertex(g, side).astype(np.int64))


@pytest.mark.parametrize("s,c", [(2, 3), (4, 5)])
def test_per_vertex_classes_closed_forms(s, c):
    """K_{s,c} all positive: every butterfly is ++/++; a U vertex lies in
    (s - 1) C(c,2) of them, a V vertex in (c - 1) C(s,2).  All negative with
    the pair on U: the same counts as --/--."""
    u, v = np.divmod(np.arange(s * c), c)
    for sg, k in ((np.ones(s * c, np.int8), 0), (-np.ones(s * c, np.int8), 2)):
        g = synth.from_edges(s, c, u, v, sg)
        pv = oracle.per_vertex_classes(g, oracle.SIDE_U)
        want = np.zeros((s + c, 6), np.uint64)
        want[:s, k] = (s - 1) * comb(c, 2)
        want[s:, k] = (c - 1) * comb(s, 2)
        np.testing.assert_array_equal(pv, want)


PV_CLASS_MUTANTS = {
    "++ centre counts itself": ("                    x[0] += p - 1;", "                    x[0] += p;"),
    "+- centre loses the ++ partners": ("                    x[3] += b - 1;\n                    x[4] += p;",
                                        "                    x[3] += b - 1;\n                    x[4] += n;"),
    "anchor w gets nothing": ("                cs[6 * (size_t)w + q] += t[q];\n", ""),
    "-- centre: mixed class swapped": ("                    x[2] += n - 1;\n                    x[5] += b;",
                                       "                    x[2] += n - 1;\n                    x[4] += b;"),
}


@pytest.mark.parametrize("name", sorted(PV_CLASS_MUTANTS))
def test_per_vertex_class_pins_catch_planted_mistakes(name, tmp_path):
    """Each plausible slip in the per-vertex class walk makes a pin fail."""
    import ctypes

    src = open(os.path.join(os.path.dirname(oracle.__file__), "bbc_oracle.c")).read()
    old, new = PV_CLASS_MUTANTS[name]
    i = src.index("int oracle_per_vertex_classes(")
    j = src.index("int oracle_brute_per_vertex_classes(")
    body = src[i:j]
    assert old in body
    mut = tmp_path / "mut.c"
    mut.write_text(src[:i] + body.replace(old, new) + src[j:])
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O1", "-shared", "-fPIC", "-o", str(so), str(mut)])
    lib = ctypes.CDLL(str(so))
    P32, P8 = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8)
    lib.oracle_per_vertex_classes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, P32, P32, P8,
                                              ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]

    def mpv(g, side):
        off = np.ascontiguousarray(g.offsets, np.int32)
        adj = np.ascontiguousarray(g.adj, np.int32)
        sg = np.ascontiguousarray(g.signs, np.int8)
        out = np.zeros((g.n_u + g.n_v, 6), np.uint64)
        lib.oracle_per_vertex_classes(g.n_u, g.n_v, adj.size, off.ctypes.data_as(P32), adj.ctypes.data_as(P32),
                                      sg.ctypes.data_as(P8), side, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
        return out

    rng = np.random.default_rng(43)
    failures = 0
    for _ in range(40):
        g = synth.small_random_graph(rng, max_n=7)
        failures += not np.array_equal(mpv(g, oracle.SIDE_U), py_per_vertex_classes(g, oracle.SIDE_U))
    assert failures > 0, f"mutant '{name}' passed every pin"
