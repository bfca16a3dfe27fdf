/* Balanced butterfly counting: serial CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU library is checked against.  Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark load it; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * What is computed (paper, Sec. "Preliminaries and Problem Definition"):
 *   - a butterfly is a 4-cycle u_i v_i u_j v_j with all four U x V edges
 *     present (Definition 1);
 *   - it is balanced when it holds an even number of negative edges
 *     (Definition 2);
 *   - the problem is the number of balanced butterflies (Problem Statement).
 *
 * Two independent computations of that number live here:
 *   oracle_brute   - enumerates every pair {u1,u2} x {v1,v2} and tests the
 *                    definition directly (tiny graphs only);
 *   oracle_count   - the bucket method of Algorithm 1 (BB2K) with k = 2: for
 *                    each anchor u, count symmetric wedges (both edges of one
 *                    sign, Definition 8) and asymmetric wedges (Definition 9)
 *                    per endpoint w, then add C(B1[w],2) + C(B2[w],2).  By
 *                    Lemma 1 a balanced butterfly is two symmetric or two
 *                    asymmetric wedges on the same endpoint pair, never a
 *                    mix.  The pair filter uses plain vertex ids (w > u):
 *                    any strict order counts each pair once, and the
 *                    algorithms of the paper use several (priority in
 *                    Algorithms 1 and 2, ids in Algorithms 3 and 4).
 *
 * Anchor side: the paper starts from the smaller side (Algorithm 2: S = V,
 * replaced by U when |V| > |U|); the count does not depend on the side
 * (Sec. "BB2K Algorithm", symmetry of the (2,2) case).  `side` selects
 * 0 = that rule, 1 = U, 2 = V.
 *
 * Per-vertex counts (the paper counts totals only; this is the reading used
 * for the optional per-vertex output): cnt[x] is the number of balanced
 * butterflies that contain x, for x in U (indices 0..n_u-1) then V
 * (n_u..n_u+n_v-1).
 *
 * Integer widths: a, b <= min(deg) < 2^31; every sum is uint64, which holds
 * any count for n_edges < 2^31 (a graph has at most m^2/4 butterflies).
 *
 * Input: CSR over U - offsets[n_u+1], adj[m] (V ids), signs[m] (+1 / -1).
 * The graph must be simple.  Functions return 0, or 1 for malformed input.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int check_csr(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                     const int8_t* sg) {
    if (n_u < 0 || n_v < 0 || m < 0) return 1;
    if (off[0] != 0 || off[n_u] != m) return 1;
    for (int32_t u = 0; u < n_u; ++u)
        if (off[u + 1] < off[u]) return 1;
    for (int64_t e = 0; e < m; ++e) {
        if (adj[e] < 0 || adj[e] >= n_v) return 1;
        if (sg[e] != 1 && sg[e] != -1) return 1;
    }
    return 0;
}

/* Adjacency of the chosen anchor side S and of the centre side C, both as
 * CSR with a sign per entry.  Built by a counting sort (the transpose). */
typedef struct {
    int32_t n_s, n_c;
    int64_t* s_off; /* n_s + 1 */
    int32_t* s_nbr; /* centres of each anchor */
    int8_t* s_sgn;
    int64_t* c_off; /* n_c + 1 */
    int32_t* c_nbr; /* anchors of each centre */
    int8_t* c_sgn;
} sides_t;

static void sides_free(sides_t* g) {
    free(g->s_off);
    free(g->s_nbr);
    free(g->s_sgn);
    free(g->c_off);
    free(g->c_nbr);
    free(g->c_sgn);
}

/* transpose of a CSR (rows n_r, columns n_col) by counting sort */
static void transpose(int32_t n_r, int32_t n_col, int64_t m, const int64_t* off, const int32_t* nbr,
                      const int8_t* sg, int64_t** t_off, int32_t** t_nbr, int8_t** t_sgn) {
    int64_t* to = (int64_t*)calloc((size_t)n_col + 1, sizeof(int64_t));
    int32_t* tn = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int8_t* ts = (int8_t*)malloc((size_t)(m > 0 ? m : 1));
    for (int64_t e = 0; e < m; ++e) to[nbr[e] + 1]++;
    for (int32_t c = 0; c < n_col; ++c) to[c + 1] += to[c];
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n_col > 0 ? n_col : 1));
    for (int32_t c = 0; c < n_col; ++c) fill[c] = to[c];
    for (int32_t r = 0; r < n_r; ++r)
        for (int64_t e = off[r]; e < off[r + 1]; ++e) {
            int64_t q = fill[nbr[e]]++;
            tn[q] = r;
            ts[q] = sg[e];
        }
    free(fill);
    *t_off = to;
    *t_nbr = tn;
    *t_sgn = ts;
}

static int pick_side(int32_t n_u, int32_t n_v, int side) {
    if (side == 1) return 1;
    if (side == 2) return 2;
    return n_u < n_v ? 1 : 2; /* the smaller side; a tie keeps V */
}

static void build_sides(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                        const int8_t* sg, int side, sides_t* g) {
    int64_t* uoff = (int64_t*)malloc(sizeof(int64_t) * ((size_t)n_u + 1));
    for (int32_t u = 0; u <= n_u; ++u) uoff[u] = off[u];
    int32_t* unbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int8_t* usg = (int8_t*)malloc((size_t)(m > 0 ? m : 1));
    memcpy(unbr, adj, sizeof(int32_t) * (size_t)m);
    memcpy(usg, sg, (size_t)m);
    int64_t* voff;
    int32_t* vnbr;
    int8_t* vsg;
    transpose(n_u, n_v, m, uoff, unbr, usg, &voff, &vnbr, &vsg);
    if (pick_side(n_u, n_v, side) == 1) {
        g->n_s = n_u;
        g->n_c = n_v;
        g->s_off = uoff;
        g->s_nbr = unbr;
        g->s_sgn = usg;
        g->c_off = voff;
        g->c_nbr = vnbr;
        g->c_sgn = vsg;
    } else {
        g->n_s = n_v;
        g->n_c = n_u;
        g->s_off = voff;
        g->s_nbr = vnbr;
        g->s_sgn = vsg;
        g->c_off = uoff;
        g->c_nbr = unbr;
        g->c_sgn = usg;
    }
}

/* C(x, 2); x < 2^32 so the product fits in 64 bits, and x = 0 gives 0 */
static inline uint64_t choose2(uint64_t x) { return x * (x - 1) / 2; }

/* Algorithm 1 (BB2K), k = 2, over the anchors a_lo <= u < a_hi.  B1 / B2 are
 * dense arrays over the anchor side with a list of touched endpoints,
 * cleared after each anchor.  *wedges receives the number of wedges u - c - w
 * with w > u that were bucketed. */
static uint64_t bb2k_range(const sides_t* g, int32_t a_lo, int32_t a_hi, uint64_t* wedges) {
    uint32_t* B1 = (uint32_t*)calloc((size_t)g->n_s + 1, sizeof(uint32_t));
    uint32_t* B2 = (uint32_t*)calloc((size_t)g->n_s + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)g->n_s + 1));
    uint64_t total = 0, nw = 0;
    for (int32_t u = a_lo; u < a_hi; ++u) {
        int32_t nt = 0;
        for (int64_t i = g->s_off[u]; i < g->s_off[u + 1]; ++i) {
            int32_t c = g->s_nbr[i];
            int8_t s1 = g->s_sgn[i];
            for (int64_t j = g->c_off[c]; j < g->c_off[c + 1]; ++j) {
                int32_t w = g->c_nbr[j];
                if (w <= u) continue; /* each endpoint pair once */
                ++nw;
                if (B1[w] == 0 && B2[w] == 0) touched[nt++] = w;
                if (g->c_sgn[j] == s1) B1[w]++; /* symmetric wedge */
                else B2[w]++;                   /* asymmetric wedge */
            }
        }
        for (int32_t k = 0; k < nt; ++k) {
            int32_t w = touched[k];
            total += choose2(B1[w]) + choose2(B2[w]);
            B1[w] = 0;
            B2[w] = 0;
        }
    }
    free(B1);
    free(B2);
    free(touched);
    *wedges = nw;
    return total;
}

int oracle_count(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                 const int8_t* sg, int side, uint64_t* out) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    sides_t g;
    build_sides(n_u, n_v, m, off, adj, sg, side, &g);
    uint64_t nw;
    *out = bb2k_range(&g, 0, g.n_s, &nw);
    sides_free(&g);
    return 0;
}

/* The same count restricted to anchors with id in [a_lo, a_hi) (a partial
 * sum; the ranges of a partition of the anchor side add up to the total).
 * Used to time the oracle on a bounded sample of a large graph. */
int oracle_count_anchors(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                         const int8_t* sg, int side, int32_t a_lo, int32_t a_hi, uint64_t* partial,
                         uint64_t* wedges) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    sides_t g;
    build_sides(n_u, n_v, m, off, adj, sg, side, &g);
    if (a_lo < 0) a_lo = 0;
    if (a_hi > g.n_s) a_hi = g.n_s;
    if (a_hi < a_lo) a_hi = a_lo;
    *partial = bb2k_range(&g, a_lo, a_hi, wedges);
    sides_free(&g);
    return 0;
}

/* Pair-level split used by the invariant checks: over every anchor pair,
 * balanced += C(a,2) + C(b,2), unbalanced += a*b (a mixed pair of wedges has
 * an odd number of negative edges, Lemma 1 case 3), and every butterfly is
 * counted once in butterflies += C(a+b,2). */
int oracle_count_kinds(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                       const int8_t* sg, int side, uint64_t* balanced, uint64_t* unbalanced,
                       uint64_t* butterflies) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    sides_t g;
    build_sides(n_u, n_v, m, off, adj, sg, side, &g);
    uint32_t* B1 = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    uint32_t* B2 = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)g.n_s + 1));
    uint64_t bal = 0, unb = 0, all = 0;
    for (int32_t u = 0; u < g.n_s; ++u) {
        int32_t nt = 0;
        for (int64_t i = g.s_off[u]; i < g.s_off[u + 1]; ++i) {
            int32_t c = g.s_nbr[i];
            for (int64_t j = g.c_off[c]; j < g.c_off[c + 1]; ++j) {
                int32_t w = g.c_nbr[j];
                if (w <= u) continue;
                if (B1[w] == 0 && B2[w] == 0) touched[nt++] = w;
                if (g.c_sgn[j] == g.s_sgn[i]) B1[w]++;
                else B2[w]++;
            }
        }
        for (int32_t k = 0; k < nt; ++k) {
            int32_t w = touched[k];
            uint64_t a = B1[w], b = B2[w];
            bal += choose2(a) + choose2(b);
            unb += a * b;
            all += choose2(a + b);
            B1[w] = 0;
            B2[w] = 0;
        }
    }
    free(B1);
    free(B2);
    free(touched);
    sides_free(&g);
    *balanced = bal;
    *unbalanced = unb;
    *butterflies = all;
    return 0;
}

/* Sign-pattern classes of the case study (Sec. "Case Study", Table 8):
 * for an anchor pair {u, w} every shared centre c carries a pattern, ++
 * (both edges positive, p of them), -- (both negative, n) or +- (the two
 * edges differ, b); a butterfly is a pair of shared centres, so its class is
 * the unordered pair of their patterns.  Per anchor pair:
 *   out[0] ++/++ C(p,2)   out[1] ++/-- p*n   out[2] --/-- C(n,2)
 *   out[3] +-/+- C(b,2)   out[4] ++/+- p*b   out[5] +-/-- n*b
 * summed over the pairs of the anchor side (the case study pairs the drugs).
 * Coherent (0-2) and incoherent (3) butterflies are balanced, mixed (4, 5)
 * unbalanced (Lemma 1).  Algorithm 1's walk with three buckets per
 * endpoint instead of two, pairs by plain id order. */
int oracle_count_classes(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                         const int8_t* sg, int side, uint64_t* out) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    sides_t g;
    build_sides(n_u, n_v, m, off, adj, sg, side, &g);
    uint32_t* P = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    uint32_t* N = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    uint32_t* B = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)g.n_s + 1));
    uint64_t c[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t u = 0; u < g.n_s; ++u) {
        int32_t nt = 0;
        for (int64_t i = g.s_off[u]; i < g.s_off[u + 1]; ++i) {
            int32_t ctr = g.s_nbr[i];
            for (int64_t j = g.c_off[ctr]; j < g.c_off[ctr + 1]; ++j) {
                int32_t w = g.c_nbr[j];
                if (w <= u) continue;
                if (P[w] == 0 && N[w] == 0 && B[w] == 0) touched[nt++] = w;
                if (g.c_sgn[j] != g.s_sgn[i]) B[w]++;
                else if (g.s_sgn[i] > 0) P[w]++;
                else N[w]++;
            }
        }
        for (int32_t k = 0; k < nt; ++k) {
            int32_t w = touched[k];
            uint64_t p = P[w], n = N[w], b = B[w];
            c[0] += choose2(p);
            c[1] += p * n;
            c[2] += choose2(n);
            c[3] += choose2(b);
            c[4] += p * b;
            c[5] += n * b;
            P[w] = N[w] = B[w] = 0;
        }
    }
    free(P);
    free(N);
    free(B);
    free(touched);
    sides_free(&g);
    for (int k = 0; k < 6; ++k) out[k] = c[k];
    return 0;
}

/* Per-vertex class counts (the case study's classes, Table 8, for every
 * vertex): cnt[6 x + k] is the number of class-k butterflies (order of
 * oracle_count_classes) that contain vertex x, U first, then V.  An anchor
 * pair {u, w} with p / n / b shared centres of pattern ++ / -- / +- closes
 * C(p,2), p n, C(n,2), C(b,2), p b and n b butterflies of the six classes,
 * each containing u and w.  A centre c of a wedge u-c-w lies in the
 * butterflies pairing that wedge with another shared centre c' of {u, w},
 * and the class is the pair of patterns (c, c'):
 *   c is ++: (p - 1) of class 0, n of class 1, b of class 4;
 *   c is --: p of class 1, (n - 1) of class 2, b of class 5;
 *   c is +-: (b - 1) of class 3, p of class 4, n of class 5.
 * Pairs by plain id order as in oracle_count_classes. */
int oracle_per_vertex_classes(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                              const int8_t* sg, int side, uint64_t* cnt) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    const int s_is_u = pick_side(n_u, n_v, side) == 1;
    sides_t g;
    build_sides(n_u, n_v, m, off, adj, sg, side, &g);
    uint64_t* cs = cnt + 6 * (size_t)(s_is_u ? 0 : n_u); /* anchor-side block */
    uint64_t* cc = cnt + 6 * (size_t)(s_is_u ? n_u : 0); /* centre-side block */
    memset(cnt, 0, sizeof(uint64_t) * 6 * ((size_t)n_u + (size_t)n_v));
    uint32_t* P = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    uint32_t* N = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    uint32_t* B = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)g.n_s + 1));
    for (int32_t u = 0; u < g.n_s; ++u) {
        int32_t nt = 0;
        for (int64_t i = g.s_off[u]; i < g.s_off[u + 1]; ++i) {
            const int32_t c = g.s_nbr[i];
            for (int64_t j = g.c_off[c]; j < g.c_off[c + 1]; ++j) {
                const int32_t w = g.c_nbr[j];
                if (w <= u) continue;
                if (P[w] == 0 && N[w] == 0 && B[w] == 0) touched[nt++] = w;
                if (g.c_sgn[j] != g.s_sgn[i]) B[w]++;
                else if (g.s_sgn[i] > 0) P[w]++;
                else N[w]++;
            }
        }
        /* second walk with the pair counts complete: the centres */
        for (int64_t i = g.s_off[u]; i < g.s_off[u + 1]; ++i) {
            const int32_t c = g.s_nbr[i];
            uint64_t* x = cc + 6 * (size_t)c;
            for (int64_t j = g.c_off[c]; j < g.c_off[c + 1]; ++j) {
                const int32_t w = g.c_nbr[j];
                if (w <= u) continue;
                const uint64_t p = P[w], n = N[w], b = B[w];
                if (g.c_sgn[j] != g.s_sgn[i]) { /* +- */
                    x[3] += b - 1;
                    x[4] += p;
                    x[5] += n;
                } else if (g.s_sgn[i] > 0) { /* ++ */
                    x[0] += p - 1;
                    x[1] += n;
                    x[4] += b;
                } else { /* -- */
                    x[1] += p;
                    x[2] += n - 1;
                    x[5] += b;
                }
            }
        }
        for (int32_t k = 0; k < nt; ++k) {
            const int32_t w = touched[k];
            const uint64_t p = P[w], n = N[w], b = B[w];
            const uint64_t t[6] = {choose2(p), p * n, choose2(n), choose2(b), p * b, n * b};
            for (int q = 0; q < 6; ++q) {
                cs[6 * (size_t)u + q] += t[q];
                cs[6 * (size_t)w + q] += t[q];
            }
            P[w] = N[w] = B[w] = 0;
        }
    }
    free(P);
    free(N);
    free(B);
    free(touched);
    sides_free(&g);
    return 0;
}

/* The same per-vertex classes by brute force over every 2 x 2 vertex
 * choice (tiny graphs): each butterfly adds one to its class at its four
 * vertices. */
int oracle_brute_per_vertex_classes(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                                    const int8_t* sg, int side, uint64_t* cnt) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    if ((int64_t)n_u * n_v > (1LL << 24)) return 1;
    const int su = pick_side(n_u, n_v, side) == 1;
    const int32_t n_s = su ? n_u : n_v, n_c = su ? n_v : n_u;
    int8_t* M = (int8_t*)calloc((size_t)n_s * (size_t)n_c + 1, 1); /* M[anchor][centre] */
    for (int32_t u = 0; u < n_u; ++u)
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            const int32_t a = su ? u : adj[e], c = su ? adj[e] : u;
            M[(size_t)a * n_c + c] = sg[e];
        }
    memset(cnt, 0, sizeof(uint64_t) * 6 * ((size_t)n_u + (size_t)n_v));
    const size_t abase = su ? 0 : (size_t)n_u, cbase = su ? (size_t)n_u : 0;
    for (int32_t a1 = 0; a1 < n_s; ++a1)
        for (int32_t a2 = a1 + 1; a2 < n_s; ++a2)
            for (int32_t c1 = 0; c1 < n_c; ++c1) {
                const int8_t x1 = M[(size_t)a1 * n_c + c1], y1 = M[(size_t)a2 * n_c + c1];
                if (!x1 || !y1) continue;
                for (int32_t c2 = c1 + 1; c2 < n_c; ++c2) {
                    const int8_t x2 = M[(size_t)a1 * n_c + c2], y2 = M[(size_t)a2 * n_c + c2];
                    if (!x2 || !y2) continue;
                    const int t1 = x1 != y1 ? 2 : (x1 > 0 ? 0 : 1);
                    const int t2 = x2 != y2 ? 2 : (x2 > 0 ? 0 : 1);
                    const int lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
                    int k;
                    if (lo == 0 && hi == 0) k = 0;
                    else if (lo == 0 && hi == 1) k = 1;
                    else if (lo == 1 && hi == 1) k = 2;
                    else if (lo == 2) k = 3;
                    else if (lo == 0) k = 4;
                    else k = 5;
                    cnt[6 * (abase + (size_t)a1) + k]++;
                    cnt[6 * (abase + (size_t)a2) + k]++;
                    cnt[6 * (cbase + (size_t)c1) + k]++;
                    cnt[6 * (cbase + (size_t)c2) + k]++;
                }
            }
    free(M);
    return 0;
}

/* Balanced (2,k)-bicliques (Definition 5; the extension named in Sec.
 * "Future Directions"): two vertices of the chosen side and k common
 * neighbours on the other, all 2k edges present, with no unbalanced
 * butterfly inside.  By Lemma 1 a butterfly of two shared centres is
 * balanced exactly when both wedges are symmetric or both asymmetric, so
 * the k centres must all be of one kind: per pair, C(a, k) + C(b, k), with
 * a / b the symmetric / asymmetric wedge counts (Algorithm 1 with general
 * k).  Unlike k = 2, the count depends on which side holds the two
 * vertices.  The BB2K section fixes the size-two side as U (its outer loop
 * runs over u in U), so side 0 (automatic) means U here; side 2 puts the
 * pair on V.
 *
 * Binomials come from Pascal's rule (a table of C(x, j), x <= the largest
 * degree of the side, j <= k), saturating at 2^128; the total is summed in
 * 128 bits.  Returns 2 when a term or the total does not fit 128 bits.
 * out[0] / out[1] receive the low / high 64 bits.  1 <= k <= 64. */
typedef unsigned __int128 u128;
static const u128 U128_MAX = ~(u128)0;

static int pascal_table(int32_t xmax, int k, u128** tab_out) {
    /* tab[x * (k + 1) + j] = C(x, j); U128_MAX marks a saturated entry */
    const size_t w = (size_t)k + 1;
    u128* tab = (u128*)calloc(((size_t)xmax + 1) * w, sizeof(u128));
    if (!tab) return 1;
    tab[0] = 1;
    for (int32_t x = 1; x <= xmax; ++x) {
        tab[(size_t)x * w] = 1;
        for (int j = 1; j <= k; ++j) {
            const u128 p = tab[(size_t)(x - 1) * w + j - 1], q = tab[(size_t)(x - 1) * w + j];
            tab[(size_t)x * w + j] = (p == U128_MAX || q == U128_MAX || p > U128_MAX - q) ? U128_MAX : p + q;
        }
    }
    *tab_out = tab;
    return 0;
}

int oracle_count_bicliques(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                           const int8_t* sg, int side, int k, uint64_t* out) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    if (k < 1 || k > 64) return 1;
    sides_t g;
    build_sides(n_u, n_v, m, off, adj, sg, side == 2 ? 2 : 1, &g);
    int32_t dmax = 0;
    for (int32_t u = 0; u < g.n_s; ++u)
        if (g.s_off[u + 1] - g.s_off[u] > dmax) dmax = (int32_t)(g.s_off[u + 1] - g.s_off[u]);
    u128* tab;
    if (pascal_table(dmax, k, &tab)) {
        sides_free(&g);
        return 1;
    }
    uint32_t* B1 = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    uint32_t* B2 = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)g.n_s + 1));
    u128 total = 0;
    int over = 0;
    for (int32_t u = 0; u < g.n_s; ++u) {
        int32_t nt = 0;
        for (int64_t i = g.s_off[u]; i < g.s_off[u + 1]; ++i) {
            const int32_t c = g.s_nbr[i];
            for (int64_t j = g.c_off[c]; j < g.c_off[c + 1]; ++j) {
                const int32_t w = g.c_nbr[j];
                if (w <= u) continue;
                if (B1[w] == 0 && B2[w] == 0) touched[nt++] = w;
                if (g.c_sgn[j] == g.s_sgn[i]) B1[w]++;
                else B2[w]++;
            }
        }
        for (int32_t t = 0; t < nt; ++t) {
            const int32_t w = touched[t];
            const u128 x = tab[(size_t)B1[w] * (k + 1) + k], y = tab[(size_t)B2[w] * (k + 1) + k];
            if (x == U128_MAX || y == U128_MAX || x > U128_MAX - y || total > U128_MAX - (x + y)) over = 1;
            else total += x + y;
            B1[w] = B2[w] = 0;
        }
    }
    free(B1);
    free(B2);
    free(touched);
    free(tab);
    sides_free(&g);
    out[0] = (uint64_t)total;
    out[1] = (uint64_t)(total >> 64);
    return over ? 2 : 0;
}

/* The same by brute force (tiny graphs): every pair of the side, every
 * k-subset of its common neighbours, kept when every butterfly inside (two
 * of the k centres) has an even number of negative edges (Definitions 2
 * and 5).  Common-neighbour sets of at most 24 vertices; 64-bit total. */
int oracle_brute_bicliques(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                           const int8_t* sg, int side, int k, uint64_t* out) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    if (k < 1 || (int64_t)n_u * n_v > (1LL << 26)) return 1;
    const int su = side != 2; /* the pair on U unless V is named, as in the walk */
    const int32_t n_s = su ? n_u : n_v, n_c = su ? n_v : n_u;
    int8_t* M = (int8_t*)calloc((size_t)n_s * (size_t)n_c + 1, 1);
    for (int32_t u = 0; u < n_u; ++u)
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            const int32_t a = su ? u : adj[e], c = su ? adj[e] : u;
            M[(size_t)a * n_c + c] = sg[e];
        }
    int32_t common[24];
    uint64_t cnt = 0;
    int rc = 0;
    for (int32_t a1 = 0; a1 < n_s && !rc; ++a1)
        for (int32_t a2 = a1 + 1; a2 < n_s && !rc; ++a2) {
            int nc = 0;
            for (int32_t c = 0; c < n_c; ++c)
                if (M[(size_t)a1 * n_c + c] && M[(size_t)a2 * n_c + c]) {
                    if (nc == 24) {
                        rc = 1;
                        break;
                    }
                    common[nc++] = c;
                }
            if (rc || nc < k) continue;
            for (uint32_t mask = 0; mask < (1u << nc); ++mask) {
                if (__builtin_popcount(mask) != k) continue;
                int ok = 1;
                for (int i = 0; i < nc && ok; ++i) {
                    if (!(mask >> i & 1)) continue;
                    for (int j = i + 1; j < nc && ok; ++j) {
                        if (!(mask >> j & 1)) continue;
                        const int32_t c1 = common[i], c2 = common[j];
                        const int prod = M[(size_t)a1 * n_c + c1] * M[(size_t)a2 * n_c + c1] *
                                         M[(size_t)a1 * n_c + c2] * M[(size_t)a2 * n_c + c2];
                        if (prod < 0) ok = 0;
                    }
                }
                cnt += (uint64_t)ok;
            }
        }
    free(M);
    *out = cnt;
    return rc;
}

/* The same classes by brute force over every 2 x 2 vertex choice (tiny
 * graphs): pairs on the anchor side, patterns read at the two centres. */
int oracle_brute_classes(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                         const int8_t* sg, int side, uint64_t* out) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    if ((int64_t)n_u * n_v > (1LL << 26)) return 1;
    const int su = pick_side(n_u, n_v, side) == 1;
    const int32_t n_s = su ? n_u : n_v, n_c = su ? n_v : n_u;
    int8_t* M = (int8_t*)calloc((size_t)n_s * (size_t)n_c + 1, 1);  // M[anchor][centre]
    for (int32_t u = 0; u < n_u; ++u)
        for (int64_t e = off[u]; e < off[u + 1]; ++e) {
            const int32_t a = su ? u : adj[e], c = su ? adj[e] : u;
            M[(size_t)a * n_c + c] = sg[e];
        }
    uint64_t cnt[6] = {0, 0, 0, 0, 0, 0};
    for (int32_t a1 = 0; a1 < n_s; ++a1)
        for (int32_t a2 = a1 + 1; a2 < n_s; ++a2)
            for (int32_t c1 = 0; c1 < n_c; ++c1) {
                const int8_t x1 = M[(size_t)a1 * n_c + c1], y1 = M[(size_t)a2 * n_c + c1];
                if (!x1 || !y1) continue;
                for (int32_t c2 = c1 + 1; c2 < n_c; ++c2) {
                    const int8_t x2 = M[(size_t)a1 * n_c + c2], y2 = M[(size_t)a2 * n_c + c2];
                    if (!x2 || !y2) continue;
                    /* pattern per centre: 0 = ++, 1 = --, 2 = +- */
                    const int t1 = x1 != y1 ? 2 : (x1 > 0 ? 0 : 1);
                    const int t2 = x2 != y2 ? 2 : (x2 > 0 ? 0 : 1);
                    const int lo = t1 < t2 ? t1 : t2, hi = t1 < t2 ? t2 : t1;
                    int k;
                    if (lo == 0 && hi == 0) k = 0;
                    else if (lo == 0 && hi == 1) k = 1;
                    else if (lo == 1 && hi == 1) k = 2;
                    else if (lo == 2) k = 3;
                    else if (lo == 0) k = 4; /* ++ with +- */
                    else k = 5;              /* -- with +- */
                    ++cnt[k];
                }
            }
    free(M);
    for (int k = 0; k < 6; ++k) out[k] = cnt[k];
    return 0;
}

/* Per-vertex counts.  For each anchor pair {u, w} with a symmetric and b
 * asymmetric wedges, the pair closes C(a,2) + C(b,2) balanced butterflies,
 * each containing u and w.  A centre c of a wedge u-c-w of one type lies in
 * every balanced butterfly that pairs this wedge with another wedge of the
 * same type on {u, w}: (a - 1) of them for a symmetric wedge, (b - 1) for an
 * asymmetric one.  Anchors are indexed on their own side; the output puts U
 * first, then V. */
int oracle_per_vertex(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                      const int8_t* sg, int side, uint64_t* cnt) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    int s_is_u = pick_side(n_u, n_v, side) == 1;
    sides_t g;
    build_sides(n_u, n_v, m, off, adj, sg, side, &g);
    uint64_t* cs = cnt + (s_is_u ? 0 : n_u); /* anchor-side block */
    uint64_t* cc = cnt + (s_is_u ? n_u : 0); /* centre-side block */
    memset(cnt, 0, sizeof(uint64_t) * ((size_t)n_u + (size_t)n_v));
    uint32_t* B1 = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    uint32_t* B2 = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
    int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)g.n_s + 1));
    for (int32_t u = 0; u < g.n_s; ++u) {
        int32_t nt = 0;
        for (int64_t i = g.s_off[u]; i < g.s_off[u + 1]; ++i) {
            int32_t c = g.s_nbr[i];
            for (int64_t j = g.c_off[c]; j < g.c_off[c + 1]; ++j) {
                int32_t w = g.c_nbr[j];
                if (w <= u) continue;
                if (B1[w] == 0 && B2[w] == 0) touched[nt++] = w;
                if (g.c_sgn[j] == g.s_sgn[i]) B1[w]++;
                else B2[w]++;
            }
        }
        /* second walk with the pair counts complete: the centres */
        for (int64_t i = g.s_off[u]; i < g.s_off[u + 1]; ++i) {
            int32_t c = g.s_nbr[i];
            for (int64_t j = g.c_off[c]; j < g.c_off[c + 1]; ++j) {
                int32_t w = g.c_nbr[j];
                if (w <= u) continue;
                uint32_t n_same = (g.c_sgn[j] == g.s_sgn[i]) ? B1[w] : B2[w];
                cc[c] += n_same - 1;
            }
        }
        for (int32_t k = 0; k < nt; ++k) {
            int32_t w = touched[k];
            uint64_t p = choose2(B1[w]) + choose2(B2[w]);
            cs[u] += p;
            cs[w] += p;
            B1[w] = 0;
            B2[w] = 0;
        }
    }
    free(B1);
    free(B2);
    free(touched);
    sides_free(&g);
    return 0;
}

/* Balanced butterflies containing x, for x on the anchor side of g, from
 * x's own 2-hop neighbourhood: every same-side vertex y sharing neighbours
 * with x gives a_xy agreeing and b_xy disagreeing common neighbours, and x
 * lies in sum_y C(a_xy,2) + C(b_xy,2) balanced butterflies. */
static uint64_t vertex_count(const sides_t* g, int32_t u, uint32_t* A, uint32_t* B, int32_t* touched) {
    int32_t nt = 0;
    for (int64_t i = g->s_off[u]; i < g->s_off[u + 1]; ++i) {
        int32_t c = g->s_nbr[i];
        for (int64_t j = g->c_off[c]; j < g->c_off[c + 1]; ++j) {
            int32_t w = g->c_nbr[j];
            if (w == u) continue;
            if (A[w] == 0 && B[w] == 0) touched[nt++] = w;
            if (g->c_sgn[j] == g->s_sgn[i]) A[w]++;
            else B[w]++;
        }
    }
    uint64_t t = 0;
    for (int32_t k = 0; k < nt; ++k) {
        t += choose2(A[touched[k]]) + choose2(B[touched[k]]);
        A[touched[k]] = 0;
        B[touched[k]] = 0;
    }
    return t;
}

/* Counts of the vertices xs[0..n) (global indices: U first, then V), for
 * spot checks on graphs too large for a full per-vertex pass. */
int oracle_vertices(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                    const int8_t* sg, const int64_t* xs, int64_t n, uint64_t* out) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    for (int64_t i = 0; i < n; ++i)
        if (xs[i] < 0 || xs[i] >= (int64_t)n_u + n_v) return 1;
    for (int side = 1; side <= 2; ++side) {
        sides_t g;
        build_sides(n_u, n_v, m, off, adj, sg, side, &g);
        uint32_t* A = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
        uint32_t* B = (uint32_t*)calloc((size_t)g.n_s + 1, sizeof(uint32_t));
        int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)g.n_s + 1));
        for (int64_t i = 0; i < n; ++i) {
            int on_u = xs[i] < n_u;
            if (on_u != (side == 1)) continue;
            out[i] = vertex_count(&g, (int32_t)(on_u ? xs[i] : xs[i] - n_u), A, B, touched);
        }
        free(A);
        free(B);
        free(touched);
        sides_free(&g);
    }
    return 0;
}

int oracle_vertex(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                  const int8_t* sg, int64_t x, uint64_t* out) {
    return oracle_vertices(n_u, n_v, m, off, adj, sg, &x, 1, out);
}

/* Definitions 1 and 2 applied directly: every {u1,u2} x {v1,v2} with all
 * four edges is a butterfly; it is balanced when the product of its four
 * signs is +1 (an even number of negative edges).  O(n_u^2 n_v^2) with a
 * dense sign matrix; for tiny graphs.  per_vertex (optional, n_u + n_v)
 * receives the balanced count of every vertex. */
int oracle_brute(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj,
                 const int8_t* sg, uint64_t* balanced, uint64_t* unbalanced, uint64_t* per_vertex) {
    if (check_csr(n_u, n_v, m, off, adj, sg)) return 1;
    if ((int64_t)n_u * n_v > (1LL << 28)) return 1;
    int8_t* M = (int8_t*)calloc((size_t)n_u * (size_t)n_v + 1, 1);
    for (int32_t u = 0; u < n_u; ++u)
        for (int64_t e = off[u]; e < off[u + 1]; ++e) M[(size_t)u * n_v + adj[e]] = sg[e];
    if (per_vertex) memset(per_vertex, 0, sizeof(uint64_t) * ((size_t)n_u + n_v));
    uint64_t bal = 0, unb = 0;
    for (int32_t u1 = 0; u1 < n_u; ++u1)
        for (int32_t u2 = u1 + 1; u2 < n_u; ++u2)
            for (int32_t v1 = 0; v1 < n_v; ++v1) {
                int8_t a = M[(size_t)u1 * n_v + v1], b = M[(size_t)u2 * n_v + v1];
                if (!a || !b) continue;
                for (int32_t v2 = v1 + 1; v2 < n_v; ++v2) {
                    int8_t c = M[(size_t)u1 * n_v + v2], d = M[(size_t)u2 * n_v + v2];
                    if (!c || !d) continue;
                    int negs = (a < 0) + (b < 0) + (c < 0) + (d < 0);
                    if (negs % 2 == 0) {
                        ++bal;
                        if (per_vertex) {
                            per_vertex[u1]++;
                            per_vertex[u2]++;
                            per_vertex[n_u + v1]++;
                            per_vertex[n_u + v2]++;
                        }
                    } else {
                        ++unb;
                    }
                }
            }
    free(M);
    *balanced = bal;
    *unbalanced = unb;
    return 0;
}
