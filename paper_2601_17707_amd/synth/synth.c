/* Seeded synthetic signed bipartite graphs (input generator only).
 *
 * This file draws inputs for both the CPU oracle and the GPU path.  It holds
 * none of the counting arithmetic.  The workloads stand in for the paper's
 * public datasets (Sec. "Datasets Description", Table 2), which are not
 * available: uniform graphs, Chung-Lu power-law graphs, a skewed graph with
 * huge hubs on the smaller side, planted dense signed blocks, and batches of
 * small graphs.
 *
 * Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014): output j of a
 * stream is a fixed bijective mix of (key + (j+1) * golden), so every draw is
 * addressed by its index and parallel loops give the same arrays as serial
 * ones on any machine and thread count.
 *
 * Edge sets are simple: endpoints are drawn independently and a pair that
 * was already drawn is drawn again (rejection sampling), done in rounds that
 * draw exactly the current deficit, so the accepted set equals sequential
 * rejection over the same draw stream.
 *
 * Output: CSR over U (rows sorted by V id), int32 offsets/adjacency, int8
 * signs (+1/-1).  Arrays are malloc'ed here and released by synth_free.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------ RNG */

typedef struct {
    uint64_t key;
} stream_t;

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static stream_t stream_make(uint64_t seed, uint64_t id) {
    stream_t s;
    s.key = mix64(seed * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL) ^ mix64(id + 0xD1B54A32D192ED03ULL);
    return s;
}

/* output j of the stream */
static inline uint64_t draw_u64(stream_t s, uint64_t j) { return mix64(s.key + (j + 1) * 0x9E3779B97F4A7C15ULL); }

/* uniform double in [0, 1) with 53 random bits */
static inline double draw_unit(stream_t s, uint64_t j) {
    return (double)(draw_u64(s, j) >> 11) * (1.0 / 9007199254740992.0);
}

/* integer in [0, n) by the multiply-high map */
static inline uint64_t draw_below(stream_t s, uint64_t j, uint64_t n) {
    return (uint64_t)(((unsigned __int128)draw_u64(s, j) * n) >> 64);
}

/* Beta(a, b) for integer shapes: X / (X + Y) with X ~ Gamma(a), Y ~ Gamma(b),
 * each a sum of exponentials; uses outputs j0 .. j0 + a + b - 1 */
static double draw_beta_int(stream_t s, uint64_t j0, int a, int b) {
    double x = 0.0, y = 0.0;
    for (int i = 0; i < a; ++i) x -= log(1.0 - draw_unit(s, j0 + (uint64_t)i));
    for (int i = 0; i < b; ++i) y -= log(1.0 - draw_unit(s, j0 + (uint64_t)(a + i)));
    return x / (x + y);
}

/* ------------------------------------------------- power-law vertex draws */

/* Continuous Chung-Lu profile: vertex i is drawn with probability
 * (H(i+1) - H(i)) / H(n), H(x) = int_0^x (t + i0)^(-alpha) dt,
 * alpha = 1/(gamma - 1).  Sampling inverts H exactly, so a draw costs one
 * pow().  i0 is solved so the head vertex expects dmax of the m draws. */
typedef struct {
    int64_t n;
    double alpha, i0, hn;
} plaw_t;

static double plaw_H(double alpha, double i0, double x) {
    if (fabs(alpha - 1.0) < 1e-12) return log1p(x / i0);
    double e = 1.0 - alpha;
    return (pow(x + i0, e) - pow(i0, e)) / e;
}

static double plaw_Hinv(double alpha, double i0, double t) {
    if (fabs(alpha - 1.0) < 1e-12) return i0 * expm1(t);
    double e = 1.0 - alpha;
    double base = pow(i0, e) + e * t;
    if (base < 0.0) base = 0.0;
    return pow(base, 1.0 / e) - i0;
}

static plaw_t plaw_make(int64_t n, double m, double gamma, double dmax) {
    plaw_t p;
    p.n = n;
    p.alpha = 1.0 / (gamma - 1.0);
    if (dmax > m) dmax = m;
    double target = dmax / m; /* head probability */
    double lo = 1e-9, hi = 1e13;
    /* the head probability decreases as i0 grows */
    double h_lo = plaw_H(p.alpha, lo, 1.0) / plaw_H(p.alpha, lo, (double)n);
    if (h_lo <= target) {
        p.i0 = lo;
    } else {
        for (int it = 0; it < 400; ++it) {
            double mid = sqrt(lo * hi);
            double h = plaw_H(p.alpha, mid, 1.0) / plaw_H(p.alpha, mid, (double)n);
            if (h > target) lo = mid;
            else hi = mid;
            if (hi / lo < 1.0 + 1e-13) break;
        }
        p.i0 = hi;
    }
    p.hn = plaw_H(p.alpha, p.i0, (double)n);
    return p;
}

static inline int64_t plaw_index(const plaw_t* p, double unit) {
    double x = plaw_Hinv(p->alpha, p->i0, unit * p->hn);
    int64_t i = (int64_t)floor(x);
    if (i < 0) i = 0;
    if (i >= p->n) i = p->n - 1;
    return i;
}

/* --------------------------------------------------------- sorting keys */

static int n_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* stable LSD radix sort of n keys using `bits` low bits; parallel passes with
 * per-thread digit counts */
static void radix_sort_u64(uint64_t* a, uint64_t* tmp, int64_t n, int bits) {
    const int D = 11, B = 1 << D;
    int T = n_threads();
    if (n < (1 << 16)) T = 1;
    int64_t* cnt = (int64_t*)malloc(sizeof(int64_t) * (size_t)B * (size_t)T);
    uint64_t *src = a, *dst = tmp;
    int passes = 0;
    for (int sh = 0; sh < bits; sh += D, ++passes) {
        memset(cnt, 0, sizeof(int64_t) * (size_t)B * (size_t)T);
#pragma omp parallel num_threads(T)
        {
            int t = 0;
#ifdef _OPENMP
            t = omp_get_thread_num();
#endif
            int64_t lo = n * t / T, hi = n * (t + 1) / T;
            int64_t* c = cnt + (size_t)t * B;
            for (int64_t i = lo; i < hi; ++i) c[(src[i] >> sh) & (B - 1)]++;
#pragma omp barrier
#pragma omp single
            {
                int64_t acc = 0;
                for (int d = 0; d < B; ++d)
                    for (int tt = 0; tt < T; ++tt) {
                        int64_t v = cnt[(size_t)tt * B + d];
                        cnt[(size_t)tt * B + d] = acc;
                        acc += v;
                    }
            }
            for (int64_t i = lo; i < hi; ++i) dst[c[(src[i] >> sh) & (B - 1)]++] = src[i];
        }
        uint64_t* t = src;
        src = dst;
        dst = t;
    }
    if (passes & 1) memcpy(a, src, sizeof(uint64_t) * (size_t)n);
    free(cnt);
}

static int bits_for(uint64_t x) {
    int b = 1;
    while (b < 64 && (x >> b)) ++b;
    return b;
}

/* sort + drop repeats; returns the new length */
static int64_t sort_unique(uint64_t* a, uint64_t* tmp, int64_t n, uint64_t maxkey) {
    if (n == 0) return 0;
    radix_sort_u64(a, tmp, n, bits_for(maxkey));
    int64_t k = 1;
    for (int64_t i = 1; i < n; ++i)
        if (a[i] != a[k - 1]) a[k++] = a[i];
    return k;
}

/* draw(ctx, j) -> key in [0, maxkey] for draw index j.  Returns m distinct
 * keys in ascending order (malloc'ed).  *next is the first unused draw
 * index. */
typedef uint64_t (*draw_fn)(const void* ctx, uint64_t j);

static uint64_t* distinct_keys(int64_t m, uint64_t maxkey, draw_fn draw, const void* ctx) {
    size_t cap = (size_t)(m > 0 ? m : 1);
    uint64_t* have = (uint64_t*)malloc(sizeof(uint64_t) * cap);
    uint64_t* batch = (uint64_t*)malloc(sizeof(uint64_t) * cap);
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * cap);
    int64_t nh = 0;
    uint64_t next = 0;
    while (nh < m) {
        int64_t need = m - nh;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < need; ++i) batch[i] = draw(ctx, next + (uint64_t)i);
        next += (uint64_t)need;
        int64_t nb = sort_unique(batch, tmp, need, maxkey);
        /* merge, keeping only batch keys not already present */
        int64_t i = 0, j = 0, k = 0;
        while (i < nh || j < nb) {
            if (j >= nb || (i < nh && have[i] < batch[j])) tmp[k++] = have[i++];
            else if (i >= nh || batch[j] < have[i]) tmp[k++] = batch[j++];
            else {
                tmp[k++] = have[i++];
                ++j;
            }
        }
        uint64_t* t = have;
        have = tmp;
        tmp = t;
        nh = k;
    }
    free(batch);
    free(tmp);
    return have;
}

/* ----------------------------------------------------------- CSR output */

typedef struct {
    int32_t n_u, n_v;
    int64_t m;
    int32_t* offsets;
    int32_t* adj;
    int8_t* signs;
} synth_graph;

/* keys are u * n_v + v, ascending; negs[e] != 0 marks a negative edge */
static void to_csr(synth_graph* g, const uint64_t* keys, const uint8_t* negs) {
    size_t mm = (size_t)(g->m > 0 ? g->m : 1);
    g->offsets = (int32_t*)calloc((size_t)g->n_u + 1, sizeof(int32_t));
    g->adj = (int32_t*)malloc(sizeof(int32_t) * mm);
    g->signs = (int8_t*)malloc(mm);
    const uint64_t nv = (uint64_t)g->n_v;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < g->m; ++e) {
        g->adj[e] = (int32_t)(keys[e] % nv);
        g->signs[e] = negs[e] ? -1 : 1;
    }
    /* rows are contiguous in key order: offsets by a single sweep */
    int64_t e = 0;
    for (int32_t u = 0; u < g->n_u; ++u) {
        g->offsets[u] = (int32_t)e;
        while (e < g->m && keys[e] / nv == (uint64_t)u) ++e;
    }
    g->offsets[g->n_u] = (int32_t)e;
}

void synth_free(synth_graph* g) {
    free(g->offsets);
    free(g->adj);
    free(g->signs);
    g->offsets = NULL;
    g->adj = NULL;
    g->signs = NULL;
}

/* ------------------------------------------------------------- uniform */

typedef struct {
    stream_t s;
    uint64_t n_u, n_v;
} uni_ctx;

static uint64_t draw_uniform(const void* c, uint64_t j) {
    const uni_ctx* u = (const uni_ctx*)c;
    uint64_t a = draw_below(u->s, 2 * j, u->n_u);
    uint64_t b = draw_below(u->s, 2 * j + 1, u->n_v);
    return a * u->n_v + b;
}

int synth_uniform(int32_t n_u, int32_t n_v, int64_t m, double p_neg, uint64_t seed, synth_graph* g) {
    if (n_u < 0 || n_v < 0 || m < 0 || (uint64_t)m > (uint64_t)n_u * (uint64_t)n_v) return 1;
    uni_ctx c = {stream_make(seed, 1), (uint64_t)n_u, (uint64_t)n_v};
    g->n_u = n_u;
    g->n_v = n_v;
    g->m = m;
    uint64_t maxkey = n_u && n_v ? (uint64_t)n_u * n_v - 1 : 0;
    uint64_t* keys = distinct_keys(m, maxkey, draw_uniform, &c);
    uint8_t* neg = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
    stream_t rs = stream_make(seed, 2);
    for (int64_t e = 0; e < m; ++e) neg[e] = draw_unit(rs, (uint64_t)e) < p_neg;
    to_csr(g, keys, neg);
    free(keys);
    free(neg);
    return 0;
}

/* ------------------------------------------------------------ Chung-Lu */

typedef struct {
    stream_t s;
    plaw_t pu, pv;
    const int64_t *perm_u, *perm_v;
    uint64_t n_v;
} cl_ctx;

static uint64_t draw_cl(const void* c, uint64_t j) {
    const cl_ctx* x = (const cl_ctx*)c;
    int64_t a = x->perm_u[plaw_index(&x->pu, draw_unit(x->s, 2 * j))];
    int64_t b = x->perm_v[plaw_index(&x->pv, draw_unit(x->s, 2 * j + 1))];
    return (uint64_t)a * x->n_v + (uint64_t)b;
}

/* Fisher-Yates with draws j = 0 .. n-2 of the stream */
static int64_t* permutation(int64_t n, stream_t s) {
    int64_t* p = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) p[i] = i;
    uint64_t j = 0;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t k = (int64_t)draw_below(s, j++, (uint64_t)(i + 1));
        int64_t t = p[i];
        p[i] = p[k];
        p[k] = t;
    }
    return p;
}

static uint64_t* chung_lu_keys(int32_t n_u, int32_t n_v, int64_t m, double gamma_u, double gamma_v,
                               double dmax_u, double dmax_v, uint64_t seed) {
    int64_t* pu = permutation(n_u, stream_make(seed, 11));
    int64_t* pv = permutation(n_v, stream_make(seed, 12));
    cl_ctx c;
    c.s = stream_make(seed, 13);
    c.pu = plaw_make(n_u, (double)m, gamma_u, dmax_u);
    c.pv = plaw_make(n_v, (double)m, gamma_v, dmax_v);
    c.perm_u = pu;
    c.perm_v = pv;
    c.n_v = (uint64_t)n_v;
    uint64_t* keys = distinct_keys(m, (uint64_t)n_u * n_v - 1, draw_cl, &c);
    free(pu);
    free(pv);
    return keys;
}

/* sign_mode 0: i.i.d. with P(-) = p_neg.
 * sign_mode 1: every vertex x draws beta_x ~ Beta(beta_a, beta_b) (integer
 * shapes); edge uv is negative w.p. min(1, beta_scale * (beta_u + beta_v)). */
static void draw_signs(int32_t n_u, int32_t n_v, int64_t m, const uint64_t* keys, int sign_mode, double p_neg,
                       int beta_a, int beta_b, double beta_scale, uint64_t seed, uint8_t* neg) {
    stream_t rs = stream_make(seed, 14);
    if (sign_mode == 0) {
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < m; ++e) neg[e] = draw_unit(rs, (uint64_t)e) < p_neg;
        return;
    }
    double* bu = (double*)malloc(sizeof(double) * (size_t)(n_u > 0 ? n_u : 1));
    double* bv = (double*)malloc(sizeof(double) * (size_t)(n_v > 0 ? n_v : 1));
    stream_t su = stream_make(seed, 15), sv = stream_make(seed, 16);
    uint64_t w = (uint64_t)(beta_a + beta_b);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n_u; ++i) bu[i] = draw_beta_int(su, w * (uint64_t)i, beta_a, beta_b);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n_v; ++i) bv[i] = draw_beta_int(sv, w * (uint64_t)i, beta_a, beta_b);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint64_t u = keys[e] / (uint64_t)n_v, v = keys[e] % (uint64_t)n_v;
        double p = beta_scale * (bu[u] + bv[v]);
        if (p > 1.0) p = 1.0;
        neg[e] = draw_unit(rs, (uint64_t)e) < p;
    }
    free(bu);
    free(bv);
}

int synth_chung_lu(int32_t n_u, int32_t n_v, int64_t m, double gamma_u, double gamma_v, double dmax_u,
                   double dmax_v, int sign_mode, double p_neg, int beta_a, int beta_b, double beta_scale,
                   uint64_t seed, synth_graph* g) {
    if (n_u <= 0 || n_v <= 0 || m < 0 || (uint64_t)m > (uint64_t)n_u * (uint64_t)n_v) return 1;
    if (gamma_u <= 1.0 || gamma_v <= 1.0) return 1;
    g->n_u = n_u;
    g->n_v = n_v;
    g->m = m;
    uint64_t* keys = chung_lu_keys(n_u, n_v, m, gamma_u, gamma_v, dmax_u, dmax_v, seed);
    uint8_t* neg = (uint8_t*)malloc((size_t)(m > 0 ? m : 1));
    draw_signs(n_u, n_v, m, keys, sign_mode, p_neg, beta_a, beta_b, beta_scale, seed, neg);
    to_csr(g, keys, neg);
    free(keys);
    free(neg);
    return 0;
}

/* --------------------------------------------------------------- hybrid */

/* Power-law background plus n_blocks planted blocks R_i x C_i (R_i of V,
 * C_i of U, pairwise disjoint, `block` vertices each).  Inside a block each
 * pair is an edge w.p. density; factions f_x in {+1,-1} are uniform; the
 * sign of rc is f_r f_c flipped w.p. flip.  Block draws replace background
 * edges inside the blocks.  rows_out / cols_out receive the block vertex ids
 * (n_blocks * block each, block-major). */
int synth_hybrid(int32_t n_u, int32_t n_v, int64_t m_bg, double gamma, double dmax, double p_neg,
                 int32_t n_blocks, int32_t block, double density, double flip, uint64_t seed, synth_graph* g,
                 int32_t* rows_out, int32_t* cols_out) {
    if (n_u <= 0 || n_v <= 0 || n_blocks < 0 || block < 0) return 1;
    if ((int64_t)n_blocks * block > n_u || (int64_t)n_blocks * block > n_v) return 1;
    if ((uint64_t)m_bg > (uint64_t)n_u * (uint64_t)n_v) return 1;
    uint64_t* bg = chung_lu_keys(n_u, n_v, m_bg, gamma, gamma, dmax, dmax, seed);
    uint8_t* bgneg = (uint8_t*)malloc((size_t)(m_bg > 0 ? m_bg : 1));
    draw_signs(n_u, n_v, m_bg, bg, 0, p_neg, 0, 0, 0.0, seed, bgneg);

    int64_t* pv = permutation(n_v, stream_make(seed, 21));
    int64_t* pu = permutation(n_u, stream_make(seed, 22));
    int32_t* blk_v = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_v);
    int32_t* blk_u = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_u);
    for (int32_t i = 0; i < n_v; ++i) blk_v[i] = -1;
    for (int32_t i = 0; i < n_u; ++i) blk_u[i] = -2;
    for (int32_t b = 0; b < n_blocks; ++b)
        for (int32_t k = 0; k < block; ++k) {
            int64_t v = pv[(int64_t)b * block + k], u = pu[(int64_t)b * block + k];
            rows_out[(int64_t)b * block + k] = (int32_t)v;
            cols_out[(int64_t)b * block + k] = (int32_t)u;
            blk_v[v] = b;
            blk_u[u] = b;
        }
    stream_t sf = stream_make(seed, 23);
    int8_t* fv = (int8_t*)malloc((size_t)n_v);
    int8_t* fu = (int8_t*)malloc((size_t)n_u);
    for (int32_t i = 0; i < n_v; ++i) fv[i] = draw_unit(sf, (uint64_t)i) < 0.5 ? -1 : 1;
    for (int32_t i = 0; i < n_u; ++i) fu[i] = draw_unit(sf, (uint64_t)n_v + (uint64_t)i) < 0.5 ? -1 : 1;

    /* background edges outside the blocks, then every block pair that is
     * drawn present; keys carry the sign in bit 0 */
    int64_t nbg = 0;
    for (int64_t e = 0; e < m_bg; ++e) {
        uint64_t u = bg[e] / (uint64_t)n_v, v = bg[e] % (uint64_t)n_v;
        if (blk_v[v] != blk_u[u]) bg[nbg++] = (bg[e] << 1) | bgneg[e];
    }
    free(bgneg);
    int64_t cells = (int64_t)n_blocks * block * block;
    uint64_t* all = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(nbg + cells > 0 ? nbg + cells : 1));
    memcpy(all, bg, sizeof(uint64_t) * (size_t)nbg);
    free(bg);
    uint8_t* keep = (uint8_t*)malloc((size_t)(cells > 0 ? cells : 1));
    uint64_t* cellkey = all + nbg;
    stream_t sd = stream_make(seed, 24);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < cells; ++q) {
        int64_t b = q / ((int64_t)block * block), r = (q / block) % block, c = q % block;
        int64_t v = rows_out[b * block + r], u = cols_out[b * block + c];
        keep[q] = draw_unit(sd, 2 * (uint64_t)q) < density;
        int s = fv[v] * fu[u];
        if (draw_unit(sd, 2 * (uint64_t)q + 1) < flip) s = -s;
        cellkey[q] = (((uint64_t)u * (uint64_t)n_v + (uint64_t)v) << 1) | (uint64_t)(s < 0);
    }
    int64_t n = nbg;
    for (int64_t q = 0; q < cells; ++q)
        if (keep[q]) all[n++] = cellkey[q];
    free(keep);
    uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    radix_sort_u64(all, tmp, n, bits_for((((uint64_t)n_u * n_v) << 1) | 1));
    free(tmp);
    uint8_t* neg = (uint8_t*)malloc((size_t)(n > 0 ? n : 1));
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n; ++e) {
        neg[e] = (uint8_t)(all[e] & 1);
        all[e] >>= 1;
    }
    g->n_u = n_u;
    g->n_v = n_v;
    g->m = n;
    to_csr(g, all, neg);
    free(all);
    free(neg);
    free(pv);
    free(pu);
    free(blk_v);
    free(blk_u);
    free(fv);
    free(fu);
    return 0;
}

/* ---------------------------------------------------------------- batch */

/* Parameters of batch member i: m log-uniform in [m_lo, m_hi]; r = |U|/|V|
 * uniform in [0.2, 5]; gamma uniform in [1.8, 2.8]; P(-) uniform in
 * [0.1, 0.5]; n = |U| + |V| is the smallest count with mean total degree at
 * most 8 and density at most 0.25; a sub-seed for the member's graph. */
void synth_batch_params(uint64_t seed, int32_t i, double m_lo, double m_hi, int64_t* m, int32_t* n_u,
                        int32_t* n_v, double* gamma, double* p_neg, uint64_t* sub_seed) {
    stream_t s = stream_make(seed, 1000003ULL + (uint64_t)i);
    double lm = log(m_lo) + draw_unit(s, 0) * (log(m_hi) - log(m_lo));
    int64_t mm = (int64_t)llround(exp(lm));
    double ratio = 0.2 + draw_unit(s, 1) * 4.8;
    *gamma = 1.8 + draw_unit(s, 2) * 1.0;
    *p_neg = 0.1 + draw_unit(s, 3) * 0.4;
    *sub_seed = draw_u64(s, 4);
    int64_t n = (mm + 3) / 4;
    if (n < 4) n = 4;
    for (;; ++n) {
        int64_t nu = (int64_t)llround((double)n * ratio / (1.0 + ratio));
        if (nu < 2) nu = 2;
        int64_t nv = n - nu;
        if (nv < 2) nv = 2;
        if (nu * nv >= 4 * mm) {
            *n_u = (int32_t)nu;
            *n_v = (int32_t)nv;
            break;
        }
    }
    *m = mm;
}
