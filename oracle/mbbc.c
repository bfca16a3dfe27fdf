/* Balanced butterfly counting: multicore CPU baseline (M-BBC style).
 *
 * TIMING BASELINE ONLY.  Like the serial oracle beside it, this is test and
 * measurement infrastructure: only the benchmark's CPU-baseline leg and the
 * test suite load it.  It shares no code, header or table with the GPU
 * library, nor with the serial oracle (it is checked against that oracle
 * in the test suite).
 *
 * It follows the shape of the paper's multicore algorithm (Algorithm 2,
 * M-BBC): the smaller side S anchors the walk; anchors are independent
 * tasks handed out dynamically to threads (OpenMP dynamic scheduling, in
 * place of TBB work stealing), heaviest first (the fanout sort of Sec.
 * "Optimization in GPU: Load balancing"); each thread keeps its own
 * symmetric / asymmetric bucket arrays (dense counters with a touched list
 * instead of hash maps); per-anchor sums are added to the total once.
 * The pair filter is the vertex priority of Definition 6: endpoint w
 * counts for anchor u when (deg w, id w) > (deg u, id u), so every pair is
 * counted once, from its lower-priority end, and each centre list is
 * sorted by priority so that the walk reads only a suffix of it.
 *
 * Input: CSR over U as elsewhere (offsets[n_u+1], adj[m] V ids, signs[m]
 * +1 / -1), assumed valid (the serial oracle validates).  Returns 0, or 1
 * when memory runs out.  *threads receives the number of threads used.
 */
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t id;
    int32_t key_deg;
} prio_t;

static int cmp_prio(const void* a, const void* b) {
    const prio_t* x = (const prio_t*)a;
    const prio_t* y = (const prio_t*)b;
    if (x->key_deg != y->key_deg) return x->key_deg < y->key_deg ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

typedef struct {
    uint64_t work;
    int32_t r;
} task_t;

static int cmp_task(const void* a, const void* b) {
    const task_t* x = (const task_t*)a;
    const task_t* y = (const task_t*)b;
    if (x->work != y->work) return x->work > y->work ? -1 : 1;
    return x->r < y->r ? -1 : (x->r > y->r);
}

int mbbc_count(int32_t n_u, int32_t n_v, int64_t m, const int32_t* off, const int32_t* adj, const int8_t* sg,
               uint64_t* total, int32_t* threads) {
    const int su = n_u < n_v; /* the smaller side anchors; a tie keeps V */
    const int32_t n_s = su ? n_u : n_v, n_c = su ? n_v : n_u;
    int ok = 1;
    /* degrees of both sides */
    int64_t* deg_s = (int64_t*)calloc((size_t)n_s + 1, sizeof(int64_t));
    int64_t* deg_c = (int64_t*)calloc((size_t)n_c + 1, sizeof(int64_t));
    if (!deg_s || !deg_c) ok = 0;
    if (ok)
        for (int32_t u = 0; u < n_u; ++u)
            for (int64_t e = off[u]; e < off[u + 1]; ++e) {
                deg_s[su ? u : adj[e]]++;
                deg_c[su ? adj[e] : u]++;
            }
    /* priority rank of every anchor: ascending (degree, id) */
    prio_t* pr = (prio_t*)malloc(sizeof(prio_t) * ((size_t)n_s + 1));
    int32_t* rank = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n_s + 1));
    if (!pr || !rank) ok = 0;
    if (ok) {
        for (int32_t a = 0; a < n_s; ++a) pr[a] = (prio_t){a, (int32_t)deg_s[a]};
        qsort(pr, (size_t)n_s, sizeof(prio_t), cmp_prio);
        for (int32_t r = 0; r < n_s; ++r) rank[pr[r].id] = r;
    }
    /* anchor lists by rank (centre, sign) and centre lists (rank, sign),
     * both by counting sort; centre lists come out rank-sorted because the
     * anchors are scattered in rank order */
    int64_t* a_off = (int64_t*)calloc((size_t)n_s + 1, sizeof(int64_t));
    int64_t* c_off = (int64_t*)calloc((size_t)n_c + 1, sizeof(int64_t));
    int32_t* a_nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int8_t* a_sg = (int8_t*)malloc((size_t)(m > 0 ? m : 1));
    int32_t* c_nbr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    int8_t* c_sg = (int8_t*)malloc((size_t)(m > 0 ? m : 1));
    int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * ((size_t)(n_s > n_c ? n_s : n_c) + 1));
    if (!a_off || !c_off || !a_nbr || !a_sg || !c_nbr || !c_sg || !fill) ok = 0;
    if (ok) {
        for (int32_t a = 0; a < n_s; ++a) a_off[rank[a] + 1] = deg_s[a];
        for (int32_t r = 0; r < n_s; ++r) a_off[r + 1] += a_off[r];
        for (int32_t c = 0; c < n_c; ++c) c_off[c + 1] = c_off[c] + deg_c[c];
        for (int32_t r = 0; r < n_s; ++r) fill[r] = a_off[r];
        for (int32_t u = 0; u < n_u; ++u)
            for (int64_t e = off[u]; e < off[u + 1]; ++e) {
                const int32_t a = su ? u : adj[e], c = su ? adj[e] : u;
                const int64_t q = fill[rank[a]]++;
                a_nbr[q] = c;
                a_sg[q] = sg[e];
            }
        for (int32_t c = 0; c < n_c; ++c) fill[c] = c_off[c];
        for (int32_t r = 0; r < n_s; ++r)
            for (int64_t i = a_off[r]; i < a_off[r + 1]; ++i) {
                const int64_t q = fill[a_nbr[i]]++;
                c_nbr[q] = r;
                c_sg[q] = a_sg[i];
            }
    }
    /* per-anchor work (the fanout: sum of centre degrees), heaviest first */
    task_t* task = (task_t*)malloc(sizeof(task_t) * ((size_t)n_s + 1));
    if (!task) ok = 0;
    if (ok)
        for (int32_t r = 0; r < n_s; ++r) {
            uint64_t w = 0;
            for (int64_t i = a_off[r]; i < a_off[r + 1]; ++i) w += (uint64_t)(c_off[a_nbr[i] + 1] - c_off[a_nbr[i]]);
            task[r] = (task_t){w, r};
        }
    if (ok) qsort(task, (size_t)n_s, sizeof(task_t), cmp_task);

    uint64_t sum = 0;
    int used = 1, fail = 0;
    if (ok) {
#pragma omp parallel reduction(+ : sum)
        {
#pragma omp single
            used = omp_get_num_threads();
            uint32_t* B1 = (uint32_t*)calloc((size_t)n_s + 1, sizeof(uint32_t));
            uint32_t* B2 = (uint32_t*)calloc((size_t)n_s + 1, sizeof(uint32_t));
            int32_t* touched = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n_s + 1));
            if (!B1 || !B2 || !touched) {
#pragma omp atomic write
                fail = 1;
            }
#pragma omp for schedule(dynamic, 1)
            for (int32_t t = 0; t < n_s; ++t) {
                if (!B1 || !B2 || !touched) continue;
                const int32_t r = task[t].r;
                int32_t nt = 0;
                for (int64_t i = a_off[r]; i < a_off[r + 1]; ++i) {
                    const int32_t c = a_nbr[i];
                    const int8_t s1 = a_sg[i];
                    /* the suffix of c's rank-sorted list above r */
                    int64_t lo = c_off[c], hi = c_off[c + 1];
                    while (lo < hi) {
                        const int64_t mid = lo + (hi - lo) / 2;
                        if (c_nbr[mid] <= r) lo = mid + 1;
                        else hi = mid;
                    }
                    for (int64_t j = lo; j < c_off[c + 1]; ++j) {
                        const int32_t w = c_nbr[j];
                        if (B1[w] == 0 && B2[w] == 0) touched[nt++] = w;
                        if (c_sg[j] == s1) B1[w]++;
                        else B2[w]++;
                    }
                }
                uint64_t part = 0;
                for (int32_t k = 0; k < nt; ++k) {
                    const int32_t w = touched[k];
                    const uint64_t a = B1[w], b = B2[w];
                    part += a * (a - (a > 0)) / 2 + b * (b - (b > 0)) / 2;
                    B1[w] = B2[w] = 0;
                }
                sum += part;
            }
            free(B1);
            free(B2);
            free(touched);
        }
    }
    free(deg_s);
    free(deg_c);
    free(pr);
    free(rank);
    free(a_off);
    free(c_off);
    free(a_nbr);
    free(a_sg);
    free(c_nbr);
    free(c_sg);
    free(fill);
    free(task);
    if (!ok || fail) return 1;
    *total = sum;
    *threads = used;
    return 0;
}
