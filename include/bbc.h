/* bbc.h - C ABI of libbbc.so: balanced butterfly counting on one AMD MI355X
 * (gfx950) GPU.
 *
 * Problem (paper, Sec. "Preliminaries and Problem Definition", Definitions 1
 * and 2 and the Problem Statement): in a signed bipartite graph
 * G = (U, V, E+ u E-), count the butterflies - 4-cycles u1 v1 u2 v2 with all
 * four U x V edges present - that hold an even number of negative edges.
 *
 * Method (Sec. "proposed algorithms", Algorithms 1-4, Lemma 1): from each
 * anchor u of one side S, walk the wedges u - c - w (c on the other side,
 * w ranked above u), count per endpoint w the wedges whose two edges agree in
 * sign (a) and disagree (b), and add C(a,2) + C(b,2).  Only pairs of agreeing
 * or pairs of disagreeing wedges close a balanced butterfly (Lemma 1), so no
 * unbalanced structure is ever formed.  Ranks follow the vertex priority of
 * Definition 6 (degree, then id).  Every step runs in the library's own HIP
 * kernels on the caller's stream; counts are exact integers.
 *
 * Entry points: bbc_count (total, optional per-vertex counts and dense
 * blocks), bbc_count_noalloc (the same without any allocation),
 * bbc_count_batched and the captured batch plans, bbc_plan_blocks
 * (dense-block planner), bbc_autotune (and its batched and dense-block
 * forms) with bbc_tune_save / _load, and the extensions bbc_count_classes
 * and bbc_count_classes_per_vertex (the six sign-pattern classes of the
 * case study, in total and per vertex), bbc_count_bicliques (balanced
 * (2,k)-bicliques) and bbc_update_delta (the change of the count under edge
 * updates).
 *
 * Conventions for every entry point
 *   - Graphs are a CSR over U: offsets[n_u + 1] (int32, offsets[0] = 0,
 *     non-decreasing, offsets[n_u] = n_edges), adj[n_edges] (int32 V ids in
 *     [0, n_v)), signs[n_edges] (int8, +1 or -1).  Rows need not be sorted.
 *     The graph must be simple: a repeated (u, v) pair is an error.
 *   - Pointers marked "device" are HIP device pointers (for example a torch
 *     tensor's data_ptr()); pointers marked "host" are ordinary host memory.
 *   - The caller owns every input and output buffer; the library never frees
 *     them.  The library owns its scratch memory, allocated inside the
 *     context and grown on demand.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     All device work is ordered on it.
 *   - On any error nothing is written to the outputs, and bbc_last_error()
 *     describes the first offending input.
 *   - A context is bound to one device and is not thread-safe: use one
 *     context per host thread.
 *   - Degenerate graphs (no edges, fewer than two vertices on a side) give 0.
 *   - n_edges must be <= INT32_MAX and n_u + n_v <= INT32_MAX, otherwise
 *     BBC_ETOOBIG.
 */
#ifndef BBC_H
#define BBC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BBC_OK = 0,
    BBC_EINVAL = 1,   /* null pointer, negative size, bad option */
    BBC_EOFFSETS = 2, /* offsets[0] != 0, decreasing offsets, or offsets[n_u] != n_edges */
    BBC_ERANGE = 3,   /* an adjacency id outside [0, n_v) */
    BBC_ESIGN = 4,    /* a sign other than +1 / -1 */
    BBC_EDUP = 5,     /* a repeated (u, v) pair */
    BBC_ENOMEM = 6,   /* device memory could not be allocated */
    BBC_EDEVICE = 7,  /* HIP runtime error; bbc_last_error has the detail */
    BBC_ETOOBIG = 8,  /* sizes beyond the int32 CSR limits */
    BBC_EOVERFLOW = 9 /* the result does not fit its integer width (bbc_count_bicliques) */
} bbc_status;

typedef struct bbc_ctx bbc_ctx;

/* anchor side: the paper starts from the smaller side, a tie keeping V
 * (Algorithm 2: S = V, replaced by U when |V| > |U|); the count is the same
 * from either side (Sec. "BB2K Algorithm").  BBC_SIDE_MIN_WEDGES takes the
 * side whose walk has fewer wedges (sum of C(deg, 2) over the other side),
 * the partition choice of the butterfly-counting prior art the paper cites
 * (Sec. "Related Work"); it measures both on the device and waits for the
 * stream once before the count, a tie following the AUTO rule.  bbc_count
 * only: batches, the planner and the class counts (whose classes depend on
 * the paired side) reject it with BBC_EINVAL. */
enum { BBC_SIDE_AUTO = 0, BBC_SIDE_U = 1, BBC_SIDE_V = 2, BBC_SIDE_MIN_WEDGES = 3 };

/* Work distribution of the wedge kernel over its persistent workgroups.
 * Anchors are listed by descending work (Sec. "Optimization in GPU: Load
 * balancing").  DYNAMIC (default): each workgroup takes the next anchor of
 * a shared atomic queue.  STATIC: workgroup b takes positions b, b + G,
 * b + 2G, ... of the list (G workgroups), a fixed deal with no queue, in the
 * manner of the paper's fixed-tile kernel (G-BBC), which wins when anchors
 * are few and heavy.  The autotuner tries both. */
enum { BBC_SCHED_DYNAMIC = 0, BBC_SCHED_STATIC = 1 };

/* optional input checks (offsets and id ranges are always checked, since
 * the kernels index with them) */
enum { BBC_CHECK_SIGNS = 1, BBC_CHECK_DUPLICATES = 2, BBC_CHECK_ALL = 3 };

/* A dense block: a set of U vertices and a set of V vertices whose edges
 * are counted on int8 matrix cores (see bbc_options.blocks).  Blocks must be
 * pairwise disjoint on both sides. */
typedef struct {
    int32_t n_u_ids, n_v_ids;
    const int32_t* u_ids; /* device, n_u_ids distinct U ids */
    const int32_t* v_ids; /* device, n_v_ids distinct V ids */
} bbc_dense_block;

typedef struct {
    uint32_t struct_size; /* sizeof(bbc_options), set by bbc_options_init */
    int32_t side;         /* BBC_SIDE_* */
    uint32_t checks;      /* BBC_CHECK_* mask, default BBC_CHECK_ALL */
    int32_t timing;       /* nonzero: record per-phase HIP event times (bbc_last_stats) */
    int32_t band_words;   /* LDS counter band in 32-bit words per workgroup, 0 = default */
    int32_t wg_size;      /* threads per wedge-kernel workgroup, 0 = default */
    int32_t wg_per_cu;    /* persistent workgroups per compute unit, 0 = as many as fit */
    /* Dense-block hybrid (bbc_count only, no per-vertex output).  For the
     * vertices of each block, with S the block's signed adjacency (entries
     * +1 / -1 / 0), S S^T = a - b and |S| |S|^T = a + b count the agreeing
     * and disagreeing wedges through the block's centres exactly (int8
     * operands, int32 accumulation).  Every other wedge - including those
     * with one block edge and one other edge - stays in the sparse walk, and
     * pairs inside a block add the cross term a_dense a_sparse +
     * b_dense b_sparse, so the count is exact for any choice of blocks.
     * Per block: at most 16384 anchor-side and 65535 centre-side ids. */
    int32_t n_blocks;
    const bbc_dense_block* blocks; /* host array of n_blocks, or NULL */
    /* Nonzero: ignore the context's tuning table (see bbc_autotune).  The
     * table is consulted only when band_words, wg_size and wg_per_cu are all
     * 0, schedule is dynamic and no per-vertex output is asked for. */
    int32_t no_tuning;
    int32_t schedule; /* BBC_SCHED_*: how wedge-kernel workgroups take anchors */
    /* Regimes of the wedge kernel (the paper's warp / block split of
     * Algorithm 4).  An anchor with at most wave_max_work wedges, at most 63
     * centres and fewer than 2^20 vertices ranked above it in its graph is
     * counted by one wavefront in a hashed LDS table of its own, with no
     * workgroup barrier; these anchors are taken 64 per queue pop.  Every
     * other anchor takes a whole workgroup, queue_chunk anchors per pop (in
     * descending work order).  wave_max_work: 0 = the kernel shape's largest
     * (1024 for the default shape; half of the table a wavefront gets from
     * the band, at most 2048 slots), -1 = no wave regime, larger values are
     * clamped to that largest.  queue_chunk: 0 = 1, at most 65536.  Only
     * bbc_count without per-vertex output and the batched calls use the wave
     * regime.  The counts never depend on either. */
    int32_t queue_chunk;
    int32_t wave_max_work;
    /* Output tile edge of the int8 matrix kernel of dense blocks: 128
     * (default) or 64 (less padding for small blocks); 0 = the tuning
     * table's choice for the graph's size class (see bbc_autotune_blocks),
     * else 128. */
    int32_t dense_tile;
    /* Largest scratch, in bytes, the call may need (the context's arena, or
     * a batch plan's own); a call that needs more fails with BBC_ENOMEM
     * before any work, its outputs and the arena untouched, and the context
     * stays usable.  0 = no limit. */
    int64_t scratch_limit;
} bbc_options;

/* Fills *opts with the defaults: auto side, all checks, no timing. */
void bbc_options_init(bbc_options* opts);

/* Creates a context on HIP device `device` (the current device if < 0).
 * *out (host) receives the context.  BBC_EDEVICE if the device is missing or
 * is not a gfx950 part. */
bbc_status bbc_create(int device, bbc_ctx** out);

/* Releases the context and its scratch memory.  NULL is accepted. */
bbc_status bbc_destroy(bbc_ctx* ctx);

/* Number of balanced butterflies of one graph (Problem Statement; computed
 * by the wedge method of Algorithms 1-4, see above).
 *   offsets, adj, signs  device, CSR over U as described above.
 *   total                host, receives the count (written only on BBC_OK).
 *   per_vertex           device or NULL; if given, n_u + n_v uint64 entries
 *                        receive the number of balanced butterflies that
 *                        contain each vertex, U ids first, then V ids (the
 *                        paper counts totals only; this is the library's
 *                        per-vertex reading).  Overwritten, not accumulated.
 *   opts                 host or NULL (defaults).  band_words / wg_size must
 *                        name an instantiated kernel shape (BBC_EINVAL
 *                        otherwise), as words/threads: 8192/256
 *                        (default), 16384/512, 16384/256, 8192/512,
 *                        32768/1024, 16384/1024, 4096/128, 8192/128,
 *                        4096/256.
 * Synchronous with respect to *total: returns after the stream has
 * produced it.  Errors: BBC_EINVAL, BBC_EOFFSETS, BBC_ERANGE, BBC_ESIGN,
 * BBC_EDUP, BBC_ENOMEM, BBC_EDEVICE, BBC_ETOOBIG. */
bbc_status bbc_count(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                     const int32_t* adj, const int8_t* signs, uint64_t* total, uint64_t* per_vertex,
                     const bbc_options* opts, void* stream);

/* Allocation-free variant of bbc_count, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, and
 * harnesses that forbid allocation.  Arguments, results, errors and
 * synchronisation are those of bbc_count, except:
 *   - the call allocates nothing (no hipMalloc / hipFree, no allocating
 *     library routine).  Its scratch is a fixed device array of
 *     BBC_NOALLOC_SCRATCH_BYTES bytes, one per GPU, held from the library's
 *     first bbc_create on that GPU until the process ends;
 *   - a graph whose scratch would exceed that size is rejected with
 *     BBC_ETOOBIG, and bbc_last_error gives the bytes it needs (41 bytes
 *     per edge, 60 per anchor-side and 24 per centre-side vertex, plus
 *     sort histograms; 64 MiB holds about 1.3M edges);
 *   - dense blocks are not accepted (BBC_EINVAL);
 *   - every call on one GPU shares that GPU's array, whose contents persist
 *     from call to call: calls that overlap on one GPU (several streams,
 *     threads or contexts) race and must be serialised by the caller.
 * The context (created beforehand, which may allocate) supplies the status
 * word, pinned result memory and the tuning table. */
#define BBC_NOALLOC_SCRATCH_BYTES (64ull << 20)
bbc_status bbc_count_noalloc(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                             const int32_t* adj, const int8_t* signs, uint64_t* total, uint64_t* per_vertex,
                             const bbc_options* opts, void* stream);

/* One graph of a batch.  Its offsets are local (offsets[0] = 0, n_u + 1
 * entries starting at offsets_cat[off_base]); its edges are adj_cat /
 * signs_cat[edge_base .. edge_base + n_edges).  Graphs may sit anywhere in
 * the concatenated arrays. */
typedef struct {
    int32_t n_u, n_v;
    int64_t n_edges;
    int64_t off_base;
    int64_t edge_base;
} bbc_graph_desc;

/* Balanced butterfly counts of n_graphs independent graphs in one pass of
 * the pipeline (the batch is counted as one disjoint union in which every
 * graph keeps its own anchor side and a contiguous range of ranks, so the
 * heavy anchors of every graph share one persistent launch).
 *   descs                host, n_graphs entries.
 *   offsets_cat, adj_cat, signs_cat  device, as described by descs.
 *   totals               device, n_graphs uint64, overwritten on BBC_OK (on
 *                        error their content is unspecified).
 * Sums over all graphs must satisfy the bbc_count size limits.  Returns
 * after the stream has produced the totals (input errors are reported). */
bbc_status bbc_count_batched(bbc_ctx* ctx, int32_t n_graphs, const bbc_graph_desc* descs,
                             const int32_t* offsets_cat, const int32_t* adj_cat, const int8_t* signs_cat,
                             uint64_t* totals, const bbc_options* opts, void* stream);

/* A batch plan: the whole batched pipeline for a fixed batch layout,
 * captured once into a HIP graph with its own scratch memory, then replayed.
 * The buffers named at creation must stay allocated while the plan lives;
 * their contents may change between launches (same sizes). */
typedef struct bbc_batch_plan bbc_batch_plan;

/* Arguments as bbc_count_batched; *out (host) receives the plan.  Allocates
 * all scratch and captures the graph; nothing is computed yet. */
bbc_status bbc_batch_plan_create(bbc_ctx* ctx, int32_t n_graphs, const bbc_graph_desc* descs,
                                 const int32_t* offsets_cat, const int32_t* adj_cat, const int8_t* signs_cat,
                                 uint64_t* totals, const bbc_options* opts, bbc_batch_plan** out);

/* Replays the captured graph on `stream` (asynchronous). */
bbc_status bbc_batch_launch(bbc_batch_plan* plan, void* stream);

/* Waits for `stream` and reports the input checks of the last launch
 * (BBC_OK, or the error bbc_count_batched would have returned). */
bbc_status bbc_batch_wait(bbc_batch_plan* plan, void* stream);

/* Releases the plan (NULL is accepted). */
bbc_status bbc_batch_plan_destroy(bbc_batch_plan* plan);

/* Facts about the last successful bbc_count on this context. */
typedef struct {
    uint32_t struct_size; /* sizeof(bbc_stats) */
    int32_t side;         /* BBC_SIDE_U or BBC_SIDE_V: the anchor side used */
    int32_t n_anchor;     /* vertices on the anchor side */
    int32_t n_centre;     /* vertices on the other side */
    int64_t n_edges;
    uint64_t wedges;      /* sum over centres c of C(deg c, 2): wedges walked once each */
    uint64_t bands;       /* LDS counter bands processed by the wedge kernel */
    int32_t grid;         /* persistent workgroups launched */
    int32_t block;        /* threads per workgroup */
    float ms_checks;      /* HIP event times on the caller's stream (timing option) */
    float ms_build;       /* degrees, ranks, degree-ordered CSR, schedule */
    float ms_count;       /* wedge aggregation kernel (and the dense blocks, if any) */
    float ms_total;
    float ms_dense;       /* int8 matrix-core kernel of the dense blocks */
    int32_t n_blocks;
    uint64_t dense_ops;   /* int8 multiply-adds x 2 of the upper-triangle block tiles */
    uint64_t wedges_all;  /* sum over centres of C(deg c, 2), dense blocks included */
    int32_t band_words;   /* LDS counter band of the wedge kernel, 32-bit words */
    int32_t tuned;        /* 1 if the kernel shape came from the tuning table */
    int32_t schedule;     /* BBC_SCHED_* of the wedge kernel */
} bbc_stats;

bbc_status bbc_last_stats(const bbc_ctx* ctx, bbc_stats* out);

/* Autotuner.  The paper fixes its launch shape by hand (warp / partial-block
 * / full-block thresholds 32 and 512, blocks in proportion to the SM count;
 * Sec. "Optimization in GPU: Load balancing", Algorithm 4); here the knobs
 * are measured instead.  bbc_autotune counts the given calibration graph
 * (arguments as bbc_count) in two stages, `reps` timed runs per
 * configuration (HIP events around the wedge kernel, best of reps; reps <= 0
 * means 2, one warm-up run before them): first every instantiated shape
 * (threads per workgroup, LDS band), persistent grid (1, 2 and as many
 * workgroups per CU as fit) and schedule (BBC_SCHED_*), then, with the
 * fastest shape and grid, both schedules x queue_chunk in {1, 2, 4, 8, 16}
 * x wave_max_work in {the shape's largest, 256, -1}.  The winner is recorded in the context's table
 * under the graph's size class: (bit length of n_S, bit length of
 * m / n_S), n_S the anchor side of the default side rule.  Later bbc_count
 * and batched calls of the same class use it unless their options fix the
 * shape or set no_tuning (queue_chunk and wave_max_work only when they are
 * 0).  *chosen (host, may be NULL) receives options holding the choice.
 * Every configuration must give the same count (BBC_EDEVICE otherwise); the
 * count never depends on them.  Errors: as bbc_count. */
bbc_status bbc_autotune(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                        const int32_t* adj, const int8_t* signs, int32_t reps, bbc_options* chosen, void* stream);

/* The same two-stage search on a batch (arguments as bbc_count_batched;
 * totals receives the last run's counts), recorded under the batch's size
 * class (n_S and m summed over its graphs), which bbc_count_batched and
 * batch plans of the same layout then use.  Every configuration must give
 * the same per-graph totals. */
bbc_status bbc_autotune_batched(bbc_ctx* ctx, int32_t n_graphs, const bbc_graph_desc* descs,
                                const int32_t* offsets_cat, const int32_t* adj_cat, const int8_t* signs_cat,
                                uint64_t* totals, int32_t reps, bbc_options* chosen, void* stream);

/* Writes the tuning table to a text file (path: host string).  One header
 * line "bbc-tune 3 gfx950", then one line per size class: "ns_bits deg_bits
 * band_words wg_size wg_per_cu schedule queue_chunk wave_max_work
 * min_degree dense_tile ms" (band_words 0: the class has only dense-block
 * choices; queue_chunk, min_degree and dense_tile 0: not tuned).
 * BBC_EINVAL if the file cannot be written. */
bbc_status bbc_tune_save(const bbc_ctx* ctx, const char* path);

/* Reads such a file (or an older one: version 2 lines end after the
 * schedule column, version 1 lines after wg_per_cu and mean the dynamic
 * schedule) and merges its entries into the table (an entry replaces the
 * one of the same class).  BBC_EINVAL, with the line number in
 * bbc_last_error, for a missing file, a wrong header, a malformed line or a
 * shape that is not instantiated; the table is unchanged on error. */
bbc_status bbc_tune_load(bbc_ctx* ctx, const char* path);

/* Sign-pattern classes of the case study (Sec. "Case Study", Table 8).
 * For a pair of anchor-side vertices (opts->side picks the side; the case
 * study pairs the drugs) every shared centre carries a pattern: ++ (both
 * edges positive), -- (both negative) or +- (the edges differ); a butterfly
 * is a pair of shared centres and its class the unordered pair of their
 * patterns.  classes (host, 6 uint64) receives, in Table 8's order:
 *   [0] coherent ++/++  [1] coherent ++/--  [2] coherent --/--
 *   [3] incoherent +-/+-  [4] mixed ++/+-  [5] mixed +-/--
 * Coherent and incoherent butterflies are balanced, mixed ones unbalanced
 * (Lemma 1), so [0] + [1] + [2] + [3] is bbc_count's total.  The same walk
 * as bbc_count with three counters per endpoint (one kernel shape: 256
 * threads, 8,192-word bands); dense blocks, per-vertex output and batches
 * are not offered here (BBC_EINVAL for blocks).  Other arguments, errors and
 * synchronisation as bbc_count. */
bbc_status bbc_count_classes(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                             const int32_t* adj, const int8_t* signs, uint64_t* classes, const bbc_options* opts,
                             void* stream);

/* The six classes for every vertex (the case study's classes, Table 8,
 * per vertex): per_vertex (device, (n_u + n_v) x 6 uint64, vertex-major,
 * U ids first, then V ids) receives, for each vertex x and class k in the
 * order of bbc_count_classes, the number of class-k butterflies that contain
 * x; classes (host, 6 uint64) receives the totals.  Each class's U entries
 * and its V entries both sum to twice its total.  Walks every anchor's whole
 * list (ranks above and below it, as bbc_count's per-vertex output does)
 * and a second time per band for the centres (one kernel shape: 256
 * threads, 8,192-word bands).  per_vertex is overwritten, not accumulated;
 * NULL is BBC_EINVAL unless the graph has no vertices.  Other arguments, errors and synchronisation as
 * bbc_count_classes. */
bbc_status bbc_count_classes_per_vertex(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges,
                                        const int32_t* offsets, const int32_t* adj, const int8_t* signs,
                                        uint64_t* classes, uint64_t* per_vertex, const bbc_options* opts,
                                        void* stream);

/* Balanced (2,k)-bicliques (Definition 5; the generalisation named in Sec.
 * "Future Directions"): two vertices of the pair side and k common
 * neighbours, all 2k edges present and no unbalanced butterfly inside.  By
 * Lemma 1 the k centres of such a biclique give wedges of one kind, so the
 * count is, over pairs {u, w} of the pair side, C(a_uw, k) + C(b_uw, k) with
 * a / b the symmetric / asymmetric wedge counts (Algorithm 1 with general
 * k).  k = 2 is bbc_count's total; k = 1 counts the wedges.  Unlike k = 2
 * the result depends on the pair side: opts->side (BBC_SIDE_U or _V).
 * The BB2K section under Algorithm 1 fixes the size-two side as U, so
 * BBC_SIDE_AUTO means U here (not the smaller side); BBC_SIDE_MIN_WEDGES
 * is rejected.
 * count (host, 2 uint64) receives the exact 128-bit result, low word
 * first; BBC_EOVERFLOW when it, or one pair's term, does not fit 128 bits.
 * 1 <= k <= BBC_BICLIQUE_MAX_K, else BBC_EINVAL.  The same walk as
 * bbc_count in one kernel shape (256 threads, 8,192-word bands); dense
 * blocks, per-vertex output and batches are not offered (BBC_EINVAL for
 * blocks).  Other arguments, errors and synchronisation as bbc_count. */
#define BBC_BICLIQUE_MAX_K 16
bbc_status bbc_count_bicliques(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                               const int32_t* adj, const int8_t* signs, int32_t k, uint64_t* count,
                               const bbc_options* opts, void* stream);

/* Dynamic graphs (the setting named in Sec. "Future Directions": edges
 * added, removed or re-signed).  For the graph G given as in bbc_count and a
 * batch of n_updates updates - pair (upd_u[i], upd_v[i]) takes the state
 * upd_state[i]: +1 / -1 (the edge is present with that sign; added if
 * absent) or 0 (absent; removed if present) - *delta (host) receives
 * T(G') - T(G), the change of the balanced butterfly count, G' being G with
 * the whole batch applied.  Pairs within a batch must be distinct; an
 * update that keeps a pair's state changes nothing.
 * Only butterflies holding an updated pair can change; each is charged to
 * the changed pair of lowest index it holds, and the walk of update i
 * visits the butterflies through its pair before and after the batch,
 * adding (balanced after) - (balanced before).  per_update (device, int64
 * [n_updates], may be NULL) receives each update's share; the shares sum to
 * *delta (on error it is left untouched).  upd_u, upd_v (int32) and upd_state (int8) are device arrays.
 * Work per update is the smaller of deg(u) deg(v) pair lookups and the
 * walk v -> w -> x (the sum of deg(w) over the neighbours w of v), each a
 * binary search, split into tasks that spread over the whole GPU.
 * Errors: BBC_EINVAL (null pointers, negative sizes, a pair repeated in the
 * batch), BBC_ERANGE / BBC_ESIGN (the graph's, or an update's id or state),
 * BBC_EOFFSETS, BBC_EDUP, BBC_ENOMEM, BBC_EDEVICE, BBC_ETOOBIG.  Waits for
 * the stream twice (after the checks, and for the result).  The graph is
 * not modified. */
bbc_status bbc_update_delta(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                            const int32_t* adj, const int8_t* signs, int32_t n_updates, const int32_t* upd_u,
                            const int32_t* upd_v, const int8_t* upd_state, int64_t* delta, int64_t* per_update,
                            void* stream);

/* Caps the number of tasks one update of bbc_update_delta is split into
 * (default 4,096; cap 0 restores the default).  With a smaller cap an
 * update's pairs go to fewer, longer tasks: whole 1,024-entry chunks of
 * its w list against every chunk of its x list once its 256 x 256 tiles
 * outnumber the cap.  The result does not depend on it.  BBC_EINVAL for a
 * NULL context or a negative cap. */
bbc_status bbc_set_update_task_cap(bbc_ctx* ctx, int32_t cap);

/* Dense-block planner options.  Candidates are the vertices of degree >=
 * min_degree.  A block grows from a seed anchor: C starts as the seed's
 * candidate centres, then twice R = the candidate anchors linked to at
 * least member_frac of C and C = the candidate centres linked to at least
 * member_frac of R; it is kept when |R| >= min_anchors, |C| >= min_centres
 * and |edges of R x C| >= min_density * |R| * |C|.  R is capped at 16,384
 * and C at 65,535 vertices (the dense kernel's limits).  The search stops
 * after max_tries seeds in a row give no block. */
typedef struct {
    uint32_t struct_size; /* sizeof(bbc_plan_options) */
    int32_t side;         /* anchor side, BBC_SIDE_* as in bbc_options */
    int32_t min_degree;   /* 0 (default) = the tuned threshold of the graph's size class
                           * (bbc_autotune_blocks), else 256 */
    float member_frac;    /* default 0.3 */
    float min_density;    /* default 0.25 */
    int32_t min_anchors;  /* default 256 */
    int32_t min_centres;  /* default 64 */
    int32_t max_tries;    /* default 32 */
} bbc_plan_options;

/* Fills *opts with the defaults above. */
bbc_status bbc_plan_options_init(bbc_plan_options* opts);

/* Finds dense blocks for the int8 matrix-core path (bbc_options.blocks).
 * The paper gives no planner (its counting is blocks-free); any choice of
 * blocks keeps the count exact, so this heuristic only decides speed.
 *   n_u, n_v, n_edges, offsets, adj  the graph as in bbc_count (device;
 *                        signs are not needed)
 *   opts                 host or NULL (defaults)
 *   max_blocks           capacity of blocks
 *   blocks               host, max_blocks entries: receive the blocks, ids
 *                        pointing into `ids`
 *   ids                  device, ids_cap int32: every block's U ids, then
 *                        its V ids; the search stops before a block that
 *                        would not fit
 *   n_blocks             host: number of blocks written
 * The blocks are pairwise disjoint and valid input for bbc_count with the
 * same anchor side.  Synchronous.  Temporary device memory (about 17 bytes
 * per edge) is allocated and freed inside the call.  Errors: BBC_EINVAL
 * (null pointers, negative sizes, bad options), BBC_EOFFSETS, BBC_ERANGE,
 * BBC_ENOMEM, BBC_EDEVICE, BBC_ETOOBIG. */
bbc_status bbc_plan_blocks(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                           const int32_t* adj, const bbc_plan_options* opts, int32_t max_blocks,
                           bbc_dense_block* blocks, int32_t* ids, int64_t ids_cap, int32_t* n_blocks, void* stream);

/* Tunes the dense-block hybrid on a calibration graph (arguments as
 * bbc_count): for the planner's degree threshold min_degree in {128, 256,
 * 512, 1024} it plans blocks (bbc_plan_blocks, default options otherwise)
 * and counts with them at both int8 tiles (dense_tile 64 and 128), each
 * count equal to the sparse-only count (BBC_EDEVICE otherwise), and keeps
 * the pair with the smallest planning time plus end-to-end count time (best
 * of reps).  The pair is recorded under the graph's size class: planner
 * calls with min_degree 0 and counts with dense_tile 0 of that class use
 * it.  *chosen_plan and *chosen (host, may be NULL) receive options holding
 * it.  Allocates a temporary id buffer (4 bytes per vertex).  Errors: as
 * bbc_count and bbc_plan_blocks. */
bbc_status bbc_autotune_blocks(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                               const int32_t* adj, const int8_t* signs, int32_t reps, bbc_plan_options* chosen_plan,
                               bbc_options* chosen, void* stream);

/* Static strings; never NULL. */
const char* bbc_status_string(bbc_status s);
const char* bbc_last_error(const bbc_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* BBC_H */
