// C ABI of libbbc.so (declared in include/bbc.h): contexts, batch plans,
// scratch arenas, the launch sequence and error mapping.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/bbc.h"
#include "bbc_internal.h"

namespace bbc {
void launch_decode_single(const int32_t* off, const int32_t* adj, const int8_t* sg, int32_t n_u, int32_t n_v,
                          int64_t m, int s_is_u, int check_sign, DevStatus* st, uint32_t* ea, uint32_t* ec,
                          uint8_t* en, uint32_t* pay, hipStream_t s);
void launch_decode_batched(const int32_t* off_cat, const int32_t* adj_cat, const int8_t* sg_cat, const DevGraph* gr,
                           const int64_t* vstart, int32_t n_graphs, int64_t m, int check_sign, DevStatus* st,
                           uint32_t* ea, uint32_t* pay, hipStream_t s);
void launch_run_degrees(const uint32_t* key, int64_t m, uint32_t* first, uint32_t* deg, int64_t n,
                        const DevStatus* st, hipStream_t s);
void launch_move_lists(const uint32_t* key, const uint32_t* pay, int64_t m, const uint32_t* first,
                       const int32_t* rank, const uint32_t* aoff, int32_t* acent, uint8_t* aneg, uint32_t* apack,
                       const DevStatus* st, hipStream_t s);
void launch_hist(const uint32_t* ids, int64_t n, uint32_t* deg, int64_t n_bins, uint32_t* scratch,
                 int64_t scratch_words, const DevStatus* st, hipStream_t s);
void launch_side_wedges(const int32_t* off, int32_t n_u, const int32_t* adj, int64_t m, int32_t n_v, uint32_t* deg,
                        unsigned long long* out, hipStream_t s);
void dyn_check(const int32_t* uu, const int32_t* vv, const int8_t* ss, int32_t q, int32_t n_u, int32_t n_v,
               DevStatus* st, hipStream_t s);
void dyn_vkeys(const uint32_t* ea, const uint32_t* ec, const uint8_t* en, int64_t m, uint32_t* key, uint32_t* pay,
               hipStream_t s);
void dyn_ukeys(const uint32_t* vkey, const uint32_t* vpay, int64_t m, uint32_t* key, uint32_t* pay, hipStream_t s);
void dyn_dup(const uint32_t* ukey, const uint32_t* urow, int64_t m, DevStatus* st, hipStream_t s);
void dyn_key_init(const int32_t* a, int32_t q, uint32_t* key, hipStream_t s);
void dyn_gather(const int32_t* src, const uint32_t* idx, int32_t q, uint32_t* key, hipStream_t s);
void dyn_key64(const int32_t* hi, const int32_t* lo, const uint32_t* idx, int32_t q, unsigned long long* key,
               uint32_t* pos, int check, DevStatus* st, hipStream_t s);
void dyn_delta(const int32_t* uoff, const uint32_t* urow, const uint32_t* voff, const uint32_t* vrow,
               const unsigned long long* uv_key, const uint32_t* uv_pos, const unsigned long long* vu_key,
               const uint32_t* vu_pos, const int32_t* upd_u, const int32_t* upd_v, const int8_t* s_new, int8_t* s_old,
               unsigned long long* wsum, int32_t n_v, int32_t q, uint32_t* n_tasks, uint32_t* task_off,
               uint32_t* span, uint8_t* mode, uint32_t* partials, long long* per_update, int32_t task_cap,
               DevStatus* st, hipStream_t s);
void launch_anchor_graph(const DevGraph* gr, int32_t n_graphs, uint32_t* agid, hipStream_t s);
void launch_gather(const uint32_t* idx, const uint32_t* src, int64_t n, uint32_t* out, hipStream_t s);
void launch_ranks(const uint32_t* inv, const uint32_t* deg_s, int64_t n_s, int32_t* rank, uint32_t* adeg,
                  const uint32_t* agid, int32_t* agraph, hipStream_t s);
void launch_check_dup(const uint32_t* ckey, const uint32_t* packed, int64_t m, DevStatus* st, hipStream_t s);
void launch_work(const uint32_t* apack, const int32_t* acent, const int32_t* back, const uint32_t* coff, int64_t m,
                 int64_t n_s, unsigned long long* work, uint32_t* key, const uint32_t* aoff, const int32_t* agraph,
                 const int64_t* rank_end, uint32_t light_w, DevStatus* st, const HybridView& hv, hipStream_t s);
void launch_block_mark(const DevBlock* blocks, int32_t n_blocks, int64_t max_ids, int32_t n_s, int32_t n_c,
                       uint32_t* agrp, int32_t* cblk, int32_t* cidx, DevStatus* st, hipStream_t s);
void launch_block_cpos(const int32_t* cblk, int32_t n_c, const DevBlock* blocks, const uint32_t* coff,
                       const uint32_t* packed, int32_t* cpos, const DevStatus* st, hipStream_t s);
void launch_block_pack(const uint32_t* ablk1, int32_t r_first, int32_t n_s, const DevBlock* blocks,
                       const uint32_t* aoff, const int32_t* acent, const uint8_t* aneg, const int32_t* cblk,
                       const int32_t* cidx, int8_t* mats, const DevStatus* st, hipStream_t s);
void launch_dense(const DevBlock* blocks, const DevTile* tiles, int32_t n_tiles, const int8_t* mats, uint32_t* tabs,
                  DevStatus* st, int tile, hipStream_t s);
void launch_bidx(const uint32_t* ckey, const uint32_t* coff, const uint32_t* packed, int64_t m, int64_t n_c, int gs,
                 uint32_t* nb, uint32_t* ioff, uint32_t* idx, int2* meta, uint32_t* partials, const DevStatus* st,
                 hipStream_t s);
void pl_scatter(const uint32_t* key, const uint32_t* val, int64_t m, const uint32_t* off, int64_t n_keys,
                uint32_t* cur, uint32_t* out, hipStream_t s);
void pl_cand_deg(const uint32_t* ea, const uint32_t* ec, int64_t m, const uint32_t* deg_a, const uint32_t* deg_c,
                 uint32_t tau, uint32_t* cd, hipStream_t s);
void pl_seed(const uint32_t* off_a, const uint32_t* adj_a, uint32_t seed, const uint32_t* deg_c, uint32_t tau,
             const uint8_t* assigned_c, uint32_t* list, uint32_t* n, uint32_t cap, hipStream_t s);
void pl_count(const uint32_t* list, const uint32_t* n, uint32_t cap, const uint32_t* off, const uint32_t* adj,
              uint32_t* cnt, hipStream_t s);
void pl_select(uint32_t* cnt, int64_t n, const uint32_t* deg, uint32_t tau, const uint8_t* assigned,
               const uint32_t* n_other, uint32_t cap_other, float frac, uint32_t* out, uint32_t* n_out, uint32_t cap,
               unsigned long long* edges, hipStream_t s);
void pl_assign(const uint32_t* list, uint32_t n, uint8_t* assigned, hipStream_t s);
bool wedge_shape_ok(int band_words, int wg);
int wedge_block(int band_words, int wg, bool full);
int wedge_blocks_per_cu(int band_words, int wg, bool full);
int wedge_class_blocks_per_cu();
int wedge_class_pv_blocks_per_cu();
int wedge_class_band();
int wedge_band(int band_words, int wg, bool full);
int wedge_shape_count();
void wedge_shape(int i, int* wg, int* band_words);
void launch_wedge(int band_words, int wg, int grid, const uint32_t* aoff, const int32_t* acent, const uint8_t* aneg,
                  const int32_t* back, const uint32_t* coff, const uint32_t* packed, const uint32_t* bidx,
                  const int2* bmeta, const uint32_t* order,
                  int32_t n_s, DevStatus* st, unsigned long long* pv, const uint32_t* inv, int64_t anchor_base,
                  int64_t centre_base, int64_t n_centre, const int32_t* agraph, const int64_t* rank_end,
                  unsigned long long* gtotals, const HybridView& hv, int kind, int32_t bic_k,
                  const unsigned long long* bic_tab, int sched, int32_t queue_chunk, int32_t light_chunk,
                  hipStream_t s);
int wedge_light_max(int band_words, int wg);
int wedge_bic_blocks_per_cu();
void launch_choose_table(int32_t k, unsigned long long* tab, hipStream_t s);

__global__ void k_status_init(DevStatus* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->flags = 0;
        st->bad_offset = st->bad_range = st->bad_sign = st->bad_dup = st->bad_block = st->bad_update = INT64_MAX;
        st->total = 0;
        for (int k = 0; k < 6; ++k) st->cls[k] = 0;
        st->wedges = 0;
        st->walked = 0;
        st->bands = 0;
        st->queue = 0;
        st->queue2 = 0;
        st->n_light = 0;
    }
}
// One entry of the tuning table: the fastest wedge-kernel shape measured
// for a size class (bit lengths of n_S and of m / n_S).
struct TuneEntry {
    int32_t ns_bits, deg_bits;
    int32_t band_words, wg_size, wg_per_cu;  // band_words = 0: shape not tuned
    int32_t schedule;       // BBC_SCHED_*
    int32_t queue_chunk;    // 0: not tuned (1)
    int32_t wave_max_work;  // 0: the shape's largest, -1: no wave regime
    int32_t min_degree;     // planner threshold; 0: not tuned (256)
    int32_t dense_tile;     // int8 matrix tile; 0: not tuned (128)
    float ms;
};
}  // namespace bbc

using namespace bbc;

struct bbc_ctx {
    int device = 0;
    int n_cu = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    DevStatus* st_dev = nullptr;
    DevStatus* st_host = nullptr;  // pinned
    hipEvent_t ev[6] = {};  // [checks, build, count, start, dense start, dense end]
    bbc_stats stats = {};
    std::string err;
    std::vector<TuneEntry> tune;
    int32_t update_task_cap = 0;  // bbc_update_delta: tasks per update (0: 4096)
    int64_t limit = 0;            // scratch_limit of the call in progress (0: none)
    char* fixed = nullptr;        // device address of this device's fixed scratch (bbc_count_noalloc)
    hipError_t fixed_err = hipSuccess;
};

struct bbc_batch_plan {
    bbc_ctx* ctx = nullptr;
    char* arena = nullptr;
    DevStatus* st_dev = nullptr;
    DevStatus* st_host = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// Fixed scratch of bbc_count_noalloc: a file-scope device array, one copy
// per GPU, held until the process ends.  Host code never uses the array's
// name as an address (it names a host-side stand-in): the device address
// comes from hipGetSymbolAddress, looked up once per device with that device
// current, and only that address reaches kernels.
constexpr size_t kFixedScratchBytes = BBC_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) char scratch[kFixedScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_fixed_mu;
char* g_fixed_ptr[kMaxDevices] = {};

// Device address of the fixed scratch on `device`, which must be current.
hipError_t fixed_scratch(int device, char** out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_fixed_mu);
    if (!g_fixed_ptr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_fixed_ptr[device] = static_cast<char*>(p);
    }
    *out = g_fixed_ptr[device];
    return hipSuccess;
}

}  // namespace

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Bump allocator over an arena (256-byte aligned pieces); with a null base
// it only measures.
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(char* b) : base(b) {}
    template <class T>
    T* take(int64_t n) {
        size_t bytes = ((size_t)(n > 0 ? n : 1) * sizeof(T) + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + used) : nullptr;
        used += bytes;
        return p;
    }
};

int bits_for(uint64_t x) {
    int b = 1;
    while (b < 64 && (x >> b)) ++b;
    return b;
}

bbc_status fail(bbc_ctx* ctx, bbc_status s, const std::string& msg) {
    if (ctx) ctx->err = msg;
    return s;
}

bbc_status hip_fail(bbc_ctx* ctx, hipError_t e, const char* where) {
    return fail(ctx, BBC_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_OR_FAIL(call)                                      \
    do {                                                       \
        hipError_t _e = (call);                                \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #call); \
    } while (0)

// Everything one pass of the pipeline needs (a single graph or a batch).
struct Job {
    bool batched = false;
    // single graph (CSR over U) or concatenated batch arrays
    const int32_t *off = nullptr, *adj = nullptr;
    const int8_t* sg = nullptr;
    int32_t n_u = 0, n_v = 0;
    bool s_is_u = false;
    bool all_su = false;  // batch: every graph's anchors are its U rows (edges already grouped by anchor)
    unsigned long long* pv = nullptr;  // single graph: per-vertex output or null
    int32_t n_graphs = 0;              // batch
    unsigned long long* totals = nullptr;
    int64_t m = 0, n_s = 0, n_c = 0;
    uint32_t checks = BBC_CHECK_ALL;
    int band_words = 0, wg_size = 0, grid = 0;
    int schedule = BBC_SCHED_DYNAMIC;
    bool tuned = false;  // shape taken from the tuning table
    int32_t queue_chunk = 1;    // workgroup-regime anchors per queue pop
    int32_t light_w = 0;        // wave regime: anchors with at most this many wedges (0: none)
    int32_t light_chunk = 64;   // wave-regime anchors per queue pop
    int32_t dense_tile = 128;   // int8 matrix output tile (64 or 128)
    bool classes = false;  // the six sign-pattern classes instead of the total
    int32_t bic_k = 0;     // > 0: balanced (2,k)-bicliques instead of the total
    // dense blocks (single graph only)
    int32_t n_blocks = 0, n_tiles = 0;
    int64_t r_first = 0;  // first rank of the block anchors (they sit at the top)
    int64_t max_ids = 0, mat_bytes = 0, tab_words = 0;
    uint64_t dense_ops = 0;
};

// All device buffers of one pass, carved from an arena in a fixed order.
struct Plan {
    uint32_t *deg_s, *deg_c;
    uint32_t *rk_ka, *rk_kb, *rk_va, *rk_vb;  // rank sort
    int32_t* rank;
    uint32_t *adeg, *aoff, *coff;
    int32_t* acent;
    uint8_t* aneg;
    uint32_t *apack, *k_a, *k_b, *v0_a, *v0_b, *v1_a, *v1_b;
    int32_t* back;
    uint32_t *wkey, *ord_a, *ord_b, *ord_va, *ord_vb;
    unsigned long long* work;  // per-anchor work (wedges walked)
    uint32_t *hist, *hist_scan, *partials;
    uint32_t* agid;    // batch: graph of each anchor id
    int32_t* agraph;   // batch: graph of each rank
    DevGraph* graphs;  // batch descriptors
    int64_t *vstart, *rank_end;
    uint32_t *agrp, *ablk1;  // dense blocks: block + 1 per anchor id / per rank
    int32_t *cblk, *cidx, *cpos;
    DevBlock* dblocks;
    DevTile* dtiles;
    int8_t* mats;
    uint32_t* tabs;
    uint32_t *bnb, *bioff, *bidx;  // band-boundary index of the centre lists
    int2* bmeta;
    unsigned long long* bic_tab;  // C(x, k) for x < 256 (biclique mode)

    size_t carve(char* base, const Job& J) {
        Carve c(base);
        const int64_t m = J.m, n_s = J.n_s, n_c = J.n_c;
        int64_t nmax = m;
        if (n_s + 1 > nmax) nmax = n_s + 1;
        if (n_c + 1 > nmax) nmax = n_c + 1;
        deg_s = c.take<uint32_t>(n_s);
        deg_c = c.take<uint32_t>(n_c);
        rk_ka = c.take<uint32_t>(n_s);
        rk_kb = c.take<uint32_t>(n_s);
        rk_va = c.take<uint32_t>(n_s);
        rk_vb = c.take<uint32_t>(n_s);
        rank = c.take<int32_t>(n_s);
        adeg = c.take<uint32_t>(n_s + 1);
        aoff = c.take<uint32_t>(n_s + 1);
        coff = c.take<uint32_t>(n_c + 1);
        acent = c.take<int32_t>(m);
        aneg = c.take<uint8_t>(m);
        apack = c.take<uint32_t>(m);
        k_a = c.take<uint32_t>(m);
        k_b = c.take<uint32_t>(m);
        v0_a = c.take<uint32_t>(m);
        v0_b = c.take<uint32_t>(m);
        v1_a = c.take<uint32_t>(m);
        v1_b = c.take<uint32_t>(m);
        back = c.take<int32_t>(m);
        wkey = c.take<uint32_t>(n_s);
        work = c.take<unsigned long long>(n_s);
        ord_a = c.take<uint32_t>(n_s);
        ord_b = c.take<uint32_t>(n_s);
        ord_va = c.take<uint32_t>(n_s);
        ord_vb = c.take<uint32_t>(n_s);
        int64_t hs = (int64_t)radix_hist_size(nmax);
        hist = c.take<uint32_t>(hs);
        hist_scan = c.take<uint32_t>(hs + 1);
        partials = c.take<uint32_t>((int64_t)scan_partials_size(hs + nmax + 8));
        agid = c.take<uint32_t>(J.batched ? n_s : 0);
        agraph = c.take<int32_t>(J.batched ? n_s : 0);
        graphs = c.take<DevGraph>(J.n_graphs);
        vstart = c.take<int64_t>(J.n_graphs + 1);
        rank_end = c.take<int64_t>(J.n_graphs + 1);
        const bool hy = J.n_blocks > 0;
        agrp = c.take<uint32_t>(hy ? n_s : 0);
        ablk1 = c.take<uint32_t>(hy ? n_s : 0);
        cblk = c.take<int32_t>(hy ? n_c : 0);
        cidx = c.take<int32_t>(hy ? n_c : 0);
        cpos = c.take<int32_t>(hy ? n_c : 0);
        dblocks = c.take<DevBlock>(J.n_blocks);
        dtiles = c.take<DevTile>(J.n_tiles);
        mats = c.take<int8_t>(J.mat_bytes);
        tabs = c.take<uint32_t>(J.tab_words);
        const bool idx = J.pv == nullptr;
        bnb = c.take<uint32_t>(idx ? n_c : 0);
        bioff = c.take<uint32_t>(idx ? n_c + 1 : 0);
        bidx = c.take<uint32_t>(idx ? m : 0);
        bmeta = c.take<int2>(idx ? n_c : 0);
        bic_tab = c.take<unsigned long long>(J.bic_k > 0 ? 512 : 0);
        return c.used;
    }
};

// Queues the whole pipeline on stream s: kernel launches only (no host
// waits, copies or allocations), so it can be captured in a graph.
// ev (optional) receives [after checks, after build, after count].
void enqueue(const Job& J, Plan& P, DevStatus* st, hipStream_t s, hipEvent_t* ev) {
    const int64_t m = J.m, n_s = J.n_s, n_c = J.n_c;
    const bool hybrid = J.n_blocks > 0;
    const int check_sign = (J.checks & BBC_CHECK_SIGNS) ? 1 : 0;
    // decoded edges (anchor id; centre id | negative << 31) in buffers that
    // are free until the centre sort
    uint32_t* ea = P.v1_a;
    uint32_t* pay = P.v1_b;
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, s, st);
    if (J.batched)
        launch_decode_batched(J.off, J.adj, J.sg, P.graphs, P.vstart, J.n_graphs, m, check_sign, st, ea, pay, s);
    else
        launch_decode_single(J.off, J.adj, J.sg, J.n_u, J.n_v, m, J.s_is_u ? 1 : 0, check_sign, st, ea, nullptr,
                             nullptr, pay, s);
    if (hybrid) {  // block of every block vertex; ids checked in range, distinct and disjoint
        fill_u32(P.agrp, 0u, n_s, s);
        fill_u32((uint32_t*)P.cblk, 0xffffffffu, n_c, s);
        launch_block_mark(P.dblocks, J.n_blocks, J.max_ids, (int32_t)n_s, (int32_t)n_c, P.agrp, P.cblk, P.cidx, st,
                          s);
    }
    if (ev) (void)hipEventRecord(ev[0], s);

    // edges grouped by anchor by a stable sort on the anchor id (CSR rows
    // are grouped already when the anchors are U): each anchor's run gives
    // its degree and its first position (held in the work array, which is
    // free until the schedule)
    const uint32_t *sk = ea, *sp = pay;
    if (!(J.batched ? J.all_su : J.s_is_u))
        radix_sort(ea, P.k_a, P.k_b, pay, P.v0_a, P.v0_b, nullptr, nullptr, nullptr, m,
                   bits_for(n_s > 0 ? (uint64_t)(n_s - 1) : 0), P.hist, P.hist_scan, P.partials, s, &sk, &sp,
                   nullptr);
    uint32_t* afirst = reinterpret_cast<uint32_t*>(P.work);
    launch_run_degrees(sk, m, afirst, P.deg_s, n_s, st, s);

    // ranks (Definition 6: degree, then id; ascending; a batch orders by
    // graph first)
    const uint32_t *rk_k = nullptr, *inv = nullptr;
    radix_sort(P.deg_s, P.rk_ka, P.rk_kb, nullptr, nullptr, nullptr, nullptr, P.rk_va, P.rk_vb, n_s,
               bits_for((uint64_t)(m > 0 ? m : 1)), P.hist, P.hist_scan, P.partials, s, &rk_k, nullptr, &inv);
    if (J.batched && n_s > 0) {
        launch_anchor_graph(P.graphs, J.n_graphs, P.agid, s);
        launch_gather(inv, P.agid, n_s, P.wkey, s);
        const uint32_t* gk = nullptr;
        radix_sort(P.wkey, P.ord_a, P.ord_b, nullptr, nullptr, nullptr, inv, P.ord_va, P.ord_vb, n_s,
                   bits_for((uint64_t)(J.n_graphs > 1 ? J.n_graphs - 1 : 1)), P.hist, P.hist_scan, P.partials, s,
                   &gk, nullptr, &inv);
    }
    if (hybrid && n_s > 0) {  // block anchors last, block by block: ranks (block, degree, id)
        launch_gather(inv, P.agrp, n_s, P.wkey, s);
        const uint32_t* gk = nullptr;
        radix_sort(P.wkey, P.ord_a, P.ord_b, nullptr, nullptr, nullptr, inv, P.ord_va, P.ord_vb, n_s,
                   bits_for((uint64_t)J.n_blocks), P.hist, P.hist_scan, P.partials, s, &gk, nullptr, &inv);
        launch_gather(inv, P.agrp, n_s, P.ablk1, s);
    }
    launch_ranks(inv, P.deg_s, n_s, P.rank, P.adeg, J.batched ? P.agid : nullptr, J.batched ? P.agraph : nullptr, s);
    scan_exclusive_u32(P.adeg, P.aoff, n_s, P.partials, s);

    // anchor lists in rank order (each anchor's run moved as a whole), then
    // centre lists by a stable sort on the centre id of the rank-ordered
    // anchor entries (each centre list comes out rank-sorted); the sort's
    // last pass writes back[] (where each anchor entry went)
    launch_move_lists(sk, sp, m, afirst, P.rank, P.aoff, P.acent, P.aneg, P.apack, st, s);
    const uint32_t *ckey = nullptr, *packed = nullptr;
    radix_sort((const uint32_t*)P.acent, P.k_a, P.k_b, P.apack, P.v0_a, P.v0_b, nullptr, P.v1_a, P.v1_b, m,
               bits_for(n_c > 0 ? (uint64_t)(n_c - 1) : 0), P.hist, P.hist_scan, P.partials, s, &ckey, &packed,
               nullptr, P.back);
    // centre degrees from the runs of the sorted centre ids (coff holds the
    // runs' first positions until the scan)
    launch_run_degrees(ckey, m, P.coff, P.deg_c, n_c, st, s);
    scan_exclusive_u32(P.deg_c, P.coff, n_c, P.partials, s);
    if (J.checks & BBC_CHECK_DUPLICATES) launch_check_dup(ckey, packed, m, st, s);
    if (!J.pv) {  // band ends of the count-mode wedge kernel fall on multiples of its granule
        int gs = 0;
        if (J.classes) {  // the narrowest class band holds a quarter of the words
            while ((4 << gs) < wedge_class_band()) ++gs;
        } else {
            while ((2 << gs) < wedge_band(J.band_words, J.wg_size, false)) ++gs;
        }
        launch_bidx(ckey, P.coff, packed, m, n_c, gs, P.bnb, P.bioff, P.bidx, P.bmeta, P.partials, st, s);
    }
    HybridView hv{nullptr, nullptr, nullptr, nullptr, nullptr};
    if (hybrid) {
        hv = HybridView{P.ablk1, P.cblk, P.cpos, P.dblocks, P.tabs};
        launch_block_cpos(P.cblk, (int32_t)n_c, P.dblocks, P.coff, packed, P.cpos, st, s);
        if (J.n_tiles > 0) {
            fill_bytes(P.mats, J.mat_bytes, s);
            launch_block_pack(P.ablk1, (int32_t)J.r_first, (int32_t)n_s, P.dblocks, P.aoff, P.acent, P.aneg, P.cblk,
                              P.cidx, P.mats, st, s);
        }
    }

    // schedule: anchors by descending work
    launch_work(P.apack, P.acent, P.back, P.coff, m, n_s, P.work, P.wkey, P.aoff, J.batched ? P.agraph : nullptr,
                J.batched ? P.rank_end : nullptr, (uint32_t)J.light_w, st, hv, s);
    const uint32_t *ok = nullptr, *order = nullptr;
    radix_sort(P.wkey, P.ord_a, P.ord_b, nullptr, nullptr, nullptr, nullptr, P.ord_va, P.ord_vb, n_s, 32, P.hist,
               P.hist_scan, P.partials, s, &ok, nullptr, &order);
    if (ev) (void)hipEventRecord(ev[1], s);

    if (J.pv) fill_bytes(J.pv, ((int64_t)J.n_u + J.n_v) * 8 * (J.classes ? 6 : 1), s);
    if (J.batched) fill_bytes(J.totals, (int64_t)J.n_graphs * 8, s);
    if (hybrid) {  // dense block products (int8 matrix cores), then the sparse walk reads their tables
        if (ev) (void)hipEventRecord(ev[4], s);
        launch_dense(P.dblocks, P.dtiles, J.n_tiles, P.mats, P.tabs, st, J.dense_tile, s);
        if (ev) (void)hipEventRecord(ev[5], s);
    }
    if (J.bic_k > 0) launch_choose_table(J.bic_k, P.bic_tab, s);
    if (n_s >= 2 && m > 0)
        launch_wedge(J.band_words, J.wg_size, J.grid, P.aoff, P.acent, P.aneg, P.back, P.coff, packed, P.bidx,
                     P.bmeta, order,
                     (int32_t)n_s, st, J.pv, inv, J.s_is_u ? 0 : J.n_u, J.s_is_u ? J.n_u : 0, n_c,
                     J.batched ? P.agraph : nullptr, J.batched ? P.rank_end : nullptr,
                     J.batched ? J.totals : nullptr, hv,
                     J.classes ? kWedgeClasses : J.bic_k > 0 ? kWedgeBicliques : kWedgeCount, J.bic_k, P.bic_tab,
                     J.schedule, J.queue_chunk, J.light_chunk, s);
    if (ev) (void)hipEventRecord(ev[2], s);
}

bbc_status grow(bbc_ctx* ctx, char** arena, size_t* have, size_t bytes) {
    if (ctx->limit > 0 && bytes > (size_t)ctx->limit)
        return fail(ctx, BBC_ENOMEM, "the call needs " + std::to_string(bytes) + " bytes of scratch, above its "
                                     "scratch_limit of " + std::to_string(ctx->limit));
    if (bytes <= *have) return BBC_OK;
    if (*arena) {
        (void)hipFree(*arena);
        *arena = nullptr;
        *have = 0;
    }
    size_t want = bytes + bytes / 8 + (1u << 20);
    if (ctx->limit > 0 && want > (size_t)ctx->limit) want = (size_t)ctx->limit;  // >= bytes
    if (hipMalloc((void**)arena, want) != hipSuccess) {
        *arena = nullptr;
        (void)hipGetLastError();
        return fail(ctx, BBC_ENOMEM, "scratch allocation of " + std::to_string(want) + " bytes failed");
    }
    *have = want;
    return BBC_OK;
}

bbc_status read_options(bbc_ctx* ctx, const bbc_options* in, bbc_options* o) {
    bbc_options_init(o);
    ctx->limit = 0;
    if (in) {
        if (in->struct_size != sizeof(bbc_options)) return fail(ctx, BBC_EINVAL, "bbc_options.struct_size");
        *o = *in;
    }
    if (o->scratch_limit < 0) return fail(ctx, BBC_EINVAL, "negative scratch_limit");
    ctx->limit = o->scratch_limit;
    if (o->side < BBC_SIDE_AUTO || o->side > BBC_SIDE_MIN_WEDGES) return fail(ctx, BBC_EINVAL, "bad side option");
    if (!wedge_shape_ok(o->band_words, o->wg_size))
        return fail(ctx, BBC_EINVAL, "no wedge kernel instance for this band_words / wg_size");
    if (o->wg_per_cu < 0) return fail(ctx, BBC_EINVAL, "negative wg_per_cu");
    if (o->schedule != BBC_SCHED_DYNAMIC && o->schedule != BBC_SCHED_STATIC)
        return fail(ctx, BBC_EINVAL, "bad schedule option");
    if (o->n_blocks < 0 || (o->n_blocks > 0 && !o->blocks)) return fail(ctx, BBC_EINVAL, "bad dense block list");
    if (o->queue_chunk < 0 || o->queue_chunk > 65536) return fail(ctx, BBC_EINVAL, "queue_chunk outside [0, 65536]");
    if (o->wave_max_work < -1) return fail(ctx, BBC_EINVAL, "wave_max_work below -1");
    if (o->dense_tile != 0 && o->dense_tile != 64 && o->dense_tile != 128)
        return fail(ctx, BBC_EINVAL, "dense_tile must be 0, 64 or 128");
    return BBC_OK;
}

// Regime knobs of a count-mode job (no wave regime with per-vertex output).
void set_regimes(Job& J, const bbc_options& o, bool full) {
    J.dense_tile = o.dense_tile ? o.dense_tile : 128;
    J.queue_chunk = o.queue_chunk > 0 ? o.queue_chunk : 1;
    const int lmax = wedge_light_max(o.band_words, o.wg_size);
    J.light_w = (full || o.wave_max_work < 0) ? 0 : o.wave_max_work == 0 ? lmax : std::min(o.wave_max_work, lmax);
}

bool side_is_u(int side, int32_t n_u, int32_t n_v) { return side == BBC_SIDE_U || (side == BBC_SIDE_AUTO && n_u < n_v); }

// The anchor side of a single-graph call.  BBC_SIDE_MIN_WEDGES measures
// both choices on the device (sum of C(deg, 2) over the centre side) and
// takes the one with fewer wedges, the default rule breaking a tie; it
// waits for the stream once.
// The measurement runs in `buf` (cap bytes) when given, else in the
// context's arena (grown to fit).
bbc_status resolve_side(bbc_ctx* ctx, int side, int32_t n_u, int32_t n_v, int64_t m, const int32_t* off,
                        const int32_t* adj, hipStream_t s, bool* su, char* buf = nullptr, size_t cap = 0) {
    if (side != BBC_SIDE_MIN_WEDGES) {
        *su = side_is_u(side, n_u, n_v);
        return BBC_OK;
    }
    const size_t bytes = 32 + (size_t)n_v * 4;
    if (buf) {
        if (bytes > cap) return fail(ctx, BBC_ENOMEM, "side measurement exceeds the fixed scratch");
    } else {
        bbc_status rc = grow(ctx, &ctx->arena, &ctx->arena_bytes, bytes);
        if (rc != BBC_OK) return rc;
        buf = ctx->arena;
    }
    unsigned long long* out = reinterpret_cast<unsigned long long*>(buf);
    launch_side_wedges(off, n_u, adj, m, n_v, reinterpret_cast<uint32_t*>(buf + 32), out, s);
    unsigned long long w[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(w, out, sizeof(w), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(ctx, e, "side choice");
    // w[0]: wedges with anchors on V (centres U); w[1]: anchors on U
    *su = w[1] < w[0] || (w[1] == w[0] && side_is_u(BBC_SIDE_AUTO, n_u, n_v));
    return BBC_OK;
}

void tune_class(int64_t n_s, int64_t m, int32_t* ns_bits, int32_t* deg_bits) {
    *ns_bits = bits_for((uint64_t)(n_s > 0 ? n_s : 0));
    *deg_bits = bits_for((uint64_t)(m / (n_s > 0 ? n_s : 1)));
}

const TuneEntry* tune_find(const bbc_ctx* ctx, int64_t n_s, int64_t m) {
    int32_t a, b;
    tune_class(n_s, m, &a, &b);
    for (const TuneEntry& e : ctx->tune)
        if (e.ns_bits == a && e.deg_bits == b) return &e;
    return nullptr;
}

// Fills what the options leave open from the tuning table: the kernel
// shape, grid and schedule (when none of them is fixed), the queue chunk
// and wave-regime threshold (when 0) and the dense tile (when 0).  Returns
// whether the shape came from the table.
bool apply_tuning(const bbc_ctx* ctx, bbc_options& o, int64_t n_s, int64_t m, bool full) {
    if (o.no_tuning || full) return false;
    const TuneEntry* e = tune_find(ctx, n_s, m);
    if (!e) return false;
    if (o.dense_tile == 0) o.dense_tile = e->dense_tile;
    if (o.band_words || o.wg_size || o.wg_per_cu || o.schedule || e->band_words == 0) return false;
    o.band_words = e->band_words;
    o.wg_size = e->wg_size;
    o.wg_per_cu = e->wg_per_cu;
    o.schedule = e->schedule;
    if (o.queue_chunk == 0) o.queue_chunk = e->queue_chunk;
    if (o.wave_max_work == 0) o.wave_max_work = e->wave_max_work;
    return true;
}

void tune_store(bbc_ctx* ctx, const TuneEntry& e) {
    for (TuneEntry& x : ctx->tune)
        if (x.ns_bits == e.ns_bits && x.deg_bits == e.deg_bits) {
            x = e;
            return;
        }
    ctx->tune.push_back(e);
}

// The entry of a size class, created empty (nothing tuned) if absent.
TuneEntry& tune_slot(bbc_ctx* ctx, int64_t n_s, int64_t m) {
    int32_t a, b;
    tune_class(n_s, m, &a, &b);
    for (TuneEntry& x : ctx->tune)
        if (x.ns_bits == a && x.deg_bits == b) return x;
    ctx->tune.push_back(TuneEntry{a, b, 0, 0, 0, 0, 0, 0, 0, 0, 0.f});
    return ctx->tune.back();
}

// Validates a batch on the host and fills the job and device descriptors.
bbc_status batch_job(bbc_ctx* ctx, int32_t n_graphs, const bbc_graph_desc* d, const int32_t* off_cat,
                     const int32_t* adj_cat, const int8_t* sg_cat, uint64_t* totals, const bbc_options& o_in, Job& J,
                     std::vector<DevGraph>& dg, std::vector<int64_t>& vstart, std::vector<int64_t>& rend) {
    if (n_graphs < 0) return fail(ctx, BBC_EINVAL, "negative n_graphs");
    bbc_options o = o_in;
    if (o.n_blocks > 0) return fail(ctx, BBC_EINVAL, "dense blocks apply to bbc_count only");
    if (o.side == BBC_SIDE_MIN_WEDGES)
        return fail(ctx, BBC_EINVAL, "BBC_SIDE_MIN_WEDGES applies to single-graph calls only");
    if (n_graphs > 0 && (!d || !off_cat || !totals)) return fail(ctx, BBC_EINVAL, "batch pointer is NULL");
    dg.resize((size_t)n_graphs);
    vstart.assign((size_t)n_graphs + 1, 0);
    rend.assign((size_t)n_graphs + 1, 0);
    int64_t m = 0, ns = 0, nc = 0;
    for (int32_t g = 0; g < n_graphs; ++g) {
        const bbc_graph_desc& x = d[g];
        if (x.n_u < 0 || x.n_v < 0 || x.n_edges < 0 || x.off_base < 0 || x.edge_base < 0)
            return fail(ctx, BBC_EINVAL, "graph " + std::to_string(g) + ": negative size or base");
        if (x.n_edges > 0 && (!adj_cat || !sg_cat)) return fail(ctx, BBC_EINVAL, "batch edge pointer is NULL");
        const bool su = side_is_u(o.side, x.n_u, x.n_v);
        DevGraph& y = dg[g];
        y.off_base = x.off_base;
        y.edge_base = x.edge_base;
        y.n_edges = x.n_edges;
        y.anchor_base = ns;
        y.centre_base = nc;
        y.n_u = x.n_u;
        y.n_v = x.n_v;
        y.s_is_u = su ? 1 : 0;
        y.pad = 0;
        vstart[g] = m;
        rend[g] = ns;
        m += x.n_edges;
        ns += su ? x.n_u : x.n_v;
        nc += su ? x.n_v : x.n_u;
        if (m > INT32_MAX || ns + nc > INT32_MAX)
            return fail(ctx, BBC_ETOOBIG, "batch exceeds INT32_MAX edges or vertices");
    }
    vstart[(size_t)n_graphs] = m;
    rend[(size_t)n_graphs] = ns;
    J.all_su = true;
    for (const DevGraph& y : dg) J.all_su = J.all_su && y.s_is_u;
    J.batched = true;
    J.off = off_cat;
    J.adj = adj_cat;
    J.sg = sg_cat;
    J.n_graphs = n_graphs;
    J.totals = (unsigned long long*)totals;
    J.m = m;
    J.n_s = ns;
    J.n_c = nc;
    J.checks = o.checks;
    J.tuned = apply_tuning(ctx, o, ns, m, false);
    J.band_words = o.band_words;
    J.schedule = o.schedule;
    J.wg_size = o.wg_size;
    set_regimes(J, o, false);
    J.grid = ctx->n_cu * (o.wg_per_cu > 0 ? o.wg_per_cu : wedge_blocks_per_cu(o.band_words, o.wg_size, false));
    return BBC_OK;
}

// Validates the dense blocks on the host (sizes, pointers) and lays out their
// device data; ids are checked on the device.  Block anchors take the top
// ranks, block by block.
bbc_status block_job(bbc_ctx* ctx, const bbc_options& o, Job& J, std::vector<DevBlock>& db,
                     std::vector<DevTile>& dt) {
    constexpr int32_t kMaxAnchors = 16384, kMaxCentres = 65535, kK = 64;
    const int32_t kTile = J.dense_tile;
    J.n_blocks = o.n_blocks;
    db.resize((size_t)o.n_blocks);
    int64_t n_anchors = 0;
    for (int32_t i = 0; i < o.n_blocks; ++i) {
        const bbc_dense_block& b = o.blocks[i];
        const std::string tag = "dense block " + std::to_string(i) + ": ";
        if (b.n_u_ids < 0 || b.n_v_ids < 0) return fail(ctx, BBC_EINVAL, tag + "negative id count");
        if ((b.n_u_ids > 0 && !b.u_ids) || (b.n_v_ids > 0 && !b.v_ids)) return fail(ctx, BBC_EINVAL, tag + "NULL ids");
        const int32_t na = J.s_is_u ? b.n_u_ids : b.n_v_ids, nk = J.s_is_u ? b.n_v_ids : b.n_u_ids;
        if (na > kMaxAnchors || nk > kMaxCentres)
            return fail(ctx, BBC_EINVAL, tag + "more than 16384 anchor-side or 65535 centre-side ids");
        DevBlock& d = db[(size_t)i];
        d.n_r = d.n_aid = na;
        d.n_k = d.n_cid = nk;
        d.aid = J.s_is_u ? b.u_ids : b.v_ids;
        d.cid = J.s_is_u ? b.v_ids : b.u_ids;
        d.rpad = (na + kTile - 1) / kTile * kTile;
        d.kpad = (nk + kK - 1) / kK * kK;
        n_anchors += na;
        if (na + nk > J.max_ids) J.max_ids = na + nk;
    }
    if (n_anchors > J.n_s) return fail(ctx, BBC_EINVAL, "dense blocks list more anchor-side ids than there are vertices");
    J.r_first = J.n_s - n_anchors;
    int64_t rank0 = J.r_first;
    for (int32_t i = 0; i < o.n_blocks; ++i) {
        DevBlock& d = db[(size_t)i];
        d.rank0 = rank0;
        rank0 += d.n_r;
        d.mat_off = d.tab_off = 0;
        if (d.n_r < 2 || d.n_k < 1) continue;  // no anchor pair: no dense wedge
        d.mat_off = J.mat_bytes;
        d.tab_off = J.tab_words;
        J.mat_bytes += (int64_t)d.rpad * d.kpad;
        J.tab_words += (int64_t)d.rpad * d.rpad;
        J.dense_ops += 2ull * (uint64_t)d.n_r * (uint64_t)(d.n_r - 1) * (uint64_t)d.n_k;
        const int32_t t = d.rpad / kTile;
        for (int32_t ti = 0; ti < t; ++ti)
            for (int32_t tj = ti; tj < t; ++tj) dt.push_back(DevTile{i, ti, tj, 0});
    }
    J.n_tiles = (int32_t)dt.size();
    return BBC_OK;
}

// Maps the device status of a finished pass to a return code.
bbc_status status_result(bbc_ctx* ctx, const DevStatus& h) {
    char buf[160];
    if (h.flags & (kBadUpdRange | kBadUpdSign | kBadUpdDup)) {
        const bbc_status st = (h.flags & kBadUpdRange) ? BBC_ERANGE : (h.flags & kBadUpdSign) ? BBC_ESIGN : BBC_EINVAL;
        snprintf(buf, sizeof buf, "update batch: %s at update %lld",
                 (h.flags & kBadUpdRange) ? "id out of range" : (h.flags & kBadUpdSign) ? "state not in {-1, 0, +1}"
                                                                                       : "repeated pair",
                 (long long)h.bad_update);
        return fail(ctx, st, buf);
    }
    if (h.flags & kBadOffsets) {
        snprintf(buf, sizeof buf, "offsets invalid at index %lld", (long long)h.bad_offset);
        return fail(ctx, BBC_EOFFSETS, buf);
    }
    if (h.flags & kBadRange) {
        snprintf(buf, sizeof buf, "adjacency id out of [0, n_v) at edge %lld", (long long)h.bad_range);
        return fail(ctx, BBC_ERANGE, buf);
    }
    if (h.flags & kBadSign) {
        snprintf(buf, sizeof buf, "sign not +1/-1 at edge %lld", (long long)h.bad_sign);
        return fail(ctx, BBC_ESIGN, buf);
    }
    if (h.flags & kBadDup) {
        snprintf(buf, sizeof buf, "repeated (u, v) pair at centre-list position %lld", (long long)h.bad_dup);
        return fail(ctx, BBC_EDUP, buf);
    }
    if (h.flags & kBadBlocks) {
        snprintf(buf, sizeof buf,
                 "dense block %lld: id at position %lld (anchor-side ids first) is out of range, repeated or in "
                 "another block",
                 (long long)(h.bad_block >> 32), (long long)(h.bad_block & 0xffffffffll));
        return fail(ctx, BBC_EINVAL, buf);
    }
    return BBC_OK;
}

void fill_stats(bbc_ctx* ctx, const Job& J, const DevStatus& h, int block) {
    bbc_stats& S = ctx->stats;
    memset(&S, 0, sizeof S);
    S.struct_size = sizeof(bbc_stats);
    S.side = J.batched ? BBC_SIDE_AUTO : (J.s_is_u ? BBC_SIDE_U : BBC_SIDE_V);
    S.n_anchor = (int32_t)J.n_s;
    S.n_centre = (int32_t)J.n_c;
    S.n_edges = J.m;
    S.wedges = h.walked;
    S.wedges_all = h.wedges;
    S.bands = h.bands;
    S.n_blocks = J.n_blocks;
    S.dense_ops = J.dense_ops;
    S.grid = J.grid;
    S.block = block;
    S.band_words = wedge_band(J.band_words, J.wg_size, J.pv != nullptr);
    S.tuned = J.tuned ? 1 : 0;
    S.schedule = J.schedule;
}

bbc_status timed_stats(bbc_ctx* ctx) {
    bbc_stats& S = ctx->stats;
    HIP_OR_FAIL(hipEventElapsedTime(&S.ms_checks, ctx->ev[3], ctx->ev[0]));
    HIP_OR_FAIL(hipEventElapsedTime(&S.ms_build, ctx->ev[0], ctx->ev[1]));
    HIP_OR_FAIL(hipEventElapsedTime(&S.ms_count, ctx->ev[1], ctx->ev[2]));
    HIP_OR_FAIL(hipEventElapsedTime(&S.ms_total, ctx->ev[3], ctx->ev[2]));
    if (S.n_blocks > 0) HIP_OR_FAIL(hipEventElapsedTime(&S.ms_dense, ctx->ev[4], ctx->ev[5]));
    return BBC_OK;
}

// Runs a job whose buffers are carved from `arena` (large enough for it) on
// stream s and waits for its status.
bbc_status run_planned(bbc_ctx* ctx, const Job& J, char* arena, const bbc_options& opts, hipStream_t s,
                       const std::vector<DevGraph>* dg, const std::vector<int64_t>* vstart,
                       const std::vector<int64_t>* rend, const std::vector<DevBlock>* db,
                       const std::vector<DevTile>* dt) {
    Plan P;
    P.carve(arena, J);
    if (dg && !dg->empty()) {
        HIP_OR_FAIL(hipMemcpyAsync(P.graphs, dg->data(), dg->size() * sizeof(DevGraph), hipMemcpyHostToDevice, s));
        HIP_OR_FAIL(hipMemcpyAsync(P.vstart, vstart->data(), vstart->size() * 8, hipMemcpyHostToDevice, s));
        HIP_OR_FAIL(hipMemcpyAsync(P.rank_end, rend->data(), rend->size() * 8, hipMemcpyHostToDevice, s));
    }
    if (db && !db->empty())
        HIP_OR_FAIL(hipMemcpyAsync(P.dblocks, db->data(), db->size() * sizeof(DevBlock), hipMemcpyHostToDevice, s));
    if (dt && !dt->empty())
        HIP_OR_FAIL(hipMemcpyAsync(P.dtiles, dt->data(), dt->size() * sizeof(DevTile), hipMemcpyHostToDevice, s));
    const bool timing = opts.timing != 0;
    if (timing) HIP_OR_FAIL(hipEventRecord(ctx->ev[3], s));
    enqueue(J, P, ctx->st_dev, s, timing ? ctx->ev : nullptr);
    HIP_OR_FAIL(hipGetLastError());
    HIP_OR_FAIL(hipMemcpyAsync(ctx->st_host, ctx->st_dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    const bbc_status rc = status_result(ctx, *ctx->st_host);
    if (rc != BBC_OK) return rc;
    fill_stats(ctx, J, *ctx->st_host, wedge_block(J.band_words, J.wg_size, J.pv != nullptr));
    return timing ? timed_stats(ctx) : BBC_OK;
}

// Runs a job on the context's arena (grown to fit) and stream and waits for
// its status.
bbc_status run_job(bbc_ctx* ctx, const Job& J, const bbc_options& opts, hipStream_t s,
                   const std::vector<DevGraph>* dg, const std::vector<int64_t>* vstart,
                   const std::vector<int64_t>* rend, const std::vector<DevBlock>* db = nullptr,
                   const std::vector<DevTile>* dt = nullptr) {
    Plan P;
    bbc_status rc = grow(ctx, &ctx->arena, &ctx->arena_bytes, P.carve(nullptr, J));
    if (rc != BBC_OK) return rc;
    return run_planned(ctx, J, ctx->arena, opts, s, dg, vstart, rend, db, dt);
}

// Autotuning of the wedge kernel, shared by the single-graph and the
// batched tuner.  `run(options, &result)` performs one call (timing on)
// and returns a result every configuration must reproduce.  Stage 1 times
// every instantiated shape x grid (1, 2 and as many workgroups per CU as
// fit) x schedule with the default regimes; stage 2 times the best shape
// and grid with both schedules x queue_chunk in {1, 2, 4, 8, 16} x
// wave_max_work in {shape's largest, 256, off}.  Each configuration runs reps + 1 times (the first warms up);
// its score is the best HIP-event time of the wedge kernel.
template <class Run>
bbc_status tune_wedge(bbc_ctx* ctx, int32_t reps, Run run, TuneEntry& best) {
    if (reps <= 0) reps = 2;
    uint64_t first = 0;
    bool counted = false, have = false;
    auto time_cfg = [&](bbc_options o, float* ms) -> bbc_status {
        o.timing = 1;
        o.no_tuning = 1;
        float t = 0.f;
        for (int r = 0; r <= reps; ++r) {
            uint64_t res = 0;
            const bbc_status rc = run(o, &res);
            if (rc != BBC_OK) return rc;
            if (!counted) {
                first = res;
                counted = true;
            } else if (res != first) {
                return fail(ctx, BBC_EDEVICE, "autotune: configurations disagree on the result");
            }
            if (r > 0 && (r == 1 || ctx->stats.ms_count < t)) t = ctx->stats.ms_count;
        }
        *ms = t;
        return BBC_OK;
    };
    const int n_shapes = wedge_shape_count();
    for (int i = 0; i < n_shapes; ++i) {
        int wg, bw;
        wedge_shape(i, &wg, &bw);
        const int occ = wedge_blocks_per_cu(bw, wg, false);
        for (int cfg = 0; cfg < 2 * occ; ++cfg) {
            const int wpc = cfg / 2 + 1, sched = cfg & 1;  // both schedules at each grid
            if (wpc > 2 && wpc < occ) continue;           // 1, 2 and as many as fit
            bbc_options o;
            bbc_options_init(&o);
            o.band_words = bw;
            o.wg_size = wg;
            o.wg_per_cu = wpc;
            o.schedule = sched;
            float ms = 0.f;
            const bbc_status rc = time_cfg(o, &ms);
            if (rc != BBC_OK) return rc;
            if (!have || ms < best.ms) {
                best = TuneEntry{0, 0, bw, wg, wpc, sched, 1, 0, 0, 0, ms};
                have = true;
            }
        }
    }
    const TuneEntry shape = best;
    // both schedules again: the best chunk can change which one wins
    for (const int32_t sched : {BBC_SCHED_DYNAMIC, BBC_SCHED_STATIC})
        for (const int32_t qc : {1, 2, 4, 8, 16})
            for (const int32_t wm : {0, 256, -1}) {
                if (qc == 1 && wm == 0) continue;  // timed in stage 1
                bbc_options o;
                bbc_options_init(&o);
                o.band_words = shape.band_words;
                o.wg_size = shape.wg_size;
                o.wg_per_cu = shape.wg_per_cu;
                o.schedule = sched;
                o.queue_chunk = qc;
                o.wave_max_work = wm;
                float ms = 0.f;
                const bbc_status rc = time_cfg(o, &ms);
                if (rc != BBC_OK) return rc;
                if (ms < best.ms) {
                    best.schedule = sched;
                    best.queue_chunk = qc;
                    best.wave_max_work = wm;
                    best.ms = ms;
                }
            }
    return BBC_OK;
}

// Records a wedge-kernel tuning result under the size class (keeping the
// class's dense-block fields) and reports it in *chosen (may be null).
void tune_keep(bbc_ctx* ctx, int64_t n_s, int64_t m, const TuneEntry& best, bbc_options* chosen) {
    TuneEntry& e = tune_slot(ctx, n_s, m);
    e.band_words = best.band_words;
    e.wg_size = best.wg_size;
    e.wg_per_cu = best.wg_per_cu;
    e.schedule = best.schedule;
    e.queue_chunk = best.queue_chunk;
    e.wave_max_work = best.wave_max_work;
    e.ms = best.ms;
    if (chosen) {
        bbc_options_init(chosen);
        chosen->band_words = best.band_words;
        chosen->wg_size = best.wg_size;
        chosen->wg_per_cu = best.wg_per_cu;
        chosen->schedule = best.schedule;
        chosen->queue_chunk = best.queue_chunk;
        chosen->wave_max_work = best.wave_max_work;
    }
}

// bbc_count_classes and bbc_count_classes_per_vertex: the class walk, with
// per_vertex (device, (n_u + n_v) x 6) when given.
bbc_status count_classes(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                         const int32_t* adj, const int8_t* signs, uint64_t* classes, uint64_t* per_vertex,
                         const bbc_options* opts_in, void* stream) {
    if (!ctx) return BBC_EINVAL;
    ctx->err.clear();
    bbc_options opts;
    bbc_status rc = read_options(ctx, opts_in, &opts);
    if (rc != BBC_OK) return rc;
    if (!classes) return fail(ctx, BBC_EINVAL, "classes is NULL");
    if (opts.n_blocks > 0) return fail(ctx, BBC_EINVAL, "dense blocks do not combine with class counts");
    if (opts.side == BBC_SIDE_MIN_WEDGES)
        return fail(ctx, BBC_EINVAL, "class counts depend on the paired side: choose BBC_SIDE_U, _V or _AUTO");
    if (n_u < 0 || n_v < 0 || n_edges < 0) return fail(ctx, BBC_EINVAL, "negative size");
    if (n_edges > INT32_MAX || (int64_t)n_u + (int64_t)n_v > INT32_MAX)
        return fail(ctx, BBC_ETOOBIG, "n_edges or n_u + n_v exceeds INT32_MAX");
    if (!offsets || (n_edges > 0 && (!adj || !signs))) return fail(ctx, BBC_EINVAL, "input pointer is NULL");

    DeviceGuard guard(ctx->device);
    Job J;
    J.off = offsets;
    J.adj = adj;
    J.sg = signs;
    J.n_u = n_u;
    J.n_v = n_v;
    J.s_is_u = side_is_u(opts.side, n_u, n_v);
    J.m = n_edges;
    J.n_s = J.s_is_u ? n_u : n_v;
    J.n_c = J.s_is_u ? n_v : n_u;
    J.checks = opts.checks;
    J.classes = true;
    J.pv = (unsigned long long*)per_vertex;
    J.band_words = wedge_class_band();
    J.schedule = opts.schedule;
    J.wg_size = 256;
    J.grid = ctx->n_cu * (opts.wg_per_cu > 0 ? opts.wg_per_cu
                                             : per_vertex ? wedge_class_pv_blocks_per_cu() : wedge_class_blocks_per_cu());
    rc = run_job(ctx, J, opts, (hipStream_t)stream, nullptr, nullptr, nullptr);
    if (rc != BBC_OK) return rc;
    for (int k = 0; k < 6; ++k) classes[k] = (uint64_t)ctx->st_host->cls[k] / (per_vertex ? 2 : 1);
    return BBC_OK;
}

// bbc_count and bbc_count_noalloc: the same pipeline, its buffers carved
// from the context's arena (grown on demand) or from the device's fixed
// scratch (no allocation; sizes beyond it are rejected).
bbc_status count_single(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                        const int32_t* adj, const int8_t* signs, uint64_t* total, uint64_t* per_vertex,
                        const bbc_options* opts_in, void* stream, bool fixed) {
    if (!ctx) return BBC_EINVAL;
    ctx->err.clear();
    bbc_options opts;
    bbc_status rc = read_options(ctx, opts_in, &opts);
    if (rc != BBC_OK) return rc;
    if (!total) return fail(ctx, BBC_EINVAL, "total is NULL");
    if (n_u < 0 || n_v < 0 || n_edges < 0) return fail(ctx, BBC_EINVAL, "negative size");
    if (n_edges > INT32_MAX || (int64_t)n_u + (int64_t)n_v > INT32_MAX)
        return fail(ctx, BBC_ETOOBIG, "n_edges or n_u + n_v exceeds INT32_MAX");
    if (!offsets || (n_edges > 0 && (!adj || !signs))) return fail(ctx, BBC_EINVAL, "input pointer is NULL");
    if (fixed) {
        if (opts.n_blocks > 0) return fail(ctx, BBC_EINVAL, "bbc_count_noalloc takes no dense blocks");
        if (!ctx->fixed) return hip_fail(ctx, ctx->fixed_err, "fixed scratch lookup (hipGetSymbolAddress)");
    }

    DeviceGuard guard(ctx->device);
    Job J;
    J.off = offsets;
    J.adj = adj;
    J.sg = signs;
    J.n_u = n_u;
    J.n_v = n_v;
    rc = resolve_side(ctx, opts.side, n_u, n_v, n_edges, offsets, adj, (hipStream_t)stream, &J.s_is_u,
                      fixed ? ctx->fixed : nullptr, fixed ? kFixedScratchBytes : 0);
    if (rc != BBC_OK) return rc;
    J.pv = (unsigned long long*)per_vertex;
    J.m = n_edges;
    J.n_s = J.s_is_u ? n_u : n_v;
    J.n_c = J.s_is_u ? n_v : n_u;
    J.checks = opts.checks;
    const bool full = per_vertex != nullptr;
    J.tuned = apply_tuning(ctx, opts, J.n_s, n_edges, full);
    J.band_words = opts.band_words;
    J.schedule = opts.schedule;
    J.wg_size = opts.wg_size;
    set_regimes(J, opts, full);
    J.grid = ctx->n_cu *
             (opts.wg_per_cu > 0 ? opts.wg_per_cu : wedge_blocks_per_cu(opts.band_words, opts.wg_size, full));
    std::vector<DevBlock> db;
    std::vector<DevTile> dt;
    if (opts.n_blocks > 0) {
        if (full) return fail(ctx, BBC_EINVAL, "dense blocks do not combine with per-vertex counts");
        rc = block_job(ctx, opts, J, db, dt);
        if (rc != BBC_OK) return rc;
    }
    if (fixed) {
        Plan P;
        const size_t need = P.carve(nullptr, J);
        if (ctx->limit > 0 && need > (size_t)ctx->limit)
            return fail(ctx, BBC_ENOMEM, "the call needs " + std::to_string(need) + " bytes of scratch, above its "
                                         "scratch_limit of " + std::to_string(ctx->limit));
        if (need > kFixedScratchBytes)
            return fail(ctx, BBC_ETOOBIG, "bbc_count_noalloc: the graph needs " + std::to_string(need) +
                                              " bytes of scratch, the fixed scratch holds " +
                                              std::to_string(kFixedScratchBytes));
        rc = run_planned(ctx, J, ctx->fixed, opts, (hipStream_t)stream, nullptr, nullptr, nullptr, nullptr, nullptr);
    } else {
        rc = run_job(ctx, J, opts, (hipStream_t)stream, nullptr, nullptr, nullptr, &db, &dt);
    }
    if (rc != BBC_OK) return rc;
    // the kernels sum twice the pair terms (per-vertex mode: every anchor's
    // pairs, seen from both ends)
    *total = (uint64_t)ctx->st_host->total / 2;
    return BBC_OK;
}

}  // namespace

// Temporary device memory of one planner call, freed on every return path.
struct PlanScratch {
    std::vector<void*> ptrs;
    ~PlanScratch() {
        for (void* p : ptrs) (void)hipFree(p);
    }
    template <class T>
    T* take(int64_t n) {
        void* p = nullptr;
        if (hipMalloc(&p, (size_t)(n > 0 ? n : 1) * sizeof(T)) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return (T*)p;
    }
};

extern "C" {

void bbc_options_init(bbc_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->struct_size = sizeof(bbc_options);
    o->side = BBC_SIDE_AUTO;
    o->checks = BBC_CHECK_ALL;
}

const char* bbc_status_string(bbc_status s) {
    switch (s) {
        case BBC_OK: return "ok";
        case BBC_EINVAL: return "invalid argument";
        case BBC_EOFFSETS: return "malformed offsets";
        case BBC_ERANGE: return "adjacency id out of range";
        case BBC_ESIGN: return "sign is not +1 or -1";
        case BBC_EDUP: return "repeated edge";
        case BBC_ENOMEM: return "out of device memory";
        case BBC_EDEVICE: return "HIP device error";
        case BBC_ETOOBIG: return "graph too large for int32 CSR";
        case BBC_EOVERFLOW: return "result does not fit its integer width";
    }
    return "unknown status";
}

const char* bbc_last_error(const bbc_ctx* ctx) {
    if (!ctx) return "no context";
    return ctx->err.c_str();
}

bbc_status bbc_create(int device, bbc_ctx** out) {
    if (!out) return BBC_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) {
        (void)hipGetLastError();
        return BBC_EDEVICE;
    }
    if (device < 0 && hipGetDevice(&device) != hipSuccess) return BBC_EDEVICE;
    if (device >= n) return BBC_EDEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return BBC_EDEVICE;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return BBC_EDEVICE;
    bbc_ctx* ctx = new (std::nothrow) bbc_ctx();
    if (!ctx) return BBC_ENOMEM;
    ctx->device = device;
    ctx->n_cu = prop.multiProcessorCount;
    DeviceGuard g(device);
    if (hipMalloc((void**)&ctx->st_dev, sizeof(DevStatus)) != hipSuccess ||
        hipHostMalloc((void**)&ctx->st_host, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        bbc_destroy(ctx);
        return BBC_ENOMEM;
    }
    for (auto& e : ctx->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            bbc_destroy(ctx);
            return BBC_EDEVICE;
        }
    // the fixed scratch of bbc_count_noalloc; a failure is reported by that
    // entry point, the others do not need it
    ctx->fixed_err = fixed_scratch(device, &ctx->fixed);
    if (ctx->fixed_err != hipSuccess) (void)hipGetLastError();
    *out = ctx;
    return BBC_OK;
}

bbc_status bbc_destroy(bbc_ctx* ctx) {
    if (!ctx) return BBC_OK;
    {
        DeviceGuard g(ctx->device);
        for (auto& e : ctx->ev)
            if (e) (void)hipEventDestroy(e);
        if (ctx->arena) (void)hipFree(ctx->arena);
        if (ctx->st_dev) (void)hipFree(ctx->st_dev);
        if (ctx->st_host) (void)hipHostFree(ctx->st_host);
    }
    delete ctx;
    return BBC_OK;
}

bbc_status bbc_last_stats(const bbc_ctx* ctx, bbc_stats* out) {
    if (!ctx || !out) return BBC_EINVAL;
    *out = ctx->stats;
    return BBC_OK;
}

bbc_status bbc_count(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                     const int32_t* adj, const int8_t* signs, uint64_t* total, uint64_t* per_vertex,
                     const bbc_options* opts_in, void* stream) {
    return count_single(ctx, n_u, n_v, n_edges, offsets, adj, signs, total, per_vertex, opts_in, stream, false);
}

bbc_status bbc_count_noalloc(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                             const int32_t* adj, const int8_t* signs, uint64_t* total, uint64_t* per_vertex,
                             const bbc_options* opts_in, void* stream) {
    return count_single(ctx, n_u, n_v, n_edges, offsets, adj, signs, total, per_vertex, opts_in, stream, true);
}

bbc_status bbc_count_classes(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                             const int32_t* adj, const int8_t* signs, uint64_t* classes, const bbc_options* opts_in,
                             void* stream) {
    return count_classes(ctx, n_u, n_v, n_edges, offsets, adj, signs, classes, nullptr, opts_in, stream);
}

bbc_status bbc_count_classes_per_vertex(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges,
                                        const int32_t* offsets, const int32_t* adj, const int8_t* signs,
                                        uint64_t* classes, uint64_t* per_vertex, const bbc_options* opts_in,
                                        void* stream) {
    if (!per_vertex && ctx && (int64_t)n_u + n_v > 0) return fail(ctx, BBC_EINVAL, "per_vertex is NULL");
    return count_classes(ctx, n_u, n_v, n_edges, offsets, adj, signs, classes, per_vertex, opts_in, stream);
}

bbc_status bbc_count_bicliques(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                               const int32_t* adj, const int8_t* signs, int32_t k, uint64_t* count,
                               const bbc_options* opts_in, void* stream) {
    if (!ctx) return BBC_EINVAL;
    ctx->err.clear();
    bbc_options opts;
    bbc_status rc = read_options(ctx, opts_in, &opts);
    if (rc != BBC_OK) return rc;
    if (!count) return fail(ctx, BBC_EINVAL, "count is NULL");
    if (k < 1 || k > BBC_BICLIQUE_MAX_K) return fail(ctx, BBC_EINVAL, "k outside [1, BBC_BICLIQUE_MAX_K]");
    if (opts.n_blocks > 0) return fail(ctx, BBC_EINVAL, "dense blocks do not combine with biclique counts");
    if (opts.side == BBC_SIDE_MIN_WEDGES)
        return fail(ctx, BBC_EINVAL, "biclique counts depend on the side of the pair: choose BBC_SIDE_U, _V or _AUTO");
    if (n_u < 0 || n_v < 0 || n_edges < 0) return fail(ctx, BBC_EINVAL, "negative size");
    if (n_edges > INT32_MAX || (int64_t)n_u + (int64_t)n_v > INT32_MAX)
        return fail(ctx, BBC_ETOOBIG, "n_edges or n_u + n_v exceeds INT32_MAX");
    if (!offsets || (n_edges > 0 && (!adj || !signs))) return fail(ctx, BBC_EINVAL, "input pointer is NULL");

    DeviceGuard guard(ctx->device);
    Job J;
    J.off = offsets;
    J.adj = adj;
    J.sg = signs;
    J.n_u = n_u;
    J.n_v = n_v;
    J.s_is_u = opts.side != BBC_SIDE_V;  // the size-two side is U unless V is named (BB2K)
    J.m = n_edges;
    J.n_s = J.s_is_u ? n_u : n_v;
    J.n_c = J.s_is_u ? n_v : n_u;
    J.checks = opts.checks;
    J.bic_k = k;
    J.band_words = 8192;
    J.schedule = opts.schedule;
    J.wg_size = 256;
    J.grid = ctx->n_cu * (opts.wg_per_cu > 0 ? opts.wg_per_cu : wedge_bic_blocks_per_cu());
    rc = run_job(ctx, J, opts, (hipStream_t)stream, nullptr, nullptr, nullptr);
    if (rc != BBC_OK) return rc;
    // 32-bit limbs summed in 64 bits: carry them into the 128-bit result
    const unsigned long long* l = ctx->st_host->cls;
    unsigned long long c = 0, w[4];
    for (int j = 0; j < 4; ++j) {
        const unsigned long long t = l[j] + c;  // l[j] < 2^63 for any graph the kernel accepts
        w[j] = t & 0xffffffffull;
        c = t >> 32;
    }
    if (c != 0 || l[4] != 0) return fail(ctx, BBC_EOVERFLOW, "(2,k)-biclique count does not fit 128 bits");
    count[0] = w[0] | (w[1] << 32);
    count[1] = w[2] | (w[3] << 32);
    return BBC_OK;
}

bbc_status bbc_update_delta(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                            const int32_t* adj, const int8_t* signs, int32_t n_updates, const int32_t* upd_u,
                            const int32_t* upd_v, const int8_t* upd_state, int64_t* delta, int64_t* per_update,
                            void* stream) {
    if (!ctx) return BBC_EINVAL;
    ctx->err.clear();
    ctx->limit = 0;
    if (!delta) return fail(ctx, BBC_EINVAL, "delta is NULL");
    if (n_u < 0 || n_v < 0 || n_edges < 0 || n_updates < 0) return fail(ctx, BBC_EINVAL, "negative size");
    if (n_edges > INT32_MAX || (int64_t)n_u + (int64_t)n_v > INT32_MAX)
        return fail(ctx, BBC_ETOOBIG, "n_edges or n_u + n_v exceeds INT32_MAX");
    if (!offsets || (n_edges > 0 && (!adj || !signs)) || (n_updates > 0 && (!upd_u || !upd_v || !upd_state)))
        return fail(ctx, BBC_EINVAL, "input pointer is NULL");
    if (n_updates == 0) {
        *delta = 0;
        return BBC_OK;
    }
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const int64_t m = n_edges, q = n_updates;
    const int64_t nmax = std::max<int64_t>(std::max<int64_t>(m, q), (int64_t)n_v + 1);
    const int64_t hs = (int64_t)radix_hist_size(nmax);
    // scratch: edge decode, two sorts of the edges, two of the updates
    struct Dyn {
        uint32_t *ea, *ec, *kin, *pin, *ka, *kb, *pa, *pb, *pa2, *pb2, *vdeg, *voff;
        uint8_t* en;
        uint32_t *qk, *qka, *qkb, *ia, *ib, *ia2, *ib2, *uv_pos, *vu_pos, *n_tasks, *task_off, *span;
        uint8_t* mode;
        unsigned long long *uv_key, *vu_key, *wsum;
        int8_t* s_old;
        uint32_t *hist, *hist_scan, *partials;
        size_t carve(char* base, int64_t m, int64_t q, int32_t n_v, int64_t hs, int64_t nmax) {
            Carve c(base);
            ea = c.take<uint32_t>(m);
            ec = c.take<uint32_t>(m);
            en = c.take<uint8_t>(m);
            kin = c.take<uint32_t>(m);
            pin = c.take<uint32_t>(m);
            ka = c.take<uint32_t>(m);
            kb = c.take<uint32_t>(m);
            pa = c.take<uint32_t>(m);
            pb = c.take<uint32_t>(m);
            pa2 = c.take<uint32_t>(m);
            pb2 = c.take<uint32_t>(m);
            vdeg = c.take<uint32_t>(n_v);
            voff = c.take<uint32_t>((int64_t)n_v + 1);
            qk = c.take<uint32_t>(q);
            qka = c.take<uint32_t>(q);
            qkb = c.take<uint32_t>(q);
            ia = c.take<uint32_t>(q);
            ib = c.take<uint32_t>(q);
            ia2 = c.take<uint32_t>(q);
            ib2 = c.take<uint32_t>(q);
            uv_pos = c.take<uint32_t>(q);
            vu_pos = c.take<uint32_t>(q);
            uv_key = c.take<unsigned long long>(q);
            vu_key = c.take<unsigned long long>(q);
            wsum = c.take<unsigned long long>(n_v);
            n_tasks = c.take<uint32_t>(q);
            task_off = c.take<uint32_t>(q + 1);
            span = c.take<uint32_t>(q);
            mode = c.take<uint8_t>(q);
            s_old = c.take<int8_t>(q);
            hist = c.take<uint32_t>(hs);
            hist_scan = c.take<uint32_t>(hs + 1);
            partials = c.take<uint32_t>((int64_t)scan_partials_size(hs + nmax + 8));
            return c.used;
        }
    } D;
    bbc_status rc = grow(ctx, &ctx->arena, &ctx->arena_bytes, D.carve(nullptr, m, q, n_v, hs, nmax));
    if (rc != BBC_OK) return rc;
    D.carve(ctx->arena, m, q, n_v, hs, nmax);
    DevStatus* st = ctx->st_dev;
    // checks first (the builds below index with the ids), one wait
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, s, st);
    launch_decode_single(offsets, adj, signs, n_u, n_v, m, 1, 1, st, D.ea, D.ec, D.en, nullptr, s);
    dyn_check(upd_u, upd_v, upd_state, (int32_t)q, n_u, n_v, st, s);
    HIP_OR_FAIL(hipMemcpyAsync(ctx->st_host, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    rc = status_result(ctx, *ctx->st_host);
    if (rc != BBC_OK) return rc;
    const int bits_u = bits_for(n_u > 0 ? (uint64_t)(n_u - 1) : 0), bits_v = bits_for(n_v > 0 ? (uint64_t)(n_v - 1) : 0);
    // V rows: stable sort of the CSR-ordered edges by v (u ascending inside)
    const uint32_t *vkey = nullptr, *vrow = nullptr, *ukey = nullptr, *urow = nullptr;
    dyn_vkeys(D.ea, D.ec, D.en, m, D.kin, D.pin, s);
    radix_sort(D.kin, D.ka, D.kb, D.pin, D.pa, D.pb, nullptr, nullptr, nullptr, m, bits_v, D.hist, D.hist_scan,
               D.partials, s, &vkey, &vrow, nullptr);
    launch_hist(D.ec, m, D.vdeg, n_v, nullptr, 0, st, s);
    scan_exclusive_u32(D.vdeg, D.voff, n_v, D.partials, s);
    // U rows sorted by v: stable sort of the V-ordered edges by u
    dyn_ukeys(vkey, vrow, m, D.kin, D.pin, s);
    radix_sort(D.kin, D.ka, D.kb, D.pin, D.pa2, D.pb2, nullptr, nullptr, nullptr, m, bits_u, D.hist, D.hist_scan,
               D.partials, s, &ukey, &urow, nullptr);
    dyn_dup(ukey, urow, m, st, s);
    // updates by (u, v) and by (v, u): two stable sorts each, carrying the index
    const uint32_t *k_out = nullptr, *i1 = nullptr, *i2 = nullptr;
    dyn_key_init(upd_v, (int32_t)q, D.qk, s);
    radix_sort(D.qk, D.qka, D.qkb, nullptr, nullptr, nullptr, nullptr, D.ia, D.ib, q, bits_v, D.hist, D.hist_scan,
               D.partials, s, &k_out, nullptr, &i1);
    dyn_gather(upd_u, i1, (int32_t)q, D.qk, s);
    radix_sort(D.qk, D.qka, D.qkb, nullptr, nullptr, nullptr, i1, D.ia2, D.ib2, q, bits_u, D.hist, D.hist_scan,
               D.partials, s, &k_out, nullptr, &i2);
    dyn_key64(upd_u, upd_v, i2, (int32_t)q, D.uv_key, D.uv_pos, 1, st, s);
    dyn_key_init(upd_u, (int32_t)q, D.qk, s);
    radix_sort(D.qk, D.qka, D.qkb, nullptr, nullptr, nullptr, nullptr, D.ia, D.ib, q, bits_u, D.hist, D.hist_scan,
               D.partials, s, &k_out, nullptr, &i1);
    dyn_gather(upd_v, i1, (int32_t)q, D.qk, s);
    radix_sort(D.qk, D.qka, D.qkb, nullptr, nullptr, nullptr, i1, D.ia2, D.ib2, q, bits_v, D.hist, D.hist_scan,
               D.partials, s, &k_out, nullptr, &i2);
    dyn_key64(upd_v, upd_u, i2, (int32_t)q, D.vu_key, D.vu_pos, 0, st, s);
    dyn_delta(offsets, urow, D.voff, vrow, D.uv_key, D.uv_pos, D.vu_key, D.vu_pos, upd_u, upd_v, upd_state, D.s_old,
              D.wsum, n_v, (int32_t)q, D.n_tasks, D.task_off, D.span, D.mode, D.partials, (long long*)per_update,
              ctx->update_task_cap, st, s);
    HIP_OR_FAIL(hipMemcpyAsync(ctx->st_host, st, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    rc = status_result(ctx, *ctx->st_host);
    if (rc != BBC_OK) return rc;
    *delta = (int64_t)ctx->st_host->total;
    return BBC_OK;
}

bbc_status bbc_set_update_task_cap(bbc_ctx* ctx, int32_t cap) {
    if (!ctx) return BBC_EINVAL;
    if (cap < 0) return fail(ctx, BBC_EINVAL, "negative task cap");
    ctx->update_task_cap = cap;
    return BBC_OK;
}

bbc_status bbc_count_batched(bbc_ctx* ctx, int32_t n_graphs, const bbc_graph_desc* descs,
                             const int32_t* offsets_cat, const int32_t* adj_cat, const int8_t* signs_cat,
                             uint64_t* totals, const bbc_options* opts_in, void* stream) {
    if (!ctx) return BBC_EINVAL;
    ctx->err.clear();
    bbc_options opts;
    bbc_status rc = read_options(ctx, opts_in, &opts);
    if (rc != BBC_OK) return rc;
    DeviceGuard guard(ctx->device);
    Job J;
    std::vector<DevGraph> dg;
    std::vector<int64_t> vstart, rend;
    rc = batch_job(ctx, n_graphs, descs, offsets_cat, adj_cat, signs_cat, totals, opts, J, dg, vstart, rend);
    if (rc != BBC_OK || n_graphs == 0) return rc;
    return run_job(ctx, J, opts, (hipStream_t)stream, &dg, &vstart, &rend);
}

bbc_status bbc_batch_plan_destroy(bbc_batch_plan* p) {
    if (!p) return BBC_OK;
    {
        DeviceGuard g(p->ctx ? p->ctx->device : 0);
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        if (p->arena) (void)hipFree(p->arena);
        if (p->st_dev) (void)hipFree(p->st_dev);
        if (p->st_host) (void)hipHostFree(p->st_host);
    }
    delete p;
    return BBC_OK;
}

bbc_status bbc_batch_plan_create(bbc_ctx* ctx, int32_t n_graphs, const bbc_graph_desc* descs,
                                 const int32_t* offsets_cat, const int32_t* adj_cat, const int8_t* signs_cat,
                                 uint64_t* totals, const bbc_options* opts_in, bbc_batch_plan** out) {
    if (!ctx || !out) return BBC_EINVAL;
    *out = nullptr;
    ctx->err.clear();
    bbc_options opts;
    bbc_status rc = read_options(ctx, opts_in, &opts);
    if (rc != BBC_OK) return rc;
    DeviceGuard guard(ctx->device);
    Job J;
    std::vector<DevGraph> dg;
    std::vector<int64_t> vstart, rend;
    rc = batch_job(ctx, n_graphs, descs, offsets_cat, adj_cat, signs_cat, totals, opts, J, dg, vstart, rend);
    if (rc != BBC_OK) return rc;
    bbc_batch_plan* p = new (std::nothrow) bbc_batch_plan();
    if (!p) return BBC_ENOMEM;
    p->ctx = ctx;
    Plan P;
    const size_t bytes = P.carve(nullptr, J);
    if (opts.scratch_limit > 0 && bytes > (size_t)opts.scratch_limit) {
        bbc_batch_plan_destroy(p);
        return fail(ctx, BBC_ENOMEM, "the plan needs " + std::to_string(bytes) + " bytes of scratch, above its "
                                     "scratch_limit of " + std::to_string(opts.scratch_limit));
    }
    if (hipMalloc((void**)&p->arena, bytes) != hipSuccess ||
        hipMalloc((void**)&p->st_dev, sizeof(DevStatus)) != hipSuccess ||
        hipHostMalloc((void**)&p->st_host, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        bbc_batch_plan_destroy(p);
        return fail(ctx, BBC_ENOMEM, "batch plan allocation failed");
    }
    P.carve(p->arena, J);
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e == hipSuccess && n_graphs > 0) {
        e = hipMemcpyAsync(P.graphs, dg.data(), dg.size() * sizeof(DevGraph), hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) e = hipMemcpyAsync(P.vstart, vstart.data(), vstart.size() * 8, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) e = hipMemcpyAsync(P.rank_end, rend.data(), rend.size() * 8, hipMemcpyHostToDevice, cs);
        if (e == hipSuccess) e = hipStreamSynchronize(cs);
    }
    if (e == hipSuccess) e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        if (n_graphs > 0) enqueue(J, P, p->st_dev, cs, nullptr);
        else hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, cs, p->st_dev);
        hipError_t le = hipGetLastError();
        e = hipStreamEndCapture(cs, &p->graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (cs) (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        bbc_batch_plan_destroy(p);
        return hip_fail(ctx, e, "batch plan capture");
    }
    *out = p;
    return BBC_OK;
}

bbc_status bbc_batch_launch(bbc_batch_plan* p, void* stream) {
    if (!p) return BBC_EINVAL;
    bbc_ctx* ctx = p->ctx;
    DeviceGuard guard(ctx->device);
    HIP_OR_FAIL(hipGraphLaunch(p->exec, (hipStream_t)stream));
    return BBC_OK;
}

bbc_status bbc_batch_wait(bbc_batch_plan* p, void* stream) {
    if (!p) return BBC_EINVAL;
    bbc_ctx* ctx = p->ctx;
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    HIP_OR_FAIL(hipMemcpyAsync(p->st_host, p->st_dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    return status_result(ctx, *p->st_host);
}

bbc_status bbc_autotune(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                        const int32_t* adj, const int8_t* signs, int32_t reps, bbc_options* chosen, void* stream) {
    if (!ctx) return BBC_EINVAL;
    TuneEntry best{};
    auto run = [&](const bbc_options& o, uint64_t* res) {
        return bbc_count(ctx, n_u, n_v, n_edges, offsets, adj, signs, res, nullptr, &o, stream);
    };
    bbc_status rc = tune_wedge(ctx, reps, run, best);
    if (rc != BBC_OK) return rc;
    const bool su = side_is_u(BBC_SIDE_AUTO, n_u, n_v);
    tune_keep(ctx, su ? n_u : n_v, n_edges, best, chosen);
    return BBC_OK;
}

bbc_status bbc_autotune_batched(bbc_ctx* ctx, int32_t n_graphs, const bbc_graph_desc* descs,
                                const int32_t* offsets_cat, const int32_t* adj_cat, const int8_t* signs_cat,
                                uint64_t* totals, int32_t reps, bbc_options* chosen, void* stream) {
    if (!ctx) return BBC_EINVAL;
    if (n_graphs < 0 || (n_graphs > 0 && (!descs || !totals))) return fail(ctx, BBC_EINVAL, "bad batch arguments");
    std::vector<uint64_t> host((size_t)(n_graphs > 0 ? n_graphs : 1));
    // the result compared across configurations: the per-graph totals,
    // folded with their positions
    auto run = [&](const bbc_options& o, uint64_t* res) {
        bbc_status rc = bbc_count_batched(ctx, n_graphs, descs, offsets_cat, adj_cat, signs_cat, totals, &o, stream);
        if (rc != BBC_OK || n_graphs == 0) return rc;
        DeviceGuard guard(ctx->device);
        HIP_OR_FAIL(hipMemcpy(host.data(), totals, (size_t)n_graphs * 8, hipMemcpyDeviceToHost));
        uint64_t h = 0;
        for (int32_t g = 0; g < n_graphs; ++g) h = h * 1000003ull + host[(size_t)g] + 1;
        *res = h;
        return BBC_OK;
    };
    TuneEntry best{};
    bbc_status rc = tune_wedge(ctx, reps, run, best);
    if (rc != BBC_OK) return rc;
    int64_t ns = 0, m = 0;
    for (int32_t g = 0; g < n_graphs; ++g) {
        m += descs[g].n_edges;
        ns += side_is_u(BBC_SIDE_AUTO, descs[g].n_u, descs[g].n_v) ? descs[g].n_u : descs[g].n_v;
    }
    tune_keep(ctx, ns, m, best, chosen);
    return BBC_OK;
}

bbc_status bbc_autotune_blocks(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                               const int32_t* adj, const int8_t* signs, int32_t reps, bbc_plan_options* chosen_plan,
                               bbc_options* chosen, void* stream) {
    if (!ctx) return BBC_EINVAL;
    if (reps <= 0) reps = 2;
    if (n_u < 0 || n_v < 0 || n_edges < 0) return fail(ctx, BBC_EINVAL, "negative size");
    if (n_edges > INT32_MAX || (int64_t)n_u + (int64_t)n_v > INT32_MAX)
        return fail(ctx, BBC_ETOOBIG, "n_edges or n_u + n_v exceeds INT32_MAX");
    constexpr int32_t kMaxBlocks = 1024;
    constexpr int32_t kTaus[] = {128, 256, 512, 1024};
    constexpr int32_t kTiles[] = {64, 128};
    // the sparse-only count is the reference every configuration must match
    uint64_t want = 0;
    bbc_options o0;
    bbc_options_init(&o0);
    o0.no_tuning = 1;
    bbc_status rc = bbc_count(ctx, n_u, n_v, n_edges, offsets, adj, signs, &want, nullptr, &o0, stream);
    if (rc != BBC_OK) return rc;
    int32_t* ids = nullptr;
    {
        DeviceGuard guard(ctx->device);
        if (hipMalloc((void**)&ids, ((size_t)n_u + (size_t)n_v + 1) * sizeof(int32_t)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, BBC_ENOMEM, "autotune: block id buffer");
        }
    }
    std::vector<bbc_dense_block> blocks((size_t)kMaxBlocks);
    double best_ms = -1.0;
    int32_t best_tau = 256, best_tile = 128;
    for (int32_t tau : kTaus) {
        bbc_plan_options po;
        bbc_plan_options_init(&po);
        po.min_degree = tau;
        int32_t nb = 0;
        const auto t0 = std::chrono::steady_clock::now();
        rc = bbc_plan_blocks(ctx, n_u, n_v, n_edges, offsets, adj, &po, kMaxBlocks, blocks.data(), ids,
                             (int64_t)n_u + n_v, &nb, stream);
        const double plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (rc != BBC_OK) break;
        for (int32_t tile : kTiles) {
            bbc_options o;
            bbc_options_init(&o);
            o.n_blocks = nb;
            o.blocks = blocks.data();
            o.dense_tile = tile;
            o.timing = 1;
            o.no_tuning = 1;
            float ms = 0.f;
            for (int r = 0; r <= reps && rc == BBC_OK; ++r) {
                uint64_t got = 0;
                rc = bbc_count(ctx, n_u, n_v, n_edges, offsets, adj, signs, &got, nullptr, &o, stream);
                if (rc == BBC_OK && got != want) rc = fail(ctx, BBC_EDEVICE, "autotune: dense blocks change the count");
                if (r > 0 && (r == 1 || ctx->stats.ms_total < ms)) ms = ctx->stats.ms_total;
            }
            if (rc != BBC_OK) break;
            const double score = plan_ms + ms;  // a one-off count plans once
            if (best_ms < 0 || score < best_ms) {
                best_ms = score;
                best_tau = tau;
                best_tile = tile;
            }
            if (nb == 0) break;  // no blocks: the tile does not matter
        }
        if (rc != BBC_OK) break;
    }
    {
        DeviceGuard guard(ctx->device);
        (void)hipFree(ids);
    }
    if (rc != BBC_OK) return rc;
    const bool su = side_is_u(BBC_SIDE_AUTO, n_u, n_v);
    TuneEntry& e = tune_slot(ctx, su ? n_u : n_v, n_edges);
    e.min_degree = best_tau;
    e.dense_tile = best_tile;
    if (e.band_words == 0) e.ms = (float)best_ms;
    if (chosen_plan) {
        bbc_plan_options_init(chosen_plan);
        chosen_plan->min_degree = best_tau;
    }
    if (chosen) {
        bbc_options_init(chosen);
        chosen->dense_tile = best_tile;
    }
    return BBC_OK;
}

bbc_status bbc_plan_options_init(bbc_plan_options* o) {
    if (!o) return BBC_EINVAL;
    *o = bbc_plan_options{sizeof(bbc_plan_options), BBC_SIDE_AUTO, 0, 0.3f, 0.25f, 256, 64, 32};
    return BBC_OK;
}

bbc_status bbc_plan_blocks(bbc_ctx* ctx, int32_t n_u, int32_t n_v, int64_t n_edges, const int32_t* offsets,
                           const int32_t* adj, const bbc_plan_options* opts_in, int32_t max_blocks,
                           bbc_dense_block* blocks, int32_t* ids, int64_t ids_cap, int32_t* n_blocks, void* stream) {
    if (!ctx) return BBC_EINVAL;
    ctx->err.clear();
    if (!n_blocks) return fail(ctx, BBC_EINVAL, "n_blocks is NULL");
    *n_blocks = 0;
    bbc_plan_options o;
    bbc_plan_options_init(&o);
    if (opts_in) {
        if (opts_in->struct_size != sizeof(bbc_plan_options))
            return fail(ctx, BBC_EINVAL, "plan options: struct_size mismatch");
        o = *opts_in;
    }
    if (o.side != BBC_SIDE_AUTO && o.side != BBC_SIDE_U && o.side != BBC_SIDE_V)
        return fail(ctx, BBC_EINVAL, "plan options: bad side");
    if (o.min_degree < 0 || !(o.member_frac > 0.f && o.member_frac <= 1.f) ||
        !(o.min_density > 0.f && o.min_density <= 1.f) || o.min_anchors < 2 || o.min_centres < 1 ||
        o.max_tries < 1)
        return fail(ctx, BBC_EINVAL, "plan options out of range");
    if (max_blocks < 0 || ids_cap < 0 || n_u < 0 || n_v < 0 || n_edges < 0)
        return fail(ctx, BBC_EINVAL, "negative size");
    if (n_edges > INT32_MAX || (int64_t)n_u + (int64_t)n_v > INT32_MAX)
        return fail(ctx, BBC_ETOOBIG, "n_edges or n_u + n_v exceeds INT32_MAX");
    if (max_blocks > 0 && (!blocks || (ids_cap > 0 && !ids))) return fail(ctx, BBC_EINVAL, "output pointer is NULL");
    if (!offsets || (n_edges > 0 && !adj)) return fail(ctx, BBC_EINVAL, "input pointer is NULL");
    if (max_blocks == 0 || n_edges == 0) return BBC_OK;

    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const bool su = side_is_u(o.side, n_u, n_v);
    const int64_t m = n_edges, n_a = su ? n_u : n_v, n_c = su ? n_v : n_u;
    if (o.min_degree == 0) {  // the tuned threshold of the graph's size class, else 256
        const TuneEntry* e = tune_find(ctx, n_a, m);
        o.min_degree = e && e->min_degree > 0 ? e->min_degree : 256;
    }
    const uint32_t tau = (uint32_t)o.min_degree;
    constexpr uint32_t kCapR = 16384, kCapC = 65535;
    PlanScratch P;
    uint32_t* ea = P.take<uint32_t>(m);
    uint32_t* ec = P.take<uint32_t>(m);
    uint32_t* adj_a = P.take<uint32_t>(m);  // anchor -> centres
    uint32_t* adj_c = P.take<uint32_t>(m);  // centre -> anchors
    uint32_t* deg_a = P.take<uint32_t>(n_a);
    uint32_t* deg_c = P.take<uint32_t>(n_c);
    uint32_t* off_a = P.take<uint32_t>(n_a + 1);
    uint32_t* off_c = P.take<uint32_t>(n_c + 1);
    uint32_t* cur = P.take<uint32_t>(std::max(n_a, n_c));
    uint32_t* cd = P.take<uint32_t>(n_a);
    uint32_t* cnt_a = P.take<uint32_t>(n_a);
    uint32_t* cnt_c = P.take<uint32_t>(n_c);
    uint8_t* asg_a = P.take<uint8_t>(n_a);
    uint8_t* asg_c = P.take<uint8_t>(n_c);
    uint32_t* list_r = P.take<uint32_t>(kCapR);
    uint32_t* list_c = P.take<uint32_t>(kCapC);
    uint32_t* small = P.take<uint32_t>(8);  // [n_r, n_c] then edges (u64) at [2..3]
    uint32_t* partials = P.take<uint32_t>((int64_t)scan_partials_size(std::max(n_a, n_c) + 8));
    uint32_t* host = nullptr;  // pinned: the three counts read back per seed
    if (!ea || !ec || !adj_a || !adj_c || !deg_a || !deg_c || !off_a || !off_c || !cur || !cd || !cnt_a || !cnt_c ||
        !asg_a || !asg_c || !list_r || !list_c || !small || !partials)
        return fail(ctx, BBC_ENOMEM, "plan: device memory");
    if (hipHostMalloc((void**)&host, 4 * sizeof(uint32_t)) != hipSuccess)
        return fail(ctx, BBC_ENOMEM, "plan: pinned host memory");
    struct HostFree {
        uint32_t* p;
        ~HostFree() { (void)hipHostFree(p); }
    } host_free{host};

    // edges as (anchor, centre) with the offset and id-range checks
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, s, ctx->st_dev);
    launch_decode_single(offsets, adj, nullptr, n_u, n_v, m, su ? 1 : 0, 0, ctx->st_dev, ea, ec, nullptr, nullptr,
                         s);
    HIP_OR_FAIL(hipMemcpyAsync(ctx->st_host, ctx->st_dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    bbc_status rc = status_result(ctx, *ctx->st_host);
    if (rc != BBC_OK) return rc;

    // both adjacency directions (degree histograms use adj_a as scratch before the scatter)
    launch_hist(ea, m, deg_a, n_a, adj_a, m, ctx->st_dev, s);
    launch_hist(ec, m, deg_c, n_c, adj_a, m, ctx->st_dev, s);
    scan_exclusive_u32(deg_a, off_a, n_a, partials, s);
    scan_exclusive_u32(deg_c, off_c, n_c, partials, s);
    pl_scatter(ea, ec, m, off_a, n_a, cur, adj_a, s);
    pl_scatter(ec, ea, m, off_c, n_c, cur, adj_c, s);
    fill_u32(cd, 0u, n_a, s);
    pl_cand_deg(ea, ec, m, deg_a, deg_c, tau, cd, s);
    fill_u32(cnt_a, 0u, n_a, s);
    fill_u32(cnt_c, 0u, n_c, s);
    fill_bytes(asg_a, n_a, s);
    fill_bytes(asg_c, n_c, s);

    // seeds: candidate anchors by decreasing (candidate centres)^2 / degree
    std::vector<uint32_t> h_deg(n_a), h_cd(n_a);
    HIP_OR_FAIL(hipMemcpyAsync(h_deg.data(), deg_a, n_a * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipMemcpyAsync(h_cd.data(), cd, n_a * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    std::vector<std::pair<double, uint32_t>> seeds;
    for (int64_t a = 0; a < n_a; ++a)
        if (h_deg[a] >= tau && h_cd[a] >= (uint32_t)o.min_centres)
            seeds.push_back({-(double)h_cd[a] * h_cd[a] / h_deg[a], (uint32_t)a});
    std::sort(seeds.begin(), seeds.end());
    std::vector<uint8_t> used(n_a, 0);

    uint32_t* n_r = small;
    uint32_t* n_cc = small + 1;
    unsigned long long* edges = (unsigned long long*)(small + 2);
    int32_t found = 0, tries = 0;
    int64_t ids_used = 0;
    std::vector<uint32_t> h_r;
    for (const auto& sd : seeds) {
        const uint32_t seed = sd.second;
        if (used[seed]) continue;
        fill_u32(small, 0u, 4, s);
        pl_seed(off_a, adj_a, seed, deg_c, tau, asg_c, list_c, n_cc, kCapC, s);
        for (int it = 0; it < 2; ++it) {
            fill_u32(small, 0u, 1, s);
            pl_count(list_c, n_cc, kCapC, off_c, adj_c, cnt_a, s);
            pl_select(cnt_a, n_a, deg_a, tau, asg_a, n_cc, kCapC, o.member_frac, list_r, n_r, kCapR,
                      edges, s);
            fill_u32(small + 1, 0u, 3, s);
            pl_count(list_r, n_r, kCapR, off_a, adj_a, cnt_c, s);
            pl_select(cnt_c, n_c, deg_c, tau, asg_c, n_r, kCapR, o.member_frac, list_c, n_cc, kCapC, edges,
                      s);
        }
        HIP_OR_FAIL(hipMemcpyAsync(host, small, 4 * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        const uint32_t nr = std::min(host[0], kCapR), nc = std::min(host[1], kCapC);
        const unsigned long long e = (unsigned long long)host[2] | ((unsigned long long)host[3] << 32);
        used[seed] = 1;
        const bool keep = nr >= (uint32_t)o.min_anchors && nc >= (uint32_t)o.min_centres &&
                          (double)e >= (double)o.min_density * nr * nc && ids_used + nr + nc <= ids_cap;
        if (!keep) {
            if (++tries >= o.max_tries) break;
            continue;
        }
        tries = 0;
        // U ids first, then V ids
        const uint32_t* lu = su ? list_r : list_c;
        const uint32_t* lv = su ? list_c : list_r;
        const uint32_t nu = su ? nr : nc, nv = su ? nc : nr;
        HIP_OR_FAIL(hipMemcpyAsync(ids + ids_used, lu, nu * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        HIP_OR_FAIL(hipMemcpyAsync(ids + ids_used + nu, lv, nv * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        blocks[found] = bbc_dense_block{(int32_t)nu, (int32_t)nv, ids + ids_used, ids + ids_used + nu};
        ids_used += nu + nv;
        pl_assign(list_r, nr, asg_a, s);
        pl_assign(list_c, nc, asg_c, s);
        h_r.resize(nr);
        HIP_OR_FAIL(hipMemcpyAsync(h_r.data(), list_r, nr * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_OR_FAIL(hipStreamSynchronize(s));
        for (uint32_t r : h_r) used[r] = 1;
        if (++found == max_blocks) break;
    }
    HIP_OR_FAIL(hipStreamSynchronize(s));
    *n_blocks = found;
    return BBC_OK;
}

bbc_status bbc_tune_save(const bbc_ctx* ctx, const char* path) {
    if (!ctx || !path) return BBC_EINVAL;
    FILE* f = fopen(path, "w");
    if (!f) return fail(const_cast<bbc_ctx*>(ctx), BBC_EINVAL, std::string("cannot write ") + path);
    bool ok = fprintf(f, "bbc-tune 3 gfx950\n") > 0;
    for (const TuneEntry& e : ctx->tune)
        ok = ok && fprintf(f, "%d %d %d %d %d %d %d %d %d %d %.4f\n", e.ns_bits, e.deg_bits, e.band_words, e.wg_size,
                           e.wg_per_cu, e.schedule, e.queue_chunk, e.wave_max_work, e.min_degree, e.dense_tile,
                           (double)e.ms) > 0;
    ok = (fclose(f) == 0) && ok;
    return ok ? BBC_OK : fail(const_cast<bbc_ctx*>(ctx), BBC_EINVAL, std::string("write failed: ") + path);
}

bbc_status bbc_tune_load(bbc_ctx* ctx, const char* path) {
    if (!ctx || !path) return BBC_EINVAL;
    FILE* f = fopen(path, "r");
    if (!f) return fail(ctx, BBC_EINVAL, std::string("cannot read ") + path);
    char line[256];
    std::vector<TuneEntry> got;
    int ln = 0, version = 0;
    bbc_status rc = BBC_OK;
    while (fgets(line, sizeof line, f)) {
        ++ln;
        if (ln == 1) {  // version 1 has no schedule column (dynamic); versions 1 and 2 no regime or block columns
            for (int v = 1; v <= 3; ++v) {
                const std::string h = "bbc-tune " + std::to_string(v) + " gfx950";
                if (h == line || h + "\n" == line) version = v;
            }
            if (!version) {
                rc = fail(ctx, BBC_EINVAL, std::string(path) + ":1: not a tuning file for gfx950");
                break;
            }
            continue;
        }
        TuneEntry e{};
        e.schedule = BBC_SCHED_DYNAMIC;
        double ms = 0;
        // whitespace-separated fields: integers, then the time; every field
        // must parse in full
        const int want = version == 1 ? 6 : version == 2 ? 7 : 11;
        int32_t* ints[10] = {&e.ns_bits,  &e.deg_bits,    &e.band_words,    &e.wg_size,    &e.wg_per_cu,
                             &e.schedule, &e.queue_chunk, &e.wave_max_work, &e.min_degree, &e.dense_tile};
        if (version == 1) ints[5] = nullptr;  // no schedule column: the time follows wg_per_cu
        int n = 0;
        bool good = true;
        char* save = nullptr;
        for (char* tok = strtok_r(line, " \t\r\n", &save); tok; tok = strtok_r(nullptr, " \t\r\n", &save), ++n) {
            char* end = nullptr;
            if (n < want - 1) {
                const long v = strtol(tok, &end, 10);
                good = good && *end == 0 && v >= INT32_MIN && v <= INT32_MAX;
                if (ints[n]) *ints[n] = (int32_t)v;
            } else if (n == want - 1) {
                ms = strtod(tok, &end);
                good = good && *end == 0;
            }
        }
        if (version == 1) e.schedule = BBC_SCHED_DYNAMIC;
        const bool shape_ok = e.band_words == 0 ? (version == 3 && e.wg_size == 0 && e.wg_per_cu == 0)
                                                : (e.wg_size > 0 && wedge_shape_ok(e.band_words, e.wg_size));
        if (!good || n != want || e.ns_bits < 0 || e.ns_bits > 64 || e.deg_bits < 0 || e.deg_bits > 64 ||
            e.wg_per_cu < 0 || e.band_words < 0 || !shape_ok ||
            (e.schedule != BBC_SCHED_DYNAMIC && e.schedule != BBC_SCHED_STATIC) || e.queue_chunk < 0 ||
            e.queue_chunk > 65536 || e.wave_max_work < -1 || e.min_degree < 0 ||
            (e.dense_tile != 0 && e.dense_tile != 64 && e.dense_tile != 128)) {
            rc = fail(ctx, BBC_EINVAL, std::string(path) + ":" + std::to_string(ln) + ": malformed tuning entry");
            break;
        }
        e.ms = (float)ms;
        got.push_back(e);
    }
    if (rc == BBC_OK && ln == 0) rc = fail(ctx, BBC_EINVAL, std::string(path) + ": empty file");
    fclose(f);
    if (rc != BBC_OK) return rc;
    for (const TuneEntry& e : got) tune_store(ctx, e);
    return BBC_OK;
}

}  // extern "C"
