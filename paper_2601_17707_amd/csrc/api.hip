// C ABI of libbbc.so (declared in include/bbc.h): context, scratch arena,
// launch sequence and error mapping.
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

#include "../../include/bbc.h"
#include "bbc_internal.h"

namespace bbc {
void launch_checks(const int32_t* off, const int32_t* adj, const int8_t* sg, int32_t n_u, int32_t n_v, int64_t m,
                   int check_sign, DevStatus* st, hipStream_t s);
void launch_degrees(const int32_t* off, const int32_t* adj, int32_t n_u, int64_t m, uint32_t* deg_u,
                    uint32_t* deg_v, int32_t n_v, hipStream_t s);
void launch_ranks(const uint32_t* inv, const uint32_t* deg_s, int32_t n_s, int32_t* rank, uint32_t* adeg,
                  hipStream_t s);
void launch_fill_anchor(const int32_t* off, const int32_t* adj, const int8_t* sg, int32_t n_u, int64_t m,
                        int s_is_u, const int32_t* rank, const uint32_t* aoff, uint32_t* fill, int32_t n_s,
                        int32_t* acent, uint8_t* aneg, uint32_t* apack, hipStream_t s);
void launch_back(const uint32_t* perm, int64_t m, int32_t* back, hipStream_t s);
void launch_check_dup(const uint32_t* ckey, const uint32_t* packed, int64_t m, DevStatus* st, hipStream_t s);
void launch_work(const uint32_t* aoff, const int32_t* acent, const int32_t* back, const uint32_t* coff, int32_t n_s,
                 uint32_t* key, DevStatus* st, hipStream_t s);
bool wedge_shape_ok(int band_words, int wg);
int wedge_block(int band_words, int wg, bool full);
int wedge_blocks_per_cu(int band_words, int wg, bool full);
void launch_wedge(int band_words, int wg, int grid, const uint32_t* aoff, const int32_t* acent, const uint8_t* aneg,
                  const int32_t* back, const uint32_t* coff, const uint32_t* packed, const uint32_t* order,
                  int32_t n_s, DevStatus* st, unsigned long long* pv, const uint32_t* inv, int64_t anchor_base,
                  int64_t centre_base, int64_t n_centre, hipStream_t s);

__global__ void k_status_init(DevStatus* st) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->flags = 0;
        st->bad_offset = st->bad_range = st->bad_sign = st->bad_dup = INT64_MAX;
        st->total = 0;
        st->wedges = 0;
        st->bands = 0;
        st->queue = 0;
    }
}
}  // namespace bbc

using namespace bbc;

struct bbc_ctx {
    int device = 0;
    int n_cu = 0;
    char* arena = nullptr;
    size_t arena_bytes = 0;
    DevStatus* st_dev = nullptr;
    DevStatus* st_host = nullptr;  // pinned
    hipEvent_t ev[5] = {};
    bbc_stats stats = {};
    std::string err;
};

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

// Bump allocator over the context arena (256-byte aligned pieces).
struct Carve {
    char* base;
    size_t used = 0;
    explicit Carve(char* b) : base(b) {}
    template <class T>
    T* take(int64_t n) {
        size_t bytes = ((size_t)(n > 0 ? n : 1) * sizeof(T) + 255) & ~(size_t)255;
        T* p = (T*)(base + used);
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

#define HIP_OR_FAIL(call)                                \
    do {                                                 \
        hipError_t _e = (call);                          \
        if (_e != hipSuccess) return hip_fail(ctx, _e, #call); \
    } while (0)

// All buffers of one call, carved from the arena in a fixed order.
struct Plan {
    int64_t m;
    int32_t n_u, n_v, n_s, n_c;
    uint32_t *deg_u, *deg_v;
    uint32_t *rk_key, *rk_ka, *rk_kb, *rk_va, *rk_vb;  // rank sort
    int32_t* rank;
    uint32_t *adeg, *aoff, *fill, *coff;
    int32_t* acent;
    uint8_t* aneg;
    uint32_t *apack, *k_a, *k_b, *v0_a, *v0_b, *v1_a, *v1_b;
    int32_t* back;
    uint32_t *wkey, *ord_a, *ord_b, *ord_va, *ord_vb;
    uint32_t *hist, *hist_scan, *partials;

    size_t carve(char* base) {
        Carve c(base);
        int64_t ns1 = (int64_t)n_s + 1, nc1 = (int64_t)n_c + 1;
        int64_t nmax = m > ns1 ? m : ns1;
        if (nc1 > nmax) nmax = nc1;
        deg_u = c.take<uint32_t>(n_u);
        deg_v = c.take<uint32_t>(n_v);
        rk_key = c.take<uint32_t>(n_s);
        rk_ka = c.take<uint32_t>(n_s);
        rk_kb = c.take<uint32_t>(n_s);
        rk_va = c.take<uint32_t>(n_s);
        rk_vb = c.take<uint32_t>(n_s);
        rank = c.take<int32_t>(n_s);
        adeg = c.take<uint32_t>(ns1);
        aoff = c.take<uint32_t>(ns1);
        fill = c.take<uint32_t>(n_s);
        coff = c.take<uint32_t>(nc1);
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
        ord_a = c.take<uint32_t>(n_s);
        ord_b = c.take<uint32_t>(n_s);
        ord_va = c.take<uint32_t>(n_s);
        ord_vb = c.take<uint32_t>(n_s);
        int64_t hs = (int64_t)radix_hist_size(nmax);
        hist = c.take<uint32_t>(hs);
        hist_scan = c.take<uint32_t>(hs + 1);
        int64_t ps = (int64_t)scan_partials_size(hs + nmax + 8);
        partials = c.take<uint32_t>(ps);
        return c.used;
    }
};

bbc_status ensure_arena(bbc_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->arena_bytes) return BBC_OK;
    if (ctx->arena) {
        (void)hipFree(ctx->arena);
        ctx->arena = nullptr;
        ctx->arena_bytes = 0;
    }
    size_t want = bytes + bytes / 8 + (1u << 20);
    hipError_t e = hipMalloc((void**)&ctx->arena, want);
    if (e != hipSuccess) {
        ctx->arena = nullptr;
        (void)hipGetLastError();
        return fail(ctx, BBC_ENOMEM, "scratch allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->arena_bytes = want;
    return BBC_OK;
}

}  // namespace

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
    if (!ctx) return BBC_EINVAL;
    ctx->err.clear();
    bbc_options opts;
    bbc_options_init(&opts);
    if (opts_in) {
        if (opts_in->struct_size != sizeof(bbc_options)) return fail(ctx, BBC_EINVAL, "bbc_options.struct_size");
        opts = *opts_in;
    }
    if (!total) return fail(ctx, BBC_EINVAL, "total is NULL");
    if (n_u < 0 || n_v < 0 || n_edges < 0) return fail(ctx, BBC_EINVAL, "negative size");
    if (n_edges > INT32_MAX || (int64_t)n_u + (int64_t)n_v > INT32_MAX)
        return fail(ctx, BBC_ETOOBIG, "n_edges or n_u + n_v exceeds INT32_MAX");
    if (!offsets || (n_edges > 0 && (!adj || !signs))) return fail(ctx, BBC_EINVAL, "input pointer is NULL");
    if (opts.side < BBC_SIDE_AUTO || opts.side > BBC_SIDE_V) return fail(ctx, BBC_EINVAL, "bad side option");
    if (!wedge_shape_ok(opts.band_words, opts.wg_size))
        return fail(ctx, BBC_EINVAL, "no wedge kernel instance for this band_words / wg_size");
    if (opts.wg_per_cu < 0) return fail(ctx, BBC_EINVAL, "negative wg_per_cu");

    hipStream_t s = (hipStream_t)stream;
    DeviceGuard guard(ctx->device);
    const int64_t m = n_edges;
    const bool s_is_u = opts.side == BBC_SIDE_U || (opts.side == BBC_SIDE_AUTO && n_u < n_v);
    Plan P;
    P.m = m;
    P.n_u = n_u;
    P.n_v = n_v;
    P.n_s = s_is_u ? n_u : n_v;
    P.n_c = s_is_u ? n_v : n_u;
    size_t need = P.carve(nullptr);
    bbc_status rc = ensure_arena(ctx, need);
    if (rc != BBC_OK) return rc;
    P.carve(ctx->arena);
    const bool timing = opts.timing != 0;

    if (timing) HIP_OR_FAIL(hipEventRecord(ctx->ev[0], s));
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, s, ctx->st_dev);
    launch_checks(offsets, adj, signs, n_u, n_v, m, (opts.checks & BBC_CHECK_SIGNS) ? 1 : 0, ctx->st_dev, s);
    HIP_OR_FAIL(hipGetLastError());
    HIP_OR_FAIL(hipMemcpyAsync(ctx->st_host, ctx->st_dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    {
        const DevStatus& h = *ctx->st_host;
        char buf[160];
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
    }
    if (timing) HIP_OR_FAIL(hipEventRecord(ctx->ev[1], s));

    // degrees and ranks (Definition 6: degree, then id; ascending)
    launch_degrees(offsets, adj, n_u, m, P.deg_u, P.deg_v, n_v, s);
    const uint32_t* deg_s = s_is_u ? P.deg_u : P.deg_v;
    const uint32_t* deg_c = s_is_u ? P.deg_v : P.deg_u;
    const uint32_t *rk_k = nullptr, *inv = nullptr;
    radix_sort(deg_s, P.rk_ka, P.rk_kb, nullptr, nullptr, nullptr, nullptr, P.rk_va, P.rk_vb, P.n_s,
               bits_for((uint64_t)P.n_c), P.hist, P.hist_scan, P.partials, s, &rk_k, nullptr, &inv);
    launch_ranks(inv, deg_s, P.n_s, P.rank, P.adeg, s);
    scan_exclusive_u32(P.adeg, P.aoff, P.n_s, P.partials, s);

    // anchor lists, then centre lists by a stable sort on the centre id of
    // the rank-ordered anchor entries (each centre list comes out rank-sorted)
    launch_fill_anchor(offsets, adj, signs, n_u, m, s_is_u ? 1 : 0, P.rank, P.aoff, P.fill, P.n_s, P.acent, P.aneg,
                       P.apack, s);
    const uint32_t *ckey = nullptr, *packed = nullptr, *perm = nullptr;
    radix_sort((const uint32_t*)P.acent, P.k_a, P.k_b, P.apack, P.v0_a, P.v0_b, nullptr, P.v1_a, P.v1_b, m,
               bits_for(P.n_c > 0 ? (uint64_t)(P.n_c - 1) : 0), P.hist, P.hist_scan, P.partials, s, &ckey, &packed,
               &perm);
    scan_exclusive_u32(deg_c, P.coff, P.n_c, P.partials, s);
    launch_back(perm, m, P.back, s);
    if (opts.checks & BBC_CHECK_DUPLICATES) launch_check_dup(ckey, packed, m, ctx->st_dev, s);

    // schedule: anchors by descending work
    launch_work(P.aoff, P.acent, P.back, P.coff, P.n_s, P.wkey, ctx->st_dev, s);
    const uint32_t *ok = nullptr, *order = nullptr;
    radix_sort(P.wkey, P.ord_a, P.ord_b, nullptr, nullptr, nullptr, nullptr, P.ord_va, P.ord_vb, P.n_s, 32, P.hist,
               P.hist_scan, P.partials, s, &ok, nullptr, &order);
    HIP_OR_FAIL(hipGetLastError());
    if (timing) HIP_OR_FAIL(hipEventRecord(ctx->ev[2], s));

    const bool full = per_vertex != nullptr;
    unsigned long long* pv = (unsigned long long*)per_vertex;
    if (full) fill_bytes(pv, ((int64_t)n_u + n_v) * 8, s);
    const int block = wedge_block(opts.band_words, opts.wg_size, full);
    const int grid =
        ctx->n_cu * (opts.wg_per_cu > 0 ? opts.wg_per_cu : wedge_blocks_per_cu(opts.band_words, opts.wg_size, full));
    if (P.n_s >= 2 && m > 0)
        launch_wedge(opts.band_words, opts.wg_size, grid, P.aoff, P.acent, P.aneg, P.back, P.coff, packed, order,
                     P.n_s, ctx->st_dev, pv, inv, s_is_u ? 0 : n_u, s_is_u ? n_u : 0, P.n_c, s);
    HIP_OR_FAIL(hipGetLastError());
    if (timing) HIP_OR_FAIL(hipEventRecord(ctx->ev[3], s));
    HIP_OR_FAIL(hipMemcpyAsync(ctx->st_host, ctx->st_dev, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    HIP_OR_FAIL(hipStreamSynchronize(s));
    const DevStatus& h = *ctx->st_host;
    if (h.flags & kBadDup) {
        char buf[160];
        snprintf(buf, sizeof buf, "repeated (u, v) pair at centre-list position %lld", (long long)h.bad_dup);
        return fail(ctx, BBC_EDUP, buf);
    }
    // per-vertex mode sums every anchor's pairs from both ends
    *total = full ? (uint64_t)h.total / 2 : (uint64_t)h.total;

    bbc_stats& S = ctx->stats;
    memset(&S, 0, sizeof S);
    S.struct_size = sizeof(bbc_stats);
    S.side = s_is_u ? BBC_SIDE_U : BBC_SIDE_V;
    S.n_anchor = P.n_s;
    S.n_centre = P.n_c;
    S.n_edges = m;
    S.wedges = h.wedges;
    S.bands = h.bands;
    S.grid = grid;
    S.block = block;
    if (timing) {
        HIP_OR_FAIL(hipEventElapsedTime(&S.ms_checks, ctx->ev[0], ctx->ev[1]));
        HIP_OR_FAIL(hipEventElapsedTime(&S.ms_build, ctx->ev[1], ctx->ev[2]));
        HIP_OR_FAIL(hipEventElapsedTime(&S.ms_count, ctx->ev[2], ctx->ev[3]));
        HIP_OR_FAIL(hipEventElapsedTime(&S.ms_total, ctx->ev[0], ctx->ev[3]));
    }
    return BBC_OK;
}

}  // extern "C"
