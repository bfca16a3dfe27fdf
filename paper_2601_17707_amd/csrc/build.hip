// Input checks and the degree-ordered CSR, built on the device.
//
// Anchor side S and centre side C: every wedge is u - c - w with u, w in S
// and c in C.  Anchors are ranked by the vertex priority of Definition 6
// (degree, then id), ascending, so "w ranked above u" is rank(w) > rank(u).
// In a batch every graph keeps its own anchor side and the ranks are
// ordered by (graph, degree, id), so each graph owns a contiguous rank range.
// Two views are built:
//   anchor lists (rank order): aoff[n_S + 1], acent[m] (centre id),
//     aneg[m] (1 = negative edge), back[m] = position of the anchor inside
//     its centre's list;
//   centre lists: coff[n_C + 1], packed[m] = rank << 1 | neg, ascending in
//     rank, so the endpoints ranked above an anchor form a suffix that starts
//     right after back[].
// The paper sorts each neighbour list by priority (Algorithm 1) and, for
// G-BBC++, sorts anchors by a fanout work estimate on the host
// (Algorithm 4); here both are device radix sorts.
//
// Every kernel after the input checks first reads the status flags and does
// nothing once an input error is flagged, so the whole sequence can be
// queued (or captured in a graph) without waiting for the checks.
#include "bbc_internal.h"

namespace bbc {

__device__ __forceinline__ void flag_bad(DevStatus* st, int32_t bit, int64_t* slot, int64_t idx) {
    atomicOr(&st->flags, bit);
    atomicMin((unsigned long long*)slot, (unsigned long long)idx);
}

__device__ __forceinline__ bool input_bad(const DevStatus* st) { return *(volatile const int32_t*)&st->flags != 0; }

#define GRID_STRIDE(i, n)                                                       \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

// ------------------------------------------------------------------ checks

// offsets[0] == 0, offsets[n_u] == m, non-decreasing
__global__ void k_check_offsets(const int32_t* off, int32_t n_u, int64_t m, DevStatus* st) {
    GRID_STRIDE(i, (int64_t)n_u + 1) {
        int32_t o = off[i];
        bool bad = (i == 0 && o != 0) || (i == n_u && (int64_t)o != m) || (i < n_u && off[i + 1] < o);
        if (bad) flag_bad(st, kBadOffsets, &st->bad_offset, i);
    }
}

// The same per graph of a batch, one workgroup per graph; the reported
// index is the position in the concatenated offsets array.
__global__ void k_check_offsets_batched(const int32_t* off_cat, const DevGraph* gr, DevStatus* st) {
    const DevGraph g = gr[blockIdx.x];
    const int32_t* off = off_cat + g.off_base;
    for (int64_t i = threadIdx.x; i <= g.n_u; i += blockDim.x) {
        int32_t o = off[i];
        bool bad = (i == 0 && o != 0) || (i == g.n_u && (int64_t)o != g.n_edges) || (i < g.n_u && off[i + 1] < o);
        if (bad) flag_bad(st, kBadOffsets, &st->bad_offset, g.off_base + i);
    }
}

// Row of CSR entry e among rows [lo, hi]: the last u with off[u] <= e (in
// range even for malformed offsets; those are flagged separately).
__device__ __forceinline__ int32_t row_in(const int32_t* off, int32_t lo, int32_t hi, int64_t e) {
    while (lo < hi) {
        int32_t mid = lo + (hi - lo + 1) / 2;
        if ((int64_t)off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Graph of batch edge j among graphs [lo, hi]: the last g with vstart[g] <= j.
__device__ __forceinline__ int32_t graph_in(const int64_t* vstart, int32_t lo, int32_t hi, int64_t j) {
    while (lo < hi) {
        int32_t mid = lo + (hi - lo + 1) / 2;
        if (vstart[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// The decode kernels give each workgroup a chunk of kDecChunk consecutive
// edges.  The rows (and graphs) of the chunk lie between those of its first
// and last edge, found once per workgroup by binary search; every row that
// starts inside the chunk marks its first edge in LDS (an empty row shares
// its start with the next row, and the larger index wins), and a running
// maximum over the chunk then gives every edge its row.
constexpr int kDecThreads = 256;
constexpr int kDecItems = 16;  // marks per thread in the running maximum
constexpr int kDecChunk = kDecThreads * kDecItems;
constexpr int kDecGroup = 4;  // edges per thread whose loads are issued together

// LDS index of chunk position i: one pad word per 16 keeps the running
// maximum (thread t reads positions 16 t ..) free of bank conflicts
__device__ __forceinline__ int dec_slot(int i) { return i + (i >> 4); }

// In-place running maximum of the chunk's marks (kDecChunk entries, -1
// where nothing starts), seeded with seed.  Ends with a barrier.
__device__ __forceinline__ void dec_running_max(int32_t* marks, int32_t seed, int32_t* wmax) {
    const int t = threadIdx.x, lane = lane_id(), wave = t / kWave;
    int32_t v[kDecItems];
    int32_t run = -1;
#pragma unroll
    for (int k = 0; k < kDecItems; ++k) {
        run = max(run, marks[dec_slot(t * kDecItems + k)]);
        v[k] = run;
    }
    int32_t x = run;  // inclusive maximum over the wave's threads
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const int32_t y = __shfl_up(x, o, kWave);
        if (lane >= o) x = max(x, y);
    }
    if (lane == kWave - 1) wmax[wave] = x;
    int32_t before = __shfl_up(x, 1, kWave);
    if (lane == 0) before = -1;
    __syncthreads();
    for (int w = 0; w < wave; ++w) before = max(before, wmax[w]);
    before = max(before, seed);
#pragma unroll
    for (int k = 0; k < kDecItems; ++k) marks[dec_slot(t * kDecItems + k)] = max(before, v[k]);
    __syncthreads();
}

// Edge e of a single graph -> anchor id ea[e] and either pay[e] = centre id
// | negative << 31 (the count) or ec[e] and en[e] (other users), with the
// id-range and sign checks.
__global__ __launch_bounds__(kDecThreads) void k_decode_single(const int32_t* off, const int32_t* adj,
                                                               const int8_t* sg, int32_t n_u, int32_t n_v, int64_t m,
                                                               int s_is_u, int check_sign, DevStatus* st, uint32_t* ea,
                                                               uint32_t* ec, uint8_t* en, uint32_t* pay) {
    __shared__ int32_t rr[2];
    __shared__ int32_t rowof[kDecChunk + kDecChunk / 16];
    __shared__ int32_t wmax[kDecThreads / kWave];
    const int t = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * kDecChunk;
    const int64_t e1 = min(m, e0 + kDecChunk);
    if (t < 2) rr[t] = row_in(off, 0, n_u - 1, t ? e1 - 1 : e0);
    for (int i = t; i < kDecChunk + kDecChunk / 16; i += kDecThreads) rowof[i] = -1;
    __syncthreads();
    const int32_t lo = rr[0], hi = rr[1];
    for (int32_t u = lo + 1 + t; u <= hi; u += kDecThreads) {
        const int64_t s = off[u];
        if (s > e0 && s < e1) atomicMax(&rowof[dec_slot((int)(s - e0))], u);
    }
    __syncthreads();
    dec_running_max(rowof, lo, wmax);
    for (int64_t e = e0 + t; e < e1; e += kDecThreads) {
        const int32_t u = rowof[dec_slot((int)(e - e0))];
        const int32_t v = adj[e];
        const int8_t s = sg ? sg[e] : (int8_t)1;  // no signs: the block planner
        if (v < 0 || v >= n_v) flag_bad(st, kBadRange, &st->bad_range, e);
        if (check_sign && s != 1 && s != -1) flag_bad(st, kBadSign, &st->bad_sign, e);
        const uint32_t neg = s < 0 ? 1u : 0u;
        ea[e] = (uint32_t)(s_is_u ? u : v);
        if (pay) {
            pay[e] = (uint32_t)(s_is_u ? v : u) | (neg << 31);
        } else {
            ec[e] = (uint32_t)(s_is_u ? v : u);
            if (en) en[e] = (uint8_t)neg;
        }
    }
}

// Edge j of a batch (graphs laid end to end by vstart, a prefix of the edge
// counts) -> global anchor id ea[j] and pay[j] = global centre id |
// negative << 31.  Each graph's anchors and centres are numbered from its
// anchor_base / centre_base.  Graph starts and row starts are marked as
// above; row u of graph g is marked by anchor_base + centre_base + u, which
// grows along the batch (each graph adds n_u + n_v to the base).
__global__ __launch_bounds__(kDecThreads) void k_decode_batched(const int32_t* __restrict__ off_cat,
                                                                const int32_t* __restrict__ adj_cat,
                                                                const int8_t* __restrict__ sg_cat,
                                                                const DevGraph* __restrict__ gr,
                                                                const int64_t* __restrict__ vstart, int32_t n_graphs,
                                                                int64_t m, int check_sign, DevStatus* st,
                                                                uint32_t* __restrict__ ea, uint32_t* __restrict__ pay) {
    __shared__ int32_t gg[2], rr[2];
    __shared__ int32_t graphof[kDecChunk + kDecChunk / 16];
    __shared__ int32_t rowof[kDecChunk + kDecChunk / 16];
    __shared__ int32_t wmax[kDecThreads / kWave];
    const int t = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * kDecChunk;
    const int64_t e1 = min(m, e0 + kDecChunk);
    if (t < 2) gg[t] = graph_in(vstart, 0, n_graphs - 1, t ? e1 - 1 : e0);
    for (int i = t; i < kDecChunk + kDecChunk / 16; i += kDecThreads) graphof[i] = rowof[i] = -1;
    __syncthreads();
    if (t < 2) {  // rows of the first and last edge inside their graphs
        const DevGraph g = gr[gg[t]];
        rr[t] = row_in(off_cat + g.off_base, 0, g.n_u - 1, (t ? e1 - 1 : e0) - vstart[gg[t]]);
    }
    const int32_t g_lo = gg[0], g_hi = gg[1];
    for (int32_t g = g_lo + 1 + t; g <= g_hi; g += kDecThreads) {
        const int64_t s = vstart[g];
        if (s > e0 && s < e1) atomicMax(&graphof[dec_slot((int)(s - e0))], g);
    }
    __syncthreads();
    for (int32_t g = g_lo; g <= g_hi; ++g) {
        const DevGraph G = gr[g];
        const int64_t vs = vstart[g];
        const int32_t u0 = g == g_lo ? rr[0] + 1 : 0, u1 = g == g_hi ? rr[1] : G.n_u - 1;
        for (int32_t u = u0 + t; u <= u1; u += kDecThreads) {
            const int64_t s = vs + off_cat[G.off_base + u];
            if (s > e0 && s < e1) atomicMax(&rowof[dec_slot((int)(s - e0))], (int32_t)(G.anchor_base + G.centre_base + u));
        }
    }
    __syncthreads();
    dec_running_max(graphof, g_lo, wmax);
    dec_running_max(rowof, (int32_t)(gr[g_lo].anchor_base + gr[g_lo].centre_base + rr[0]), wmax);
    // kDecGroup edges per thread at a time, every load of the group issued
    // before any of its values is used (the graph of an edge decides where
    // its adjacency entry lies)
    for (int64_t jb = e0 + t; jb < e1; jb += kDecGroup * kDecThreads) {
        int32_t gi[kDecGroup], uu[kDecGroup];
#pragma unroll
        for (int q = 0; q < kDecGroup; ++q) {
            const int64_t j = jb + q * kDecThreads;
            const int slot = dec_slot((int)(min(j, e1 - 1) - e0));
            gi[q] = graphof[slot];
            uu[q] = rowof[slot];
        }
        int64_t pe[kDecGroup], ab[kDecGroup], cb[kDecGroup];
        int32_t nv[kDecGroup], su[kDecGroup];
#pragma unroll
        for (int q = 0; q < kDecGroup; ++q) {
            const DevGraph& g = gr[gi[q]];
            pe[q] = g.edge_base + (min(jb + q * kDecThreads, e1 - 1) - vstart[gi[q]]);
            ab[q] = g.anchor_base;
            cb[q] = g.centre_base;
            nv[q] = g.n_v;
            su[q] = g.s_is_u;
        }
        int32_t v[kDecGroup];
        int8_t sv[kDecGroup];
#pragma unroll
        for (int q = 0; q < kDecGroup; ++q) {
            v[q] = adj_cat[pe[q]];
            sv[q] = sg_cat[pe[q]];
        }
#pragma unroll
        for (int q = 0; q < kDecGroup; ++q) {
            const int64_t j = jb + q * kDecThreads;
            if (j >= e1) continue;
            const int32_t u = uu[q] - (int32_t)(ab[q] + cb[q]);
            if (v[q] < 0 || v[q] >= nv[q]) flag_bad(st, kBadRange, &st->bad_range, pe[q]);
            if (check_sign && sv[q] != 1 && sv[q] != -1) flag_bad(st, kBadSign, &st->bad_sign, pe[q]);
            ea[j] = (uint32_t)(ab[q] + (su[q] ? u : v[q]));
            pay[j] = (uint32_t)(cb[q] + (su[q] ? v[q] : u)) | ((sv[q] < 0 ? 1u : 0u) << 31);
        }
    }
}

// Degrees from a sorted id array: every id's entries form one run, so the
// run's first position goes to first[id] and its end to deg[id] (zeroed
// beforehand); k_run_degrees then leaves the run length in deg (0 for ids
// that never occur).  Nothing runs after an input error (ids may be out of
// range then).
__global__ void k_run_bounds(const uint32_t* key, int64_t m, uint32_t* first, uint32_t* deg, const DevStatus* st) {
    if (input_bad(st)) return;
    GRID_STRIDE(p, m) {
        const uint32_t k = key[p];
        if (p == 0 || key[p - 1] != k) first[k] = (uint32_t)p;
        if (p == m - 1 || key[p + 1] != k) deg[k] = (uint32_t)(p + 1);
    }
}

__global__ void k_run_degrees(const uint32_t* first, int64_t n, uint32_t* deg) {
    GRID_STRIDE(i, n) {
        const uint32_t end = deg[i];
        deg[i] = end ? end - first[i] : 0u;
    }
}

// Anchor lists in rank order from the edges sorted (stably) by anchor id:
// the run of anchor a moves, in its order, to aoff[rank[a]]; each entry
// becomes centre id, sign, and the packed rank << 1 | neg that goes into
// the centre lists.
__global__ void k_move_lists(const uint32_t* __restrict__ key, const uint32_t* __restrict__ pay, int64_t m,
                             const uint32_t* __restrict__ first, const int32_t* __restrict__ rank,
                             const uint32_t* __restrict__ aoff, int32_t* __restrict__ acent,
                             uint8_t* __restrict__ aneg, uint32_t* __restrict__ apack, const DevStatus* st) {
    if (input_bad(st)) return;
    constexpr int U = 4;  // entries per thread whose gathers are in flight together
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * U;
    for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x * U + threadIdx.x; p0 < m; p0 += stride) {
        uint32_t a[U], c[U], f[U], o[U];
        int32_t r[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = p0 + (int64_t)u * blockDim.x;
            a[u] = p < m ? key[p] : 0u;
            c[u] = p < m ? pay[p] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = p0 + (int64_t)u * blockDim.x;
            r[u] = p < m ? rank[a[u]] : 0;
            f[u] = p < m ? first[a[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = p0 + (int64_t)u * blockDim.x;
            o[u] = p < m ? aoff[r[u]] : 0u;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = p0 + (int64_t)u * blockDim.x;
            if (p < m) {
                const int64_t q = (int64_t)o[u] + (p - (int64_t)f[u]);
                acent[q] = (int32_t)(c[u] & 0x7fffffffu);
                aneg[q] = (uint8_t)(c[u] >> 31);
                apack[q] = ((uint32_t)r[u] << 1) | (c[u] >> 31);
            }
        }
    }
}

// ------------------------------------------------------------------ degrees

__global__ void k_hist(const uint32_t* ids, int64_t n, uint32_t* deg, const DevStatus* st) {
    if (input_bad(st)) return;
    GRID_STRIDE(i, n) atomicAdd(&deg[ids[i]], 1u);
}

// The same histogram over nrep zeroed replicas: workgroup b adds into
// replica b % nrep (consecutive workgroups run on different XCDs), which
// spreads the atomics on the few ids of very high degree; k_hist_sum then
// adds the replicas up into deg.
__global__ void k_hist_rep(const uint32_t* ids, int64_t n, uint32_t* rep, int64_t n_bins, int nrep,
                           const DevStatus* st) {
    if (input_bad(st)) return;
    uint32_t* h = rep + (int64_t)(blockIdx.x % nrep) * n_bins;
    GRID_STRIDE(i, n) atomicAdd(&h[ids[i]], 1u);
}

__global__ void k_hist_sum(const uint32_t* rep, int64_t n_bins, int nrep, uint32_t* deg) {
    GRID_STRIDE(v, n_bins) {
        uint32_t s = 0;
        for (int c = 0; c < nrep; ++c) s += rep[(int64_t)c * n_bins + v];
        deg[v] = s;
    }
}

// Wedges of each anchor-side choice: the walk from anchors on one side
// visits every pair of neighbours of every centre once, sum of C(deg, 2)
// over the other side.  k_side_rows adds C(deg, 2) of the U rows into
// out[0] (the walk from anchors on V); k_side_hist counts V degrees (ids
// outside [0, n_v) are skipped: the count's own checks report them) and
// k_side_bins adds their C(deg, 2) into out[1] (anchors on U).  Rows with
// decreasing offsets count as empty here.
__device__ __forceinline__ unsigned long long choose2_u64(long long d) {
    return d > 1 ? (unsigned long long)d * (unsigned long long)(d - 1) / 2ull : 0ull;
}

__global__ void k_side_rows(const int32_t* off, int32_t n_u, unsigned long long* out) {
    unsigned long long acc = 0;
    GRID_STRIDE(i, n_u) acc += choose2_u64((long long)off[i + 1] - (long long)off[i]);
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(&out[0], acc);
}

__global__ void k_side_hist(const int32_t* adj, int64_t m, int32_t n_v, uint32_t* deg) {
    GRID_STRIDE(i, m) {
        const int32_t v = adj[i];
        if (v >= 0 && v < n_v) atomicAdd(&deg[v], 1u);
    }
}

__global__ void k_side_bins(const uint32_t* deg, int32_t n_v, unsigned long long* out) {
    unsigned long long acc = 0;
    GRID_STRIDE(i, n_v) acc += choose2_u64(deg[i]);
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(&out[1], acc);
}

// graph id of every anchor of a batch (one workgroup per graph)
__global__ void k_anchor_graph(const DevGraph* gr, uint32_t* agid) {
    const DevGraph g = gr[blockIdx.x];
    const int64_t n_s = g.s_is_u ? g.n_u : g.n_v;
    for (int64_t i = threadIdx.x; i < n_s; i += blockDim.x) agid[g.anchor_base + i] = blockIdx.x;
}

__global__ void k_gather(const uint32_t* idx, const uint32_t* src, int64_t n, uint32_t* out) {
    GRID_STRIDE(i, n) out[i] = src[idx[i]];
}

// inv[r] = anchor id of rank r (the sorted payload); rank[id] = r;
// adeg[r] = degree of that anchor; agraph[r] = its graph (batches)
__global__ void k_ranks(const uint32_t* inv, const uint32_t* deg_s, int64_t n_s, int32_t* rank, uint32_t* adeg,
                        const uint32_t* agid, int32_t* agraph) {
    GRID_STRIDE(r, n_s) {
        uint32_t id = inv[r];
        rank[id] = (int32_t)r;
        adeg[r] = deg_s[id];
        if (agraph) agraph[r] = (int32_t)agid[id];
    }
}

// A repeated (u, v) pair shows up as the same anchor rank twice in a row of
// one centre's sorted list.
__global__ void k_check_dup(const uint32_t* ckey, const uint32_t* packed, int64_t m, DevStatus* st) {
    if (input_bad(st)) return;
    GRID_STRIDE(q, m - 1) {
        if (ckey[q] == ckey[q + 1] && (packed[q] >> 1) == (packed[q + 1] >> 1))
            flag_bad(st, kBadDup, &st->bad_dup, q);
    }
}

// Per-anchor work: the number of wedges the anchor walks, i.e. the suffix
// lengths of its centres' lists (ranked-above endpoints; an anchor of a
// dense block starts past the block's anchors in the block's centres).  One
// thread per anchor-list entry; the entries of an anchor are contiguous, so
// a wave sums runs of equal rank with a segmented scan and adds each run
// once.  st->wedges receives the sum over centres of C(deg, 2), st->walked
// the wedges the walk visits.
__global__ __launch_bounds__(256) void k_work(const uint32_t* __restrict__ apack, const int32_t* __restrict__ acent,
                                              const int32_t* __restrict__ back, const uint32_t* __restrict__ coff,
                                              int64_t m, unsigned long long* __restrict__ work, DevStatus* st,
                                              HybridView hv) {
    if (input_bad(st)) return;
    constexpr int U = 4;  // entries per thread whose loads are in flight together
    __shared__ unsigned long long red[256 / kWave];
    const int lane = lane_id();
    unsigned long long all = 0, walked = 0;
    // whole waves walk the entries, so the scan below sees every lane
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * U;
    for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x * U; p0 < m; p0 += stride) {
        uint32_t r[U];
        unsigned long long wk[U];
        int32_t c[U];
        uint32_t bk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t p = p0 + u * blockDim.x + threadIdx.x;
            r[u] = 0xffffffffu;
            c[u] = 0;
            bk[u] = 0;
            if (p < m) {
                r[u] = apack[p] >> 1;
                c[u] = acent[p];
                bk[u] = (uint32_t)back[p];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            wk[u] = 0;
            if (r[u] != 0xffffffffu) {
                const uint32_t suffix = coff[c[u] + 1] - bk[u] - 1u;
                all += suffix;
                wk[u] = suffix;
                if (hv.ablk1) {
                    const int32_t blk = (int32_t)hv.ablk1[r[u]] - 1;
                    if (blk >= 0 && hv.cblk[c[u]] == blk) wk[u] = coff[c[u] + 1] - (uint32_t)hv.cpos[c[u]];
                }
                walked += wk[u];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // inclusive segmented sum over lanes of equal rank
            unsigned long long x = wk[u];
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const unsigned long long y = __shfl_up(x, o, kWave);
                const uint32_t ry = __shfl_up(r[u], o, kWave);
                if (lane >= o && ry == r[u]) x += y;
            }
            const uint32_t rn = __shfl_down(r[u], 1, kWave);
            if (r[u] != 0xffffffffu && (lane == kWave - 1 || rn != r[u]) && x) atomicAdd(&work[r[u]], x);
        }
    }
    all = block_sum<256>(all, red);
    walked = block_sum<256>(walked, red);
    if (threadIdx.x == 0 && all) atomicAdd(&st->wedges, all);
    if (threadIdx.x == 0 && walked) atomicAdd(&st->walked, walked);
}

// Sort key of each anchor: the bitwise complement of its clamped work, so an
// ascending sort orders anchors by descending work (heavy anchors start
// first, as in the fanout ordering of Algorithm 4).
// Sort keys of the schedule (ascending): anchors of the workgroup regime by
// descending work in [0, 2^31), then the wave regime (light anchors, see
// kLightMaxWork) in [2^31, 2^32): a batch keeps each graph's light anchors
// together (key = graph), a single graph orders them by descending work.
// light_w = 0 puts every anchor in the workgroup regime.  st->n_light
// receives the number of light anchors (one atomic per workgroup).
__global__ __launch_bounds__(256) void k_work_keys(const unsigned long long* work, int64_t n_s, uint32_t* key,
                                                   const uint32_t* aoff, const int32_t* agraph,
                                                   const int64_t* rank_end, const uint32_t* ablk1, uint32_t light_w,
                                                   DevStatus* st) {
    __shared__ unsigned long long red[256 / kWave];
    unsigned long long n_light = 0;
    GRID_STRIDE(r, n_s) {
        const unsigned long long w = work[r];
        const uint32_t deg = aoff[r + 1] - aoff[r];
        const int64_t n_end = agraph ? rank_end[agraph[r] + 1] : n_s;
        const bool light = light_w > 0 && w <= light_w && deg <= (uint32_t)kLightMaxDeg && n_end - r <= (1ll << kLightKeyBits) &&
                           !(ablk1 && ablk1[r]);
        const uint32_t wc = w > 0x7fffffffull ? 0x7fffffffu : (uint32_t)w;
        if (light) {
            key[r] = 0x80000000u | (agraph ? (uint32_t)agraph[r] : 0x7fffffffu - wc);
            ++n_light;
        } else {
            key[r] = 0x7fffffffu - wc;
        }
    }
    n_light = block_sum<256>(n_light, red);
    if (threadIdx.x == 0 && n_light) atomicAdd(&st->n_light, (unsigned int)n_light);
}

// ------------------------------------------------------ band-boundary index
//
// The wedge kernel walks each centre list in bands of endpoint ranks whose
// ends are multiples of a granule G = 2^gs.  For every centre c it needs
// pos(c, k) = the first position of its list with rank >= k G.  Below the
// granule of the list's first entry that is the list start, above the
// granule of its last entry the list end; the positions in between,
// klo = (first rank >> gs) + 1 <= k <= khi = last rank >> gs, are stored
// once per call as idx[ioff[c] + k - klo] -- but only for lists with at
// least as many entries as boundaries (khi - klo + 1 <= length), so the
// index never exceeds m entries.  Shorter lists spread over many granules
// are not indexed: the kernel finds their band ends by stepping forward
// from its cursor (each entry is passed once per anchor).

// Number of index entries of list c: its boundary count, or 0 if the list
// is shorter than that (or the input is bad).
__device__ __forceinline__ uint32_t bidx_entries(const uint32_t* coff, const uint32_t* packed, int64_t c, int gs) {
    const uint32_t a = coff[c], b = coff[c + 1];
    if (a == b) return 0u;
    const uint32_t nbr = ((packed[b - 1] >> 1) >> gs) - ((packed[a] >> 1) >> gs);
    return nbr <= b - a ? nbr : 0u;
}

__global__ void k_bidx_count(const uint32_t* coff, const uint32_t* packed, int64_t n_c, int gs, uint32_t* nb,
                             const DevStatus* st) {
    const bool bad = input_bad(st);
    GRID_STRIDE(c, n_c) nb[c] = bad ? 0u : bidx_entries(coff, packed, c, gs);
}

// One thread per list entry q > list start of an indexed list: the granule
// boundaries that fall between the previous entry's rank and its own point
// at q.
// The neighbour entries are read first (coalesced): an entry that starts
// its list or crosses no boundary needs no lookup of its centre.
__global__ void k_bidx_fill(const uint32_t* __restrict__ ckey, const uint32_t* __restrict__ coff,
                            const uint32_t* __restrict__ packed, int64_t m, int gs, const uint32_t* __restrict__ ioff,
                            uint32_t* __restrict__ idx, const DevStatus* st) {
    if (input_bad(st)) return;
    GRID_STRIDE(q, m) {
        if (q == 0) continue;
        const uint32_t c = ckey[q];
        const uint32_t g = (packed[q] >> 1) >> gs, gp = (packed[q - 1] >> 1) >> gs;
        if (ckey[q - 1] != c || g == gp) continue;  // list start, or no granule boundary crossed
        const uint32_t i0 = ioff[c];
        if (ioff[c + 1] == i0) continue;  // list not indexed
        const uint32_t klo = ((packed[coff[c]] >> 1) >> gs) + 1u;
        for (uint32_t k = gp + 1; k <= g; ++k) idx[i0 + (k - klo)] = (uint32_t)q;
    }
}

// Per centre: (x, khi) with pos(c, k) = k > khi ? list end : idx[x + k] for
// every k >= klo; x = kBidxNone for a list without index entries.
__global__ void k_bidx_meta(const uint32_t* coff, const uint32_t* packed, const uint32_t* ioff, int64_t n_c, int gs,
                            int2* meta, const DevStatus* st) {
    if (input_bad(st)) return;
    GRID_STRIDE(c, n_c) {
        const uint32_t a = coff[c], b = coff[c + 1];
        int2 v{kBidxNone, -1};
        if (a != b) {
            const int32_t klo = (int32_t)(((packed[a] >> 1) >> gs) + 1u);
            v.y = (int32_t)((packed[b - 1] >> 1) >> gs);
            if (ioff[c + 1] != ioff[c]) v.x = (int32_t)ioff[c] - klo;
        }
        meta[c] = v;
    }
}

// ------------------------------------------------------------ host launchers

static int grid_for(int64_t n, int threads, int cap = 16384) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void launch_decode_single(const int32_t* off, const int32_t* adj, const int8_t* sg, int32_t n_u, int32_t n_v,
                          int64_t m, int s_is_u, int check_sign, DevStatus* st, uint32_t* ea, uint32_t* ec,
                          uint8_t* en, uint32_t* pay, hipStream_t s) {
    hipLaunchKernelGGL(k_check_offsets, dim3(grid_for((int64_t)n_u + 1, 256)), dim3(256), 0, s, off, n_u, m, st);
    if (m > 0)
        hipLaunchKernelGGL(k_decode_single, dim3((unsigned)((m + kDecChunk - 1) / kDecChunk)), dim3(kDecThreads), 0, s,
                           off, adj, sg, n_u, n_v, m, s_is_u, check_sign, st, ea, ec, en, pay);
}

void launch_decode_batched(const int32_t* off_cat, const int32_t* adj_cat, const int8_t* sg_cat, const DevGraph* gr,
                           const int64_t* vstart, int32_t n_graphs, int64_t m, int check_sign, DevStatus* st,
                           uint32_t* ea, uint32_t* pay, hipStream_t s) {
    if (n_graphs <= 0) return;
    hipLaunchKernelGGL(k_check_offsets_batched, dim3(n_graphs), dim3(256), 0, s, off_cat, gr, st);
    if (m > 0)
        hipLaunchKernelGGL(k_decode_batched, dim3((unsigned)((m + kDecChunk - 1) / kDecChunk)), dim3(kDecThreads), 0,
                           s, off_cat, adj_cat, sg_cat, gr, vstart, n_graphs, m, check_sign, st, ea, pay);
}

// deg[id] = number of entries of id in the sorted key array (n ids);
// first[id] = position of its first entry (ids that occur)
void launch_run_degrees(const uint32_t* key, int64_t m, uint32_t* first, uint32_t* deg, int64_t n,
                        const DevStatus* st, hipStream_t s) {
    if (n <= 0) return;
    fill_u32(deg, 0u, n, s);
    if (m > 0) hipLaunchKernelGGL(k_run_bounds, dim3(grid_for(m, 256)), dim3(256), 0, s, key, m, first, deg, st);
    hipLaunchKernelGGL(k_run_degrees, dim3(grid_for(n, 256)), dim3(256), 0, s, first, n, deg);
}

void launch_move_lists(const uint32_t* key, const uint32_t* pay, int64_t m, const uint32_t* first,
                       const int32_t* rank, const uint32_t* aoff, int32_t* acent, uint8_t* aneg, uint32_t* apack,
                       const DevStatus* st, hipStream_t s) {
    if (m > 0)
        hipLaunchKernelGGL(k_move_lists, dim3(grid_for(m, 256)), dim3(256), 0, s, key, pay, m, first, rank, aoff,
                           acent, aneg, apack, st);
}

void launch_hist(const uint32_t* ids, int64_t n, uint32_t* deg, int64_t n_bins, uint32_t* scratch,
                 int64_t scratch_words, const DevStatus* st, hipStream_t s) {
    const int nrep = n_bins > 0 ? (int)std::min<int64_t>(8, scratch_words / n_bins) : 0;
    if (nrep < 2) {  // no room for replicas: one histogram
        fill_u32(deg, 0u, n_bins, s);
        if (n > 0) hipLaunchKernelGGL(k_hist, dim3(grid_for(n, 256)), dim3(256), 0, s, ids, n, deg, st);
        return;
    }
    fill_u32(scratch, 0u, (int64_t)nrep * n_bins, s);
    if (n > 0)
        hipLaunchKernelGGL(k_hist_rep, dim3(grid_for(n, 256)), dim3(256), 0, s, ids, n, scratch, n_bins, nrep, st);
    hipLaunchKernelGGL(k_hist_sum, dim3(grid_for(n_bins, 256)), dim3(256), 0, s, scratch, n_bins, nrep, deg);
}

void launch_side_wedges(const int32_t* off, int32_t n_u, const int32_t* adj, int64_t m, int32_t n_v, uint32_t* deg,
                        unsigned long long* out, hipStream_t s) {
    fill_u32(reinterpret_cast<uint32_t*>(out), 0u, 4, s);
    fill_u32(deg, 0u, n_v, s);
    if (n_u > 0) hipLaunchKernelGGL(k_side_rows, dim3(grid_for(n_u, 256)), dim3(256), 0, s, off, n_u, out);
    if (m > 0) hipLaunchKernelGGL(k_side_hist, dim3(grid_for(m, 256)), dim3(256), 0, s, adj, m, n_v, deg);
    if (n_v > 0) hipLaunchKernelGGL(k_side_bins, dim3(grid_for(n_v, 256)), dim3(256), 0, s, deg, n_v, out);
}

void launch_anchor_graph(const DevGraph* gr, int32_t n_graphs, uint32_t* agid, hipStream_t s) {
    if (n_graphs > 0) hipLaunchKernelGGL(k_anchor_graph, dim3(n_graphs), dim3(256), 0, s, gr, agid);
}

void launch_gather(const uint32_t* idx, const uint32_t* src, int64_t n, uint32_t* out, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, s, idx, src, n, out);
}

void launch_ranks(const uint32_t* inv, const uint32_t* deg_s, int64_t n_s, int32_t* rank, uint32_t* adeg,
                  const uint32_t* agid, int32_t* agraph, hipStream_t s) {
    if (n_s > 0)
        hipLaunchKernelGGL(k_ranks, dim3(grid_for(n_s, 256)), dim3(256), 0, s, inv, deg_s, n_s, rank, adeg, agid,
                           agraph);
}

void launch_check_dup(const uint32_t* ckey, const uint32_t* packed, int64_t m, DevStatus* st, hipStream_t s) {
    if (m > 1) hipLaunchKernelGGL(k_check_dup, dim3(grid_for(m, 256)), dim3(256), 0, s, ckey, packed, m, st);
}

void launch_work(const uint32_t* apack, const int32_t* acent, const int32_t* back, const uint32_t* coff, int64_t m,
                 int64_t n_s, unsigned long long* work, uint32_t* key, const uint32_t* aoff, const int32_t* agraph,
                 const int64_t* rank_end, uint32_t light_w, DevStatus* st, const HybridView& hv, hipStream_t s) {
    if (n_s <= 0) return;
    fill_bytes(work, n_s * 8, s);
    if (m > 0)
        hipLaunchKernelGGL(k_work, dim3(grid_for(m, 256, 4096)), dim3(256), 0, s, apack, acent, back, coff, m, work,
                           st, hv);
    hipLaunchKernelGGL(k_work_keys, dim3(grid_for(n_s, 256)), dim3(256), 0, s, work, n_s, key, aoff, agraph,
                       rank_end, hv.ablk1, light_w, st);
}

void launch_bidx(const uint32_t* ckey, const uint32_t* coff, const uint32_t* packed, int64_t m, int64_t n_c, int gs,
                 uint32_t* nb, uint32_t* ioff, uint32_t* idx, int2* meta, uint32_t* partials, const DevStatus* st,
                 hipStream_t s) {
    if (n_c <= 0) return;
    hipLaunchKernelGGL(k_bidx_count, dim3(grid_for(n_c, 256)), dim3(256), 0, s, coff, packed, n_c, gs, nb, st);
    scan_exclusive_u32(nb, ioff, n_c, partials, s);
    if (m > 0)
        hipLaunchKernelGGL(k_bidx_fill, dim3(grid_for(m, 256)), dim3(256), 0, s, ckey, coff, packed, m, gs, ioff, idx,
                           st);
    hipLaunchKernelGGL(k_bidx_meta, dim3(grid_for(n_c, 256)), dim3(256), 0, s, coff, packed, ioff, n_c, gs, meta, st);
}

}  // namespace bbc
