// Input checks and the degree-ordered CSR, built on the device.
//
// Anchor side S and centre side C: every wedge is u - c - w with u, w in S
// and c in C.  Anchors are ranked by the vertex priority of Definition 6
// (degree, then id), ascending, so "w ranked above u" is rank(w) > rank(u).
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
#include "bbc_internal.h"

namespace bbc {

__device__ __forceinline__ void flag_bad(DevStatus* st, int32_t bit, int64_t* slot, int64_t idx) {
    atomicOr(&st->flags, bit);
    atomicMin((unsigned long long*)slot, (unsigned long long)idx);
}

// offsets[0] == 0, offsets[n_u] == m, non-decreasing
__global__ void k_check_offsets(const int32_t* off, int32_t n_u, int64_t m, DevStatus* st) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i <= n_u; i += stride) {
        int32_t o = off[i];
        bool bad = (i == 0 && o != 0) || (i == n_u && (int64_t)o != m) || (i < n_u && off[i + 1] < o);
        if (bad) flag_bad(st, kBadOffsets, &st->bad_offset, i);
    }
}

__global__ void k_check_edges(const int32_t* adj, const int8_t* sg, int64_t m, int32_t n_v, int check_sign,
                              DevStatus* st) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) {
        int32_t v = adj[i];
        if (v < 0 || v >= n_v) flag_bad(st, kBadRange, &st->bad_range, i);
        if (check_sign) {
            int8_t s = sg[i];
            if (s != 1 && s != -1) flag_bad(st, kBadSign, &st->bad_sign, i);
        }
    }
}

__global__ void k_degrees_u(const int32_t* off, int32_t n_u, uint32_t* deg_u) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n_u; i += stride) deg_u[i] = (uint32_t)(off[i + 1] - off[i]);
}

__global__ void k_degrees_v(const int32_t* adj, int64_t m, uint32_t* deg_v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < m; i += stride) atomicAdd(&deg_v[adj[i]], 1u);
}

// inv[r] = anchor id of rank r (the sorted payload); rank[id] = r;
// adeg[r] = degree of that anchor
__global__ void k_ranks(const uint32_t* inv, const uint32_t* deg_s, int32_t n_s, int32_t* rank, uint32_t* adeg) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; r < n_s; r += stride) {
        uint32_t id = inv[r];
        rank[id] = (int32_t)r;
        adeg[r] = deg_s[id];
    }
}

// Row of CSR entry e: the u with off[u] <= e < off[u + 1].
__device__ __forceinline__ int32_t row_of(const int32_t* off, int32_t n_u, int64_t e) {
    int32_t lo = 0, hi = n_u - 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo + 1) / 2;
        if ((int64_t)off[mid] <= e) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Scatter every input edge into its anchor's list (rank order).  With
// S = U an anchor's entries keep their row order; with S = V they are placed
// by an atomic fill counter (their order inside an anchor list is free).
__global__ void k_fill_anchor(const int32_t* off, const int32_t* adj, const int8_t* sg, int32_t n_u, int64_t m,
                              int s_is_u, const int32_t* rank, const uint32_t* aoff, uint32_t* fill,
                              int32_t* acent, uint8_t* aneg, uint32_t* apack) {
    int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; e < m; e += stride) {
        int32_t u = row_of(off, n_u, e);
        int32_t v = adj[e];
        uint32_t neg = sg[e] < 0 ? 1u : 0u;
        int32_t anchor = s_is_u ? u : v, centre = s_is_u ? v : u;
        int32_t r = rank[anchor];
        uint32_t slot = s_is_u ? aoff[r] + (uint32_t)(e - off[u]) : aoff[r] + atomicAdd(&fill[r], 1u);
        acent[slot] = centre;
        aneg[slot] = (uint8_t)neg;
        apack[slot] = ((uint32_t)r << 1) | neg;
    }
}

// back[perm[q]] = q: where each anchor entry sits in its centre's list
__global__ void k_back(const uint32_t* perm, int64_t m, int32_t* back) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; q < m; q += stride) back[perm[q]] = (int32_t)q;
}

// A repeated (u, v) pair shows up as the same anchor rank twice in a row of
// one centre's sorted list.
__global__ void k_check_dup(const uint32_t* ckey, const uint32_t* packed, int64_t m, DevStatus* st) {
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; q + 1 < m; q += stride)
        if (ckey[q] == ckey[q + 1] && (packed[q] >> 1) == (packed[q + 1] >> 1))
            flag_bad(st, kBadDup, &st->bad_dup, q);
}

// Per-anchor work: the number of wedges the anchor walks, i.e. the suffix
// lengths of its centres' lists (ranked-above endpoints).  One wave per
// anchor.  key = bitwise complement of the clamped work, so an ascending
// sort orders anchors by descending work (heavy anchors start first, as in
// the fanout ordering of Algorithm 4).
__global__ __launch_bounds__(256) void k_work(const uint32_t* aoff, const int32_t* acent, const int32_t* back,
                                              const uint32_t* coff, int32_t n_s, uint32_t* key, DevStatus* st) {
    const int lane = lane_id();
    int64_t wv = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    int64_t nwv = ((int64_t)gridDim.x * blockDim.x) / kWave;
    unsigned long long all = 0;
    for (int64_t r = wv; r < n_s; r += nwv) {
        uint32_t a0 = aoff[r], a1 = aoff[r + 1];
        unsigned long long w = 0;
        for (uint32_t p = a0 + lane; p < a1; p += kWave) {
            int32_t c = acent[p];
            w += (unsigned long long)(coff[c + 1] - (uint32_t)back[p] - 1u);
        }
        w = wave_sum(w);
        if (lane == 0) {
            uint32_t cl = w > 0xffffffffull ? 0xffffffffu : (uint32_t)w;
            key[r] = ~cl;
        }
        all += w;
    }
    if (lane == 0 && all) atomicAdd(&st->wedges, all);
}

// ------------------------------------------------------------ host launchers

static int grid_for(int64_t n, int threads, int cap = 16384) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void launch_checks(const int32_t* off, const int32_t* adj, const int8_t* sg, int32_t n_u, int32_t n_v, int64_t m,
                   int check_sign, DevStatus* st, hipStream_t s) {
    hipLaunchKernelGGL(k_check_offsets, dim3(grid_for((int64_t)n_u + 1, 256)), dim3(256), 0, s, off, n_u, m, st);
    if (m > 0)
        hipLaunchKernelGGL(k_check_edges, dim3(grid_for(m, 256)), dim3(256), 0, s, adj, sg, m, n_v, check_sign,
                           st);
}

void launch_degrees(const int32_t* off, const int32_t* adj, int32_t n_u, int64_t m, uint32_t* deg_u,
                    uint32_t* deg_v, int32_t n_v, hipStream_t s) {
    fill_u32(deg_v, 0u, n_v, s);
    if (n_u > 0) hipLaunchKernelGGL(k_degrees_u, dim3(grid_for(n_u, 256)), dim3(256), 0, s, off, n_u, deg_u);
    if (m > 0) hipLaunchKernelGGL(k_degrees_v, dim3(grid_for(m, 256)), dim3(256), 0, s, adj, m, deg_v);
}

void launch_ranks(const uint32_t* inv, const uint32_t* deg_s, int32_t n_s, int32_t* rank, uint32_t* adeg,
                  hipStream_t s) {
    if (n_s > 0) hipLaunchKernelGGL(k_ranks, dim3(grid_for(n_s, 256)), dim3(256), 0, s, inv, deg_s, n_s, rank, adeg);
}

void launch_fill_anchor(const int32_t* off, const int32_t* adj, const int8_t* sg, int32_t n_u, int64_t m,
                        int s_is_u, const int32_t* rank, const uint32_t* aoff, uint32_t* fill, int32_t n_s,
                        int32_t* acent, uint8_t* aneg, uint32_t* apack, hipStream_t s) {
    if (!s_is_u) fill_u32(fill, 0u, n_s, s);
    if (m > 0)
        hipLaunchKernelGGL(k_fill_anchor, dim3(grid_for(m, 256)), dim3(256), 0, s, off, adj, sg, n_u, m, s_is_u,
                           rank, aoff, fill, acent, aneg, apack);
}

void launch_back(const uint32_t* perm, int64_t m, int32_t* back, hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_back, dim3(grid_for(m, 256)), dim3(256), 0, s, perm, m, back);
}

void launch_check_dup(const uint32_t* ckey, const uint32_t* packed, int64_t m, DevStatus* st, hipStream_t s) {
    if (m > 1) hipLaunchKernelGGL(k_check_dup, dim3(grid_for(m, 256)), dim3(256), 0, s, ckey, packed, m, st);
}

void launch_work(const uint32_t* aoff, const int32_t* acent, const int32_t* back, const uint32_t* coff, int32_t n_s,
                 uint32_t* key, DevStatus* st, hipStream_t s) {
    if (n_s > 0)
        hipLaunchKernelGGL(k_work, dim3(grid_for((int64_t)n_s * kWave, 256)), dim3(256), 0, s, aoff, acent, back,
                           coff, n_s, key, st);
}

}  // namespace bbc
