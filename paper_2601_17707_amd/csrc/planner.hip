// Dense-block planner: finds pairs (R, C) of anchor-side and centre-side
// vertex sets whose edges are dense, for the int8 matrix-core path.
//
// Any partition of the edges into dense-block and sparse parts gives the
// exact count (the pair terms split into a dense part, a sparse part and a
// cross term), so the planner only decides speed.  It works on the
// candidates, the vertices of degree >= tau, and grows one block at a time
// from a seed anchor:
//   C <- the seed's candidate centres;
//   twice: R <- candidate anchors linked to at least frac * |C| of C,
//          C <- candidate centres linked to at least frac * |R| of R;
// and keeps the block when |R|, |C| and the edge density of R x C reach
// their minimums.  Members of kept blocks are never used again.  Seeds are
// tried in decreasing order of (candidate centres)^2 / degree, which favours
// anchors whose neighbours are mostly candidates.
//
// The kernels below are the data-parallel steps; the loop over seeds runs
// on the host (bbc_plan_blocks in api.hip), one synchronisation per seed.
#include "bbc_internal.h"

namespace bbc {

#define PL_STRIDE(i, n)                                                         \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

static int pl_grid(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    return (int)(g < 1 ? 1 : g > 16384 ? 16384 : g);
}

// out[cur[key[i]]++] = val[i]: lists of val grouped by key (order within a
// list arbitrary); cur starts as the list offsets.
__global__ void k_pl_scatter(const uint32_t* key, const uint32_t* val, int64_t m, uint32_t* cur, uint32_t* out) {
    PL_STRIDE(i, m) out[atomicAdd(&cur[key[i]], 1u)] = val[i];
}

__global__ void k_pl_copy(const uint32_t* in, int64_t n, uint32_t* out) { PL_STRIDE(i, n) out[i] = in[i]; }

// cd[a] = number of candidate centres among the neighbours of candidate
// anchor a.
__global__ void k_pl_cand_deg(const uint32_t* ea, const uint32_t* ec, int64_t m, const uint32_t* deg_a,
                              const uint32_t* deg_c, uint32_t tau, uint32_t* cd) {
    PL_STRIDE(i, m) {
        const uint32_t a = ea[i], c = ec[i];
        if (deg_a[a] >= tau && deg_c[c] >= tau) atomicAdd(&cd[a], 1u);
    }
}

// The seed's unassigned candidate centres, appended to list (count *n).
__global__ void k_pl_seed(const uint32_t* off_a, const uint32_t* adj_a, uint32_t seed, const uint32_t* deg_c,
                          uint32_t tau, const uint8_t* assigned_c, uint32_t* list, uint32_t* n, uint32_t cap) {
    const uint32_t b = off_a[seed], e = off_a[seed + 1];
    for (uint32_t k = b + blockIdx.x * blockDim.x + threadIdx.x; k < e; k += gridDim.x * blockDim.x) {
        const uint32_t c = adj_a[k];
        if (deg_c[c] >= tau && !assigned_c[c]) {
            const uint32_t p = atomicAdd(n, 1u);
            if (p < cap) list[p] = c;
        }
    }
}

// For every member x of list (its first min(*n, cap) entries) and every
// neighbour y of x: cnt[y] += 1.  Workgroups stride over the members,
// threads over a member's neighbours.
__global__ void k_pl_count(const uint32_t* list, const uint32_t* n, uint32_t cap, const uint32_t* off,
                           const uint32_t* adj, uint32_t* cnt) {
    const uint32_t nl = min(*n, cap);
    for (uint32_t k = blockIdx.x; k < nl; k += gridDim.x) {
        const uint32_t x = list[k];
        for (uint32_t e = off[x] + threadIdx.x; e < off[x + 1]; e += blockDim.x) atomicAdd(&cnt[adj[e]], 1u);
    }
}

// Vertices i with cnt[i] >= max(1, ceil(frac * min(*n_other, cap_other))),
// degree >= tau and not yet assigned, appended to out (count *n_out, at
// most cap stored); *edges += cnt[i] for every stored one.  Every cnt entry
// is reset to zero for the next count.
__global__ void k_pl_select(uint32_t* cnt, int64_t n, const uint32_t* deg, uint32_t tau, const uint8_t* assigned,
                            const uint32_t* n_other, uint32_t cap_other, float frac, uint32_t* out, uint32_t* n_out,
                            uint32_t cap, unsigned long long* edges) {
    const float other = (float)min(*n_other, cap_other);
    const uint32_t thresh = max(1u, (uint32_t)ceilf(frac * other));
    PL_STRIDE(i, n) {
        const uint32_t c = cnt[i];
        if (c) {
            cnt[i] = 0;
            if (c >= thresh && deg[i] >= tau && !assigned[i]) {
                const uint32_t p = atomicAdd(n_out, 1u);
                if (p < cap) {
                    out[p] = (uint32_t)i;
                    atomicAdd(edges, (unsigned long long)c);
                }
            }
        }
    }
}

__global__ void k_pl_assign(const uint32_t* list, uint32_t n, uint8_t* assigned) {
    PL_STRIDE(i, (int64_t)n) assigned[list[i]] = 1;
}

// ------------------------------------------------------------------ launchers

void pl_scatter(const uint32_t* key, const uint32_t* val, int64_t m, const uint32_t* off, int64_t n_keys,
                uint32_t* cur, uint32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_pl_copy, dim3(pl_grid(n_keys, 256)), dim3(256), 0, s, off, n_keys, cur);
    if (m > 0) hipLaunchKernelGGL(k_pl_scatter, dim3(pl_grid(m, 256)), dim3(256), 0, s, key, val, m, cur, out);
}

void pl_cand_deg(const uint32_t* ea, const uint32_t* ec, int64_t m, const uint32_t* deg_a, const uint32_t* deg_c,
                 uint32_t tau, uint32_t* cd, hipStream_t s) {
    if (m > 0)
        hipLaunchKernelGGL(k_pl_cand_deg, dim3(pl_grid(m, 256)), dim3(256), 0, s, ea, ec, m, deg_a, deg_c, tau, cd);
}

void pl_seed(const uint32_t* off_a, const uint32_t* adj_a, uint32_t seed, const uint32_t* deg_c, uint32_t tau,
             const uint8_t* assigned_c, uint32_t* list, uint32_t* n, uint32_t cap, hipStream_t s) {
    hipLaunchKernelGGL(k_pl_seed, dim3(64), dim3(256), 0, s, off_a, adj_a, seed, deg_c, tau, assigned_c, list, n,
                       cap);
}

void pl_count(const uint32_t* list, const uint32_t* n, uint32_t cap, const uint32_t* off, const uint32_t* adj,
              uint32_t* cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_pl_count, dim3(4096), dim3(256), 0, s, list, n, cap, off, adj, cnt);
}

void pl_select(uint32_t* cnt, int64_t n, const uint32_t* deg, uint32_t tau, const uint8_t* assigned,
               const uint32_t* n_other, uint32_t cap_other, float frac, uint32_t* out, uint32_t* n_out, uint32_t cap,
               unsigned long long* edges, hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_pl_select, dim3(pl_grid(n, 256)), dim3(256), 0, s, cnt, n, deg, tau, assigned, n_other,
                           cap_other, frac, out, n_out, cap, edges);
}

void pl_assign(const uint32_t* list, uint32_t n, uint8_t* assigned, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_pl_assign, dim3(pl_grid(n, 256)), dim3(256), 0, s, list, n, assigned);
}

}  // namespace bbc
