// Dynamic graphs: the change of the balanced count under a batch of edge
// updates (edges added, removed or re-signed; the setting named in the
// paper's Sec. "Future Directions").
//
// Only butterflies that hold an updated pair can change.  Each one is
// charged to the first changed pair it holds (lowest update index): the
// walk of update i visits every butterfly u - v - w - x through its pair
// (u, v), before or after the batch (w adjacent to v and x adjacent to u in
// either graph, (w, x) present in either), skips those holding a changed
// pair of lower index, and adds balanced-after minus balanced-before
// (Definition 2: an even number of negative edges, all four present).
// Summed over the batch this is T(after) - T(before) exactly.
//
// Device data: both CSRs of the graph with every row sorted by neighbour
// id (entries id << 1 | negative), and the update pairs sorted by (u, v)
// and by (v, u) as 64-bit keys, so that every edge state is a binary
// search away.  One workgroup walks one update; its threads stride over the
// (w, x) candidate pairs.
#include "bbc_internal.h"

namespace bbc {

#define DYN_STRIDE(i, n)                                                        \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); \
         i += (int64_t)gridDim.x * blockDim.x)

static int dyn_grid(int64_t n, int threads) {
    int64_t g = (n + threads - 1) / threads;
    return (int)(g < 1 ? 1 : g > 16384 ? 16384 : g);
}

__device__ __forceinline__ bool dyn_bad(const DevStatus* st) { return *(volatile const int32_t*)&st->flags != 0; }

__device__ __forceinline__ void dyn_flag(DevStatus* st, int32_t bit, int64_t* slot, int64_t idx) {
    atomicOr(&st->flags, bit);
    atomicMin(reinterpret_cast<long long*>(slot), (long long)idx);
}

// Update checks: ids in range, new state +1 / -1 / 0.
__global__ void k_dyn_check(const int32_t* uu, const int32_t* vv, const int8_t* ss, int32_t q, int32_t n_u,
                            int32_t n_v, DevStatus* st) {
    DYN_STRIDE(i, q) {
        if (uu[i] < 0 || uu[i] >= n_u || vv[i] < 0 || vv[i] >= n_v) dyn_flag(st, kBadUpdRange, &st->bad_update, i);
        if (ss[i] < -1 || ss[i] > 1) dyn_flag(st, kBadUpdSign, &st->bad_update, i);
    }
}

// Sort keys of the edges: v, with payload u << 1 | negative (for the stable
// sort by v that yields the V rows with u ascending).
__global__ void k_dyn_vkeys(const uint32_t* ea, const uint32_t* ec, const uint8_t* en, int64_t m, uint32_t* key,
                            uint32_t* pay) {
    DYN_STRIDE(e, m) {
        key[e] = ec[e];
        pay[e] = (ea[e] << 1) | (en[e] ? 1u : 0u);
    }
}

// From the V rows (key v, payload u << 1 | neg): keys u and payload
// v << 1 | neg for the stable sort by u that yields the U rows with v
// ascending.
__global__ void k_dyn_ukeys(const uint32_t* vkey, const uint32_t* vpay, int64_t m, uint32_t* key, uint32_t* pay) {
    DYN_STRIDE(e, m) {
        key[e] = vpay[e] >> 1;
        pay[e] = (vkey[e] << 1) | (vpay[e] & 1u);
    }
}

// Repeated pairs: neighbours of one row sorted, so repeats are adjacent.
__global__ void k_dyn_dup(const uint32_t* ukey, const uint32_t* urow, int64_t m, DevStatus* st) {
    DYN_STRIDE(e, m) {
        if (e > 0 && ukey[e] == ukey[e - 1] && (urow[e] >> 1) == (urow[e - 1] >> 1))
            dyn_flag(st, kBadDup, &st->bad_dup, e);
    }
}

// Update keys: a = first id, b = second id (as ints), index as payload.
__global__ void k_dyn_ukey_init(const int32_t* a, int32_t q, uint32_t* key) {
    DYN_STRIDE(i, q) key[i] = (uint32_t)a[i];
}

__global__ void k_dyn_gather(const int32_t* src, const uint32_t* idx, int32_t q, uint32_t* key) {
    DYN_STRIDE(i, q) key[i] = (uint32_t)src[idx[i]];
}

// 64-bit keys (hi << 32 | lo) in sorted order, and repeated update pairs.
__global__ void k_dyn_key64(const int32_t* hi, const int32_t* lo, const uint32_t* idx, int32_t q,
                            unsigned long long* key, uint32_t* pos, int check, DevStatus* st) {
    DYN_STRIDE(i, q) {
        const uint32_t j = idx[i];
        key[i] = ((unsigned long long)(uint32_t)hi[j] << 32) | (uint32_t)lo[j];
        pos[i] = j;
    }
    if (check) {
        DYN_STRIDE(i, q) {
            if (i > 0 && hi[idx[i]] == hi[idx[i - 1]] && lo[idx[i]] == lo[idx[i - 1]])
                dyn_flag(st, kBadUpdDup, &st->bad_update, idx[i]);
        }
    }
}

// Position of the first key >= x in key[0, n).
__device__ __forceinline__ int32_t lower_bound64(const unsigned long long* key, int32_t n, unsigned long long x) {
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (key[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Sign (+1 / -1) of the edge (a, b) in a sorted row (entries id << 1 | neg),
// 0 when absent.
__device__ __forceinline__ int32_t row_state(const uint32_t* row, uint32_t beg, uint32_t end, uint32_t b) {
    uint32_t lo = beg, hi = end;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((row[mid] >> 1) < b) lo = mid + 1;
        else hi = mid;
    }
    if (lo < end && (row[lo] >> 1) == b) return (row[lo] & 1u) ? -1 : 1;
    return 0;
}

struct DynView {
    const int32_t* uoff;  // U rows (the input offsets)
    const uint32_t* urow;
    const uint32_t* voff;  // V rows
    const uint32_t* vrow;
    const unsigned long long* uv_key;  // update pairs by (u, v)
    const uint32_t* uv_pos;            // their update indices
    const unsigned long long* vu_key;  // by (v, u)
    const uint32_t* vu_pos;
    const int32_t* upd_u;
    const int32_t* upd_v;
    const int8_t* s_new;  // by update index
    int8_t* s_old;        // state before the batch, filled by k_dyn_old
    int32_t q;
};

// Index of the update on pair (a, b), or -1.
__device__ __forceinline__ int32_t find_update(const DynView& d, uint32_t a, uint32_t b) {
    const unsigned long long x = ((unsigned long long)a << 32) | b;
    const int32_t p = lower_bound64(d.uv_key, d.q, x);
    return (p < d.q && d.uv_key[p] == x) ? (int32_t)d.uv_pos[p] : -1;
}

__global__ void k_dyn_old(DynView d, DevStatus* st) {
    if (dyn_bad(st)) return;
    DYN_STRIDE(i, d.q) {
        const uint32_t u = (uint32_t)d.upd_u[i], v = (uint32_t)d.upd_v[i];
        d.s_old[i] = (int8_t)row_state(d.urow, (uint32_t)d.uoff[u], (uint32_t)d.uoff[u + 1], v);
    }
}

__device__ __forceinline__ bool changed(const DynView& d, int32_t j) { return d.s_old[j] != d.s_new[j]; }

// One workgroup per update (grid-stride over updates).  Candidates: w from
// the V row of v (before) and from the updates on v that insert an edge;
// x from the U row of u and from the updates on u that insert one.
template <int WG>
__global__ __launch_bounds__(WG) void k_dyn_delta(DynView d, long long* per_update, DevStatus* st) {
    if (dyn_bad(st)) return;
    __shared__ long long tmp[WG / kWave + 1];
    for (int32_t i = blockIdx.x; i < d.q; i += gridDim.x) {
        long long acc = 0;
        if (changed(d, i)) {
            const uint32_t u = (uint32_t)d.upd_u[i], v = (uint32_t)d.upd_v[i];
            const int32_t s_uv0 = d.s_old[i], s_uv1 = d.s_new[i];
            const uint32_t a_beg = d.voff[v], a_g = d.voff[v + 1] - a_beg;  // w before the batch
            const int32_t a_ub = lower_bound64(d.vu_key, d.q, (unsigned long long)v << 32);
            const int32_t a_ue = lower_bound64(d.vu_key, d.q, (unsigned long long)(v + 1) << 32);
            const uint32_t b_beg = (uint32_t)d.uoff[u], b_g = (uint32_t)d.uoff[u + 1] - b_beg;  // x before
            const int32_t b_ub = lower_bound64(d.uv_key, d.q, (unsigned long long)u << 32);
            const int32_t b_ue = lower_bound64(d.uv_key, d.q, (unsigned long long)(u + 1) << 32);
            const uint64_t n_a = a_g + (uint64_t)(a_ue - a_ub), n_b = b_g + (uint64_t)(b_ue - b_ub);
            const uint64_t n_p = n_a * n_b;
            for (uint64_t p = threadIdx.x; p < n_p; p += WG) {
                const uint64_t ia = p / n_b, ib = p - ia * n_b;
                uint32_t w, x;
                int32_t s_wv0, s_wv1, s_ux0, s_ux1, j2, j3;
                if (ia < a_g) {
                    const uint32_t e = d.vrow[a_beg + ia];
                    w = e >> 1;
                    s_wv0 = (e & 1u) ? -1 : 1;
                    j2 = find_update(d, w, v);
                    s_wv1 = j2 >= 0 ? d.s_new[j2] : s_wv0;
                } else {
                    j2 = (int32_t)d.vu_pos[a_ub + (int32_t)(ia - a_g)];
                    if (d.s_old[j2] != 0 || d.s_new[j2] == 0) continue;  // only insertions are new w
                    w = (uint32_t)d.upd_u[j2];
                    s_wv0 = 0;
                    s_wv1 = d.s_new[j2];
                }
                if (w == u) continue;
                if (ib < b_g) {
                    const uint32_t e = d.urow[b_beg + ib];
                    x = e >> 1;
                    s_ux0 = (e & 1u) ? -1 : 1;
                    j3 = find_update(d, u, x);
                    s_ux1 = j3 >= 0 ? d.s_new[j3] : s_ux0;
                } else {
                    j3 = (int32_t)d.uv_pos[b_ub + (int32_t)(ib - b_g)];
                    if (d.s_old[j3] != 0 || d.s_new[j3] == 0) continue;
                    x = (uint32_t)d.upd_v[j3];
                    s_ux0 = 0;
                    s_ux1 = d.s_new[j3];
                }
                if (x == v) continue;
                const int32_t s_wx0 = row_state(d.urow, (uint32_t)d.uoff[w], (uint32_t)d.uoff[w + 1], x);
                const int32_t j4 = find_update(d, w, x);
                const int32_t s_wx1 = j4 >= 0 ? d.s_new[j4] : s_wx0;
                if (s_wx0 == 0 && s_wx1 == 0) continue;
                // charged to the changed pair of lowest index
                if ((j2 >= 0 && j2 < i && changed(d, j2)) || (j3 >= 0 && j3 < i && changed(d, j3)) ||
                    (j4 >= 0 && j4 < i && changed(d, j4)))
                    continue;
                const int32_t b0 = s_uv0 * s_wv0 * s_ux0 * s_wx0 > 0, b1 = s_uv1 * s_wv1 * s_ux1 * s_wx1 > 0;
                acc += b1 - b0;
            }
        }
        const long long sum = block_sum<WG>(acc, tmp);
        if (threadIdx.x == 0) {
            if (per_update) per_update[i] = sum;
            if (sum) atomicAdd(&st->total, (unsigned long long)sum);
        }
    }
}

// ------------------------------------------------------------------ launchers

void dyn_check(const int32_t* uu, const int32_t* vv, const int8_t* ss, int32_t q, int32_t n_u, int32_t n_v,
               DevStatus* st, hipStream_t s) {
    if (q > 0) hipLaunchKernelGGL(k_dyn_check, dim3(dyn_grid(q, 256)), dim3(256), 0, s, uu, vv, ss, q, n_u, n_v, st);
}

void dyn_vkeys(const uint32_t* ea, const uint32_t* ec, const uint8_t* en, int64_t m, uint32_t* key, uint32_t* pay,
               hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_dyn_vkeys, dim3(dyn_grid(m, 256)), dim3(256), 0, s, ea, ec, en, m, key, pay);
}

void dyn_ukeys(const uint32_t* vkey, const uint32_t* vpay, int64_t m, uint32_t* key, uint32_t* pay, hipStream_t s) {
    if (m > 0) hipLaunchKernelGGL(k_dyn_ukeys, dim3(dyn_grid(m, 256)), dim3(256), 0, s, vkey, vpay, m, key, pay);
}

void dyn_dup(const uint32_t* ukey, const uint32_t* urow, int64_t m, DevStatus* st, hipStream_t s) {
    if (m > 1) hipLaunchKernelGGL(k_dyn_dup, dim3(dyn_grid(m, 256)), dim3(256), 0, s, ukey, urow, m, st);
}

void dyn_key_init(const int32_t* a, int32_t q, uint32_t* key, hipStream_t s) {
    if (q > 0) hipLaunchKernelGGL(k_dyn_ukey_init, dim3(dyn_grid(q, 256)), dim3(256), 0, s, a, q, key);
}

void dyn_gather(const int32_t* src, const uint32_t* idx, int32_t q, uint32_t* key, hipStream_t s) {
    if (q > 0) hipLaunchKernelGGL(k_dyn_gather, dim3(dyn_grid(q, 256)), dim3(256), 0, s, src, idx, q, key);
}

void dyn_key64(const int32_t* hi, const int32_t* lo, const uint32_t* idx, int32_t q, unsigned long long* key,
               uint32_t* pos, int check, DevStatus* st, hipStream_t s) {
    if (q > 0)
        hipLaunchKernelGGL(k_dyn_key64, dim3(dyn_grid(q, 256)), dim3(256), 0, s, hi, lo, idx, q, key, pos, check, st);
}

void dyn_delta(const int32_t* uoff, const uint32_t* urow, const uint32_t* voff, const uint32_t* vrow,
               const unsigned long long* uv_key, const uint32_t* uv_pos, const unsigned long long* vu_key,
               const uint32_t* vu_pos, const int32_t* upd_u, const int32_t* upd_v, const int8_t* s_new, int8_t* s_old,
               int32_t q, long long* per_update, DevStatus* st, hipStream_t s) {
    if (q <= 0) return;
    const DynView d{uoff, urow, voff, vrow, uv_key, uv_pos, vu_key, vu_pos, upd_u, upd_v, s_new, s_old, q};
    hipLaunchKernelGGL(k_dyn_old, dim3(dyn_grid(q, 256)), dim3(256), 0, s, d, st);
    hipLaunchKernelGGL(k_dyn_delta<256>, dim3((unsigned)(q < 65536 ? q : 65536)), dim3(256), 0, s, d, per_update, st);
}

}  // namespace bbc
