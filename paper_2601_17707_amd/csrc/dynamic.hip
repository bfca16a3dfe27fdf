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
#include <algorithm>

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

// Sort keys of the updates for the first (least significant) pass: one id
// of every update, in update order.
__global__ void k_dyn_ukey_init(const int32_t* a, int32_t q, uint32_t* key) {
    DYN_STRIDE(i, q) key[i] = (uint32_t)a[i];
}

// Keys of the second pass: the other id, in the order the first pass left.
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
    const unsigned long long* wsum;  // per V vertex v: sum of deg(w) over its neighbours w
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

// wsum[v] = sum of deg(w) over the neighbours w of v (one wave per v): the
// length of the walk v -> w -> x.
__global__ void k_dyn_wsum(const uint32_t* voff, const uint32_t* vrow, const int32_t* uoff, int32_t n_v,
                           unsigned long long* wsum) {
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t n_waves = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t v = wave; v < n_v; v += n_waves) {
        unsigned long long acc = 0;
        for (uint32_t e = voff[v] + lane_id(); e < voff[v + 1]; e += kWave) {
            const uint32_t w = vrow[e] >> 1;
            acc += (unsigned long long)(uoff[w + 1] - uoff[w]);
        }
        acc = wave_sum(acc);
        if (lane_id() == 0) wsum[v] = acc;
    }
}

// Position of pair key in the sorted update keys [lo, hi), or -1.
__device__ __forceinline__ int32_t find_in(const DynView& d, int32_t lo, int32_t hi, unsigned long long key) {
    const int32_t end = hi;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (d.uv_key[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return (lo < end && d.uv_key[lo] == key) ? (int32_t)d.uv_pos[lo] : -1;
}

// Update range [lo, hi) of the pairs (a, *) in the (u, v)-sorted keys.
__device__ __forceinline__ void update_row(const DynView& d, uint32_t a, int32_t& lo, int32_t& hi) {
    lo = lower_bound64(d.uv_key, d.q, (unsigned long long)a << 32);
    hi = lower_bound64(d.uv_key, d.q, (unsigned long long)(a + 1) << 32);
}

// Sign of (a, b) in a sorted row, searched from whichever side has the
// shorter list: U row of a (entries v << 1 | neg) or V row of b (u << 1 | neg).
__device__ __forceinline__ int32_t pair_state(const DynView& d, uint32_t a, uint32_t ua0, uint32_t ua1, uint32_t b,
                                              uint32_t vb0, uint32_t vb1) {
    return (ua1 - ua0 <= vb1 - vb0) ? row_state(d.urow, ua0, ua1, b) : row_state(d.vrow, vb0, vb1, a);
}

// LDS lists of one workgroup: candidates w (neighbours of v before or after
// the batch) and x (of u), with what a pair needs besides the state of
// (w, x).
template <int CH>
struct DynShared {
    uint32_t a_w[CH], a_r0[CH], a_r1[CH];  // w, its U row bounds
    int32_t a_lo[CH], a_hi[CH];           // updates on row w
    int8_t a_s0[CH], a_s1[CH], a_ok[CH];   // (w, v) before / after; candidate kept
    uint32_t b_x[CH], b_r0[CH], b_r1[CH];  // x, its V row bounds
    int8_t b_s0[CH], b_s1[CH], b_ok[CH];   // (u, x) before / after; candidate kept
    unsigned long long a_pre[CH];          // walk mode: first walk element of each w
    unsigned long long scan_tmp[CH / kWave + 1];
    long long tmp[CH / kWave + 1];
};

// Entry t of the w list: position a0 + t of [V row of v before the batch,
// then the updates on v].  Kept when it is a neighbour of v before or after
// (updates that do not insert add nothing new), is not u, and (w, v) is not
// a changed pair of lower index than i.
template <int CH>
__device__ __forceinline__ void fill_w(const DynView& d, DynShared<CH>& sh, int32_t i, uint32_t u, uint32_t v,
                                       uint32_t a_beg, uint32_t a_g, int32_t a_ub, uint32_t ia, uint32_t t) {
    uint32_t w;
    int32_t s0, s1, j2;
    bool ok = true;
    if (ia < a_g) {
        const uint32_t e = d.vrow[a_beg + ia];
        w = e >> 1;
        s0 = (e & 1u) ? -1 : 1;
        j2 = find_update(d, w, v);
        s1 = j2 >= 0 ? d.s_new[j2] : s0;
    } else {
        j2 = (int32_t)d.vu_pos[a_ub + (int32_t)(ia - a_g)];
        w = (uint32_t)d.upd_u[j2];
        s0 = 0;
        s1 = d.s_new[j2];
        ok = d.s_old[j2] == 0 && s1 != 0;
    }
    ok = ok && w != u && !(j2 >= 0 && j2 < i && changed(d, j2));
    sh.a_w[t] = w;
    sh.a_s0[t] = (int8_t)s0;
    sh.a_s1[t] = (int8_t)s1;
    sh.a_ok[t] = ok;
    if (ok) {
        sh.a_r0[t] = (uint32_t)d.uoff[w];
        sh.a_r1[t] = (uint32_t)d.uoff[w + 1];
        int32_t lo, hi;
        update_row(d, w, lo, hi);
        sh.a_lo[t] = lo;
        sh.a_hi[t] = hi;
    }
}

// Per-update scalars of the walk: the w list (V row of v, then the updates
// on v) and the x list (U row of u, then the updates on u).
struct DynUpd {
    uint32_t u, v, a_beg, a_g, b_beg, b_g, n_a, n_b;
    int32_t a_ub, b_ub, b_ue;
};

__device__ __forceinline__ DynUpd dyn_upd(const DynView& d, int32_t i) {
    DynUpd r;
    r.u = (uint32_t)d.upd_u[i];
    r.v = (uint32_t)d.upd_v[i];
    r.a_beg = d.voff[r.v];
    r.a_g = d.voff[r.v + 1] - r.a_beg;
    r.a_ub = lower_bound64(d.vu_key, d.q, (unsigned long long)r.v << 32);
    const int32_t a_ue = lower_bound64(d.vu_key, d.q, (unsigned long long)(r.v + 1) << 32);
    r.b_beg = (uint32_t)d.uoff[r.u];
    r.b_g = (uint32_t)d.uoff[r.u + 1] - r.b_beg;
    update_row(d, r.u, r.b_ub, r.b_ue);
    r.n_a = r.a_g + (uint32_t)(a_ue - r.a_ub);
    r.n_b = r.b_g + (uint32_t)(r.b_ue - r.b_ub);
    return r;
}

// Work plan: every changed update is split into at most max_tasks tasks;
// unchanged updates get none.  mode 1, the walk: spans of the w list
// holding about kWalkBudget walk elements (from wsum), so a hub's heavy
// neighbours spread over many workgroups; mode 2, pairs: one WG x WG tile
// of (w, x) pairs per task (span = tiles per w chunk); mode 0, pairs when
// the tiles are too many: spans of whole w chunks against every x chunk.  mode[i] = 1 for the
// walk.
constexpr unsigned long long kWalkBudget = 1ull << 15;

template <int WG, int CH>
__global__ void k_dyn_plan(DynView d, uint32_t max_tasks, uint32_t* n_tasks, uint32_t* span, uint8_t* mode,
                           long long* per_update, const DevStatus* st) {
    const bool bad = dyn_bad(st);
    DYN_STRIDE(i, d.q) {
        // the shares start at zero only when the batch was accepted (every
        // check ran earlier on the stream), so a rejected batch leaves them
        if (per_update && !bad) per_update[i] = 0;
        uint32_t c = 0, sp = 0;
        uint8_t walk = 0;
        if (!bad && changed(d, (int32_t)i)) {
            const DynUpd r = dyn_upd(d, (int32_t)i);
            walk = d.wsum[r.v] < (unsigned long long)r.n_a * r.n_b;
            if (walk) {  // spans of w's holding about kWalkBudget walk elements each
                const unsigned long long want = (d.wsum[r.v] + kWalkBudget - 1) / kWalkBudget;
                c = (uint32_t)min(want, (unsigned long long)min(max_tasks, r.n_a));
                if (c == 0 && r.n_a > 0) c = 1;
                sp = c ? (r.n_a + c - 1) / c : 0;
                c = sp ? (r.n_a + sp - 1) / sp : 0;
            } else {
                const uint32_t ca = (r.n_a + WG - 1) / WG, cb = (r.n_b + WG - 1) / WG;
                if ((unsigned long long)ca * cb <= max_tasks) {  // one WG x WG tile of pairs per task
                    walk = 2;
                    c = ca * cb;
                    sp = cb;
                } else {  // spans of whole CH-chunks of the w list, every x chunk
                    const uint32_t cc = (r.n_a + CH - 1) / CH;
                    c = min(cc, max_tasks);
                    sp = c ? ((cc + c - 1) / c) * CH : 0;
                    c = sp ? (r.n_a + sp - 1) / sp : 0;
                }
            }
        }
        n_tasks[i] = c;
        span[i] = sp;
        mode[i] = walk;
    }
}

// One workgroup per task (grid-stride over the tasks).  Two ways to visit
// the butterflies through (u, v), the cheaper one taken per update:
//   pairs: every (w, x) of the w list times the x list (neighbours of u and
//          the updates on u that insert), the state of (w, x) by a binary
//          search in the shorter of the two rows: deg(v) deg(u) searches;
//   walk:  every w of the w list and every x of w's row (and of the updates
//          on row w that insert), the state of (u, x) by a binary search in
//          u's row: sum of deg(w) over w, which wsum[v] gives up front.
// Both lists go through LDS in chunks; the walk flattens a chunk of w's row
// lengths with a workgroup prefix sum.
template <int WG, int CH>
__global__ __launch_bounds__(WG) void k_dyn_delta(DynView d, const uint32_t* task_off, const uint32_t* span,
                                                  const uint8_t* mode, long long* per_update, DevStatus* st) {
    static_assert(CH >= WG, "one w per thread in walk mode");
    if (dyn_bad(st)) return;
    __shared__ DynShared<CH> sh;
    const uint32_t n_tasks = task_off[d.q];
    for (uint32_t task = blockIdx.x; task < n_tasks; task += gridDim.x) {
        int32_t i;
        {  // the update of this task: last i with task_off[i] <= task
            int32_t lo = 0, hi = d.q - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (task_off[mid] <= task) lo = mid;
                else hi = mid - 1;
            }
            i = lo;
        }
        long long acc = 0;
        {
            const DynUpd r = dyn_upd(d, i);
            const uint32_t u = r.u, v = r.v, a_beg = r.a_beg, a_g = r.a_g, b_beg = r.b_beg, b_g = r.b_g;
            const int32_t a_ub = r.a_ub, b_ub = r.b_ub, b_ue = r.b_ue;
            const uint32_t n_b = r.n_b;
            const int32_t s_uv0 = d.s_old[i], s_uv1 = d.s_new[i];
            // this task's part: w list [a_lo_t, n_a), x list [b_lo_t, b_hi_t)
            const uint32_t k_t = task - task_off[i];
            uint32_t a_lo_t, n_a, b_lo_t = 0, b_hi_t = n_b;
            if (mode[i] == 2) {
                a_lo_t = (k_t / span[i]) * WG;
                n_a = min(r.n_a, a_lo_t + WG);
                b_lo_t = (k_t % span[i]) * WG;
                b_hi_t = min(n_b, b_lo_t + WG);
            } else {
                a_lo_t = k_t * span[i];
                n_a = min(r.n_a, a_lo_t + span[i]);
            }
            if (mode[i] == 1) {
                // u's row, searched once per walk element, sits in LDS when it fits
                // (the x list's slots are free in this mode)
                const bool u_lds = b_g <= (uint32_t)CH;
                if (u_lds) {
                    for (uint32_t t = threadIdx.x; t < b_g; t += WG) sh.b_x[t] = d.urow[b_beg + t];
                    __syncthreads();
                }
                for (uint32_t a0 = a_lo_t; a0 < n_a; a0 += WG) {
                    const uint32_t na = min((uint32_t)WG, n_a - a0), t = threadIdx.x;
                    unsigned long long cnt = 0;
                    if (t < na) {
                        fill_w(d, sh, i, u, v, a_beg, a_g, a_ub, a0 + t, t);
                        if (sh.a_ok[t]) cnt = (sh.a_r1[t] - sh.a_r0[t]) + (unsigned long long)(sh.a_hi[t] - sh.a_lo[t]);
                    }
                    unsigned long long n_e;
                    const unsigned long long pre = block_exclusive_scan<WG>(cnt, sh.scan_tmp, &n_e);
                    sh.a_pre[t] = pre;
                    __syncthreads();
                    for (unsigned long long e = threadIdx.x; e < n_e; e += WG) {
                        uint32_t lo = 0, hi = na - 1;  // last entry whose first element is <= e
                        while (lo < hi) {
                            const uint32_t mid = (lo + hi + 1) >> 1;
                            if (sh.a_pre[mid] <= e) lo = mid;
                            else hi = mid - 1;
                        }
                        const uint32_t ta = lo;
                        const unsigned long long k = e - sh.a_pre[ta];
                        const uint32_t w = sh.a_w[ta], deg_w = sh.a_r1[ta] - sh.a_r0[ta];
                        uint32_t x;
                        int32_t s_wx0, s_wx1, j4;
                        if (k < deg_w) {
                            const uint32_t ent = d.urow[sh.a_r0[ta] + (uint32_t)k];
                            x = ent >> 1;
                            s_wx0 = (ent & 1u) ? -1 : 1;
                            j4 = sh.a_lo[ta] < sh.a_hi[ta]
                                     ? find_in(d, sh.a_lo[ta], sh.a_hi[ta], ((unsigned long long)w << 32) | x)
                                     : -1;
                            s_wx1 = j4 >= 0 ? d.s_new[j4] : s_wx0;
                        } else {
                            j4 = (int32_t)d.uv_pos[sh.a_lo[ta] + (int32_t)(k - deg_w)];
                            if (d.s_old[j4] != 0 || d.s_new[j4] == 0) continue;  // only insertions add an x
                            x = (uint32_t)d.upd_v[j4];
                            s_wx0 = 0;
                            s_wx1 = d.s_new[j4];
                        }
                        if (x == v || (j4 >= 0 && j4 < i && changed(d, j4))) continue;
                        const int32_t s_ux0 = u_lds ? row_state(sh.b_x, 0, b_g, x) : row_state(d.urow, b_beg, b_beg + b_g, x);
                        const int32_t j3 = b_ub < b_ue ? find_in(d, b_ub, b_ue, ((unsigned long long)u << 32) | x) : -1;
                        const int32_t s_ux1 = j3 >= 0 ? d.s_new[j3] : s_ux0;
                        if ((s_ux0 == 0 && s_ux1 == 0) || (j3 >= 0 && j3 < i && changed(d, j3))) continue;
                        const int32_t b_before = s_uv0 * sh.a_s0[ta] * s_ux0 * s_wx0 > 0;
                        const int32_t b_after = s_uv1 * sh.a_s1[ta] * s_ux1 * s_wx1 > 0;
                        acc += b_after - b_before;
                    }
                    __syncthreads();  // the chunk is reloaded next
                }
            } else {
                for (uint32_t a0 = a_lo_t; a0 < n_a; a0 += CH) {
                    const uint32_t na = min((uint32_t)CH, n_a - a0);
                    for (uint32_t t = threadIdx.x; t < na; t += WG) fill_w(d, sh, i, u, v, a_beg, a_g, a_ub, a0 + t, t);
                    for (uint32_t b0 = b_lo_t; b0 < b_hi_t; b0 += CH) {
                        const uint32_t nb = min((uint32_t)CH, b_hi_t - b0);
                        if (a0 == a_lo_t || b_hi_t - b_lo_t > CH) {  // the x chunk is loaded once when it fits
                            for (uint32_t t = threadIdx.x; t < nb; t += WG) {
                                const uint32_t ib = b0 + t;
                                uint32_t x;
                                int32_t s0, s1, j3;
                                bool ok = true;
                                if (ib < b_g) {
                                    const uint32_t e = d.urow[b_beg + ib];
                                    x = e >> 1;
                                    s0 = (e & 1u) ? -1 : 1;
                                    j3 = b_ub < b_ue ? find_in(d, b_ub, b_ue, ((unsigned long long)u << 32) | x) : -1;
                                    s1 = j3 >= 0 ? d.s_new[j3] : s0;
                                } else {
                                    j3 = (int32_t)d.uv_pos[b_ub + (int32_t)(ib - b_g)];
                                    x = (uint32_t)d.upd_v[j3];
                                    s0 = 0;
                                    s1 = d.s_new[j3];
                                    ok = d.s_old[j3] == 0 && s1 != 0;
                                }
                                ok = ok && x != v && !(j3 >= 0 && j3 < i && changed(d, j3));
                                sh.b_x[t] = x;
                                sh.b_s0[t] = (int8_t)s0;
                                sh.b_s1[t] = (int8_t)s1;
                                sh.b_ok[t] = ok;
                                if (ok) {
                                    sh.b_r0[t] = d.voff[x];
                                    sh.b_r1[t] = d.voff[x + 1];
                                }
                            }
                        }
                        __syncthreads();
                        const uint32_t n_p = na * nb;
                        for (uint32_t p = threadIdx.x; p < n_p; p += WG) {
                            const uint32_t ja = p / nb, jb = p - ja * nb;
                            if (!sh.a_ok[ja] || !sh.b_ok[jb]) continue;
                            const uint32_t w = sh.a_w[ja], x = sh.b_x[jb];
                            const int32_t s_wx0 =
                                pair_state(d, w, sh.a_r0[ja], sh.a_r1[ja], x, sh.b_r0[jb], sh.b_r1[jb]);
                            int32_t s_wx1 = s_wx0;
                            if (sh.a_lo[ja] < sh.a_hi[ja]) {  // row w has updates: is (w, x) one of them?
                                const int32_t j4 =
                                    find_in(d, sh.a_lo[ja], sh.a_hi[ja], ((unsigned long long)w << 32) | x);
                                if (j4 >= 0) {
                                    if (j4 < i && changed(d, j4)) continue;  // charged to update j4
                                    s_wx1 = d.s_new[j4];
                                }
                            }
                            if (s_wx0 == 0 && s_wx1 == 0) continue;
                            const int32_t b_before = s_uv0 * sh.a_s0[ja] * sh.b_s0[jb] * s_wx0 > 0;
                            const int32_t b_after = s_uv1 * sh.a_s1[ja] * sh.b_s1[jb] * s_wx1 > 0;
                            acc += b_after - b_before;
                        }
                        __syncthreads();  // the chunks are reloaded next
                    }
                }
            }
        }
        const long long sum = block_sum<WG>(acc, sh.tmp);
        if (threadIdx.x == 0 && sum) {
            if (per_update) atomicAdd((unsigned long long*)&per_update[i], (unsigned long long)sum);
            atomicAdd(&st->total, (unsigned long long)sum);
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
               unsigned long long* wsum, int32_t n_v, int32_t q, uint32_t* n_tasks, uint32_t* task_off,
               uint32_t* span, uint8_t* mode, uint32_t* partials, long long* per_update, int32_t task_cap,
               DevStatus* st, hipStream_t s) {
    if (q <= 0) return;
    constexpr int WG = 256, CH = 1024;
    const DynView d{uoff, urow, voff, vrow, uv_key, uv_pos, vu_key, vu_pos, upd_u, upd_v, s_new, s_old, wsum, q};
    if (n_v > 0)
        hipLaunchKernelGGL(k_dyn_wsum, dim3(dyn_grid((int64_t)n_v * kWave, 256)), dim3(256), 0, s, voff, vrow, uoff,
                           n_v, wsum);
    hipLaunchKernelGGL(k_dyn_old, dim3(dyn_grid(q, 256)), dim3(256), 0, s, d, st);
    // at most task_cap (default 4096) tasks per update and 2^31 in all
    const int64_t cap = task_cap > 0 ? task_cap : 4096;
    const uint32_t max_tasks = (uint32_t)std::max<int64_t>(1, std::min<int64_t>(cap, (int64_t)INT32_MAX / q));
    hipLaunchKernelGGL((k_dyn_plan<WG, CH>), dim3(dyn_grid(q, 256)), dim3(256), 0, s, d, max_tasks, n_tasks, span,
                       mode, per_update, (const DevStatus*)st);
    scan_exclusive_u32(n_tasks, task_off, q, partials, s);
    hipLaunchKernelGGL((k_dyn_delta<WG, CH>), dim3(65536), dim3(WG), 0, s, d, (const uint32_t*)task_off,
                       (const uint32_t*)span, (const uint8_t*)mode, per_update, st);
}

}  // namespace bbc
