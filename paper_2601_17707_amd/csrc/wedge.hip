// Wedge aggregation: the hot loop of balanced butterfly counting.
//
// For each anchor u (rank r) and each endpoint w ranked above it, a_uw counts
// the wedges u - c - w whose two edges agree in sign and b_uw those that
// disagree; u contributes sum_w C(a_uw,2) + C(b_uw,2) (Algorithm 1 with k = 2;
// Lemma 1: only two agreeing or two disagreeing wedges close a balanced
// butterfly).  The paper keeps these counters in per-thread hash maps
// (Algorithm 2), in shared-memory tiles over the 2-hop set (Algorithm 3) or
// in per-block global buffers behind an atomic task counter (Algorithm 4).
//
// MI355X design:
//   - persistent workgroups pull anchors from an atomic queue, heaviest
//     first (the order comes from a device sort of per-anchor work);
//   - the counters of one anchor live in LDS as a dense "band" over a
//     contiguous range of endpoint ranks.  Centre lists are sorted by rank,
//     so the wedges of a band are one contiguous slice of every centre's
//     list; a band is counted, reduced and cleared before the next one;
//   - counter width follows the anchor degree d (a, b <= d): 4-bit pairs for
//     d <= 15, 8-bit for d <= 255, 16-bit for d <= 65535, else 32-bit, so a
//     64 KiB band spans 64K, 32K, 16K or 8K endpoint ranks;
//   - the slices of a band are flattened across all lanes (prefix sum over
//     slice lengths), so a wave reads consecutive entries of one list
//     (coalesced 4-byte reads) regardless of how uneven the lists are;
//   - the first increment of a counter word sets a bit in an LDS bitmap, so
//     the reduction only visits touched words;
//   - sums stay in registers across tasks and are reduced once per wave at
//     exit (one 64-bit atomic per wave).
#include "bbc_internal.h"

namespace bbc {

// first position q in [lo, hi) of a rank-sorted list with rank(q) >= target
__device__ __forceinline__ int32_t lower_bound_rank(const uint32_t* __restrict__ packed, int32_t lo, int32_t hi,
                                                    uint32_t target) {
    while (lo < hi) {
        int32_t mid = lo + ((hi - lo) >> 1);
        if ((packed[mid] >> 1) < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Sum of C(x,2) over the counter fields of one LDS word.
template <int MODE>
__device__ __forceinline__ unsigned long long word_pairs(uint32_t v) {
    if constexpr (MODE == 0) {  // eight 4-bit fields
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            uint32_t x = (v >> (4 * i)) & 15u;
            s += x * (x - 1u) / 2u;
        }
        return s;
    } else if constexpr (MODE == 1) {  // four 8-bit fields
        uint32_t s = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            uint32_t x = (v >> (8 * i)) & 255u;
            s += x * (x - 1u) / 2u;
        }
        return s;
    } else if constexpr (MODE == 2) {  // two 16-bit fields
        unsigned long long a = v & 0xffffu, b = v >> 16;
        return a * (a - (a > 0)) / 2 + b * (b - (b > 0)) / 2;
    } else {  // one 32-bit field
        unsigned long long a = v;
        return a * (a - (a > 0)) / 2;
    }
}

// LDS word and increment for endpoint slot `slot` (rank - band start) and
// wedge type t (0 = signs agree, 1 = disagree).
template <int MODE>
__device__ __forceinline__ void slot_word(uint32_t slot, uint32_t t, uint32_t& word, uint32_t& inc) {
    if constexpr (MODE == 0) {
        word = slot >> 2;
        inc = 1u << (((slot & 3u) << 3) + (t << 2));
    } else if constexpr (MODE == 1) {
        word = slot >> 1;
        inc = 1u << (((slot & 1u) << 4) + (t << 3));
    } else if constexpr (MODE == 2) {
        word = slot;
        inc = 1u << (t << 4);
    } else {
        word = (slot << 1) + t;
        inc = 1u;
    }
}

template <int MODE>
__host__ __device__ constexpr int slots_per_word_x2() {
    return MODE == 0 ? 8 : MODE == 1 ? 4 : MODE == 2 ? 2 : 1;  // twice the slots per word
}

constexpr int kUnroll = 4;

template <int WG, int BAND_WORDS>
struct WedgeShared {
    uint32_t cnt[BAND_WORDS];
    uint32_t bmp[BAND_WORDS / 32];
    uint32_t c_start[WG];  // slice start | negative-edge bit << 31
    int32_t c_pre[WG + 1];
    int32_t scan_tmp[WG / kWave + 1];
    int32_t task;
};

// Count one band [lo, hi) of anchor r.  Returns the sum of pair terms seen
// by this thread.
template <int MODE, int WG, int BAND_WORDS>
__device__ unsigned long long count_band(WedgeShared<WG, BAND_WORDS>& sh, const int32_t* __restrict__ acent,
                                         const uint8_t* __restrict__ aneg, const int32_t* __restrict__ back,
                                         const uint32_t* __restrict__ coff, const uint32_t* __restrict__ packed,
                                         int32_t a0, int32_t deg, int32_t r, int64_t lo, int64_t hi, int64_t n_s) {
    const int tid = threadIdx.x;
    const bool first = lo == (int64_t)r + 1, last = hi == n_s;
    const uint32_t band = (uint32_t)(hi - lo);
    for (int32_t k0 = 0; k0 < deg; k0 += WG) {
        const int32_t nk = min(WG, deg - k0);
        int32_t len = 0;
        if (tid < nk) {
            const int32_t p = a0 + k0 + tid;
            const int32_t c = acent[p];
            const int32_t ce = (int32_t)coff[c + 1];
            const int32_t sfx = back[p] + 1;
            const int32_t s = first ? sfx : lower_bound_rank(packed, sfx, ce, (uint32_t)lo);
            const int32_t e = last ? ce : lower_bound_rank(packed, s, ce, (uint32_t)hi);
            sh.c_start[tid] = (uint32_t)s | ((uint32_t)aneg[p] << 31);
            len = e - s;
        }
        int32_t total;
        int32_t ex = block_exclusive_scan<WG>(len, sh.scan_tmp, &total);
        if (tid < nk) sh.c_pre[tid] = ex;
        if (tid == 0) sh.c_pre[nk] = total;
        __syncthreads();

        for (int32_t j0 = 0; j0 < total; j0 += WG * kUnroll) {
            uint32_t x[kUnroll], ng[kUnroll];
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int32_t j = j0 + u * WG + tid;
                x[u] = 0xffffffffu;
                ng[u] = 0;
                if (j < total) {
                    // slice holding flattened wedge j: largest k with c_pre[k] <= j
                    int32_t a = 0, b = nk - 1;
                    while (a < b) {
                        int32_t mid = (a + b + 1) >> 1;
                        if (sh.c_pre[mid] <= j) a = mid;
                        else b = mid - 1;
                    }
                    const uint32_t st = sh.c_start[a];
                    x[u] = packed[(st & 0x7fffffffu) + (uint32_t)(j - sh.c_pre[a])];
                    ng[u] = st >> 31;
                }
            }
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const uint32_t slot = (x[u] >> 1) - (uint32_t)lo;
                if (slot < band) {  // also rejects the padding lanes
                    uint32_t word, inc;
                    slot_word<MODE>(slot, (x[u] ^ ng[u]) & 1u, word, inc);
                    const uint32_t old = atomicAdd(&sh.cnt[word], inc);
                    if (old == 0) atomicOr(&sh.bmp[word >> 5], 1u << (word & 31u));
                }
            }
        }
        __syncthreads();  // slice tables are rewritten by the next chunk
    }

    // reduce and clear the touched words of this band
    unsigned long long acc = 0;
    const uint32_t nwords = MODE == 3 ? 2u * band : (band * 2u + slots_per_word_x2<MODE>() - 1u) /
                                                        (uint32_t)slots_per_word_x2<MODE>();
    const uint32_t nbm = (nwords + 31u) >> 5;
    for (uint32_t b = tid; b < nbm; b += WG) {
        uint32_t bits = sh.bmp[b];
        if (bits) {
            sh.bmp[b] = 0;
            while (bits) {
                const uint32_t i = __ffs(bits) - 1;
                bits &= bits - 1u;
                const uint32_t wd = (b << 5) + i;
                acc += word_pairs<MODE>(sh.cnt[wd]);
                sh.cnt[wd] = 0;
            }
        }
    }
    __syncthreads();
    return acc;
}

template <int WG, int BAND_WORDS>
__global__ __launch_bounds__(WG) void k_wedge(const uint32_t* __restrict__ aoff, const int32_t* __restrict__ acent,
                                              const uint8_t* __restrict__ aneg, const int32_t* __restrict__ back,
                                              const uint32_t* __restrict__ coff, const uint32_t* __restrict__ packed,
                                              const uint32_t* __restrict__ order, int32_t n_s, DevStatus* st) {
    __shared__ WedgeShared<WG, BAND_WORDS> sh;
    const int tid = threadIdx.x;
    for (int i = tid; i < BAND_WORDS; i += WG) sh.cnt[i] = 0;
    for (int i = tid; i < BAND_WORDS / 32; i += WG) sh.bmp[i] = 0;
    unsigned long long acc = 0, bands = 0;
    for (;;) {
        __syncthreads();
        if (tid == 0) sh.task = (int32_t)atomicAdd(&st->queue, 1u);
        __syncthreads();
        const int32_t task = sh.task;
        if (task >= n_s) break;
        const int32_t r = (int32_t)order[task];
        const int32_t a0 = (int32_t)aoff[r], deg = (int32_t)aoff[r + 1] - a0;
        if (deg < 2 || r >= n_s - 1) continue;  // no endpoint pair can close a butterfly
        int64_t band_slots;
        int mode;
        if (deg <= 15) {
            mode = 0;
            band_slots = (int64_t)BAND_WORDS * 4;
        } else if (deg <= 255) {
            mode = 1;
            band_slots = (int64_t)BAND_WORDS * 2;
        } else if (deg <= 65535) {
            mode = 2;
            band_slots = BAND_WORDS;
        } else {
            mode = 3;
            band_slots = BAND_WORDS / 2;
        }
        for (int64_t lo = (int64_t)r + 1; lo < n_s; lo += band_slots) {
            const int64_t hi = min((int64_t)n_s, lo + band_slots);
            if (mode == 0)
                acc += count_band<0, WG, BAND_WORDS>(sh, acent, aneg, back, coff, packed, a0, deg, r, lo, hi, n_s);
            else if (mode == 1)
                acc += count_band<1, WG, BAND_WORDS>(sh, acent, aneg, back, coff, packed, a0, deg, r, lo, hi, n_s);
            else if (mode == 2)
                acc += count_band<2, WG, BAND_WORDS>(sh, acent, aneg, back, coff, packed, a0, deg, r, lo, hi, n_s);
            else
                acc += count_band<3, WG, BAND_WORDS>(sh, acent, aneg, back, coff, packed, a0, deg, r, lo, hi, n_s);
            ++bands;
        }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(&st->total, acc);
    if (tid == 0 && bands) atomicAdd(&st->bands, bands);
}

// ------------------------------------------------------------------ launch

constexpr int kWedgeWG = 512;
constexpr int kBandWords = 16384;  // 64 KiB of counters per workgroup

int wedge_block() { return kWedgeWG; }

int wedge_blocks_per_cu() {
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_wedge<kWedgeWG, kBandWords>, kWedgeWG, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

void launch_wedge(int grid, const uint32_t* aoff, const int32_t* acent, const uint8_t* aneg, const int32_t* back,
                  const uint32_t* coff, const uint32_t* packed, const uint32_t* order, int32_t n_s, DevStatus* st,
                  hipStream_t s) {
    hipLaunchKernelGGL((k_wedge<kWedgeWG, kBandWords>), dim3(grid), dim3(kWedgeWG), 0, s, aoff, acent, aneg, back,
                       coff, packed, order, n_s, st);
}

}  // namespace bbc
