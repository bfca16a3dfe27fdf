// Device-wide building blocks: fills, exclusive scan and a stable LSD radix
// sort, used to build the degree-ordered CSR on the GPU.
#include "bbc_internal.h"

namespace bbc {

// ------------------------------------------------------------------ fills

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

__global__ void k_zero_bytes(uint8_t* p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = 0;
}

static int grid_for(int64_t n, int threads, int cap = 8192) {
    int64_t g = (n + threads - 1) / threads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (int)g;
}

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, v, n);
}

void fill_bytes(void* p, int64_t bytes, hipStream_t s) {
    if (bytes <= 0) return;
    if (bytes % 4 == 0 && ((uintptr_t)p % 4) == 0) {
        fill_u32((uint32_t*)p, 0u, bytes / 4, s);
        return;
    }
    hipLaunchKernelGGL(k_zero_bytes, dim3(grid_for(bytes, 256)), dim3(256), 0, s, (uint8_t*)p, bytes);
}

// ------------------------------------------------------------------- scan

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

size_t scan_partials_size(int64_t n) { return (size_t)((n + kScanTile - 1) / kScanTile) + 2; }

__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const uint32_t* in, int64_t n, uint32_t* partial) {
    __shared__ uint32_t tmp[kScanThreads / kWave];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    s = block_sum<kScanThreads>(s, tmp);
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// exclusive scan of nb partials by one workgroup, in place
__global__ __launch_bounds__(1024) void k_scan_partials(uint32_t* partial, int64_t nb) {
    __shared__ uint32_t tmp[1024 / kWave + 1];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
        int64_t i = b0 + threadIdx.x;
        uint32_t v = i < nb ? partial[i] : 0u;
        uint32_t tot;
        uint32_t ex = block_exclusive_scan<1024>(v, tmp, &tot);
        uint32_t c = carry;
        if (i < nb) partial[i] = c + ex;
        __syncthreads();
        if (threadIdx.x == 0) carry = c + tot;
        __syncthreads();
    }
}

// Each thread owns kScanItems consecutive inputs, staged through LDS so the
// global reads and writes stay coalesced.  partial == NULL: a single tile
// (no partial sums to add).
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(const uint32_t* in, uint32_t* out, int64_t n,
                                                             const uint32_t* partial) {
    __shared__ uint32_t stage[kScanTile];
    __shared__ uint32_t tmp[kScanThreads / kWave + 1];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        stage[k * kScanThreads + threadIdx.x] = i < n ? in[i] : 0u;
    }
    __syncthreads();
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        v[k] = stage[threadIdx.x * kScanItems + k];
        s += v[k];
    }
    uint32_t tot;
    uint32_t ex = block_exclusive_scan<kScanThreads>(s, tmp, &tot) + (partial ? partial[blockIdx.x] : 0u);
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        stage[threadIdx.x * kScanItems + k] = ex;
        ex += v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (i < n) out[i] = stage[k * kScanThreads + threadIdx.x];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == kScanThreads - 1) out[n] = ex;
}

void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials, hipStream_t s) {
    if (n <= 0) {
        fill_u32(out, 0u, 1, s);
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb == 1) {  // one tile: one launch
        hipLaunchKernelGGL(k_scan_apply, dim3(1), dim3(kScanThreads), 0, s, in, out, n, (const uint32_t*)nullptr);
        return;
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, partials);
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partials, nb);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, n,
                       (const uint32_t*)partials);
}

// ------------------------------------------------------------- radix sort

constexpr int kRsThreads = 256;  // one thread per digit value
constexpr int kRsRounds = 16;
constexpr int kRsTile = kRsThreads * kRsRounds;
constexpr int kRsWaves = kRsThreads / kWave;

size_t radix_hist_size(int64_t n) { return (size_t)256 * (size_t)((n + kRsTile - 1) / kRsTile) + 1; }

// Tile of workgroup b.  Workgroups are dealt round robin over the eight
// XCDs, so XCD x = b % 8 is given a contiguous range of tiles: consecutive
// tiles write neighbouring pieces of every digit's output run (and of the
// digit-major histogram), which then meet in the same L2.
__device__ __forceinline__ int64_t rs_tile(int64_t b, int64_t nblk) {
    const int64_t x = b & 7, i = b >> 3, q = nblk >> 3, r = nblk & 7;
    return x * q + (x < r ? x : r) + i;
}

// Lanes of the wave holding the same 8-bit digit d (eight ballots), among
// the lanes where valid is set.
__device__ __forceinline__ unsigned long long digit_peers(uint32_t d, bool valid) {
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
        const int on = (d >> bit) & 1u;
        const unsigned long long m = __ballot(on);
        peers &= on ? m : ~m;
    }
    return peers;
}

// Digit counts of one tile; hist is digit-major: hist[d * nblk + tile].
// When every lane of a wave holds the same digit (the high digits of
// narrow or grouped keys) one lane adds them all, instead of 64 atomics on
// one LDS word.
__global__ __launch_bounds__(kRsThreads) void k_rs_hist(const uint32_t* keys, int64_t n, int shift, uint32_t* hist,
                                                        int64_t nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile = rs_tile(blockIdx.x, nblk);
    const int64_t base = tile * kRsTile;
#pragma unroll 4
    for (int r = 0; r < kRsRounds; ++r) {
        const int64_t i = base + (int64_t)r * kRsThreads + threadIdx.x;
        const bool valid = i < n;
        const uint32_t d = valid ? (keys[i] >> shift) & 255u : 0u;
        const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
        if (__all(d == d0 || !valid)) {
            const unsigned long long vm = __ballot(valid);
            if (lane_id() == 0 && vm) atomicAdd(&h[d0], (uint32_t)__popcll(vm));
        } else if (valid) {
            atomicAdd(&h[d], 1u);
        }
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + tile] = h[threadIdx.x];
}

// Stable scatter of one tile, staged through LDS so that global writes are
// runs of consecutive positions.  Wave w owns the tile's items
// [w * 1024, (w + 1) * 1024), visited in 16 rounds of 64, so the input
// order is (wave, round, lane).  Within a round the lanes that share a
// digit are found with eight ballots; an item's place among its wave's
// items of that digit is the wave's running count of the digit plus the
// number of such lanes below it (the lowest of them then advances the
// count; a wave's LDS operations complete in order).  After one barrier
// every digit's places are offset by the counts of the waves before.  The
// key, then each payload, goes to its place in the tile sorted by digit
// (one LDS buffer, reused) and is written out in order, every digit's run
// at its global offset (the digit of each place is kept in LDS for the
// payloads).  Keys and places stay in registers between the phases; each
// payload is read when its turn comes.  One buffer and few registers let
// six tiles run per CU (26 KB of LDS each).  With inv_out the
// second payload is not moved: inv_out[v1] receives the item's new position
// instead (the inverse of the permutation that payload tracks).
__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(const uint32_t* keys, uint32_t* keys_out,
                                                           const uint32_t* v0, uint32_t* v0_out,
                                                           const uint32_t* v1, uint32_t* v1_out, int v1_iota,
                                                           int32_t* inv_out, int64_t n, int shift,
                                                           const uint32_t* hist, const uint32_t* hist_scan,
                                                           int64_t nblk) {
    __shared__ uint32_t s_buf[kRsTile];
    __shared__ uint8_t s_dig[kRsTile];
    __shared__ uint32_t lstart[256];  // first place of each digit in the sorted tile
    __shared__ uint32_t gstart[256];  // global position of that place
    __shared__ uint32_t wcnt[kRsWaves][256];
    __shared__ uint32_t scan_tmp[kRsWaves + 1];
    const int t = threadIdx.x, w = t / kWave, lane = lane_id();
    // the inverse scatter's writes go anywhere: tiles in launch order there
    const int64_t tile = inv_out ? (int64_t)blockIdx.x : rs_tile(blockIdx.x, nblk);
    const uint32_t cnt = hist[(int64_t)t * nblk + tile];
    uint32_t tot;
    const uint32_t ls = block_exclusive_scan<kRsThreads>(cnt, scan_tmp, &tot);
    lstart[t] = ls;
    gstart[t] = hist_scan[(int64_t)t * nblk + tile];
#pragma unroll
    for (int k = 0; k < kRsWaves; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const bool with_v0 = v0 != nullptr, with_v1 = v1_out != nullptr || inv_out != nullptr;
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    // 32-bit positions (n < 2^31)
    const uint32_t n32 = (uint32_t)n;
    const uint32_t base = (uint32_t)tile * kRsTile + (uint32_t)(w * (kRsRounds * kWave));
    uint32_t key[kRsRounds], place[kRsRounds];
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const uint32_t i = base + (uint32_t)(r * kWave + lane);
        key[r] = i < n32 ? keys[i] : 0u;
    }
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const bool valid = base + (uint32_t)(r * kWave + lane) < n32;
        const uint32_t d = (key[r] >> shift) & 255u;
        const unsigned long long peers = digit_peers(d, valid);
        const uint32_t rk = (uint32_t)__popcll(peers & below);
        const uint32_t run = wcnt[w][d];
        place[r] = run + rk;
        if (valid && rk == 0) wcnt[w][d] = run + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {  // digit t: offset of each wave's places
        uint32_t off = lstart[t];
#pragma unroll
        for (int k = 0; k < kRsWaves; ++k) {
            const uint32_t c = wcnt[k][t];
            wcnt[k][t] = off;
            off += c;
        }
    }
    __syncthreads();
    // places in the sorted tile (invalid items get none)
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        const uint32_t d = (key[r] >> shift) & 255u;
        place[r] = base + (uint32_t)(r * kWave + lane) < n32 ? wcnt[w][d] + place[r] : 0xffffffffu;
    }
    const uint32_t tbase = (uint32_t)tile * kRsTile;
    const uint32_t tile_n = min((uint32_t)kRsTile, n32 - tbase);
    // keys (and the digit of every place)
#pragma unroll
    for (int r = 0; r < kRsRounds; ++r) {
        if (place[r] != 0xffffffffu) {
            s_buf[place[r]] = key[r];
            s_dig[place[r]] = (uint8_t)((key[r] >> shift) & 255u);
        }
    }
    __syncthreads();
    for (uint32_t p = t; p < tile_n; p += kRsThreads) {
        const uint32_t d = s_dig[p];
        keys_out[gstart[d] + (p - lstart[d])] = s_buf[p];
    }
    if (with_v0) {
        uint32_t a[kRsRounds];
#pragma unroll
        for (int r = 0; r < kRsRounds; ++r) a[r] = place[r] != 0xffffffffu ? v0[base + (uint32_t)(r * kWave + lane)] : 0u;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRsRounds; ++r)
            if (place[r] != 0xffffffffu) s_buf[place[r]] = a[r];
        __syncthreads();
        for (uint32_t p = t; p < tile_n; p += kRsThreads) {
            const uint32_t d = s_dig[p];
            v0_out[gstart[d] + (p - lstart[d])] = s_buf[p];
        }
    }
    if (with_v1) {
        uint32_t b[kRsRounds];
#pragma unroll
        for (int r = 0; r < kRsRounds; ++r) {
            const uint32_t i = base + (uint32_t)(r * kWave + lane);
            b[r] = place[r] != 0xffffffffu ? (v1_iota ? i : v1[i]) : 0u;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRsRounds; ++r)
            if (place[r] != 0xffffffffu) s_buf[place[r]] = b[r];
        __syncthreads();
        for (uint32_t p = t; p < tile_n; p += kRsThreads) {
            const uint32_t d = s_dig[p];
            const uint32_t g = gstart[d] + (p - lstart[d]);
            if (inv_out) inv_out[s_buf[p]] = (int32_t)g;
            else v1_out[g] = s_buf[p];
        }
    }
}

// Every pass of a sort of at most one tile (n <= kRsTile) in one
// workgroup: the items stay in LDS between the passes, read back in the
// (wave, round, lane) order the ranking uses, so each pass is stable as in
// k_rs_scatter.  Used for the small sorts (per-anchor keys of small graphs),
// where the launches of the multi-tile passes would dominate.
__global__ __launch_bounds__(kRsThreads) void k_rs_single(const uint32_t* keys, uint32_t* keys_out,
                                                          const uint32_t* v0, uint32_t* v0_out, const uint32_t* v1,
                                                          uint32_t* v1_out, int v1_iota, int32_t* inv_out, int n,
                                                          int bits) {
    __shared__ uint32_t s_key[kRsTile];
    __shared__ uint32_t s_v0[kRsTile];
    __shared__ uint32_t s_v1[kRsTile];
    __shared__ uint32_t wcnt[kRsWaves][256];
    __shared__ uint32_t scan_tmp[kRsWaves + 1];
    const int t = threadIdx.x, w = t / kWave, lane = lane_id();
    const bool with_v0 = v0 != nullptr, with_v1 = v1_out != nullptr || inv_out != nullptr;
    for (int i = t; i < n; i += kRsThreads) {
        s_key[i] = keys[i];
        if (with_v0) s_v0[i] = v0[i];
        if (with_v1) s_v1[i] = v1_iota ? (uint32_t)i : v1[i];
    }
    const unsigned long long below = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const int base = w * (kRsRounds * kWave);
    for (int shift = 0; shift < bits; shift += 8) {
        __syncthreads();  // the previous pass's items are in place
        uint32_t key[kRsRounds], a[kRsRounds], b[kRsRounds], place[kRsRounds];
#pragma unroll
        for (int r = 0; r < kRsRounds; ++r) {
            const int i = base + r * kWave + lane;
            const bool valid = i < n;
            key[r] = valid ? s_key[i] : 0u;
            a[r] = (valid && with_v0) ? s_v0[i] : 0u;
            b[r] = (valid && with_v1) ? s_v1[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < kRsWaves; ++k) wcnt[k][t] = 0;
        __syncthreads();  // every item read; counts cleared
#pragma unroll
        for (int r = 0; r < kRsRounds; ++r) {
            const bool valid = base + r * kWave + lane < n;
            const uint32_t d = (key[r] >> shift) & 255u;
            const unsigned long long peers = digit_peers(d, valid);
            const uint32_t rk = (uint32_t)__popcll(peers & below);
            const uint32_t run = wcnt[w][d];
            place[r] = run + rk;
            if (valid && rk == 0) wcnt[w][d] = run + (uint32_t)__popcll(peers);
        }
        __syncthreads();
        uint32_t c_all = 0;  // digit t over all waves
#pragma unroll
        for (int k = 0; k < kRsWaves; ++k) c_all += wcnt[k][t];
        uint32_t tot;
        uint32_t off = block_exclusive_scan<kRsThreads>(c_all, scan_tmp, &tot);
#pragma unroll
        for (int k = 0; k < kRsWaves; ++k) {
            const uint32_t c = wcnt[k][t];
            wcnt[k][t] = off;
            off += c;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kRsRounds; ++r) {
            if (base + r * kWave + lane < n) {
                const uint32_t pos = wcnt[w][(key[r] >> shift) & 255u] + place[r];
                s_key[pos] = key[r];
                if (with_v0) s_v0[pos] = a[r];
                if (with_v1) s_v1[pos] = b[r];
            }
        }
    }
    __syncthreads();
    for (int i = t; i < n; i += kRsThreads) {
        keys_out[i] = s_key[i];
        if (with_v0) v0_out[i] = s_v0[i];
        if (inv_out) inv_out[s_v1[i]] = i;
        else if (with_v1) v1_out[i] = s_v1[i];
    }
}

void radix_sort(const uint32_t* k_in, uint32_t* k_a, uint32_t* k_b, const uint32_t* v0_in, uint32_t* v0_a,
                uint32_t* v0_b, const uint32_t* v1_in, uint32_t* v1_a, uint32_t* v1_b, int64_t n, int bits,
                uint32_t* hist, uint32_t* hist_scan, uint32_t* partials, hipStream_t s, const uint32_t** k_out,
                const uint32_t** v0_out, const uint32_t** v1_out, int32_t* inv_out) {
    const uint32_t *ks = k_in, *v0s = v0_in, *v1s = v1_in;
    int v1_iota = (v1_a != nullptr && v1_in == nullptr) ? 1 : 0;
    int64_t nblk = (n + kRsTile - 1) / kRsTile;
    if (bits < 1) bits = 1;
    if (n > 0 && nblk == 1) {  // one tile: every pass in one launch
        uint32_t* v0d = v0_in ? v0_a : nullptr;
        uint32_t* v1d = (v1_a && !inv_out) ? v1_a : nullptr;
        hipLaunchKernelGGL(k_rs_single, dim3(1), dim3(kRsThreads), 0, s, k_in, k_a, v0_in, v0d, v1_in, v1d, v1_iota,
                           inv_out, (int)n, bits);
        *k_out = k_a;
        if (v0_out) *v0_out = v0d;
        if (v1_out) *v1_out = v1d;
        return;
    }
    const int n_pass = (bits + 7) / 8;
    int pass = 0;
    for (int shift = 0; shift < bits && n > 0; shift += 8, ++pass) {
        uint32_t* kd = (pass & 1) ? k_b : k_a;
        uint32_t* v0d = v0_in ? ((pass & 1) ? v0_b : v0_a) : nullptr;
        int32_t* inv = (inv_out && pass == n_pass - 1) ? inv_out : nullptr;
        uint32_t* v1d = (v1_a && !inv) ? ((pass & 1) ? v1_b : v1_a) : nullptr;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nblk), dim3(kRsThreads), 0, s, ks, n, shift, hist, nblk);
        scan_exclusive_u32(hist, hist_scan, 256 * nblk, partials, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nblk), dim3(kRsThreads), 0, s, ks, kd, v0s, v0d, v1s,
                           v1d, v1_iota, inv, n, shift, (const uint32_t*)hist,
                           (const uint32_t*)hist_scan, nblk);
        ks = kd;
        v0s = v0d;
        v1s = v1d;
        v1_iota = 0;
    }
    *k_out = ks;
    if (v0_out) *v0_out = v0s;
    if (v1_out) *v1_out = v1s;
}

}  // namespace bbc
