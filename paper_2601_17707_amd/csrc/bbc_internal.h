// Internal declarations shared by the HIP sources of libbbc.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bbc {

constexpr int kWave = 64;

// Device-side status and accumulators of one bbc_count call.
struct DevStatus {
    int32_t flags;  // kBad* bits
    unsigned int queue2;  // second work queue head (the wave-regime launch of count mode)
    int64_t bad_offset;  // first offending index (atomicMin)
    int64_t bad_range;
    int64_t bad_sign;
    int64_t bad_dup;
    int64_t bad_block;          // first offending dense-block vertex (block * 2^32 + position)
    int64_t bad_update;         // first offending update of a batch
    unsigned long long total;   // twice the balanced butterflies
    unsigned long long wedges;  // sum over centres of C(deg, 2)
    unsigned long long walked;  // wedges the sparse walk visits (dense-block wedges excluded)
    unsigned long long bands;   // counter bands processed
    unsigned long long cls[6];  // sign-pattern classes (class mode); biclique limbs and overflows
    unsigned int queue;         // persistent work queue head
    unsigned int n_light;       // anchors of the wave regime (listed after every other anchor)
};

enum : int32_t {
    kBadOffsets = 1,
    kBadRange = 2,
    kBadSign = 4,
    kBadDup = 8,
    kBadBlocks = 16,
    kBadUpdRange = 32,  // update batches: id out of range,
    kBadUpdSign = 64,   // new state not in {-1, 0, +1},
    kBadUpdDup = 128    // repeated pair
};

// What the wedge kernel sums: the balanced count, the six sign-pattern
// classes, or balanced (2,k)-bicliques.
enum : int { kWedgeCount = 0, kWedgeClasses = 1, kWedgeBicliques = 2 };

// Wave regime of the wedge kernel: an anchor with at most kLightMaxWork
// wedges, at most kLightMaxDeg centres and fewer than 2^kLightKeyBits ranks
// above it in its graph is counted by one wave in a hashed LDS table of its
// own (20-bit endpoint key, two 6-bit counters per slot).  Such anchors are
// listed after all others; the rest take a whole workgroup each.
constexpr int kLightMaxDeg = 63;
constexpr int kLightKeyBits = 20;
constexpr int kLightMaxWork = 1024;

// Band-boundary index: meta.x of a centre list that has no index entries.
constexpr int32_t kBidxNone = INT32_MIN;

// One dense block as the device sees it.
struct DevBlock {
    // matrix and table exist only for blocks with n_r >= 2 and n_k >= 1
    int64_t mat_off;  // int8 matrix [rpad][kpad] (anchor rows x centre columns)
    int64_t tab_off;  // uint32 table [rpad][rpad]: a_dense | b_dense << 16 per anchor pair (u < w)
    int64_t rank0;    // first rank of the block's anchors (they are contiguous)
    int32_t n_r, n_k; // anchors, centres
    int32_t rpad, kpad;    // padded rows (multiple of 128) and columns (multiple of 64)
    int32_t n_aid, n_cid;  // caller's id counts on the anchor and centre side
    const int32_t* aid;    // anchor-side ids (device)
    const int32_t* cid;    // centre-side ids (device)
};

// One 128 x 128 upper-triangle output tile of a block product.
struct DevTile {
    int32_t blk, ti, tj, pad;
};

// Dense-block data the wedge kernel reads (ablk1 is null without blocks).
struct HybridView {
    const uint32_t* ablk1;  // per rank: block + 1 of the anchor, 0 for none
    const int32_t* cblk;    // per centre id: block, or -1
    const int32_t* cpos;    // per centre id of a block: list position past the block's anchors
    const DevBlock* blocks;
    const uint32_t* tabs;   // per block: a_dense | b_dense << 16 for anchor pairs (upper triangle)
};

// One graph of a batch, as the device sees it.
struct DevGraph {
    int64_t off_base;     // first offset in the concatenated offsets array
    int64_t edge_base;    // first edge in the concatenated adjacency / sign arrays
    int64_t n_edges;
    int64_t anchor_base;  // first global anchor id (and first rank) of this graph
    int64_t centre_base;  // first global centre id
    int32_t n_u, n_v;
    int32_t s_is_u;       // anchor side of this graph
    int32_t pad;
};

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

template <class T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// A lane's value from `CTRL` (a DPP row shift or row broadcast), or 0 where
// the source lane is out of reach or the lane's row is masked off.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ uint32_t dpp_take(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROW_MASK, 0xf, false);
}

// Inclusive max / sum over the lanes of a wave, in registers: shifts by 1,
// 2, 4 and 8 lanes within each row of 16 (row_shr), then lane 15 of each row
// into the next row (row_bcast:15, rows 1 and 3) and lane 31 into rows 2 and
// 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_inclusive_max_dpp(uint32_t x) {
    x = max(x, dpp_take<0x111, 0xf>(x));
    x = max(x, dpp_take<0x112, 0xf>(x));
    x = max(x, dpp_take<0x114, 0xf>(x));
    x = max(x, dpp_take<0x118, 0xf>(x));
    x = max(x, dpp_take<0x142, 0xa>(x));
    x = max(x, dpp_take<0x143, 0xc>(x));
    return x;
}

__device__ __forceinline__ uint32_t wave_inclusive_sum_dpp(uint32_t x) {
    x += dpp_take<0x111, 0xf>(x);
    x += dpp_take<0x112, 0xf>(x);
    x += dpp_take<0x114, 0xf>(x);
    x += dpp_take<0x118, 0xf>(x);
    x += dpp_take<0x142, 0xa>(x);
    x += dpp_take<0x143, 0xc>(x);
    return x;
}

template <class T>
__device__ __forceinline__ T wave_inclusive_scan(T x) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T y = __shfl_up(x, o, kWave);
        if (lane >= o) x += y;
    }
    return x;
}

// Exclusive scan over a workgroup of NT threads; `tmp` holds NT/64 + 1
// entries of LDS.  Returns this thread's exclusive prefix; *total receives
// the sum.  Must be reached by every thread of the workgroup.
template <int NT, class T>
__device__ __forceinline__ T block_exclusive_scan(T x, T* tmp, T* total) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave, lane = lane_id();
    T inc = wave_inclusive_scan(x);
    if (lane == kWave - 1) tmp[w] = inc;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int i = 0; i < NW; ++i) {
            T v = tmp[i];
            tmp[i] = run;
            run += v;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    T r = tmp[w] + inc - x;
    *total = tmp[NW];
    __syncthreads();  // tmp may be reused right after
    return r;
}

template <int NT, class T>
__device__ __forceinline__ T block_sum(T x, T* tmp) {
    constexpr int NW = NT / kWave;
    const int w = threadIdx.x / kWave;
    x = wave_sum(x);
    if (lane_id() == 0) tmp[w] = x;
    __syncthreads();
    T s = 0;
    for (int i = 0; i < NW; ++i) s += tmp[i];
    __syncthreads();
    return s;
}

// ------------------------------------------------------------ host launchers

// Exclusive scan: out[i] = sum(in[0..i)), out[n] = total.  `partials` needs
// scan_partials_size(n) elements of Tacc.  in and out must not alias.
size_t scan_partials_size(int64_t n);
void scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* partials, hipStream_t s);

// Stable LSD radix sort of n uint32 keys on their low `bits` bits, carrying
// up to two uint32 payloads.  The inputs are read only; the result lands in
// one of the two ping-pong buffers, returned through *_out.  v0_in may be
// NULL (no payload 0); v1_in == NULL with v1 buffers set means payload 1 is
// the input index.  `hist` needs radix_hist_size(n) uint32 and `partials`
// scan_partials_size(radix_hist_size(n)).  With inv_out (n int32), payload
// 1 is not returned: inv_out[payload 1 of an item] = its sorted position
// (with v1_in == NULL: inv_out[i] = where input item i went).
size_t radix_hist_size(int64_t n);
void radix_sort(const uint32_t* k_in, uint32_t* k_a, uint32_t* k_b, const uint32_t* v0_in, uint32_t* v0_a,
                uint32_t* v0_b, const uint32_t* v1_in, uint32_t* v1_a, uint32_t* v1_b, int64_t n, int bits,
                uint32_t* hist, uint32_t* hist_scan, uint32_t* partials, hipStream_t s, const uint32_t** k_out,
                const uint32_t** v0_out, const uint32_t** v1_out, int32_t* inv_out = nullptr);

void fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
void fill_bytes(void* p, int64_t bytes, hipStream_t s);  // zero fill

}  // namespace bbc
