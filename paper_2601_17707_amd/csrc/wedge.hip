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
//   - the non-empty slices of a band are flattened into rows of 64 wedges
//     (prefix sum over slice lengths); waves own contiguous runs of rows and
//     lanes keep a cursor on their slice, so a wave reads consecutive entries
//     of one list (coalesced 4-byte reads) however uneven the lists are;
//   - endpoint slots are scattered over the band by an odd multiplier so
//     that rank-sorted lists do not pile onto a few LDS banks;
//   - the first increment of a counter word sets a bit in an LDS bitmap, so
//     the reduction only visits touched words;
//   - sums stay in registers across tasks and are reduced once per wave at
//     exit (one 64-bit atomic per wave).
//
// Per-vertex mode (FULL): every anchor walks its whole 2-hop range (endpoints
// ranked above and below it), so cnt[u] = sum over w != u of
// C(a_uw,2) + C(b_uw,2) is summed locally and stored once, and the total is
// half the sum over anchors.  A second walk of each band, with the counters
// complete, adds n_t(u,w) - 1 for every wedge u - c - w of type t to the
// centre c (the balanced butterflies pairing that wedge with another of its
// type); every unordered pair is seen from both ends, so centre sums are
// halved at the end.  No endpoint count is ever scattered.
#include "bbc_internal.h"


namespace bbc {

// First position q in [lo, hi) of a rank-sorted list with rank(q) >= target
// (hi if none), found by one wave: each round probes 64 evenly spaced
// positions and keeps the gap where the ranks cross the target, so a list of
// length L takes ceil(log64 L) dependent loads.  Every lane of the wave must
// call it with the same arguments; every lane returns the answer.
__device__ __forceinline__ int32_t wave_lower_bound(const uint32_t* __restrict__ packed, int32_t lo, int32_t hi,
                                                    uint32_t target) {
    const int lane = lane_id();
    while (lo < hi) {  // the answer lies in [lo, hi]
        const int32_t len = hi - lo;
        const int32_t step = (len + kWave - 1) / kWave;
        const int32_t off = lane * step;
        const bool probe = off < len;
        const bool ge = probe && (packed[lo + off] >> 1) >= target;
        const unsigned long long b = __ballot(ge);
        if (b == 0) {
            const unsigned long long pm = __ballot(probe);
            const int last = 63 - __clzll(pm);
            lo += last * step + 1;
        } else {
            const int f = __ffsll(b) - 1;
            if (f == 0) return lo;
            hi = lo + f * step;
            lo += (f - 1) * step + 1;
        }
    }
    return lo;
}

// Pair terms of the counter fields of LDS words: sum over fields x of
// C(x,2) = (x^2 - x) / 2.  The sum of x^2 over a word is one packed
// dot-product instruction (the word with itself), so no field is unpacked.
// In count mode (TWICE) only the squares are summed: the band's sum of x is
// its number of wedges, which the caller subtracts once, and the kernel
// carries twice the pair terms.  Otherwise the sum of x is the dot product
// with a word of ones and x^2 - x, always even, is halved per thread.
// Modes 0 and 1 keep 32-bit partial sums per band and thread (at most 64
// words per thread and band, each below 2^18); modes 2 and 3 widen per
// word (in mode 2, a + b <= 65535, so a^2 + b^2 fits 32 bits).
template <int MODE, bool TWICE>
struct PairSum {
    uint32_t sq = 0, lin = 0;
    unsigned long long wide = 0;
    __device__ __forceinline__ void add(uint32_t v) {
        if constexpr (MODE == 0) {  // eight 4-bit fields
            sq = __builtin_amdgcn_udot8(v, v, sq, false);
            if constexpr (!TWICE) lin = __builtin_amdgcn_udot8(v, 0x11111111u, lin, false);
        } else if constexpr (MODE == 1) {  // four 8-bit fields
            sq = __builtin_amdgcn_udot4(v, v, sq, false);
            if constexpr (!TWICE) lin = __builtin_amdgcn_udot4(v, 0x01010101u, lin, false);
        } else if constexpr (MODE == 2) {  // a and b of one endpoint
            typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
            const u16x2 h = __builtin_bit_cast(u16x2, v);
            const uint32_t q = __builtin_amdgcn_udot2(h, h, 0u, false);
            if constexpr (TWICE) wide += q;
            else wide += (q - ((v & 0xffffu) + (v >> 16))) >> 1;
        } else {  // one 32-bit field
            const unsigned long long a = v;
            if constexpr (TWICE) wide += a * a;
            else wide += a * (a - (a > 0)) / 2;
        }
    }
    // The sums added so far, and restarts.
    __device__ __forceinline__ unsigned long long take() {
        unsigned long long r = wide;
        if constexpr (MODE <= 1) r += TWICE ? (unsigned long long)sq : (unsigned long long)((sq - lin) >> 1);
        sq = lin = 0;
        wide = 0;
        return r;
    }
};

// Band capacity in endpoint slots for a counter mode (a power of two).
// Modes 0-3 count two wedge types per slot (agree, disagree) in 4, 8, 16 or
// 32-bit fields; modes 4-7 count three for the sign-pattern classes (both
// edges positive, both negative, different) in a slot of four such fields.
template <int MODE, int BAND_WORDS>
__host__ __device__ constexpr uint32_t band_capacity() {
    constexpr uint32_t bw = BAND_WORDS;
    return MODE == 0 ? bw * 4u : MODE == 1 ? bw * 2u : MODE == 2 ? bw : MODE == 3 ? bw / 2u
         : MODE == 4 ? bw * 2u : MODE == 5 ? bw : MODE == 6 ? bw / 2u : bw / 4u;
}

// Multiplier of the slot scatter.  Centre lists are sorted by rank, so the
// lanes of a wave read endpoints at a near-regular stride; mapped straight
// onto LDS words that stride lands on a few banks.  Any bijection between
// the endpoint ranks of a band and counter fields is valid (the reduction
// sums every touched field), so an endpoint's slot is its rank times an odd
// multiplier modulo the power-of-two band capacity: a band never spans more
// ranks than its capacity, and distinct residues stay distinct under the
// multiplication.
constexpr uint32_t kSlotMul = 0x9E377u;  // times 8 still below 2^24: a full-rate 24-bit multiply

// Inverse of an odd number modulo 2^32 (Newton iteration; each step doubles
// the number of correct low bits).
constexpr uint32_t inverse_odd(uint32_t m) {
    uint32_t x = m;  // correct to 3 bits
    for (int i = 0; i < 5; ++i) x *= 2u - m * x;
    return x;
}
constexpr uint32_t kSlotInv = inverse_odd(kSlotMul);
static_assert(kSlotMul * kSlotInv == 1u, "slot scatter must be invertible");
static_assert(kSlotMul * 8u < (1u << 24), "scaled multipliers must fit a 24-bit multiply");

// Low 32 bits of a 24 x 24-bit product (full rate; the compiler drops the
// masks that would let it pick this form, since only the low bits are used).
// The low k <= 24 bits of the product depend only on the low k bits of the
// operands, so ranks above 2^24 map correctly modulo the band capacity.
__device__ __forceinline__ uint32_t mul_u24(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// Counter field of endpoint rank `rank` and wedge type t (0 = signs agree,
// 1 = disagree): byte offset of its LDS word in the band and bit shift of
// the field.  Slot = rank * kSlotMul mod capacity; fields per word: mode 0
// four slots of (a, b) nibbles, mode 1 two slots of (a, b) bytes, mode 2 one
// slot of (a, b) halves, mode 3 one 32-bit word per slot and type.  The
// multiplier is pre-scaled so that the product lands at the byte offset.
template <int MODE, int BAND_WORDS>
__device__ __forceinline__ void slot_field(uint32_t rank, uint32_t t, uint32_t& byte, uint32_t& shift) {
    static_assert(band_capacity<MODE, BAND_WORDS>() <= (1u << 24), "band slots must fit a 24-bit multiply");
    constexpr uint32_t wmask = (uint32_t)(BAND_WORDS - 1) << 2;
    if constexpr (MODE == 0) {
        const uint32_t p = mul_u24(rank, kSlotMul);  // slot = p mod 4 BW; word = slot / 4
        byte = p & wmask;
        shift = ((p & 3u) << 3) | (t << 2);
    } else if constexpr (MODE == 1) {
        const uint32_t p = mul_u24(rank, kSlotMul * 2u);  // slot = p / 2 mod 2 BW; word = slot / 2
        byte = p & wmask;
        shift = ((p & 2u) << 3) | (t << 3);
    } else if constexpr (MODE == 2) {
        const uint32_t p = mul_u24(rank, kSlotMul * 4u);  // slot = p / 4 mod BW; word = slot
        byte = p & wmask;
        shift = t << 4;
    } else if constexpr (MODE == 3) {
        const uint32_t p = mul_u24(rank, kSlotMul * 8u);  // slot = p / 8 mod BW / 2; word = 2 slot + t
        byte = (p & ((uint32_t)(BAND_WORDS / 2 - 1) << 3)) | (t << 2);
        shift = 0;
    } else {  // classes, t in {0, 1, 2}: field t of the slot's four
        const uint32_t slot = mul_u24(rank, kSlotMul) & (band_capacity<MODE, BAND_WORDS>() - 1u);
        if constexpr (MODE == 4) {  // 4-bit fields, two slots per word
            byte = (slot >> 1) << 2;
            shift = ((slot & 1u) << 4) | (t << 2);
        } else if constexpr (MODE == 5) {  // 8-bit fields, a word per slot
            byte = slot << 2;
            shift = t << 3;
        } else if constexpr (MODE == 6) {  // 16-bit fields, two words per slot
            byte = (slot << 3) | ((t >> 1) << 2);
            shift = (t & 1u) << 4;
        } else {  // 32-bit fields, four words per slot
            byte = (slot << 4) | (t << 2);
            shift = 0;
        }
    }
}

// Endpoint rank of slot `slot` in the band starting at lo (the inverse of
// the scatter: the one rank in [lo, lo + capacity) with that residue).
template <int MODE, int BAND_WORDS>
__device__ __forceinline__ int64_t slot_rank(uint32_t slot, int64_t lo) {
    constexpr uint32_t mask = band_capacity<MODE, BAND_WORDS>() - 1u;
    return lo + (int64_t)((slot * kSlotInv - (uint32_t)lo) & mask);
}

// The dense-block table row of an anchor inside a block (row == null
// otherwise): entries for endpoint ranks rank0 .. rank0 + n_r - 1.
struct CrossRow {
    const uint32_t* row;
    int64_t rank0;
    int64_t n_r;
};

// Cross term a_dense * a_sparse + b_dense * b_sparse of every counter field
// of word wd (value v) whose endpoint lies in the anchor's block: the slot
// of a field is recovered by inverting the scatter.
template <int MODE, int BAND_WORDS>
__device__ __forceinline__ unsigned long long cross_term(uint32_t wd, uint32_t v, int64_t lo, const CrossRow& cr) {
    unsigned long long acc = 0;
    if constexpr (MODE == 3) {  // word = slot * 2 + type
        const int64_t i = slot_rank<MODE, BAND_WORDS>(wd >> 1, lo) - cr.rank0;
        if ((uint64_t)i < (uint64_t)cr.n_r) {
            const uint32_t t = cr.row[i];
            acc = (unsigned long long)v * ((wd & 1u) ? (t >> 16) : (t & 0xffffu));
        }
    } else {
        constexpr int F = MODE == 0 ? 4 : MODE == 1 ? 2 : 1;     // slots per word
        constexpr int FB = MODE == 0 ? 8 : MODE == 1 ? 16 : 32;  // bits per slot: a, then b
        constexpr uint32_t fm = (1u << (FB / 2)) - 1u;
#pragma unroll
        for (int f = 0; f < F; ++f) {
            const uint32_t x = v >> (f * FB);
            const uint32_t a = x & fm, b = (x >> (FB / 2)) & fm;
            if (a | b) {
                const int64_t i = slot_rank<MODE, BAND_WORDS>(wd * (uint32_t)F + (uint32_t)f, lo) - cr.rank0;
                if ((uint64_t)i < (uint64_t)cr.n_r) {
                    const uint32_t t = cr.row[i];
                    acc += (unsigned long long)a * (t & 0xffffu) + (unsigned long long)b * (t >> 16);
                }
            }
        }
    }
    return acc;
}

constexpr int kUnroll = 8;

// Compacted slices of one band: start | negative-edge bit << 31 of the
// non-empty slices and the exclusive prefix of their lengths.
template <int WG>
struct SliceTable {
    uint32_t start[WG];
    int32_t pre[WG + 1];
};

template <int WG, int BAND_WORDS, bool FULL>
struct WedgeShared {
    alignas(16) uint32_t cnt[BAND_WORDS];  // counters
    uint32_t bmp[BAND_WORDS / 32];
    uint32_t c_cur[WG];     // cursor of each centre: next list position | negative-edge bit << 31
    int32_t c_ce[FULL ? WG : 1];  // per-vertex mode: end of the centre's whole list
    // count mode compacts the next band while the current one is reduced
    SliceTable<WG> tab[FULL ? 1 : 2];
    long long scan_tmp[WG / kWave + 1];
    uint32_t ctab[16];  // biclique mode: C(x, k) for x < 16 (at most C(15, 7) = 6435)
    // per-vertex mode only
    int32_t c_id[FULL ? WG : 1];                // centre id of each chunk entry
    int32_t w_k[FULL ? WG : 1];                 // chunk entry of each compacted slice
    unsigned long long c_sum[FULL ? WG : 1];    // centre contributions of this anchor
    int32_t task;
};

// Per-centre values that stay in the registers of the thread owning the
// centre in count mode: the end of its whole list and its band-boundary
// index (pos(k) = k > khi ? ce : idx[base + k]).
struct CentreMeta {
    int32_t ce, base, khi;
};

// Loads the centres k0 .. k0+nk-1 of the anchor list starting at a0: the
// slice start (just past the anchor's own entry in the centre list, the
// ranked-above suffix; or the list start in per-vertex mode), the list end,
// and the sign of the anchor edge.  Thread k owns centre k.
template <bool FULL, int WG, int BAND_WORDS>
__device__ __forceinline__ CentreMeta load_centres(WedgeShared<WG, BAND_WORDS, FULL>& sh,
                                             const int32_t* __restrict__ acent, const uint8_t* __restrict__ aneg,
                                             const int32_t* __restrict__ back, const uint32_t* __restrict__ coff,
                                             const int2* __restrict__ bmeta, int32_t a0, int32_t k0, int32_t nk,
                                             int32_t blk, const HybridView& hv) {
    const int tid = threadIdx.x;
    CentreMeta cm{0, kBidxNone, -1};
    if (tid < nk) {
        const int32_t p = a0 + k0 + tid;
        const int32_t c = acent[p];
        uint32_t start = FULL ? coff[c] : (uint32_t)(back[p] + 1);
        // an anchor of a dense block skips the block's anchors in the lists
        // of the block's centres (those wedges are counted on matrix cores)
        if (!FULL && blk >= 0 && hv.cblk[c] == blk) start = (uint32_t)hv.cpos[c];
        sh.c_cur[tid] = start | ((uint32_t)aneg[p] << 31);
        cm.ce = (int32_t)coff[c + 1];
        if constexpr (FULL) {
            sh.c_ce[tid] = cm.ce;
            sh.c_id[tid] = c;
            sh.c_sum[tid] = 0;
        } else {
            const int2 bm = bmeta[c];
            cm.base = bm.x;
            cm.khi = bm.y;
        }
    }
    return cm;
}

// Position of the first compacted slice holding flattened wedge jq.
template <int WG>
__device__ __forceinline__ int32_t slice_of(const SliceTable<WG>& t, int32_t nkc, int32_t jq) {
    int32_t k = 0, b = nkc - 1;
    while (k < b) {
        const int32_t mid = (k + b + 1) >> 1;
        if (t.pre[mid] <= jq) k = mid;
        else b = mid - 1;
    }
    return k;
}

// Counts the wedges of the centres in the slice tables whose endpoint rank
// lies in [lo, hi).  Slices start at the cursors in c_cur; when
// `seek_start` they are first advanced to the first rank >= lo.  Cursors
// move to the slice ends.  `self` is the anchor's own rank (its entries are
// skipped in the per-vertex centre walk).  `phases`: bit 0 counts the
// wedges, bit 1 runs the per-vertex centre walk, which needs the band's
// counters complete over every centre of the anchor.
//
// Slice ends: in count mode every band but the last ends on a multiple of
// the granule 2^gs, so the end is one read of the band-boundary index (lo,
// when seeking, is such a multiple too); per-vertex mode searches the list
// with one wave per centre.
//
// A band holding at least BAND_WORDS / 16 wedges is "dense": its increments
// need no return value (no touched-word bitmap) and the reduction scans the
// whole band; sparser bands mark touched words.  Returns whether the band
// was dense.
//
// The non-empty slices are compacted and flattened into rows of 64 wedges;
// each wave owns a contiguous run of rows and each lane keeps a cursor on
// the slice holding its wedge, so moving to the next row costs a compare
// (and a short advance when the lane crosses into the next slice).  Lanes
// of a wave read consecutive entries of a list: coalesced 4-byte loads.
// Slices of the current band (search and compaction).  Leaves the
// compacted slice table in t and ends with a barrier; *total and *nkc
// receive the band's wedges and non-empty slices.
template <bool FULL, int WG, int BAND_WORDS>
__device__ __forceinline__ void compact_band(WedgeShared<WG, BAND_WORDS, FULL>& sh, SliceTable<WG>& t,
                                             const uint32_t* __restrict__ packed, const uint32_t* __restrict__ bidx,
                                             int gs, int32_t nk, int64_t lo, int64_t hi, bool seek_start, bool last,
                                             int32_t& pre, bool use_pre, int64_t next_hi, const CentreMeta& cm,
                                             int32_t& total_out, int32_t& nkc_out) {
    constexpr int NW = WG / kWave;
    const int tid = threadIdx.x, wave = tid / kWave, lane = lane_id();
    // slice of each centre: start (per-vertex mode: in t.start, scratch
    // until the compaction), end as the new cursor in c_cur
    uint32_t slice = 0;
    if constexpr (FULL) {
        for (int32_t k = wave; k < nk; k += NW) {
            const uint32_t cur = sh.c_cur[k];
            int32_t st = (int32_t)(cur & 0x7fffffffu);
            const int32_t ce = sh.c_ce[k];
            if (seek_start) st = wave_lower_bound(packed, st, ce, (uint32_t)lo);
            const int32_t en = last ? ce : wave_lower_bound(packed, st, ce, (uint32_t)hi);
            if (lane == 0) {
                t.start[k] = (uint32_t)st | (cur & 0x80000000u);
                sh.c_cur[k] = (uint32_t)en | (cur & 0x80000000u);
            }
        }
        __syncthreads();
        if (tid < nk) slice = t.start[tid];
    } else if (tid < nk) {
        // thread k owns centre k from here to the compaction: no barrier
        const uint32_t cur = sh.c_cur[tid];
        int32_t st = (int32_t)(cur & 0x7fffffffu);
        const int32_t ce = cm.ce, base = cm.base, khi = cm.khi;
        // first position at or after q with rank >= bound (a granule
        // multiple above the anchor's own entry, so bound >> gs is at least
        // the first indexed granule of every list holding the anchor)
        auto seek = [&](int32_t q, int64_t bound) {
            const int32_t kk = (int32_t)(bound >> gs);
            if (kk > khi) return ce;
            if (base != kBidxNone) return max(q, (int32_t)bidx[base + kk]);
            while (q < ce && (int64_t)(packed[q] >> 1) < bound) ++q;  // short list: step forward
            return q;
        };
        if (seek_start) st = seek(st, lo);
        int32_t en = ce;
        if (!last) en = (use_pre && base != kBidxNone) ? max(st, pre) : seek(st, hi);
        // the end of the next band of an indexed list, read now and used one band later
        if (next_hi >= 0 && base != kBidxNone) {
            const int32_t kk = (int32_t)(next_hi >> gs);
            pre = kk > khi ? ce : (int32_t)bidx[base + kk];
        }
        slice = (uint32_t)st | (cur & 0x80000000u);
        sh.c_cur[tid] = (uint32_t)en | (cur & 0x80000000u);
    }

    // compact the non-empty slices: one scan carries (length, count << 40)
    const uint32_t cur = slice;
    const int32_t len = tid < nk ? (int32_t)(sh.c_cur[tid] & 0x7fffffffu) - (int32_t)(cur & 0x7fffffffu) : 0;
    long long tot;
    const long long ex =
        block_exclusive_scan<WG>((long long)len + ((long long)(len > 0) << 40), sh.scan_tmp, &tot);
    const int32_t total = (int32_t)(tot & ((1ll << 40) - 1));
    const int32_t nkc = (int32_t)(tot >> 40);
    if (len > 0) {
        const int32_t idx = (int32_t)(ex >> 40);
        t.start[idx] = cur;
        t.pre[idx] = (int32_t)(ex & ((1ll << 40) - 1));
        if constexpr (FULL) sh.w_k[idx] = tid;
    }
    if (tid == 0) t.pre[nkc] = total;
    __syncthreads();
    // the same for every lane: keep them in scalar registers
    total_out = __builtin_amdgcn_readfirstlane(total);
    nkc_out = __builtin_amdgcn_readfirstlane(nkc);
}

// One wave's walk over its rows of the compacted band: row range, the
// per-lane slice cursor and the batch loaded ahead.
struct RowWalk {
    int32_t r, r1;      // next row, end of the wave's rows
    int32_t total;      // wedges in the band
    int32_t j, k, nb;   // this lane's next wedge, its slice and the slice end
    uint32_t st;        // slice start | negative-edge bit << 31
    int32_t base;       // list position of wedge j is base + j
};

// A batch of kUnroll rows (one element per lane and row) and the signs of
// its anchor edges (bit u: the anchor edge of row u is negative); the signs
// are applied when the batch is counted, so that the loads stay in flight
// until then.  A full batch (the same for every lane of the wave) lies
// inside each lane's current slice: every element is a wedge and ngmask is
// all ones or zero.  Otherwise only the first `rows` rows belong to the
// wave (the same for every lane) and bit u of vmask says whether row u
// holds a wedge for this lane (lanes past the band's last wedge hold none).
struct Batch {
    uint32_t x[kUnroll];
    uint32_t ngmask;
    uint32_t vmask;
    int32_t rows;
    bool full;
};

// Loads the batch of kUnroll rows at row w.r into x.  Advances the slice
// cursor, not w.j.
template <int WG>
__device__ __forceinline__ Batch load_batch(const SliceTable<WG>& t, const uint32_t* __restrict__ packed,
                                            RowWalk& w) {
    Batch bt;
    uint32_t(&x)[kUnroll] = bt.x;
    if (w.r + kUnroll <= w.r1 && __all(w.j + (kUnroll - 1) * kWave < w.nb)) {
        // whole batch inside each lane's current slice: one address,
        // immediate offsets
        const uint32_t* row = packed + (uint32_t)(w.base + w.j);
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) x[u] = row[u * kWave];
        bt.ngmask = (w.st >> 31) ? 0xffffffffu : 0u;
        bt.vmask = (1u << kUnroll) - 1u;
        bt.rows = kUnroll;
        bt.full = true;
    } else {
        uint32_t ngm = 0, vm = 0;
        const uint32_t spread = (uint32_t)lane_id() << 1;  // lanes with no wedge add zero to distinct words
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int32_t jj = w.j + u * kWave;
            x[u] = spread;
            if (w.r + u < w.r1 && jj < w.total) {
                while (jj >= w.nb) {  // stays below nkc: t.pre[nkc] = total > jj
                    ++w.k;
                    w.nb = t.pre[w.k + 1];
                    w.st = t.start[w.k];
                    w.base = (int32_t)(w.st & 0x7fffffffu) - t.pre[w.k];
                }
                x[u] = packed[(uint32_t)(w.base + jj)];
                ngm |= (w.st >> 31) << u;
                vm |= 1u << u;
            }
        }
        bt.ngmask = ngm;
        bt.vmask = vm;
        bt.rows = min(kUnroll, w.r1 - w.r);
        bt.full = false;
    }
    return bt;
}

// Counts the wedges of one batch in two steps: count_prep takes each
// loaded element to its counter field (byte offset in the band, increment),
// count_apply adds the increments.  Every loaded element lies in the current
// band (slices are cut at the band's ends), so no range test is needed.  In
// MASKED batches rows past the wave's last row are skipped and lanes holding
// no wedge add zero.  Dense bands increment without a return value; sparse
// ones mark the first increment of a word in the touched-word bitmap.
template <int MODE, bool MASKED, int BAND_WORDS>
__device__ __forceinline__ void count_prep(const Batch& b, uint32_t (&byte)[kUnroll], uint32_t (&inc)[kUnroll]) {
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
        const uint32_t ng = (MASKED ? b.ngmask >> u : b.ngmask) & 1u;
        // agree / disagree; in class mode both positive 0, both negative 1, different 2
        const uint32_t t = MODE >= 4 ? (((b.x[u] & 1u) != ng) ? 2u : ng) : (b.x[u] ^ ng) & 1u;
        uint32_t shift;
        slot_field<MODE, BAND_WORDS>(b.x[u] >> 1, t, byte[u], shift);
        const uint32_t one = MASKED ? (b.vmask >> u) & 1u : 1u;
        inc[u] = (MODE == 3 || MODE == 7) ? one : one << shift;
    }
}

template <int MODE, bool MASKED, int WG, int BAND_WORDS, bool FULL>
__device__ __forceinline__ void count_apply(WedgeShared<WG, BAND_WORDS, FULL>& sh, const uint32_t (&byte)[kUnroll],
                                            const uint32_t (&inc)[kUnroll], int32_t rows, bool dense) {
    char* base = reinterpret_cast<char*>(sh.cnt);
    if (dense) {  // no return value needed: the reduction scans the band
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (!MASKED || u < rows)
                (void)__hip_atomic_fetch_add(reinterpret_cast<uint32_t*>(base + byte[u]), inc[u], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP);
    } else {
        uint32_t old[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            old[u] = (!MASKED || u < rows) ? atomicAdd(reinterpret_cast<uint32_t*>(base + byte[u]), inc[u]) : 1u;
#pragma unroll
        for (int u = 0; u < kUnroll; ++u)
            if (old[u] == 0 && inc[u] != 0) atomicOr(&sh.bmp[byte[u] >> 7], 1u << ((byte[u] >> 2) & 31u));
    }
}

// Sets up this wave's rows of a compacted band (contiguous runs of rows per
// wave) and issues the loads of its first batch.
template <int WG>
__device__ __forceinline__ void walk_start(const SliceTable<WG>& t, const uint32_t* __restrict__ packed,
                                           int32_t total, int32_t nkc, RowWalk& w, Batch& next, bool& have_next) {
    constexpr int NW = WG / kWave;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)), lane = lane_id();
    const int32_t rows = (total + kWave - 1) / kWave;
    const int32_t rpw = (rows + NW - 1) / NW;
    w.r = wave * rpw;
    w.r1 = min(rows, w.r + rpw);
    w.total = total;
    have_next = false;
    if (w.r < w.r1) {
        w.j = w.r * kWave + lane;
        w.k = slice_of(t, nkc, min(w.j, total - 1));
        w.nb = t.pre[w.k + 1];
        w.st = t.start[w.k];
        w.base = (int32_t)(w.st & 0x7fffffffu) - t.pre[w.k];
        next = load_batch(t, packed, w);
        have_next = true;
    }
}

// Counts the wedges of this wave's rows.  walk_start has loaded the first
// batch (next, have_next set when the wave has rows); each step loads the
// batch after the current one (a full batch by one address, else through
// the slice cursors) before the current one's increments are applied.
template <int MODE, int WG, int BAND_WORDS, bool FULL>
__device__ __forceinline__ void walk_rows(WedgeShared<WG, BAND_WORDS, FULL>& sh, const SliceTable<WG>& t,
                                          const uint32_t* __restrict__ packed, bool dense, RowWalk& w, Batch& next,
                                          bool& have_next) {
    while (w.r < w.r1) {
        const Batch cur = next;
        w.j += kUnroll * kWave;
        w.r += kUnroll;
        // the current batch's fields first, then the next batch's loads:
        // a wave's loads complete in order, so a use of the current batch
        // placed after the next batch's loads would wait for those as well
        uint32_t byte[kUnroll], inc[kUnroll];
        if (cur.full) count_prep<MODE, false, BAND_WORDS>(cur, byte, inc);
        else count_prep<MODE, true, BAND_WORDS>(cur, byte, inc);
        __builtin_amdgcn_sched_barrier(0);
        have_next = w.r < w.r1;
        if (have_next) next = load_batch(t, packed, w);
        __builtin_amdgcn_sched_barrier(0);
        if (cur.full) count_apply<MODE, false>(sh, byte, inc, kUnroll, dense);
        else count_apply<MODE, true>(sh, byte, inc, cur.rows, dense);
    }
}

// A band holding at least BAND_WORDS / 16 wedges is "dense": its increments
// need no return value (no touched-word bitmap) and the reduction scans the
// whole band; sparser bands mark touched words.
template <int MODE, int BAND_WORDS>
__device__ __forceinline__ bool dense_band(int32_t total) { return MODE >= 6 || total >= BAND_WORDS / 16; }

// The three counters (both edges positive, both negative, different) of
// an endpoint's slot in a class layout (modes 4-7).
template <int MODE, int BAND_WORDS>
__device__ __forceinline__ void class_fields(const uint32_t* cnt, uint32_t rank, uint32_t& p, uint32_t& n,
                                             uint32_t& b) {
    uint32_t byte, shift;
    slot_field<MODE, BAND_WORDS>(rank, 0u, byte, shift);
    const uint32_t w = byte >> 2;
    if constexpr (MODE == 4) {
        const uint32_t v = cnt[w] >> shift;
        p = v & 15u;
        n = (v >> 4) & 15u;
        b = (v >> 8) & 15u;
    } else if constexpr (MODE == 5) {
        const uint32_t v = cnt[w];
        p = v & 255u;
        n = (v >> 8) & 255u;
        b = (v >> 16) & 255u;
    } else if constexpr (MODE == 6) {
        p = cnt[w] & 0xffffu;
        n = cnt[w] >> 16;
        b = cnt[w + 1] & 0xffffu;
    } else {
        p = cnt[w];
        n = cnt[w + 1];
        b = cnt[w + 2];
    }
}

// Per-vertex class mode: an anchor walking its whole list meets itself
// once per centre (a wedge u - c - u of pattern ++ or --); its slot is
// cleared before the band is reduced.  Ends with a barrier.
template <int MODE, int WG, int BAND_WORDS, bool FULL>
__device__ __forceinline__ void clear_self(WedgeShared<WG, BAND_WORDS, FULL>& sh, int32_t self, int64_t lo,
                                           int64_t hi) {
    if (threadIdx.x == 0 && (int64_t)self >= lo && (int64_t)self < hi) {
        uint32_t byte, shift;
        slot_field<MODE, BAND_WORDS>((uint32_t)self, 0u, byte, shift);
        const uint32_t w = byte >> 2;
        if constexpr (MODE == 4) sh.cnt[w] &= ~(0xfffu << shift);
        else if constexpr (MODE == 5) sh.cnt[w] = 0u;
        else if constexpr (MODE == 6) sh.cnt[w] = sh.cnt[w + 1] = 0u;
        else sh.cnt[w] = sh.cnt[w + 1] = sh.cnt[w + 2] = 0u;
    }
    __syncthreads();
}

// One band in one call: compaction, walk, and in per-vertex mode the centre
// walk (phases: bit 0 counts the wedges, bit 1 runs the centre walk, which
// needs the band's counters complete over every centre of the anchor).
// Returns the band's wedges.
template <int MODE, bool FULL, int WG, int BAND_WORDS>
__device__ __forceinline__ int32_t walk_band(WedgeShared<WG, BAND_WORDS, FULL>& sh, const uint32_t* __restrict__ packed,
                                          const uint32_t* __restrict__ bidx, int gs, int32_t nk, int64_t lo,
                                          int64_t hi, bool seek_start, bool last, int32_t self, int phases,
                                          int32_t& pre, bool use_pre, int64_t next_hi, const CentreMeta& cm,
                                          unsigned long long* __restrict__ pv = nullptr, int64_t centre_base = 0) {
    constexpr int NW = WG / kWave;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave)), lane = lane_id();
    SliceTable<WG>& t = sh.tab[0];
    int32_t total, nkc;
    compact_band(sh, t, packed, bidx, gs, nk, lo, hi, seek_start, last, pre, use_pre, next_hi, cm, total, nkc);
    const bool dense = dense_band<MODE, BAND_WORDS>(total);
    const int32_t rows = (total + kWave - 1) / kWave;
    const int32_t rpw = (rows + NW - 1) / NW;
    const int32_t r0 = wave * rpw, r1 = min(rows, r0 + rpw);
    if (phases & 1) {
        RowWalk w;
        Batch next;
        bool have_next;
        walk_start(t, packed, total, nkc, w, next, have_next);
        walk_rows<MODE>(sh, t, packed, dense, w, next, have_next);
    }
    __syncthreads();

    if constexpr (FULL && MODE >= 4) {
        // per-vertex classes: the centre of every wedge u - c - w lies in
        // the butterflies pairing it with another shared centre of {u, w};
        // by the pattern t of this wedge (0 ++, 1 --, 2 +-) and the
        // endpoint's counters p, n, b:
        //   ++: p - 1 of ++/++, n of ++/--, b of ++/+-
        //   --: p of ++/--, n - 1 of --/--, b of +-/--
        //   +-: b - 1 of +-/+-, p of ++/+-, n of +-/--
        // summed per lane and added to the centre's six global counters
        // when the lane leaves the slice (halved at the end: every pair is
        // walked from both ends)
        if ((phases & 2) && r0 < r1) {
            int32_t j = r0 * kWave + lane;
            int32_t k = slice_of(t, nkc, min(j, total - 1));
            int32_t nb = t.pre[k + 1];
            uint32_t st = t.start[k];
            int32_t base = (int32_t)(st & 0x7fffffffu) - t.pre[k];
            unsigned long long run[6] = {0, 0, 0, 0, 0, 0};
            auto flush = [&](int32_t kk) {
                unsigned long long* dst = pv + (centre_base + sh.c_id[sh.w_k[kk]]) * 6;
#pragma unroll
                for (int q = 0; q < 6; ++q) {
                    if (run[q]) atomicAdd(&dst[q], run[q]);
                    run[q] = 0;
                }
            };
            for (int32_t r = r0; r < r1; ++r, j += kWave) {
                if (j >= total) continue;
                while (j >= nb) {
                    flush(k);
                    ++k;
                    nb = t.pre[k + 1];
                    st = t.start[k];
                    base = (int32_t)(st & 0x7fffffffu) - t.pre[k];
                }
                const uint32_t x = packed[(uint32_t)(base + j)];
                if ((int32_t)(x >> 1) != self) {
                    const uint32_t ng = st >> 31;
                    const uint32_t pat = ((x & 1u) != ng) ? 2u : ng;
                    uint32_t p, n, b;
                    class_fields<MODE, BAND_WORDS>(sh.cnt, x >> 1, p, n, b);
                    if (pat == 0u) {
                        run[0] += p - 1u;
                        run[1] += n;
                        run[4] += b;
                    } else if (pat == 1u) {
                        run[1] += p;
                        run[2] += n - 1u;
                        run[5] += b;
                    } else {
                        run[3] += b - 1u;
                        run[4] += p;
                        run[5] += n;
                    }
                }
            }
            flush(k);
        }
        __syncthreads();
    } else if constexpr (FULL) {
        // centre walk over the same rows with the band's counters complete
        if ((phases & 2) && r0 < r1) {
            constexpr uint32_t fmask = MODE == 0 ? 15u : MODE == 1 ? 255u : MODE == 2 ? 0xffffu : 0xffffffffu;
            int32_t j = r0 * kWave + lane;
            int32_t k = slice_of(t, nkc, min(j, total - 1));
            int32_t nb = t.pre[k + 1];
            uint32_t st = t.start[k];
            int32_t base = (int32_t)(st & 0x7fffffffu) - t.pre[k];
            unsigned long long run = 0;
            for (int32_t r = r0; r < r1; ++r, j += kWave) {
                if (j >= total) continue;
                while (j >= nb) {
                    if (run) atomicAdd(&sh.c_sum[sh.w_k[k]], run);
                    run = 0;
                    ++k;
                    nb = t.pre[k + 1];
                    st = t.start[k];
                    base = (int32_t)(st & 0x7fffffffu) - t.pre[k];
                }
                const uint32_t x = packed[(uint32_t)(base + j)];
                if ((int32_t)(x >> 1) != self) {
                    uint32_t byte, shift;
                    slot_field<MODE, BAND_WORDS>(x >> 1, (x ^ (st >> 31)) & 1u, byte, shift);
                    run += ((sh.cnt[byte >> 2] >> shift) & fmask) - 1u;
                }
            }
            if (run) atomicAdd(&sh.c_sum[sh.w_k[k]], run);
        }
        __syncthreads();
    }
    return total;
}

// Sums of the six sign-pattern classes, per thread: for an endpoint with p
// wedges whose edges are both positive, n both negative and b different,
// ++/++ C(p,2), ++/-- p n, --/-- C(n,2), +-/+- C(b,2), ++/+- p b, +-/-- n b.
struct ClassSums {
    unsigned long long c[6] = {0, 0, 0, 0, 0, 0};
    __device__ __forceinline__ void add(uint32_t p, uint32_t n, uint32_t b) {
        if (!(p | n | b)) return;
        const unsigned long long P = p, N = n, B = b;
        c[0] += P * (P - (P > 0)) / 2;
        c[1] += P * N;
        c[2] += N * (N - (N > 0)) / 2;
        c[3] += B * (B - (B > 0)) / 2;
        c[4] += P * B;
        c[5] += N * B;
    }
};

// Per-band class sums of narrow slots (4- and 8-bit fields) in 32 bits:
// a thread visits at most 64 slots of a band, each adding at most 255^2
// per class.  take() moves C(p,2) = (p^2 - p) / 2 and the products into the
// 64-bit sums.
struct NarrowClassSums {
    uint32_t pp = 0, nn = 0, bb = 0, pn = 0, pb = 0, nb = 0, p1 = 0, n1 = 0, b1 = 0;
    __device__ __forceinline__ void add(uint32_t p, uint32_t n, uint32_t b) {
        pp += p * p;
        nn += n * n;
        bb += b * b;
        pn += p * n;
        pb += p * b;
        nb += n * b;
        p1 += p;
        n1 += n;
        b1 += b;
    }
    __device__ __forceinline__ void take(ClassSums& cs) const {
        cs.c[0] += (pp - p1) >> 1;
        cs.c[1] += pn;
        cs.c[2] += (nn - n1) >> 1;
        cs.c[3] += (bb - b1) >> 1;
        cs.c[4] += pb;
        cs.c[5] += nb;
    }
};

// The slots of one counter word in the narrow class layouts: two 16-bit
// slots of 4-bit fields (p, n, b gathered into nibbles 0 and 4 of three
// words, then nibble dot products), or one slot of 8-bit fields.
template <int MODE>
__device__ __forceinline__ void narrow_word(NarrowClassSums& ns, uint32_t w) {
    if constexpr (MODE == 4) {
        const uint32_t P = w & 0x000f000fu, N = (w >> 4) & 0x000f000fu, B = (w >> 8) & 0x000f000fu;
        ns.pp = __builtin_amdgcn_udot8(P, P, ns.pp, false);
        ns.nn = __builtin_amdgcn_udot8(N, N, ns.nn, false);
        ns.bb = __builtin_amdgcn_udot8(B, B, ns.bb, false);
        ns.pn = __builtin_amdgcn_udot8(P, N, ns.pn, false);
        ns.pb = __builtin_amdgcn_udot8(P, B, ns.pb, false);
        ns.nb = __builtin_amdgcn_udot8(N, B, ns.nb, false);
        ns.p1 = __builtin_amdgcn_udot8(P, 0x11111111u, ns.p1, false);
        ns.n1 = __builtin_amdgcn_udot8(N, 0x11111111u, ns.n1, false);
        ns.b1 = __builtin_amdgcn_udot8(B, 0x11111111u, ns.b1, false);
    } else {
        ns.add(w & 255u, (w >> 8) & 255u, (w >> 16) & 255u);
    }
}

// Four slots of 8-bit fields (one per word): byte k of each word gathered
// into one word by byte permutes, then byte dot products.
__device__ __forceinline__ void narrow_quad8(NarrowClassSums& ns, const uint4& v) {
    // v_perm_b32: selector byte s picks byte s of {hi, lo} (lo = bytes 0-3), 0x0c gives zero
    const uint32_t P = __builtin_amdgcn_perm(v.y, v.x, 0x0c0c0400u) | __builtin_amdgcn_perm(v.w, v.z, 0x04000c0cu);
    const uint32_t N = __builtin_amdgcn_perm(v.y, v.x, 0x0c0c0501u) | __builtin_amdgcn_perm(v.w, v.z, 0x05010c0cu);
    const uint32_t B = __builtin_amdgcn_perm(v.y, v.x, 0x0c0c0602u) | __builtin_amdgcn_perm(v.w, v.z, 0x06020c0cu);
    ns.pp = __builtin_amdgcn_udot4(P, P, ns.pp, false);
    ns.nn = __builtin_amdgcn_udot4(N, N, ns.nn, false);
    ns.bb = __builtin_amdgcn_udot4(B, B, ns.bb, false);
    ns.pn = __builtin_amdgcn_udot4(P, N, ns.pn, false);
    ns.pb = __builtin_amdgcn_udot4(P, B, ns.pb, false);
    ns.nb = __builtin_amdgcn_udot4(N, B, ns.nb, false);
    ns.p1 = __builtin_amdgcn_udot4(P, 0x01010101u, ns.p1, false);
    ns.n1 = __builtin_amdgcn_udot4(N, 0x01010101u, ns.n1, false);
    ns.b1 = __builtin_amdgcn_udot4(B, 0x01010101u, ns.b1, false);
}

// Class mode: the class sums of every touched slot of the band, clearing
// the counters.  A dense band is scanned four words at a time (slots never
// straddle them); a sparse one (narrow layouts only) through the
// touched-word bitmap.  Ends with a barrier.
template <int MODE, int WG, int BAND_WORDS, bool FULL>
__device__ __forceinline__ void reduce_classes(WedgeShared<WG, BAND_WORDS, FULL>& sh, ClassSums& cs, bool dense) {
    if constexpr (MODE <= 5) {
        NarrowClassSums ns;
        if (dense) {
            for (uint32_t w4 = threadIdx.x; w4 < (uint32_t)BAND_WORDS / 4u; w4 += WG) {
                uint4* q = reinterpret_cast<uint4*>(&sh.cnt[w4 * 4u]);
                const uint4 v = *q;
                if (!(v.x | v.y | v.z | v.w)) continue;
                *q = uint4{0u, 0u, 0u, 0u};
                if constexpr (MODE == 5) {
                    narrow_quad8(ns, v);
                } else {
                    narrow_word<MODE>(ns, v.x);
                    narrow_word<MODE>(ns, v.y);
                    narrow_word<MODE>(ns, v.z);
                    narrow_word<MODE>(ns, v.w);
                }
            }
        } else {
            for (uint32_t b = threadIdx.x; b < (uint32_t)BAND_WORDS / 32u; b += WG) {
                uint32_t bits = sh.bmp[b];
                if (bits) {
                    sh.bmp[b] = 0;
                    while (bits) {
                        const uint32_t wd = (b << 5) + (uint32_t)(__ffs(bits) - 1);
                        bits &= bits - 1u;
                        narrow_word<MODE>(ns, sh.cnt[wd]);
                        sh.cnt[wd] = 0;
                    }
                }
            }
        }
        ns.take(cs);
    } else {
        for (uint32_t w4 = threadIdx.x; w4 < (uint32_t)BAND_WORDS / 4u; w4 += WG) {
            uint4* q = reinterpret_cast<uint4*>(&sh.cnt[w4 * 4u]);
            const uint4 v = *q;
            if (!(v.x | v.y | v.z | v.w)) continue;
            *q = uint4{0u, 0u, 0u, 0u};
            if constexpr (MODE == 6) {
                cs.add(v.x & 0xffffu, v.x >> 16, v.y & 0xffffu);
                cs.add(v.z & 0xffffu, v.z >> 16, v.w & 0xffffu);
            } else {
                cs.add(v.x, v.y, v.z);
            }
        }
    }
    __syncthreads();
}

// Balanced (2,k)-bicliques: per endpoint pair C(a, k) + C(b, k) as exact
// 128-bit integers.  tab holds C(x, k) for x < 256 (low, high words);
// larger counts use the multiplicative formula.
struct BicView {
    int32_t k;  // 1..16
    const unsigned long long* __restrict__ tab;
};

// C(x, k) in four 32-bit limbs: after step i the limbs hold C(x, i + 1),
// since C(x, i) (x - i) is divisible by i + 1.  ovf is set when a partial
// product leaves 128 bits.
__device__ inline void choose_u128(uint32_t x, int k, unsigned long long& lo, unsigned long long& hi, bool& ovf) {
    uint32_t l[4] = {1u, 0u, 0u, 0u};
    for (int i = 0; i < k; ++i) {
        const unsigned long long f = x - (uint32_t)i;
        unsigned long long carry = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const unsigned long long t = (unsigned long long)l[j] * f + carry;
            l[j] = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) ovf = true;
        const unsigned long long d = (unsigned long long)(i + 1);
        unsigned long long r = 0;
#pragma unroll
        for (int j = 3; j >= 0; --j) {
            const unsigned long long t = (r << 32) | l[j];
            l[j] = (uint32_t)(t / d);
            r = t % d;
        }
    }
    lo = ((unsigned long long)l[1] << 32) | l[0];
    hi = ((unsigned long long)l[3] << 32) | l[2];
}

// Biclique sums ride in a ClassSums: c[0..3] are 32-bit limbs of the 128-bit
// sum kept in 64-bit registers (carried once per band), c[4] counts terms
// that do not fit 128 bits.
__device__ __forceinline__ void bic_field(ClassSums& cs, const BicView& bv, uint32_t x) {
    if (x < (uint32_t)bv.k) return;
    unsigned long long lo, hi;
    if (x < 256u) {
        lo = bv.tab[2 * x];
        hi = bv.tab[2 * x + 1];
    } else {
        bool ovf = false;
        choose_u128(x, bv.k, lo, hi, ovf);
        if (ovf) {
            cs.c[4] += 1;
            return;
        }
    }
    cs.c[0] += lo & 0xffffffffull;
    cs.c[1] += lo >> 32;
    cs.c[2] += hi & 0xffffffffull;
    cs.c[3] += hi >> 32;
}

__device__ __forceinline__ void bic_carry(ClassSums& cs) {
    cs.c[1] += cs.c[0] >> 32;
    cs.c[0] &= 0xffffffffull;
    cs.c[2] += cs.c[1] >> 32;
    cs.c[1] &= 0xffffffffull;
    cs.c[3] += cs.c[2] >> 32;
    cs.c[2] &= 0xffffffffull;
}

// Fields of one counter word in the count layouts (a and b alike).  4-bit
// fields read C(x, k) from the small LDS table.
template <int MODE>
__device__ __forceinline__ void bic_word(ClassSums& cs, const BicView& bv, const uint32_t* ctab, uint32_t v) {
    if constexpr (MODE == 0) {
#pragma unroll
        for (int f = 0; f < 8; ++f) {
            const uint32_t x = (v >> (4 * f)) & 15u;
            if (x >= (uint32_t)bv.k) cs.c[0] += ctab[x];
        }
    } else if constexpr (MODE == 1) {
#pragma unroll
        for (int f = 0; f < 4; ++f) bic_field(cs, bv, (v >> (8 * f)) & 255u);
    } else if constexpr (MODE == 2) {
        bic_field(cs, bv, v & 0xffffu);
        bic_field(cs, bv, v >> 16);
    } else {
        bic_field(cs, bv, v);
    }
}

// Biclique mode: C(x, k) of every field of every touched word (a full scan
// of a dense band, the touched-word bitmap otherwise), clearing the
// counters.  Ends with a barrier.
template <int MODE, int WG, int BAND_WORDS, bool FULL>
__device__ __forceinline__ void reduce_bic(WedgeShared<WG, BAND_WORDS, FULL>& sh, const BicView& bv, ClassSums& cs,
                                           bool dense) {
    if (dense) {
        for (uint32_t w4 = threadIdx.x; w4 < (uint32_t)BAND_WORDS / 4u; w4 += WG) {
            uint4* q = reinterpret_cast<uint4*>(&sh.cnt[w4 * 4u]);
            const uint4 v = *q;
            if (!(v.x | v.y | v.z | v.w)) continue;
            *q = uint4{0u, 0u, 0u, 0u};
            bic_word<MODE>(cs, bv, sh.ctab, v.x);
            bic_word<MODE>(cs, bv, sh.ctab, v.y);
            bic_word<MODE>(cs, bv, sh.ctab, v.z);
            bic_word<MODE>(cs, bv, sh.ctab, v.w);
        }
    } else {
        for (uint32_t b = threadIdx.x; b < (uint32_t)BAND_WORDS / 32u; b += WG) {
            uint32_t bits = sh.bmp[b];
            if (bits) {
                sh.bmp[b] = 0;
                while (bits) {
                    const uint32_t wd = (b << 5) + (uint32_t)(__ffs(bits) - 1);
                    bits &= bits - 1u;
                    bic_word<MODE>(cs, bv, sh.ctab, sh.cnt[wd]);
                    sh.cnt[wd] = 0;
                }
            }
        }
    }
    bic_carry(cs);
    __syncthreads();
}

// C(x, k) for x = 0..255 (one workgroup of 256 threads); x < k gives 0.
__global__ void k_choose_table(int32_t k, unsigned long long* tab) {
    const uint32_t x = threadIdx.x;
    unsigned long long lo = 0, hi = 0;
    bool ovf = false;
    if (x >= (uint32_t)k) choose_u128(x, k, lo, hi, ovf);  // C(255, 16) < 2^81: no overflow here
    tab[2 * x] = lo;
    tab[2 * x + 1] = hi;
}

// Sum of the pair terms of every touched counter word, and clears them.
// A dense band is scanned word by word; otherwise the touched-word bitmap
// is scanned in full (slots are scattered over the whole band capacity).
// In per-vertex mode the anchor's own slot (w = u), if in [lo, hi), is left
// out.  For an anchor of a dense block the cross term of endpoints in the
// same block is added.  Ends with a barrier.
template <int MODE, bool FULL, int WG, int BAND_WORDS>
__device__ __forceinline__ unsigned long long reduce_band(WedgeShared<WG, BAND_WORDS, FULL>& sh, int64_t lo,
                                                          int64_t hi, int32_t self, const CrossRow& cr, bool dense,
                                                          int32_t total) {
    const bool cross = cr.row && lo < cr.rank0 + cr.n_r && hi > cr.rank0;
    uint32_t sw0 = 0xffffffffu, sm0 = 0, sw1 = 0xffffffffu, sm1 = 0;
    if constexpr (FULL) {
        if ((int64_t)self >= lo && (int64_t)self < hi) {
            constexpr uint32_t fmask = MODE == 0 ? 15u : MODE == 1 ? 255u : MODE == 2 ? 0xffffu : 0xffffffffu;
            uint32_t sh0, sh1;
            slot_field<MODE, BAND_WORDS>((uint32_t)self, 0u, sw0, sh0);
            slot_field<MODE, BAND_WORDS>((uint32_t)self, 1u, sw1, sh1);
            sw0 >>= 2;
            sw1 >>= 2;
            sm0 = fmask << sh0;
            sm1 = fmask << sh1;
        }
    }
    unsigned long long acc = 0;
    PairSum<MODE, !FULL> ps;
    auto word_terms = [&](uint32_t wd, uint32_t v) {
        if constexpr (FULL) {
            if (wd == sw0) v &= ~sm0;
            if (wd == sw1) v &= ~sm1;
        }
        ps.add(v);
        if (cross && v) acc += cross_term<MODE, BAND_WORDS>(wd, v, lo, cr);
    };
    if (dense) {  // every word, four at a time
        for (uint32_t w4 = threadIdx.x; w4 < (uint32_t)BAND_WORDS / 4u; w4 += WG) {
            uint4* p = reinterpret_cast<uint4*>(&sh.cnt[w4 * 4u]);
            const uint4 v = *p;
            if (v.x | v.y | v.z | v.w) *p = uint4{0u, 0u, 0u, 0u};
            if (FULL || cross) {
                word_terms(w4 * 4u + 0u, v.x);
                word_terms(w4 * 4u + 1u, v.y);
                word_terms(w4 * 4u + 2u, v.z);
                word_terms(w4 * 4u + 3u, v.w);
            } else {  // zero words add nothing
                ps.add(v.x);
                ps.add(v.y);
                ps.add(v.z);
                ps.add(v.w);
            }
        }
    } else {
        for (uint32_t b = threadIdx.x; b < (uint32_t)BAND_WORDS / 32u; b += WG) {
            uint32_t bits = sh.bmp[b];
            if (bits) {
                sh.bmp[b] = 0;
                while (bits) {
                    const uint32_t i = __ffs(bits) - 1;
                    bits &= bits - 1u;
                    const uint32_t wd = (b << 5) + i;
                    const uint32_t v = sh.cnt[wd];
                    sh.cnt[wd] = 0;
                    word_terms(wd, v);
                }
            }
        }
    }
    __syncthreads();
    if constexpr (FULL) return acc + ps.take();
    // count mode: twice the pair terms, the band's wedges subtracted once
    // (modular arithmetic: only the workgroup's sum is meaningful)
    return 2 * acc + ps.take() - (threadIdx.x == 0 ? (unsigned long long)total : 0ull);
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Granule of band ends in count mode: the band capacity of the widest
// counters, so every band capacity is a multiple of it.
template <int BAND_WORDS>
constexpr int granule_shift() { return ilog2(BAND_WORDS) - 1; }

// In class mode the narrowest band holds BAND_WORDS / 4 slots.
template <int MODE, int BAND_WORDS>
constexpr int mode_granule_shift() { return MODE >= 4 ? ilog2(BAND_WORDS) - 2 : granule_shift<BAND_WORDS>(); }

// All bands of anchor r (rank), list start a0, deg entries.  Anchors with
// at most WG centres keep one slice cursor per centre across bands (each
// band starts where the previous one ended); wider anchors re-load their
// centres per chunk and seek the band start.  In count mode the first band
// is [r + 1, the last granule multiple <= r + 1 + capacity), the next ones
// start and end on granule multiples.  Returns this thread's share of the
// anchor's pair terms (twice the pair terms in count mode; the shares are
// meaningful only summed over the workgroup).
template <int MODE, bool FULL, bool BIC, int WG, int BAND_WORDS>
__device__ __forceinline__ unsigned long long count_anchor(WedgeShared<WG, BAND_WORDS, FULL>& sh, const int32_t* __restrict__ acent,
                                           const uint8_t* __restrict__ aneg, const int32_t* __restrict__ back,
                                           const uint32_t* __restrict__ coff, const uint32_t* __restrict__ packed,
                                           const uint32_t* __restrict__ bidx, const int2* __restrict__ bmeta,
                                           int32_t a0, int32_t deg, int32_t r, int64_t n_s,
                                           unsigned long long* __restrict__ pv, int64_t centre_base,
                                           unsigned long long& bands, const HybridView& hv, ClassSums& cs,
                                           const BicView& bv) {
    constexpr int64_t band_slots = band_capacity<MODE, BAND_WORDS>();
    constexpr int gs = mode_granule_shift<MODE, BAND_WORDS>();
    auto band_end = [&](int64_t lo) {
        const int64_t hi = FULL ? lo + band_slots : ((lo + band_slots) >> gs) << gs;
        return hi < n_s ? hi : n_s;
    };
    const int64_t lo0 = FULL ? 0 : (int64_t)r + 1;
    unsigned long long acc = 0;
    int32_t blk = -1;
    CrossRow cr{nullptr, 0, 0};
    if (!FULL && hv.ablk1) {
        blk = (int32_t)hv.ablk1[r] - 1;
        const DevBlock& B = hv.blocks[blk < 0 ? 0 : blk];
        if (blk >= 0 && B.n_r >= 2 && B.n_k >= 1) {  // blocks without an anchor pair have no table
            cr.rank0 = B.rank0;
            cr.n_r = B.n_r;
            cr.row = hv.tabs + B.tab_off + (int64_t)(r - B.rank0) * B.rpad;
        }
    }
    if (deg <= WG && !FULL) {
        // count mode, one chunk of centres: the next band is compacted and
        // its first loads are issued before the current band is reduced, so
        // the loads travel while the counters are summed and cleared
        const CentreMeta cm = load_centres<FULL>(sh, acent, aneg, back, coff, bmeta, a0, 0, deg, blk, hv);
        __syncthreads();
        int32_t pre = 0;  // prefetched end of the band after the current one
        int64_t lo = lo0, hi = band_end(lo);
        int buf = 0;
        int32_t total, nkc;
        RowWalk w;
        Batch next;
        bool have_next;
        {
            const int64_t nh = hi < n_s ? band_end(hi) : -1;
            compact_band(sh, sh.tab[0], packed, bidx, gs, deg, lo, hi, false, hi == n_s, pre, false,
                         nh < n_s ? nh : -1, cm, total, nkc);
            walk_start(sh.tab[0], packed, total, nkc, w, next, have_next);
        }
        for (;;) {
            const bool dense = dense_band<MODE, BAND_WORDS>(total);
            walk_rows<MODE>(sh, sh.tab[buf], packed, dense, w, next, have_next);
            __syncthreads();
            const bool more = hi < n_s;
            const int64_t lo2 = hi;
            int64_t hi2 = hi;
            int32_t total2 = 0, nkc2 = 0;
            RowWalk w2;
            Batch next2;
            bool have_next2 = false;
            if (more) {
                hi2 = band_end(lo2);
                const int64_t nh = hi2 < n_s ? band_end(hi2) : -1;
                compact_band(sh, sh.tab[buf ^ 1], packed, bidx, gs, deg, lo2, hi2, false, hi2 == n_s, pre, true,
                             nh < n_s ? nh : -1, cm, total2, nkc2);
                walk_start(sh.tab[buf ^ 1], packed, total2, nkc2, w2, next2, have_next2);
            }
            if constexpr (MODE >= 4) reduce_classes<MODE>(sh, cs, dense);
            else if constexpr (BIC) reduce_bic<MODE>(sh, bv, cs, dense);
            else acc += reduce_band<MODE, FULL>(sh, lo, hi, r, cr, dense, total);
            ++bands;
            if (!more) break;
            lo = lo2;
            hi = hi2;
            total = total2;
            nkc = nkc2;
            w = w2;
            next = next2;
            have_next = have_next2;
            buf ^= 1;
        }
    } else if (deg <= WG) {
        const CentreMeta cm = load_centres<FULL>(sh, acent, aneg, back, coff, bmeta, a0, 0, deg, blk, hv);
        __syncthreads();
        int32_t pre = 0;  // prefetched end of the band after the current one
        for (int64_t lo = lo0, hi; lo < n_s; lo = hi) {
            hi = band_end(lo);
            // the next band's end is a granule multiple unless it is the last band
            const int64_t nh = hi < n_s ? band_end(hi) : -1;
            const int32_t total = walk_band<MODE, FULL>(sh, packed, bidx, gs, deg, lo, hi, false, hi == n_s, r,
                                                        FULL ? 3 : 1, pre, lo != lo0, nh < n_s ? nh : -1, cm, pv,
                                                        centre_base);
            if constexpr (FULL && MODE >= 4) clear_self<MODE>(sh, r, lo, hi);
            if constexpr (MODE >= 4) reduce_classes<MODE>(sh, cs, dense_band<MODE, BAND_WORDS>(total));
            else if constexpr (BIC) reduce_bic<MODE>(sh, bv, cs, dense_band<MODE, BAND_WORDS>(total));
            else acc += reduce_band<MODE, FULL>(sh, lo, hi, r, cr, dense_band<MODE, BAND_WORDS>(total), total);
            ++bands;
        }
        if constexpr (FULL && MODE < 4) {
            if (threadIdx.x < deg && sh.c_sum[threadIdx.x])
                atomicAdd(&pv[centre_base + sh.c_id[threadIdx.x]], sh.c_sum[threadIdx.x]);
        }
    } else {
        for (int64_t lo = lo0, hi; lo < n_s; lo = hi) {
            hi = band_end(lo);
            const bool first = lo == lo0;
            bool dense = false;  // any chunk dense: the band is reduced by a full scan
            int32_t total = 0;
            for (int32_t k0 = 0; k0 < deg; k0 += WG) {
                const int32_t nk = min(WG, deg - k0);
                const CentreMeta cm =
                    load_centres<FULL>(sh, acent, aneg, back, coff, bmeta, a0, k0, nk, blk, hv);
                __syncthreads();
                int32_t pre = 0;
                const int32_t tc = walk_band<MODE, FULL>(sh, packed, bidx, gs, nk, lo, hi, !first, hi == n_s, r, 1,
                                                         pre, false, -1, cm);
                dense |= dense_band<MODE, BAND_WORDS>(tc);
                total += tc;
            }
            if constexpr (FULL) {
                // second pass over the chunks once every wedge of the band is counted
                for (int32_t k0 = 0; k0 < deg; k0 += WG) {
                    const int32_t nk = min(WG, deg - k0);
                    const CentreMeta cm =
                        load_centres<FULL>(sh, acent, aneg, back, coff, bmeta, a0, k0, nk, blk, hv);
                    __syncthreads();
                    int32_t pre = 0;
                    walk_band<MODE, FULL>(sh, packed, bidx, gs, nk, lo, hi, !first, hi == n_s, r, 2, pre, false, -1,
                                          cm, pv, centre_base);
                    if constexpr (MODE < 4) {
                        if (threadIdx.x < nk && sh.c_sum[threadIdx.x])
                            atomicAdd(&pv[centre_base + sh.c_id[threadIdx.x]], sh.c_sum[threadIdx.x]);
                    }
                }
            }
            if constexpr (FULL && MODE >= 4) clear_self<MODE>(sh, r, lo, hi);
            if constexpr (MODE >= 4) reduce_classes<MODE>(sh, cs, dense);
            else if constexpr (BIC) reduce_bic<MODE>(sh, bv, cs, dense);
            else acc += reduce_band<MODE, FULL>(sh, lo, hi, r, cr, dense, total);
            ++bands;
        }
    }
    return acc;
}

// ------------------------------------------------------------ wave regime
//
// Light anchors (at most kLightMaxWork wedges and kLightMaxDeg centres; the
// paper's warp regime, Algorithm 4) are counted by one wave each, with no
// workgroup barrier: the wave's share of the counter band becomes a hashed
// table of TW slots, a slot holding the endpoint key (rank - anchor rank,
// 20 bits) above its two 6-bit counters (agree, disagree; both <= degree).
// An anchor has at most TW / 2 wedges, so the table is never more than half
// full and a linear probe always ends.  The pair terms are summed while
// counting: raising a counter from x to x + 1 adds C(x+1,2) - C(x,2) = x, so
// the value an increment returns is its share and no reduction pass is
// needed; the table is then cleared.

template <int TW>
__device__ __forceinline__ uint32_t light_hash(uint32_t key) {
    return (key * 0x9E3779B1u) >> (32 - ilog2(TW));
}

// Slot of `key` for wedge type t, probing from slot h: claims an empty slot
// or increments the key's counter; returns the counter's value before the
// increment.  A slot, once claimed, keeps its key until the table is
// cleared, so every probe for a key stops at the same slot whatever the
// order of the insertions.
template <int TW>
__device__ __forceinline__ uint32_t light_insert(uint32_t* __restrict__ tab, uint32_t key, uint32_t t, uint32_t h) {
    const uint32_t sh = 6u * t;
    const uint32_t inc = 1u << sh;
    for (;;) {
        const uint32_t old = atomicCAS(&tab[h], 0u, (key << 12) | inc);
        if (old == 0u) return 0u;
        if ((old >> 12) == key) return (atomicAdd(&tab[h], inc) >> sh) & 63u;
        h = (h + 1u) & (uint32_t)(TW - 1);
    }
}

// The inserts of N rows (row u valid where bit u of vm is set), taken in
// lock step: the first probes of all rows go out together, then the
// increments of the rows whose key was there already; rows that met another
// key probe on one by one.  Returns the sum of the counters' values before
// their increments.
template <int TW, int N>
__device__ __forceinline__ uint32_t light_insert_rows(uint32_t* __restrict__ tab, const uint32_t (&key)[N],
                                                      const uint32_t (&t)[N], uint32_t vm) {
    uint32_t h[N], old[N];
#pragma unroll
    for (int u = 0; u < N; ++u) {
        h[u] = light_hash<TW>(key[u]);
        old[u] = ((vm >> u) & 1u) ? atomicCAS(&tab[h[u]], 0u, (key[u] << 12) | (1u << (6u * t[u]))) : 0u;
    }
    uint32_t acc = 0;
#pragma unroll
    for (int u = 0; u < N; ++u)
        if (old[u] != 0u && (old[u] >> 12) == key[u])
            acc += (atomicAdd(&tab[h[u]], 1u << (6u * t[u])) >> (6u * t[u])) & 63u;
#pragma unroll
    for (int u = 0; u < N; ++u)
        if (old[u] != 0u && (old[u] >> 12) != key[u])
            acc += light_insert<TW>(tab, key[u], t[u], (h[u] + 1u) & (uint32_t)(TW - 1));
    return acc;
}

// Rows of 64 wedges loaded together by the wave regime.
constexpr int kLightRows = 4;

// A wave-regime anchor read ahead of its walk, in steps a wave can issue
// while it still walks the anchors before: its rank r (-1: none), then its
// list range (a0, deg) and, in a batch, its graph g, then each lane's centre
// (lane < deg: back-pointer, centre id, sign of the anchor edge), then the
// end of that centre's list.
struct LightAhead {
    int32_t r, a0, deg, g;
    int32_t bk, ce;
    uint32_t ng, cend;
};

__device__ __forceinline__ void light_head(LightAhead& n, const uint32_t* __restrict__ aoff,
                                           const int32_t* __restrict__ agraph) {
    n.a0 = 0;
    n.deg = 0;
    n.g = -1;
    if (n.r >= 0) {
        n.a0 = (int32_t)aoff[n.r];
        n.deg = (int32_t)aoff[n.r + 1] - n.a0;
        if (agraph) n.g = agraph[n.r];
    }
}

__device__ __forceinline__ void light_lanes(LightAhead& n, const int32_t* __restrict__ acent,
                                            const uint8_t* __restrict__ aneg, const int32_t* __restrict__ back) {
    const int lane = lane_id();
    n.bk = 0;
    n.ce = 0;
    n.ng = 0;
    if (n.deg >= 2 && lane < n.deg) {
        const int32_t p = n.a0 + lane;
        n.bk = back[p];
        n.ce = acent[p];
        n.ng = aneg[p];
    }
}

__device__ __forceinline__ void light_ends(LightAhead& n, const uint32_t* __restrict__ coff) {
    n.cend = (n.deg >= 2 && lane_id() < n.deg) ? coff[n.ce + 1] : 0u;
}

// A wave-regime anchor whose walk has begun.  Lane k holds centre k's
// slice (the suffix of its list above the anchor): pp its first position in
// the flattened walk (exclusive prefix of the lengths) | one past its last
// << 16 (a walk has at most kLightMaxWork positions), sv its list start |
// sign of the anchor edge << 31.  carry is one more than
// the slice holding the last position of the rows loaded so far (0 before
// the first).  The next kLightRows rows are loaded: row u in x[u], bit u of
// ngm the sign of the anchor edge, bit u of vm set where the lane holds a
// wedge.  total = 0: nothing to count and the hashed table left untouched.
static_assert(kLightMaxWork < 65536, "walk positions must fit 16 bits");
struct LightWalk {
    int32_t r, g, total;
    uint32_t pp, sv, carry;
    uint32_t x[kLightRows];
    uint32_t ngm, vm;
};

// Loads rows j0 .. j0 + kLightRows - 1 of the walk (one wedge per lane and
// row).  The slice of position j is the last non-empty slice starting at or
// before j: each non-empty slice marks its start in the wave's LDS marks
// (mark u + (p & 63) for a start p in row u, value slice + 1), and a running
// maximum over the lanes, carried from row to row, gives every lane its
// slice; the marks are zeroed again as they are read.  A lane loads only
// when its position lies inside the slice found, so every load stays in
// the slice's list.
__device__ __forceinline__ void light_rows(LightWalk& w, int32_t j0, uint32_t* __restrict__ mark,
                                           const uint32_t* __restrict__ packed) {
    const int lane = lane_id();
    const int32_t d = (int32_t)(w.pp & 0xffffu) - j0;
    if ((w.pp >> 16) > (w.pp & 0xffffu) && d >= 0 && d < kLightRows * kWave) mark[d] = (uint32_t)lane + 1u;
    __builtin_amdgcn_wave_barrier();
    uint32_t m[kLightRows];
#pragma unroll
    for (int u = 0; u < kLightRows; ++u) m[u] = mark[u * kWave + lane];
#pragma unroll
    for (int u = 0; u < kLightRows; ++u) mark[u * kWave + lane] = 0u;
    __builtin_amdgcn_wave_barrier();
    uint32_t ngm = 0, vm = 0;
#pragma unroll
    for (int u = 0; u < kLightRows; ++u) {
        const uint32_t kk = max(wave_inclusive_max_dpp(m[u]), w.carry);
        w.carry = (uint32_t)__builtin_amdgcn_readlane((int)kk, kWave - 1);
        const int src = ((int)kk - 1) & (kWave - 1);
        const uint32_t sp = (uint32_t)__shfl((int)w.pp, src, kWave);
        const int32_t s0 = (int32_t)(sp & 0xffffu), s1 = (int32_t)(sp >> 16);
        const uint32_t st = (uint32_t)__shfl((int)w.sv, src, kWave);
        const int32_t j = j0 + u * kWave + lane;
        w.x[u] = 0u;
        if (kk != 0u && j < w.total && j >= s0 && j < s1) {
            w.x[u] = packed[(st & 0x7fffffffu) + (uint32_t)(j - s0)];
            ngm |= (st >> 31) << u;
            vm |= 1u << u;
        }
    }
    w.ngm = ngm;
    w.vm = vm;
}

// Begins the walk of light anchor c and loads its first rows.
__device__ __forceinline__ void light_start(LightWalk& w, uint32_t* __restrict__ mark,
                                            const uint32_t* __restrict__ packed, const LightAhead& c) {
    const int lane = lane_id();
    w.r = c.r;
    w.g = c.g;
    w.total = 0;
    if (c.deg < 2) return;
    int32_t len = 0;
    w.sv = 0;
    if (lane < c.deg) {
        const uint32_t s0 = (uint32_t)c.bk + 1u;
        len = (int32_t)(c.cend - s0);
        w.sv = s0 | (c.ng << 31);
    }
    const int32_t inc = (int32_t)wave_inclusive_sum_dpp((uint32_t)len);
    const int32_t total = __builtin_amdgcn_readlane(inc, kWave - 1);
    if (total < 2) return;
    w.total = total;
    w.pp = (uint32_t)(inc - len) | ((uint32_t)inc << 16);
    w.carry = 0;
    light_rows(w, 0, mark, packed);
}

// Turns the loaded rows of walk w into table keys (endpoint rank minus the
// anchor's rank, in x) and wedge types (bit u of ngm: 0 signs agree, 1
// differ).
__device__ __forceinline__ void light_prep(LightWalk& w) {
    uint32_t tm = 0;
#pragma unroll
    for (int u = 0; u < kLightRows; ++u) {
        tm |= ((w.x[u] ^ (w.ngm >> u)) & 1u) << u;
        w.x[u] = (w.x[u] >> 1) - (uint32_t)w.r;
    }
    w.ngm = tm;
}

// Twice the pair terms of the anchor whose walk w began, its loaded rows
// prepared (light_prep), summed over the wave's lanes (each lane returns
// its share): counts the loaded rows, then loads and counts the rest.
template <int TW>
__device__ __forceinline__ uint32_t light_finish(LightWalk& w, uint32_t* __restrict__ tab, uint32_t* __restrict__ mark,
                                                 const uint32_t* __restrict__ packed) {
    uint32_t acc = 0;  // at most kLightMaxWork increments of at most 63
    for (int32_t j0 = 0;;) {
        uint32_t t[kLightRows];
#pragma unroll
        for (int u = 0; u < kLightRows; ++u) t[u] = (w.ngm >> u) & 1u;
        acc += light_insert_rows<TW>(tab, w.x, t, w.vm);
        j0 += kWave * kLightRows;
        if (j0 >= w.total) break;
        light_rows(w, j0, mark, packed);
        light_prep(w);
    }
    return 2u * acc;
}

template <int TW>
__device__ __forceinline__ void light_clear(uint32_t* __restrict__ tab) {
    uint4* t4 = reinterpret_cast<uint4*>(tab);
    for (int i = lane_id(); i < TW / 4; i += kWave) t4[i] = uint4{0u, 0u, 0u, 0u};
    __builtin_amdgcn_wave_barrier();
}

// How the persistent workgroups take work: positions [0, n_s - n_light) of
// the schedule one anchor each (workgroup regime), queue_chunk anchors per
// pop; the light positions after them light_chunk anchors per pop, dealt
// to the waves of the workgroup.
struct SchedArgs {
    int32_t statik;       // nonzero: fixed deal of the tasks instead of the queue
    int32_t queue_chunk;  // >= 1
    int32_t light_chunk;  // >= 1
};

// Batched launches pass agraph (graph of each rank), rank_end (first rank of
// each graph, n_graphs + 1 entries) and per-graph totals; an anchor's
// endpoints then stop at the end of its graph's rank range.
// CLS: the six sign-pattern classes instead of the balanced total (count
// mode only), summed into st->cls.  BIC: balanced (2,k)-bicliques, the
// 128-bit sum as 32-bit limbs in st->cls[0..3] and the count of terms
// beyond 128 bits in st->cls[4].
// PH: 0 runs every anchor; count mode runs in two launches, PH = 1 for the
// workgroup-regime anchors (queue st->queue) and PH = 2 for the wave-regime
// anchors (queue st->queue2), so that neither path's registers weigh on the
// other (in one kernel the wave path made the compiler spill the workgroup
// path's per-anchor state).
template <int WG, int BAND_WORDS, bool FULL, bool CLS = false, bool BIC = false, int PH = 0>
__global__ __launch_bounds__(WG, 1024 / WG) void k_wedge(const uint32_t* __restrict__ aoff, const int32_t* __restrict__ acent,
                                              const uint8_t* __restrict__ aneg, const int32_t* __restrict__ back,
                                              const uint32_t* __restrict__ coff, const uint32_t* __restrict__ packed,
                                              const uint32_t* __restrict__ bidx, const int2* __restrict__ bmeta,
                                              const uint32_t* __restrict__ order, int32_t n_s, DevStatus* st,
                                              unsigned long long* __restrict__ pv, const uint32_t* __restrict__ inv,
                                              int64_t anchor_base, int64_t centre_base,
                                              const int32_t* __restrict__ agraph,
                                              const int64_t* __restrict__ rank_end,
                                              unsigned long long* __restrict__ gtotals, HybridView hv, BicView bv,
                                              SchedArgs sc) {
    if (*(volatile const int32_t*)&st->flags) return;  // input error: nothing to count
    __shared__ WedgeShared<WG, BAND_WORDS, FULL> sh;
    const int tid = threadIdx.x;
    for (int i = tid; i < BAND_WORDS; i += WG) sh.cnt[i] = 0;
    for (int i = tid; i < BAND_WORDS / 32; i += WG) sh.bmp[i] = 0;
    if (BIC && tid < 16) sh.ctab[tid] = (uint32_t)bv.tab[2 * tid];
    unsigned long long acc = 0, bands = 0;
    ClassSums cs;
    constexpr bool kCount = !FULL && !CLS && !BIC;
    constexpr bool kLight = kCount && PH != 1;  // this launch runs wave-regime anchors
    constexpr bool kHeavy = PH != 2;            // this launch runs workgroup-regime anchors
    constexpr int NW = WG / kWave;
    constexpr int TW = BAND_WORDS / NW < 2048 ? BAND_WORDS / NW : 2048;  // light table slots per wave
    const uint32_t n_light = kCount ? *(volatile const uint32_t*)&st->n_light : 0u;
    const uint32_t n_heavy = (uint32_t)n_s - n_light;
    // 32-bit task arithmetic: n_s < 2^31 and both chunks are at most 2^16
    const uint32_t qc = (uint32_t)sc.queue_chunk, lc = (uint32_t)sc.light_chunk;
    const uint32_t heavy_tasks = (n_heavy + qc - 1) / qc;
    const uint32_t light_tasks = kLight ? (n_light + lc - 1) / lc : 0u;
    // tasks of this launch are [t_first, n_tasks)
    const uint32_t t_first = PH == 2 ? heavy_tasks : 0u;
    const uint32_t n_tasks = heavy_tasks + light_tasks;
    unsigned int* queue = PH == 2 ? &st->queue2 : &st->queue;

    // one anchor of the workgroup regime (schedule position pos)
    auto heavy = [&](uint32_t pos) {
        const int32_t r = (int32_t)order[pos];
        const int32_t a0 = (int32_t)aoff[r], deg = (int32_t)aoff[r + 1] - a0;
        const int64_t n_end = agraph ? rank_end[agraph[r] + 1] : (int64_t)n_s;
        // fewer than two centres (k in biclique mode): no endpoint pair
        // shares enough wedges
        if (deg < (BIC ? bv.k : 2) || (!FULL && r >= n_end - 1)) return;
        constexpr int M0 = CLS ? 4 : 0;  // counter mode of degree class 0; classes use modes 4-7
        unsigned long long a;
        // per-vertex classes: the anchor's own six sums, then the totals
        ClassSums ca;
        ClassSums& csa = (FULL && CLS) ? ca : cs;
        if (deg <= 15)
            a = count_anchor<M0 + 0, FULL, BIC>(sh, acent, aneg, back, coff, packed, bidx, bmeta, a0, deg, r, n_end,
                                                  pv, centre_base, bands, hv, csa, bv);
        else if (deg <= 255)
            a = count_anchor<M0 + 1, FULL, BIC>(sh, acent, aneg, back, coff, packed, bidx, bmeta, a0, deg, r, n_end,
                                                  pv, centre_base, bands, hv, csa, bv);
        else if (deg <= 65535)
            a = count_anchor<M0 + 2, FULL, BIC>(sh, acent, aneg, back, coff, packed, bidx, bmeta, a0, deg, r, n_end,
                                                  pv, centre_base, bands, hv, csa, bv);
        else
            a = count_anchor<M0 + 3, FULL, BIC>(sh, acent, aneg, back, coff, packed, bidx, bmeta, a0, deg, r, n_end,
                                                  pv, centre_base, bands, hv, csa, bv);
        if constexpr (FULL && CLS) {
#pragma unroll
            for (int q = 0; q < 6; ++q) {
                const unsigned long long s = block_sum<WG>(ca.c[q], (unsigned long long*)sh.scan_tmp);
                if (tid == 0) pv[(anchor_base + inv[r]) * 6 + q] = s;
                cs.c[q] += ca.c[q];
            }
        } else if constexpr (FULL) {
            const unsigned long long s = block_sum<WG>(a, (unsigned long long*)sh.scan_tmp);
            if (tid == 0) pv[anchor_base + inv[r]] = s;
        } else if (gtotals) {
            const unsigned long long s = block_sum<WG>(a, (unsigned long long*)sh.scan_tmp);
            if (tid == 0 && s) atomicAdd(&gtotals[agraph[r]], s >> 1);  // twice the pair terms
        }
        acc += a;
    };

    uint32_t snext = t_first + blockIdx.x;  // static deal: tasks b, b + grid, b + 2 grid, ... (< 2^32)
    for (;;) {
        __syncthreads();
        uint32_t task;
        if (sc.statik) {
            task = snext;
            snext += gridDim.x;
        } else {  // dynamic: the next task of the shared queue
            if (tid == 0) sh.task = (int32_t)atomicAdd(queue, 1u);
            __syncthreads();
            task = t_first + (uint32_t)sh.task;
        }
        if (task >= n_tasks) break;
        if (task < heavy_tasks) {
            if constexpr (kHeavy) {
                const uint32_t p1 = min(n_heavy, (task + 1) * qc);
                for (uint32_t pos = task * qc; pos < p1; ++pos) {
                    if (pos > task * qc) __syncthreads();
                    heavy((uint32_t)pos);
                }
            }
        } else if constexpr (kLight) {
            // a chunk of light anchors, dealt round robin to the waves
            const int wave = tid / kWave;
            uint32_t* tab = sh.cnt + wave * TW;
            const uint32_t p0 = n_heavy + (task - heavy_tasks) * lc;
            const uint32_t p1 = min((uint32_t)n_s, p0 + lc);
            int32_t g_cur = -1;
            uint32_t g_acc = 0;  // this lane's share of the current graph's total (batches)
            // the wave's anchors pos, pos + NW, ... in a pipeline four deep:
            // while anchor A is counted, the first rows of B are in flight,
            // C's list ends and D's list range; D's centres while A's table
            // is cleared.  The marks of the row loads: kLightRows * 64 words
            // per wave, in the slice tables (unused by wave-regime anchors),
            // zero between loads.
            static_assert(sizeof(sh.tab) >= (size_t)NW * kLightRows * kWave * 4, "light marks must fit");
            uint32_t* const mark = reinterpret_cast<uint32_t*>(&sh.tab[0]) + wave * (kLightRows * kWave);
#pragma unroll
            for (int u = 0; u < kLightRows; ++u) mark[u * kWave + lane_id()] = 0u;
            __builtin_amdgcn_wave_barrier();
            uint32_t pos = p0 + wave;
            LightAhead B, C, D;
            B.r = pos < p1 ? (int32_t)order[pos] : -1;
            light_head(B, aoff, agraph);
            light_lanes(B, acent, aneg, back);
            light_ends(B, coff);
            LightWalk A;
            light_start(A, mark, packed, B);
            B.r = pos + NW < p1 ? (int32_t)order[pos + NW] : -1;
            light_head(B, aoff, agraph);
            light_lanes(B, acent, aneg, back);
            light_ends(B, coff);
            C.r = pos + 2 * NW < p1 ? (int32_t)order[pos + 2 * NW] : -1;
            light_head(C, aoff, agraph);
            light_lanes(C, acent, aneg, back);
            D.r = pos + 3 * NW < p1 ? (int32_t)order[pos + 3 * NW] : -1;
            for (; pos < p1; pos += NW) {
                // A's rows are used before any load below is issued: a wave's
                // loads complete in order, so a use placed after newer loads
                // would wait for those too
                if (A.total > 0) light_prep(A);
                __builtin_amdgcn_sched_barrier(0);
                LightWalk Bw;
                light_start(Bw, mark, packed, B);
                light_ends(C, coff);
                light_head(D, aoff, agraph);
                const int32_t r_n = pos + 4 * NW < p1 ? (int32_t)order[pos + 4 * NW] : -1;
                if (gtotals) {
                    const int32_t g = A.g;
                    if (g != g_cur) {
                        const uint32_t t = wave_sum(g_acc);
                        if (lane_id() == 0 && t && g_cur >= 0) atomicAdd(&gtotals[g_cur], (unsigned long long)(t >> 1));
                        g_cur = g;
                        g_acc = 0;
                    }
                }
                const bool touched = A.total > 0;
                const uint32_t a = touched ? light_finish<TW>(A, tab, mark, packed) : 0u;
                light_lanes(D, acent, aneg, back);
                if (touched) light_clear<TW>(tab);
                acc += a;
                g_acc += a;
                A = Bw;
                B = C;
                C = D;
                D.r = r_n;
            }
            if (gtotals) {
                const unsigned long long t = wave_sum((unsigned long long)g_acc);
                if (lane_id() == 0 && t && g_cur >= 0) atomicAdd(&gtotals[g_cur], t >> 1);
            }
        }
    }
    acc = wave_sum(acc);
    if (lane_id() == 0 && acc) atomicAdd(&st->total, acc);
    if constexpr (CLS || BIC) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const unsigned long long v = wave_sum(cs.c[k]);
            if (lane_id() == 0 && v) atomicAdd(&st->cls[k], v);
        }
    }
    if (tid == 0 && bands) atomicAdd(&st->bands, bands);
}

// In per-vertex mode every unordered endpoint pair is seen from both ends:
// halve the centre sums.
__global__ void k_halve(unsigned long long* pv, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) pv[i] >>= 1;
}

// ------------------------------------------------------------------ launch

struct WedgeArgs {
    const uint32_t* aoff;
    const int32_t* acent;
    const uint8_t* aneg;
    const int32_t* back;
    const uint32_t* coff;
    const uint32_t* packed;
    const uint32_t* bidx;
    const int2* bmeta;
    const uint32_t* order;
    int32_t n_s;
    DevStatus* st;
    unsigned long long* pv;
    const uint32_t* inv;
    int64_t anchor_base, centre_base;
    const int32_t* agraph;
    const int64_t* rank_end;
    unsigned long long* gtotals;
    HybridView hv;
    BicView bv;
    SchedArgs sc;
};

template <int WG, int BW, bool FULL, bool CLS = false, bool BIC = false, int PH = 0>
static void launch_phase(const WedgeArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_wedge<WG, BW, FULL, CLS, BIC, PH>), dim3(grid), dim3(WG), 0, s, a.aoff, a.acent, a.aneg,
                       a.back, a.coff, a.packed, a.bidx, a.bmeta, a.order, a.n_s, a.st, a.pv, a.inv, a.anchor_base,
                       a.centre_base, a.agraph, a.rank_end, a.gtotals, a.hv, a.bv, a.sc);
}

// Count mode: the workgroup-regime anchors, then the wave-regime ones.
template <int WG, int BW, bool FULL, bool CLS = false, bool BIC = false>
static void launch_shape(const WedgeArgs& a, int grid, hipStream_t s) {
    if constexpr (!FULL && !CLS && !BIC) {
        launch_phase<WG, BW, false, false, false, 1>(a, grid, s);
        launch_phase<WG, BW, false, false, false, 2>(a, grid, s);
    } else {
        launch_phase<WG, BW, FULL, CLS, BIC>(a, grid, s);
    }
}

template <int WG, int BW, bool FULL, bool CLS = false, bool BIC = false>
static int occupancy() {
    constexpr int PH = (!FULL && !CLS && !BIC) ? 1 : 0;
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_wedge<WG, BW, FULL, CLS, BIC, PH>, WG, 0) != hipSuccess)
        return 1;
    return n > 0 ? n : 1;
}

// Instantiated shapes: (threads per workgroup, counter words per band).
// The first is the default.  Per-vertex mode uses one shape of its own.
struct WedgeShape {
    int wg, band_words;
    int (*occ)();
    void (*launch)(const WedgeArgs&, int, hipStream_t);
};
#define BBC_SHAPE(W, B) {W, B, occupancy<W, B, false>, launch_shape<W, B, false>}
static const WedgeShape kShapes[] = {BBC_SHAPE(256, 8192),  BBC_SHAPE(512, 16384), BBC_SHAPE(256, 16384),
                                     BBC_SHAPE(512, 8192),  BBC_SHAPE(1024, 32768), BBC_SHAPE(1024, 16384),
                                     BBC_SHAPE(128, 4096),  BBC_SHAPE(128, 8192),   BBC_SHAPE(256, 4096)};
#undef BBC_SHAPE
constexpr int kFullWG = 256, kFullBW = 16384;
constexpr int kFullClsWG = 256, kFullClsBW = 8192;  // per-vertex classes
constexpr int kClsWG = 256, kClsBW = 8192;  // sign-pattern classes: one shape
constexpr int kBicWG = 256, kBicBW = 8192;  // (2,k)-bicliques: one shape, the count layouts

static int shape_index(int band_words, int wg) {
    int n = (int)(sizeof(kShapes) / sizeof(kShapes[0]));
    for (int i = 0; i < n; ++i)
        if ((band_words == 0 || kShapes[i].band_words == band_words) && (wg == 0 || kShapes[i].wg == wg)) return i;
    return -1;
}

bool wedge_shape_ok(int band_words, int wg) { return shape_index(band_words, wg) >= 0; }

int wedge_block(int band_words, int wg, bool full) { return full ? kFullWG : kShapes[shape_index(band_words, wg)].wg; }

int wedge_band(int band_words, int wg, bool full) {
    return full ? kFullBW : kShapes[shape_index(band_words, wg)].band_words;
}

int wedge_shape_count() { return (int)(sizeof(kShapes) / sizeof(kShapes[0])); }

// Largest wedge count of a light anchor for a count-mode shape: half the
// hashed table each wave carves from the band (at most 2048 slots).
int wedge_light_max(int band_words, int wg) {
    const int i = shape_index(band_words, wg);
    if (i < 0) return 0;
    int tw = kShapes[i].band_words / (kShapes[i].wg / kWave);
    if (tw > 2048) tw = 2048;
    return tw / 2;
}

void wedge_shape(int i, int* wg, int* band_words) {
    *wg = kShapes[i].wg;
    *band_words = kShapes[i].band_words;
}

int wedge_class_blocks_per_cu() { return occupancy<kClsWG, kClsBW, false, true>(); }

int wedge_class_pv_blocks_per_cu() { return occupancy<kFullClsWG, kFullClsBW, true, true>(); }

int wedge_class_band() { return kClsBW; }

int wedge_bic_blocks_per_cu() { return occupancy<kBicWG, kBicBW, false, false, true>(); }

void launch_choose_table(int32_t k, unsigned long long* tab, hipStream_t s) {
    hipLaunchKernelGGL(k_choose_table, dim3(1), dim3(256), 0, s, k, tab);
}

int wedge_blocks_per_cu(int band_words, int wg, bool full) {
    if (full) return occupancy<kFullWG, kFullBW, true>();
    const int i = shape_index(band_words, wg);
    return i >= 0 ? kShapes[i].occ() : 1;
}

void launch_wedge(int band_words, int wg, int grid, const uint32_t* aoff, const int32_t* acent, const uint8_t* aneg,
                  const int32_t* back, const uint32_t* coff, const uint32_t* packed, const uint32_t* bidx,
                  const int2* bmeta, const uint32_t* order, int32_t n_s, DevStatus* st, unsigned long long* pv,
                  const uint32_t* inv, int64_t anchor_base, int64_t centre_base, int64_t n_centre,
                  const int32_t* agraph, const int64_t* rank_end, unsigned long long* gtotals, const HybridView& hv,
                  int kind, int32_t bic_k, const unsigned long long* bic_tab, int sched, int32_t queue_chunk,
                  int32_t light_chunk, hipStream_t s) {
    const WedgeArgs a{aoff,        acent,       aneg,   back,     coff,    packed, bidx,
                      bmeta,       order,       n_s,    st,       pv,      inv,    anchor_base,
                      centre_base, agraph,      rank_end, gtotals, hv,     BicView{bic_k, bic_tab},
                      SchedArgs{sched == 1 ? 1 : 0, queue_chunk > 0 ? queue_chunk : 1,
                                light_chunk > 0 ? light_chunk : 1}};
    if (pv) {
        // per-vertex output: U ids first, then V ids; six counters per
        // vertex in class mode
        const int64_t per = kind == kWedgeClasses ? 6 : 1;
        if (kind == kWedgeClasses) launch_shape<kFullClsWG, kFullClsBW, true, true>(a, grid, s);
        else launch_shape<kFullWG, kFullBW, true>(a, grid, s);
        if (n_centre > 0) {
            int64_t g = (n_centre * per + 255) / 256;
            hipLaunchKernelGGL(k_halve, dim3((unsigned)(g > 4096 ? 4096 : g)), dim3(256), 0, s,
                               pv + centre_base * per, n_centre * per);
        }
        return;
    }
    if (kind == kWedgeClasses) {
        launch_shape<kClsWG, kClsBW, false, true>(a, grid, s);
        return;
    }
    if (kind == kWedgeBicliques) {
        launch_shape<kBicWG, kBicBW, false, false, true>(a, grid, s);
        return;
    }
    const int i = shape_index(band_words, wg);
    if (i >= 0) kShapes[i].launch(a, grid, s);
}

}  // namespace bbc
