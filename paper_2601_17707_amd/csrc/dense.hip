// Dense-block hybrid: the wedges of dense anchor x centre blocks counted on
// int8 matrix cores.
//
// A block is a set R of anchors and a set C of centres; its dense edges are
// the graph's edges between R and C.  With S the |R| x |C| signed adjacency
// of those edges (+1, -1, 0 when absent), the wedges u - c - w with both
// edges dense give, for every anchor pair,
//     (S S^T)[u][w]     = a - b   (agreeing minus disagreeing wedges)
//     (|S| |S|^T)[u][w] = a + b
// so a and b come out of two int8 products with exact int32 accumulation.
// By Lemma 1 the pair contributes C(a,2) + C(b,2).  The paper counts every
// wedge through hash maps or shared-memory tiles (Algorithms 2-4); this
// split is the library's own.  It is exact for any choice of blocks: per
// pair, with a = a_dense + a_sparse (likewise b),
//     C(a,2) = C(a_dense,2) + C(a_sparse,2) + a_dense * a_sparse,
// so the sparse walk skips exactly the dense wedges (an anchor of R walking
// a centre of C jumps past R's run of that centre's rank-sorted list) and,
// for endpoint pairs inside R, adds the cross term from a table of
// (a_dense, b_dense) written here.
//
// Layout: each block's anchors take a contiguous rank range at the top of
// the rank order (ranks by (block, degree, id)); the block matrix is int8,
// row-major, rows in rank order (padded to 128), columns in the caller's
// centre order (padded to 64).  |S| is S & 1 per byte, formed in registers.
// Each workgroup computes one 128 x 128 tile of the upper triangle with
// v_mfma_i32_32x32x32_i8: four waves, each 64 x 64 (2 x 2 MFMA tiles, two
// products), operands staged through two LDS buffers 128 bytes of K at a
// time (the next slice is loaded while the current one computes, one
// barrier per slice); two workgroups per CU.  A 64 x 64 tile (one MFMA tile
// per wave, four workgroups per CU) is the alternative the autotuner can
// pick for small blocks.
#include <type_traits>

#include "bbc_internal.h"

namespace bbc {

__device__ __forceinline__ void flag_block(DevStatus* st, int64_t idx) {
    atomicOr(&st->flags, kBadBlocks);
    atomicMin((unsigned long long*)&st->bad_block, (unsigned long long)idx);
}

__device__ __forceinline__ bool status_bad(const DevStatus* st) { return *(volatile const int32_t*)&st->flags != 0; }

// Marks the block of every listed anchor (agrp[id] = block + 1) and centre
// (cblk[id] = block, cidx[id] = position in the block's centre list).  An id
// out of range, repeated, or listed by two blocks flags kBadBlocks with
// bad_block = block * 2^32 + position (anchor list first, then centre list
// positions offset by the anchor count).  agrp starts at 0, cblk at -1.
__global__ void k_block_mark(const DevBlock* blocks, int32_t n_s, int32_t n_c, uint32_t* agrp, int32_t* cblk,
                             int32_t* cidx, DevStatus* st) {
    const int32_t b = blockIdx.y;
    const DevBlock B = blocks[b];
    const int64_t tot = (int64_t)B.n_aid + B.n_cid;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < tot; p += (int64_t)gridDim.x * blockDim.x) {
        const int64_t tag = ((int64_t)b << 32) + p;
        if (p < B.n_aid) {
            const int32_t x = B.aid[p];
            if (x < 0 || x >= n_s || atomicCAS(&agrp[x], 0u, (uint32_t)b + 1u) != 0u) flag_block(st, tag);
        } else {
            const int32_t q = (int32_t)(p - B.n_aid);
            const int32_t c = B.cid[q];
            if (c < 0 || c >= n_c || atomicCAS(&cblk[c], -1, b) != -1) flag_block(st, tag);
            else cidx[c] = q;
        }
    }
}

// For each centre of a block: the first position of its list past the
// block's anchors (their ranks form [rank0, rank0 + n_r)).
__global__ void k_block_cpos(const int32_t* cblk, int32_t n_c, const DevBlock* blocks, const uint32_t* coff,
                             const uint32_t* packed, int32_t* cpos, const DevStatus* st) {
    if (status_bad(st)) return;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n_c; c += (int64_t)gridDim.x * blockDim.x) {
        const int32_t b = cblk[c];
        if (b < 0) continue;
        const uint32_t end_rank = (uint32_t)(blocks[b].rank0 + blocks[b].n_r);
        uint32_t lo = coff[c], hi = coff[c + 1];
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if ((packed[mid] >> 1) < end_rank) lo = mid + 1;
            else hi = mid;
        }
        cpos[c] = (int32_t)lo;
    }
}

// One wave per block anchor: writes its dense edges into the block matrix
// (already zeroed): +1 or -1 at (rank - rank0, position of the centre).
__global__ void k_block_pack(const uint32_t* ablk1, int32_t r_first, int32_t n_s, const DevBlock* blocks,
                             const uint32_t* aoff, const int32_t* acent, const uint8_t* aneg, const int32_t* cblk,
                             const int32_t* cidx, int8_t* mats, const DevStatus* st) {
    if (status_bad(st)) return;
    const int lane = lane_id();
    const int64_t nwv = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t r = r_first + ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; r < n_s; r += nwv) {
        const int32_t b = (int32_t)ablk1[r] - 1;
        if (b < 0) continue;
        const DevBlock B = blocks[b];
        if (B.n_r < 2 || B.n_k < 1) continue;  // no anchor pair: the block has no matrix
        int8_t* row = mats + B.mat_off + (r - B.rank0) * (int64_t)B.kpad;
        for (uint32_t p = aoff[r] + lane; p < aoff[r + 1]; p += kWave) {
            const int32_t c = acent[p];
            if (cblk[c] == b) row[cidx[c]] = aneg[p] ? (int8_t)-1 : (int8_t)1;
        }
    }
}

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kDK = 128;         // K bytes per LDS stage
constexpr int kDRow = kDK + 16;  // LDS row pitch in bytes (padding spreads banks)
constexpr int kDRowsPerPass = 256 * 16 / kDK;  // rows one pass of the workgroup's 16-byte loads covers

// Output element of accumulator i in lane l of a 32 x 32 MFMA tile: column
// l % 32, row 8 * (i / 4) + 4 * (l / 32) + i % 4.
__device__ __forceinline__ int mfma_row(int i, int lane) { return 8 * (i >> 2) + 4 * (lane >> 5) + (i & 3); }

// One TILE x TILE output tile of the upper triangle of a block product per
// workgroup, operands staged through registers into two LDS buffers
// (TILE = 64: four waves of 32 x 32, one MFMA tile each; the 64-row tile
// option runs this kernel, the 128-row default runs k_dense_lds below).
template <int TILE>
__global__ __launch_bounds__(256, TILE == 128 ? 2 : 4) void k_dense(const DevBlock* __restrict__ blocks,
                                                                    const DevTile* __restrict__ tiles,
                                                                    const int8_t* __restrict__ mats,
                                                                    uint32_t* __restrict__ tabs, DevStatus* st) {
    constexpr int WT = TILE / 2;           // wave tile edge
    constexpr int NT = WT / 32;            // MFMA tiles per wave tile edge
    constexpr int kLoads = TILE / kDRowsPerPass;  // 16-byte loads per thread and matrix per stage
    if (status_bad(st)) return;
    // two LDS stages: the next K slice is stored into one while the other
    // feeds the matrix cores
    __shared__ __align__(16) int8_t As[2][TILE * kDRow];
    __shared__ __align__(16) int8_t Bs[2][TILE * kDRow];
    const DevTile T = tiles[blockIdx.x];
    const DevBlock B = blocks[T.blk];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int wr = wave >> 1, wc = wave & 1;
    // on a diagonal tile the lower-left wave's outputs all lie below the
    // diagonal (u > w): it loads and stores its share of the operands but
    // issues no matrix instruction
    const bool idle = T.ti == T.tj && wr > wc;
    const int8_t* arow = mats + B.mat_off + (int64_t)T.ti * TILE * B.kpad;
    const int8_t* brow = mats + B.mat_off + (int64_t)T.tj * TILE * B.kpad;

    v16i accD[NT][NT], accP[NT][NT];
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            accD[i][j] = v16i{};
            accP[i][j] = v16i{};
        }

    // staging: TILE rows x kDK bytes per matrix in 16-byte pieces, kLoads
    // per thread and matrix, held in registers while the previous slice
    // computes; columns past kpad (a block whose K is not a multiple of kDK)
    // are read as zero
    const int lr = tid / (kDK / 16), lc = (tid % (kDK / 16)) * 16;
    int4 ga[kLoads], gb[kLoads];
    auto load_stage = [&](int k0) {
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int64_t row = (int64_t)(lr + i * kDRowsPerPass) * B.kpad;
            const bool in = k0 + lc < B.kpad;
            ga[i] = in ? *(const int4*)(arow + row + k0 + lc) : int4{0, 0, 0, 0};
            gb[i] = in ? *(const int4*)(brow + row + k0 + lc) : int4{0, 0, 0, 0};
        }
    };
    auto store_stage = [&](int buf) {
#pragma unroll
        for (int i = 0; i < kLoads; ++i) {
            const int so = (lr + i * kDRowsPerPass) * kDRow + lc;
            *(int4*)&As[buf][so] = ga[i];
            *(int4*)&Bs[buf][so] = gb[i];
        }
    };
    load_stage(0);
    store_stage(0);
    __syncthreads();
    int buf = 0;
    for (int k0 = 0; k0 < B.kpad; k0 += kDK, buf ^= 1) {
        const bool more = k0 + kDK < B.kpad;
        if (more) load_stage(k0 + kDK);
        if (!idle) {
#pragma unroll
            for (int ks = 0; ks < kDK; ks += 32) {
                v4i a[NT], b[NT], aa[NT], ba[NT];
                const int kk = ks + 16 * (lane >> 5);
#pragma unroll
                for (int i = 0; i < NT; ++i) {
                    a[i] = *(const v4i*)&As[buf][(wr * WT + i * 32 + (lane & 31)) * kDRow + kk];
                    b[i] = *(const v4i*)&Bs[buf][(wc * WT + i * 32 + (lane & 31)) * kDRow + kk];
                    aa[i] = a[i] & 0x01010101;
                    ba[i] = b[i] & 0x01010101;
                }
#pragma unroll
                for (int i = 0; i < NT; ++i)
#pragma unroll
                    for (int j = 0; j < NT; ++j) {
                        accD[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], accD[i][j], 0, 0, 0);
                        accP[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aa[i], ba[j], accP[i][j], 0, 0, 0);
                    }
            }
        }
        // the other stage was last read before the previous barrier
        if (more) store_stage(buf ^ 1);
        __syncthreads();
    }
    if (idle) return;

    // epilogue: pair terms of the upper triangle and the (a, b) table;
    // a, b <= 65535, so a (a - 1) / 2 fits 32 bits
    unsigned long long acc = 0;
    uint32_t* tab = tabs + B.tab_off;
#pragma unroll
    for (int i = 0; i < NT; ++i)
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const int gw = T.tj * TILE + wc * WT + j * 32 + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int gu = T.ti * TILE + wr * WT + i * 32 + mfma_row(e, lane);
                if (gu < gw && gw < B.n_r) {
                    const uint32_t P = (uint32_t)accP[i][j][e], D = (uint32_t)accD[i][j][e];
                    const uint32_t a = (P + D) >> 1, b = (P - D) >> 1;
                    acc += (unsigned long long)(a * (a - (a > 0u))) + b * (b - (b > 0u));  // twice the pair terms
                    tab[(int64_t)gu * B.rpad + gw] = a | (b << 16);
                }
            }
        }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomicAdd(&st->total, acc);
}

// The 128 x 128 tile with operands loaded straight into LDS
// (global_load_lds_dwordx4: a wave's load fills 1,024 consecutive LDS
// bytes, 16 per lane) through kQStages stages of kQK bytes of K, so three
// stages are in flight while one feeds the matrix cores and no registers
// hold staged operands.  A stage holds 128 rows of kQK = 64 bytes per
// matrix; the four 16-byte chunks of row r sit at chunk c ^ qswz(r), which
// spreads the rows one wave reads at one K offset over all LDS banks (the
// loads pick their global chunk to match).  Each wave waits for its own
// loads of a stage, then one barrier makes every wave's loads visible and
// frees the stage read before it, which is refilled at once.
constexpr int kQK = 64;
constexpr int kQStages = 4;
constexpr int kQTile = 128;
constexpr int kQStageBytes = kQTile * kQK;

__device__ __forceinline__ int qswz(int r) { return ((r >> 1 ^ r >> 3) & 1) | ((r >> 1) & 2); }

// s_waitcnt with at most n vector memory operations outstanding (expcnt and
// lgkmcnt left at their maximum)
template <int N>
__device__ __forceinline__ void wait_vm() {
    static_assert(N >= 0 && N < 16, "vmcnt field");
    __builtin_amdgcn_s_waitcnt(0x0F70 | N);
}

// kQWaves waves per workgroup in a 2 x kQWaves/2 grid, each owning a 64 x
// (256 / kQWaves) piece of the tile; wave w loads rows 128 / kQWaves * w ..
// of both matrices, 16 rows per load.  Four waves of 64 x 64 (two
// workgroups, eight waves per CU) measured faster than eight of 64 x 32
// (four waves per SIMD, but half the reuse of each fragment read).
constexpr int kQWaves = 4;
__global__ __launch_bounds__(kQWaves * kWave, 2) void k_dense_lds(const DevBlock* __restrict__ blocks,
                                                                 const DevTile* __restrict__ tiles,
                                                                 const int8_t* __restrict__ mats,
                                                                 uint32_t* __restrict__ tabs, DevStatus* st) {
    constexpr int NWAVE = kQWaves;
    constexpr int WC = NWAVE / 2;                 // wave columns
    constexpr int WTR = kQTile / 2, WTC = kQTile / WC;  // wave tile rows, columns
    constexpr int NTR = WTR / 32, NTC = WTC / 32;  // MFMA tiles per wave tile edge
    constexpr int RPW = kQTile / NWAVE;            // rows each wave loads per matrix
    constexpr int LPM = RPW / 16;                  // loads per wave, matrix and stage
    constexpr int kInFlight = 2 * 2 * LPM;         // loads of the two stages after the one waited for
    typedef __attribute__((address_space(3))) void lds_t;
    if (status_bad(st)) return;
    // one LDS object per stage and matrix: the compiler then sees that a
    // stage's loads do not touch the stage being read and adds no wait of
    // its own (the waits below are the ones needed)
    __shared__ __align__(1024) int8_t A0[kQStageBytes], A1[kQStageBytes], A2[kQStageBytes], A3[kQStageBytes];
    __shared__ __align__(1024) int8_t B0[kQStageBytes], B1[kQStageBytes], B2[kQStageBytes], B3[kQStageBytes];
    const DevTile T = tiles[blockIdx.x];
    const DevBlock B = blocks[T.blk];
    const int tid = threadIdx.x, lane = lane_id(), wave = tid / kWave;
    const int wr = wave / WC, wc = wave % WC;
    // on a diagonal tile a wave whose outputs all lie below the diagonal
    // (u > w) loads its share of the operands but issues no matrix
    // instruction
    const bool idle = T.ti == T.tj && wr * WTR > wc * WTC + WTC - 1;
    // this lane's pieces: load j of the wave covers rows RPW w + 16 j ..,
    // lane l row RPW w + 16 j + l / 4, slot l % 4
    const int rl = RPW * wave + (lane >> 2), slot = lane & 3;
    const int64_t kp = B.kpad;
    const int8_t* ga[LPM];
    const int8_t* gb[LPM];
#pragma unroll
    for (int j = 0; j < LPM; ++j) {
        const int r = rl + 16 * j;
        ga[j] = mats + B.mat_off + ((int64_t)T.ti * kQTile + r) * kp + 16 * (slot ^ qswz(r));
        gb[j] = mats + B.mat_off + ((int64_t)T.tj * kQTile + r) * kp + 16 * (slot ^ qswz(r));
    }
    const int n_st = (int)(kp / kQK);  // kpad is a multiple of 64

    v16i accD[NTR][NTC], accP[NTR][NTC];
#pragma unroll
    for (int i = 0; i < NTR; ++i)
#pragma unroll
        for (int j = 0; j < NTC; ++j) {
            accD[i][j] = v16i{};
            accP[i][j] = v16i{};
        }

    // stage k (K bytes 64 k ..) into stage buffers S (= k % kQStages)
    auto issue = [&](auto S, int k) {
        constexpr int I = decltype(S)::value;
        int8_t* as = I == 0 ? A0 : I == 1 ? A1 : I == 2 ? A2 : A3;
        int8_t* bs = I == 0 ? B0 : I == 1 ? B1 : I == 2 ? B2 : B3;
        const int64_t k0 = (int64_t)k * kQK;
#pragma unroll
        for (int j = 0; j < LPM; ++j) {
            __builtin_amdgcn_global_load_lds(ga[j] + k0, (lds_t*)(as + (RPW * wave + 16 * j) * kQK), 16, 0, 0);
            __builtin_amdgcn_global_load_lds(gb[j] + k0, (lds_t*)(bs + (RPW * wave + 16 * j) * kQK), 16, 0, 0);
        }
    };
    // stage k from buffers S: wait for it (every step issues the same number
    // of loads, so those of the two later stages may stay in flight), refill
    // the buffers read before it with stage k + 3 (past the last stage the
    // last one is loaded again, which keeps the count uniform), then feed
    // the matrix cores
    auto step = [&](auto S, int k) {
        constexpr int I = decltype(S)::value;
        wait_vm<kInFlight>();
        __builtin_amdgcn_s_barrier();
        issue(std::integral_constant<int, (I + kQStages - 1) % kQStages>{}, min(k + kQStages - 1, n_st - 1));
        if (idle) return;
        const int8_t* as = I == 0 ? A0 : I == 1 ? A1 : I == 2 ? A2 : A3;
        const int8_t* bs = I == 0 ? B0 : I == 1 ? B1 : I == 2 ? B2 : B3;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            v4i a[NTR], b[NTC], aa[NTR], ba[NTC];
            const int c = 2 * ks + (lane >> 5);  // logical 16-byte chunk of this lane
#pragma unroll
            for (int i = 0; i < NTR; ++i) {
                const int ra = wr * WTR + i * 32 + (lane & 31);
                a[i] = *(const v4i*)&as[ra * kQK + 16 * (c ^ qswz(ra))];
                aa[i] = a[i] & 0x01010101;
            }
#pragma unroll
            for (int j = 0; j < NTC; ++j) {
                const int rb = wc * WTC + j * 32 + (lane & 31);
                b[j] = *(const v4i*)&bs[rb * kQK + 16 * (c ^ qswz(rb))];
                ba[j] = b[j] & 0x01010101;
            }
#pragma unroll
            for (int i = 0; i < NTR; ++i)
#pragma unroll
                for (int j = 0; j < NTC; ++j) {
                    accD[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a[i], b[j], accD[i][j], 0, 0, 0);
                    accP[i][j] = __builtin_amdgcn_mfma_i32_32x32x32_i8(aa[i], ba[j], accP[i][j], 0, 0, 0);
                }
        }
    };
    // n_st >= 1 (a block has a centre)
    issue(std::integral_constant<int, 0>{}, 0);
    issue(std::integral_constant<int, 1>{}, min(1, n_st - 1));
    issue(std::integral_constant<int, 2>{}, min(2, n_st - 1));
    int k = 0;
    for (; k + kQStages <= n_st; k += kQStages) {
        step(std::integral_constant<int, 0>{}, k);
        step(std::integral_constant<int, 1>{}, k + 1);
        step(std::integral_constant<int, 2>{}, k + 2);
        step(std::integral_constant<int, 3>{}, k + 3);
    }
    if (k < n_st) step(std::integral_constant<int, 0>{}, k);
    if (k + 1 < n_st) step(std::integral_constant<int, 1>{}, k + 1);
    if (k + 2 < n_st) step(std::integral_constant<int, 2>{}, k + 2);
    wait_vm<0>();  // no load may still be writing LDS when the workgroup ends
    if (idle) return;

    unsigned long long acc = 0;
    uint32_t* tab = tabs + B.tab_off;
#pragma unroll
    for (int i = 0; i < NTR; ++i)
#pragma unroll
        for (int j = 0; j < NTC; ++j) {
            const int gw = T.tj * kQTile + wc * WTC + j * 32 + (lane & 31);
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int gu = T.ti * kQTile + wr * WTR + i * 32 + mfma_row(e, lane);
                if (gu < gw && gw < B.n_r) {
                    const uint32_t P = (uint32_t)accP[i][j][e], D = (uint32_t)accD[i][j][e];
                    const uint32_t a = (P + D) >> 1, b = (P - D) >> 1;
                    acc += (unsigned long long)(a * (a - (a > 0u))) + b * (b - (b > 0u));  // twice the pair terms
                    tab[(int64_t)gu * B.rpad + gw] = a | (b << 16);
                }
            }
        }
    acc = wave_sum(acc);
    if (lane == 0 && acc) atomicAdd(&st->total, acc);
}

// ------------------------------------------------------------ host launchers

void launch_block_mark(const DevBlock* blocks, int32_t n_blocks, int64_t max_ids, int32_t n_s, int32_t n_c,
                       uint32_t* agrp, int32_t* cblk, int32_t* cidx, DevStatus* st, hipStream_t s) {
    if (n_blocks <= 0 || max_ids <= 0) return;
    int64_t g = (max_ids + 255) / 256;
    hipLaunchKernelGGL(k_block_mark, dim3((unsigned)(g > 1024 ? 1024 : g), (unsigned)n_blocks), dim3(256), 0, s,
                       blocks, n_s, n_c, agrp, cblk, cidx, st);
}

void launch_block_cpos(const int32_t* cblk, int32_t n_c, const DevBlock* blocks, const uint32_t* coff,
                       const uint32_t* packed, int32_t* cpos, const DevStatus* st, hipStream_t s) {
    if (n_c <= 0) return;
    int64_t g = ((int64_t)n_c + 255) / 256;
    hipLaunchKernelGGL(k_block_cpos, dim3((unsigned)(g > 4096 ? 4096 : g)), dim3(256), 0, s, cblk, n_c, blocks, coff,
                       packed, cpos, st);
}

void launch_block_pack(const uint32_t* ablk1, int32_t r_first, int32_t n_s, const DevBlock* blocks,
                       const uint32_t* aoff, const int32_t* acent, const uint8_t* aneg, const int32_t* cblk,
                       const int32_t* cidx, int8_t* mats, const DevStatus* st, hipStream_t s) {
    const int64_t rows = (int64_t)n_s - r_first;
    if (rows <= 0) return;
    int64_t g = (rows * kWave + 255) / 256;
    hipLaunchKernelGGL(k_block_pack, dim3((unsigned)(g > 8192 ? 8192 : g)), dim3(256), 0, s, ablk1, r_first, n_s,
                       blocks, aoff, acent, aneg, cblk, cidx, mats, st);
}

// tile: 64 or 128 (the output tile edge the tile list was built for)
void launch_dense(const DevBlock* blocks, const DevTile* tiles, int32_t n_tiles, const int8_t* mats, uint32_t* tabs,
                  DevStatus* st, int tile, hipStream_t s) {
    if (n_tiles <= 0) return;
    if (tile == 64)
        hipLaunchKernelGGL(k_dense<64>, dim3((unsigned)n_tiles), dim3(256), 0, s, blocks, tiles, mats, tabs, st);
    else
        hipLaunchKernelGGL(k_dense_lds, dim3((unsigned)n_tiles), dim3(kQWaves * kWave), 0, s, blocks, tiles, mats, tabs,
                           st);
}

}  // namespace bbc
