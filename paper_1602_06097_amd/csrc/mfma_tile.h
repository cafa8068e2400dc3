// mfma_tile.h -- the int8-limb MFMA tiles shared by the GEMM kernels.
//
// Every residue x in [0, p), p <= 65521, is centred into
//     r = x            if x <= 32639
//     r = x - p        otherwise            (r in [-32881, 32639])
// and split into two signed 8-bit limbs r = 256 h + l with
//     h = floor((r + 128) / 256) in [-128, 127],  l = r - 256 h in [-128, 127].
// Then  sum_k A B = 65536 S_hh + 256 (S_hl + S_lh) + S_ll  with four int8 GEMMs
// accumulated exactly in int32 (v_mfma_i32_16x16x64_i8): |h h'| <= 2^14, so a
// K-chunk of at most kKChunk = 65472 terms keeps |S_hh|, |S_ll| < 2^30 and the
// shared middle accumulator |S_hl + S_lh| < 2^31.  The three partials are
// combined into S = 65536 S_hh + 256 S_mid + S_ll and reduced mod p in
// double precision (combine_limbs): every intermediate is an integer below
// 2^53 in magnitude, so all of it is exact except the quotient estimate,
// which only selects a candidate remainder that two comparisons correct.
//
// The tiles are device functions so that both the one-problem kernels and
// the kernels that serve many problems in one launch (one problem per
// workgroup, looked up in a table) run the same code.
#pragma once

#include "fl_internal.h"

namespace fl_mfma {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 64;
constexpr uint32_t kKChunk = 65472;  // multiple of BK, < 65536
constexpr int kLdsRow = BK + 16;     // padded LDS row (bytes) against bank conflicts
constexpr int kOutLd = BN + 4;       // u16 row stride of the epilogue tile (8-byte aligned rows)
constexpr uint32_t kStages = 4;                 // operand ring depth (K steps)
constexpr uint32_t kPlaneBytes = BM * BK;       // one plane tile: 128 rows x 64 bytes
constexpr uint32_t kStageBytes = 4 * kPlaneBytes;
constexpr int kGemmLds = kStages * kStageBytes;  // bytes of LDS of one GEMM tile
constexpr int kRank64Ld = 128 + 4;          // u16 row stride of the rank-k residue tile

// The residue of S = 65536 S_hh + 256 S_mid + S_ll mod p from the three int32
// limb sums, in double precision (full-rate FP64 on the vector units,
// against four quarter-rate 32-bit multiplies per Barrett reduction):
//   t = 256 S_hh + S_mid and S = 256 t + S_ll are exact fused multiply-adds
//   (|S| < 2^47 for sums of at most kKChunk terms);
//   q = floor(S * (1/p)) is within 1 of floor(S / p), because the relative
//   error of the product is below 2^-50 and |S / p| < 2^46;
//   r = S - q p is exact (an integer below 2^53), lies in [-p, 2p), and two
//   conditional corrections bring it into [0, p).
struct LimbCombine {
    double pd, inv;
    int p;
};
__device__ __forceinline__ LimbCombine limb_combine(const fl::Mod &md) {
    LimbCombine c;
    c.p = (int)md.p;
    c.pd = (double)md.p;
    c.inv = 1.0 / c.pd;
    return c;
}
__device__ __forceinline__ uint32_t combine_limbs(const LimbCombine &c, int hh, int mid, int ll) {
    const double t = __builtin_fma((double)hh, 256.0, (double)mid);
    const double S = __builtin_fma(t, 256.0, (double)ll);
    const double q = __builtin_floor(S * c.inv);
    int r = (int)__builtin_fma(-q, c.pd, S);
    r += r < 0 ? c.p : 0;
    r -= r >= c.p ? c.p : 0;
    return (uint32_t)r;
}

// bias: the smallest multiple of p that is >= 2^31, so s + bias >= 0 and
// s + bias < 2^32 for |s| < 2^31 - 2^16.
inline uint32_t gemm_bias(uint32_t p) { return (uint32_t)((((uint64_t)1 << 31) + p - 1) / p * p); }
inline uint32_t gemm_c16(uint32_t p) { return (uint32_t)((1u << 16) % p); }

// 256 threads = 4 waves in a 2 x 2 arrangement, 64 x 64 outputs per wave as
// 4 x 4 tiles of 16 x 16.  The next K-tile is loaded into registers while
// the current one is multiplied, so global latency overlaps the MFMAs.
__device__ __forceinline__ void mfma_gemm_tile(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                               const GemmPlanes &g, uint32_t bx, uint32_t by,
                                               int8_t *smem) {
    static_assert(BM * kOutLd * 2 <= kGemmLds, "epilogue tile must fit the operand buffers");
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t wm = wave >> 1, wn = wave & 1;
    const uint32_t m0 = by * BM, n0 = bx * BN;
    // C row of each tile row (0xffffffff: past M or unmapped), read by the
    // epilogue after its barrier
    __shared__ uint32_t rows_s[BM];
    if (tid < BM) {
        const uint32_t row = m0 + tid;
        rows_s[tid] = row < g.M ? (g.row_map ? g.row_map[row] : row) : 0xffffffffu;
    }
    uint32_t kbeg = g.kbeg, kend = g.kend;
    if (g.krange) {
        kbeg = g.krange[2 * by];
        kend = g.krange[2 * by + 1];
    }
    if (g.krange_n) {  // per column block: intersect
        const uint32_t b = g.krange_n[2 * bx], e = g.krange_n[2 * bx + 1];
        kbeg = b > kbeg ? b : kbeg;
        kend = e < kend ? e : kend;
    }
    if (g.klen_dev) {
        const uint32_t kd = (*g.klen_dev + BK - 1) / BK * BK;
        if (kend > kd) kend = kd;
    }
    v4i acc_hh[4][4], acc_mid[4][4], acc_ll[4][4];
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            acc_hh[i][j] = v4i{0, 0, 0, 0};
            acc_mid[i][j] = v4i{0, 0, 0, 0};
            acc_ll[i][j] = v4i{0, 0, 0, 0};
        }
    // Operand pipeline: the four plane tiles of a K step (128 rows x 64 bytes
    // each) are copied global -> LDS by the DMA path (global_load_lds, no
    // registers involved) into a ring of kStages slots, issued kStages - 1
    // steps ahead, so HBM latency is covered by several steps of MFMA work.
    // A wave's DMA instruction fills a 1 KiB block (16 rows x 4 chunks of 16
    // bytes, lane L -> row L / 4, slot L % 4); chunk c of row r sits in slot
    // c ^ ((r >> 2) & 3) so that the 16-row reads below hit all LDS banks.
    const uint32_t ring = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) int8_t *)smem;
    const uint32_t lrow = lane >> 2, lslot = lane & 3;
    uint64_t goff[8];      // per DMA instruction of this wave: plane row offset + chunk
    const int8_t *gbase[8];
    uint32_t loff[8];      // LDS offset of the instruction's block within a slot
#pragma unroll
    for (int i = 0; i < 8; i++) {
        const uint32_t plane = i >> 1, rb = wave * 2 + (i & 1);
        const uint32_t r = rb * 16 + lrow;
        const uint32_t c = lslot ^ ((r >> 2) & 3);
        const bool isA = plane < 2;
        gbase[i] = plane == 0 ? g.Ah : plane == 1 ? g.Al : plane == 2 ? g.Bh : g.Bl;
        goff[i] = isA ? (uint64_t)(m0 + r) * g.lda + g.a_k0 + c * 16 : (uint64_t)(n0 + r) * g.ldb + g.b_k0 + c * 16;
        loff[i] = plane * kPlaneBytes + rb * 1024;
    }
    // one K step into ring slot `slot` (steps past kend re-read the last valid
    // step, so every step issues the same 8 instructions per wave)
    auto issue = [&](uint32_t k0, uint32_t slot) {
        const uint32_t kk = k0 < kend ? k0 : kend - BK;
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int8_t *src = gbase[i] + goff[i] + kk;
            const uint32_t dst = __builtin_amdgcn_readfirstlane(ring + slot * kStageBytes + loff[i]);
            asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(dst), "v"(src) : "memory");
        }
    };
    if (kbeg < kend) {
#pragma unroll
        for (uint32_t s = 0; s + 1 < kStages; s++) issue(kbeg + s * BK, s);
    }
    uint32_t slot = 0;
    for (uint32_t k0 = kbeg; k0 < kend; k0 += BK) {
        // this step's slot is complete when at most the (kStages - 2) later
        // steps' instructions are outstanding; the barrier extends that to
        // every wave's instructions and retires the reads of the slot
        // refilled next
        asm volatile("s_waitcnt vmcnt(%0)" ::"n"((kStages - 2) * 8) : "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        issue(k0 + (kStages - 1) * BK, slot == 0 ? kStages - 1 : slot - 1);
        const int8_t *st = smem + slot * kStageBytes;
        v4i ah[4], al[4], bh[4], bl[4];
        const uint32_t kc = lane >> 4;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const uint32_t ra = wm * 64 + t * 16 + (lane & 15);
            const uint32_t rb = wn * 64 + t * 16 + (lane & 15);
            const uint32_t oa = ra * 64 + ((kc ^ ((ra >> 2) & 3)) << 4);
            const uint32_t ob = rb * 64 + ((kc ^ ((rb >> 2) & 3)) << 4);
            ah[t] = *(const v4i *)(st + oa);
            al[t] = *(const v4i *)(st + kPlaneBytes + oa);
            bh[t] = *(const v4i *)(st + 2 * kPlaneBytes + ob);
            bl[t] = *(const v4i *)(st + 3 * kPlaneBytes + ob);
        }
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int j = 0; j < 4; j++) {
                acc_hh[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[i], bh[j], acc_hh[i][j], 0, 0, 0);
                acc_mid[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[i], bl[j], acc_mid[i][j], 0, 0, 0);
                acc_mid[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[i], bh[j], acc_mid[i][j], 0, 0, 0);
                acc_ll[i][j] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[i], bl[j], acc_ll[i][j], 0, 0, 0);
            }
        slot = slot + 1 == kStages ? 0 : slot + 1;
    }
    // drain the DMA path before the ring is reused for the output tile
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (kbeg >= kend) return;  // nothing to subtract
    // the C tile (128 rows x 32 chunks of 4 columns, 16 chunks per thread) is
    // loaded before the residues are formed, so its latency overlaps that
    // work; every load is issued (chunks outside the tile read C[0])
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    typedef __attribute__((address_space(1))) uint64_t gu64w;
    uint64_t cvals[16];
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const uint32_t ch = tid + u * 256, r = ch / (BN / 4), c4 = (ch % (BN / 4)) * 4;
        const uint32_t orow = rows_s[r], col = n0 + c4;
        const bool ok = orow != 0xffffffffu && col + 4 <= g.N;
        cvals[u] = *(gu64 *)(ok ? g.C + (uint64_t)orow * g.ldc + col : g.C);
    }
    // epilogue: residues of the 128 x 128 tile go through LDS (the operand
    // buffers are free now), then C is read, reduced and written back with
    // coalesced 8-byte accesses.  Output element (row 4*(lane/16) + e,
    // column lane%16) of each 16 x 16 tile is held by the wave.
    uint16_t *sOut = (uint16_t *)smem;
    const LimbCombine lc = limb_combine(md);
    (void)bias;
    (void)c16;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t col = wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t row = wm * 64 + i * 16 + (lane >> 4) * 4 + e;
                sOut[row * kOutLd + col] = (uint16_t)combine_limbs(lc, acc_hh[i][j][e], acc_mid[i][j][e], acc_ll[i][j][e]);
            }
        }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; u++) {
        const uint32_t ch = tid + u * 256, r = ch / (BN / 4), c4 = (ch % (BN / 4)) * 4;
        const uint32_t orow = rows_s[r], col = n0 + c4;
        if (orow == 0xffffffffu || col >= g.N) continue;
        uint16_t *o = g.C + (uint64_t)orow * g.ldc + col;
        const uint64_t sv = *(const uint64_t *)(sOut + r * kOutLd + c4);
        if (col + 4 <= g.N) {
            const uint64_t ov = cvals[u];
            uint64_t nv = 0;
#pragma unroll
            for (int c = 0; c < 4; c++)
                nv |= (uint64_t)fl::submod((uint32_t)(ov >> (16 * c)) & 0xffffu,
                                           (uint32_t)(sv >> (16 * c)) & 0xffffu, md.p) << (16 * c);
            *(gu64w *)o = nv;
        } else {
            for (uint32_t c = 0; col + c < g.N; c++)
                o[c] = (uint16_t)fl::submod(o[c], (uint32_t)(sv >> (16 * c)) & 0xffffu, md.p);
        }
    }
}

// Rank-k update, k <= 64 KS (Gauss-Jordan panel and block updates, TRSM near
// updates): KS
// MFMA K-steps, so the kernel is bound by the read-modify-write of C and its
// epilogue.  A block owns 64 rows x 128 columns; rows are taken through an
// optional row list (row_map, M rows: only rows with nonzero multipliers),
// the C tile is loaded first with row-contiguous 8-byte accesses (latency
// overlapping the operand loads and MFMAs), residues are staged through LDS
// and C is written back with 8-byte accesses.  A planes are indexed by the C
// row (lda bytes per row), B planes by the C column (ldb bytes per column).
// With K <= 64, |S_hh|, |S_ll| <= 2^20 and |S_mid| <= 2^21, so
// 256 S_mid + S_ll fits 32 bits and the recombination needs three Barrett
// reductions; with K <= 384 the three sums are reduced separately.
// One 64-row x 128-column tile (row block by, column block bx) of the
// update.  sv: kRank64Ld * 64 u16, rows_s: 64 u32 in LDS.  Callers looping
// over row blocks must synchronise between tiles.
// The row block's part of a rank-k tile: its row list entries (rows_s, LDS)
// and its A fragments, kept in registers for any number of column tiles.
// A row block of RT x 64 rows: wave w holds the A fragments (both limb
// planes, K = 64 KS) of its RT row tiles of 16, rows (w RT + rt) 16 + [0, 16).
template <int KS, int RT = 1> struct RankkRows {
    v4i ah[RT][KS], al[RT][KS];
};

template <int KS, int RT = 1>
__device__ __forceinline__ void rankk_rows(const int8_t *__restrict__ Ah, const int8_t *__restrict__ Al,
                                           uint32_t lda, const uint32_t *__restrict__ row_map, uint32_t M,
                                           uint32_t by, uint32_t *rows_s, RankkRows<KS, RT> &R) {
    static_assert(KS >= 1 && KS <= 6, "K up to 384");
    static_assert(RT == 1 || RT == 2, "16 or 32 rows per wave");
    typedef __attribute__((address_space(1))) const v4i gv4i;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t m0 = by * 64 * RT;
    if (tid < 64 * RT) rows_s[tid] = (m0 + tid < M) ? (row_map ? row_map[m0 + tid] : m0 + tid) : 0xffffffffu;
    __syncthreads();
    const uint32_t cl = lane & 15, kq = (lane >> 4) * 16;
#pragma unroll
    for (int rt = 0; rt < RT; rt++) {
        const uint32_t arow = rows_s[(wave * RT + rt) * 16 + cl];
        const uint32_t ar = arow != 0xffffffffu ? arow : rows_s[0];  // row m0 exists
#pragma unroll
        for (int s = 0; s < KS; s++) {
            R.ah[rt][s] = *(gv4i *)(Ah + (uint64_t)ar * lda + s * 64 + kq);
            R.al[rt][s] = *(gv4i *)(Al + (uint64_t)ar * lda + s * 64 + kq);
        }
        if (arow == 0xffffffffu) {
#pragma unroll
            for (int s = 0; s < KS; s++) R.ah[rt][s] = R.al[rt][s] = v4i{0, 0, 0, 0};
        }
    }
}

// One column tile bx (16 NJ columns, NJ = 8 or 4) of the row block set up by
// rankk_rows (sv: 64 RT rows of kRank64Ld residues).  Callers looping over column tiles must
// synchronise between tiles (sv is reused).  Each B fragment feeds the RT
// row tiles of the wave.
template <int KS, int RT = 1, int NJ = 8>
__device__ __forceinline__ void rankk_cols(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                           const RankkRows<KS, RT> &R, const int8_t *__restrict__ Bh,
                                           const int8_t *__restrict__ Bl, uint32_t ldb, uint16_t *C, uint64_t ldc,
                                           uint32_t N, uint32_t bx, uint16_t *sv, const uint32_t *rows_s) {
    // every operand lives in device memory: global (not flat) accesses, so
    // that loads are counted apart from LDS traffic and can stay in flight
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    typedef __attribute__((address_space(1))) uint64_t gu64w;
    typedef __attribute__((address_space(1))) const v4i gv4i;
    constexpr int kLd = kRank64Ld;
    static_assert(NJ == 8 || NJ == 4, "128 or 64 columns per tile");
    constexpr int kCpr = 4 * NJ;        // C chunks of 4 columns per row
    constexpr int kChunks = NJ * RT;    // C chunks per thread
    (void)c16;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t n0 = bx * 16 * NJ;
    // C tile: 64 RT rows x kCpr chunks of 4 columns; every load is issued
    // (chunks outside the tile read C[0])
    uint64_t cv[kChunks];
#pragma unroll
    for (int u = 0; u < kChunks; u++) {
        const uint32_t ch = tid + u * 256, r = ch / kCpr, c4 = (ch % kCpr) * 4;
        const uint32_t row = rows_s[r], col = n0 + c4;
        const bool ok = row != 0xffffffffu && col + 4 <= N;
        cv[u] = *(gu64 *)(ok ? C + (uint64_t)row * ldc + col : C);
    }
    const uint32_t rq = (lane >> 4) * 4, cl = lane & 15, kq = (lane >> 4) * 16;
    // B fragments of column tile j + 1 are fetched while tile j is multiplied
    v4i bh[2][KS], bl[2][KS];
#pragma unroll
    for (int s = 0; s < KS; s++) {
        const uint64_t b = (uint64_t)(n0 + cl) * ldb + s * 64 + kq;
        bh[0][s] = *(gv4i *)(Bh + b);
        bl[0][s] = *(gv4i *)(Bl + b);
    }
    const LimbCombine lc = limb_combine(md);
    (void)bias;
#pragma unroll
    for (int j = 0; j < NJ; j++) {
        const int cur = j & 1, nxt = cur ^ 1;
        if (j + 1 < NJ) {
#pragma unroll
            for (int s = 0; s < KS; s++) {
                const uint64_t b = (uint64_t)(n0 + (j + 1) * 16 + cl) * ldb + s * 64 + kq;
                bh[nxt][s] = *(gv4i *)(Bh + b);
                bl[nxt][s] = *(gv4i *)(Bl + b);
            }
        }
        v4i hh[RT], mid[RT], ll[RT];
#pragma unroll
        for (int rt = 0; rt < RT; rt++) hh[rt] = mid[rt] = ll[rt] = v4i{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; s++)
#pragma unroll
            for (int rt = 0; rt < RT; rt++) {
                hh[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(R.ah[rt][s], bh[cur][s], hh[rt], 0, 0, 0);
                mid[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(R.ah[rt][s], bl[cur][s], mid[rt], 0, 0, 0);
                mid[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(R.al[rt][s], bh[cur][s], mid[rt], 0, 0, 0);
                ll[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(R.al[rt][s], bl[cur][s], ll[rt], 0, 0, 0);
            }
#pragma unroll
        for (int rt = 0; rt < RT; rt++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t v = combine_limbs(lc, hh[rt][e], mid[rt][e], ll[rt][e]);
                sv[((wave * RT + rt) * 16 + rq + e) * kLd + j * 16 + cl] = (uint16_t)v;
            }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kChunks; u++) {
        const uint32_t ch = tid + u * 256, r = ch / kCpr, c4 = (ch % kCpr) * 4;
        const uint32_t row = rows_s[r], col = n0 + c4;
        if (row == 0xffffffffu || col >= N) continue;
        const uint64_t s4 = *(const uint64_t *)(sv + r * kLd + c4);
        uint16_t *o = C + (uint64_t)row * ldc + col;
        if (col + 4 <= N) {
            uint64_t nv = 0;
#pragma unroll
            for (int c = 0; c < 4; c++)
                nv |= (uint64_t)fl::submod((uint32_t)(cv[u] >> (16 * c)) & 0xffffu,
                                           (uint32_t)(s4 >> (16 * c)) & 0xffffu, md.p) << (16 * c);
            *(gu64w *)o = nv;
        } else {
            for (uint32_t c = 0; col + c < N; c++)
                o[c] = (uint16_t)fl::submod(o[c], (uint32_t)(s4 >> (16 * c)) & 0xffffu, md.p);
        }
    }
}


template <int KS, int NJ = 8>
__device__ __forceinline__ void mfma_rankk_tile(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                                const int8_t *__restrict__ Ah, const int8_t *__restrict__ Al,
                                                uint32_t lda, const int8_t *__restrict__ Bh,
                                                const int8_t *__restrict__ Bl, uint32_t ldb,
                                                const uint32_t *__restrict__ row_map, uint32_t M, uint16_t *C,
                                                uint64_t ldc, uint32_t N, uint32_t bx, uint32_t by, uint16_t *sv,
                                                uint32_t *rows_s) {
    RankkRows<KS> R;
    rankk_rows<KS>(Ah, Al, lda, row_map, M, by, rows_s, R);
    rankk_cols<KS, 1, NJ>(md, bias, c16, R, Bh, Bl, ldb, C, ldc, N, bx, sv, rows_s);
}

// K <= 64 with 64-byte A rows and B columns.
__device__ __forceinline__ void mfma_rank64_tile(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                                 const int8_t *__restrict__ Ah,
                                                 const int8_t *__restrict__ Al,
                                                 const int8_t *__restrict__ Bh,
                                                 const int8_t *__restrict__ Bl,
                                                 const uint32_t *__restrict__ row_map, uint32_t M,
                                                 uint16_t *C, uint64_t ldc, uint32_t N, uint32_t bx,
                                                 uint32_t by, uint16_t *sv, uint32_t *rows_s) {
    mfma_rankk_tile<1>(md, bias, c16, Ah, Al, 64, Bh, Bl, 64, row_map, M, C, ldc, N, bx, by, sv, rows_s);
}

}  // namespace fl_mfma
