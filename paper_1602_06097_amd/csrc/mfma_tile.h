// mfma_tile.h -- the int8-limb MFMA tiles shared by the GEMM kernels.
//
// Every residue x in [0, p), p <= 65521, is centred into
//     r = x            if x <= 32639
//     r = x - p        otherwise            (r in [-32881, 32639])
// and split into two signed 8-bit limbs r = 256 h + l with
//     h = floor((r + 128) / 256) in [-128, 127],  l = r - 256 h in [-128, 127].
// (For p < 256 the symmetric residue in [-127, 127] is the single limb l and
// h = 0: the GEMM tile then runs only the S_ll product, one int8 GEMM.)
// Then  sum_k A B = 65536 S_hh + 256 (S_hl + S_lh) + S_ll  with four int8 GEMMs
// accumulated exactly in int32 (v_mfma_i32_16x16x64_i8).  Per K term
// |h h'|, |l l'| <= 2^14 and |h l' + l h'| <= 32512 (the largest pair sum of
// two limb pairs of the window above, at r = -32641 = 256 (-128) + 127), so a
// K-chunk of at most kKChunk = 65472 terms keeps |S_hh|, |S_ll| < 2^30 and the
// shared middle accumulator |S_mid| <= 65472 * 32512 < 2^31.  A tile whose K
// range is longer folds its accumulators every kKChunk terms: the residue of
// the chunk's sum goes into S_ll (it has 2^20 of headroom) and S_hh, S_mid
// restart at zero.  The three partials are combined and reduced mod p with
// 32-bit integer operations only (combine_limbs).
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
constexpr int kOutLd = BN + 4;       // u16 row stride of the epilogue tile (8-byte aligned rows)
constexpr uint32_t kPairRow = 2 * BK;                // bytes of a plane row in a ring slot (two K steps)
constexpr uint32_t kPairPlane = BM * kPairRow;       // one plane tile of a slot: 128 rows x 128 bytes
constexpr uint32_t kPairBytes = 4 * kPairPlane;      // one ring slot: the four plane tiles
constexpr int kGemmLds = 2 * kPairBytes;             // bytes of LDS of one GEMM tile (two slots)
constexpr int kRank64Ld = 128 + 4;          // u16 row stride of the rank-k residue tile

// The residue of S = 65536 S_hh + 256 S_mid + S_ll mod p from the three int32
// limb sums (|S_hh| < 2^30, |S_mid| < 2^31, |S_ll| < 2^30 + 2^16), in 32-bit
// integer arithmetic:
//   carry the low byte of S_ll into S_mid and the low byte of that into S_hh,
//     m1 = S_mid + (S_ll >> 8),  h1 = S_hh + (m1 >> 8)      (arithmetic shifts:
//     |m1| < 2^31 - 2^23, |h1| < 2^30 + 2^23),
//   so that S = 65536 h1 + L with L = 256 (m1 & 255) + (S_ll & 255) in [0, 2^16);
//   r1 = (h1 + bias) mod p, bias the smallest multiple of p >= 2^31 (so
//   h1 + bias lies in [0, 2^32));
//   S = r1 c16 + L (mod p) with c16 = 2^16 mod p, and r1 c16 + L <=
//   (p - 1)^2 + 2^16 - 1 < 2^32, so one more reduction gives the residue.
// Both reductions are fl::reduce32 (Barrett, exact for every 32-bit value).
struct LimbCombine {
    fl::Mod md;
    uint32_t bias, c16;
};
__device__ __forceinline__ LimbCombine limb_combine(const fl::Mod &md, uint32_t bias, uint32_t c16) {
    LimbCombine c;
    c.md = md;
    c.bias = bias;
    c.c16 = c16;
    return c;
}
__device__ __forceinline__ uint32_t combine_limbs(const LimbCombine &c, int hh, int mid, int ll) {
    const int m1 = mid + (ll >> 8);
    const int h1 = hh + (m1 >> 8);
    const uint32_t L = (((uint32_t)m1 & 255u) << 8) | ((uint32_t)ll & 255u);
    const uint32_t r1 = fl::reduce32((uint32_t)h1 + c.bias, c.md);
    return fl::reduce32(r1 * c.c16 + L, c.md);
}
// reduce32 for p >= 256: the quotient estimate floor(x mu / 2^32) <= x / p
// is below 2^24, so q p is the full-rate 24-bit product.
__device__ __forceinline__ uint32_t reduce32_q24(uint32_t x, const fl::Mod &m) {
    const uint32_t q = __umulhi(x, m.mu);
    const uint32_t r = x - __umul24(q, m.p);
    return r >= m.p ? r - m.p : r;
}
// combine_limbs for p >= 256 (two limbs), with full-rate 24-bit products
// only: r1 < p and c16 < p are below 2^16.
__device__ __forceinline__ uint32_t combine_limbs_2(const LimbCombine &c, int hh, int mid, int ll) {
    const int m1 = mid + (ll >> 8);
    const int h1 = hh + (m1 >> 8);
    const uint32_t L = (((uint32_t)m1 & 255u) << 8) | ((uint32_t)ll & 255u);
    const uint32_t r1 = reduce32_q24((uint32_t)h1 + c.bias, c.md);
    return reduce32_q24(__umul24(r1, c.c16) + L, c.md);
}
// The residue of a single-limb sum S_ll (p < 256, |S_ll| < 2^30: at most
// kKChunk products of two limbs in [-127, 127], plus a folded residue):
// S_ll + bias lies in [0, 2^32).
__device__ __forceinline__ uint32_t combine_limbs_1(const LimbCombine &c, int ll) {
    return fl::reduce32((uint32_t)ll + c.bias, c.md);
}
// The GEMM tile's combine: ONE = single-limb operands (p < 256); BIG =
// p >= 256 is known; otherwise any p.
template <bool ONE, bool BIG>
__device__ __forceinline__ uint32_t combine_limbs_t(const LimbCombine &c, int hh, int mid, int ll) {
    if constexpr (ONE) {
        (void)hh;
        (void)mid;
        return combine_limbs_1(c, ll);
    } else if constexpr (BIG) {
        return combine_limbs_2(c, hh, mid, ll);
    } else {
        return combine_limbs(c, hh, mid, ll);
    }
}

// bias: the smallest multiple of p that is >= 2^31 (combine_limbs);
// c16 = 2^16 mod p.
inline uint32_t gemm_bias(uint32_t p) { return (uint32_t)((((uint64_t)1 << 31) + p - 1) / p * p); }
inline uint32_t gemm_c16(uint32_t p) { return (uint32_t)((1u << 16) % p); }

// One 128 x 128 output tile per workgroup of kGemmThreads = 512 threads: 8
// waves in a 2 x 4 arrangement, 64 x 32 outputs per wave as 4 x 2 tiles of
// 16 x 16 (three int32 accumulators each: 96 registers), so two waves share
// each SIMD and one wave's MFMAs cover the other's waits.
constexpr int kGemmThreads = 512;
// The epilogue stages the residues of half a tile (64 rows) at a time.
constexpr int kGemmOutBytes = (BM / 2) * kOutLd * 2;
// LDS of the persistent GEMM kernel: the operand ring and, beside it, the
// epilogue's staging area, so that the next tile's operands can be fetched
// while the current tile is written back.
constexpr int kGemmLdsP = kGemmLds + kGemmOutBytes;

// The K range [kbeg, kend) of tile (bx, by) of g (empty when kbeg >= kend).
__device__ __forceinline__ void gemm_tile_krange(const GemmPlanes &g, uint32_t bx, uint32_t by, uint32_t &kbeg,
                                                 uint32_t &kend) {
    kbeg = g.kbeg;
    kend = g.kend;
    if (g.krange) {  // per row block: intersect
        const uint32_t b = g.krange[2 * by], e = g.krange[2 * by + 1];
        kbeg = b > kbeg ? b : kbeg;
        kend = e < kend ? e : kend;
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
    if (g.kcap_n) {  // rows of B past the column tile's last nonzero row: zero
        const uint32_t cap = g.kcap_n[bx];
        const uint32_t rel = cap > g.b_k0 ? (cap - g.b_k0 + BK - 1) / BK * BK : 0u;
        // (a cap that would leave less than one K step keeps the range)
        if (rel < kend && (rel <= kbeg || rel - kbeg >= BK)) kend = rel;
    }
}

// C row of row r of the row tile starting at m0 (0xffffffff: past M).
__device__ __forceinline__ uint32_t gemm_tile_row(const GemmPlanes &g, uint32_t m0, uint32_t r) {
    const uint32_t row = m0 + r;
    return row < g.M ? (g.row_map ? g.row_map[row] : row) : 0xffffffffu;
}

// Operand pipeline: K steps are fetched in pairs, so that every row of a
// plane tile is read as one whole 128-byte line (two 64-byte steps).  A
// ring of two slots holds pairs of the four plane tiles (128 rows x 128
// bytes each), copied global -> LDS by the DMA path (global_load_lds, no
// registers involved).  Wave w fills rows 64 (w & 1) .. + 63 of plane
// w / 2, 8 rows per instruction (lane L -> row L / 8, slot L % 8); global
// chunk c (16 bytes) of row r sits in slot c ^ swz(r), swz(r) =
// ((r >> 1) & 7) ^ (4 (r & 1)), so that the 16-row fragment reads below
// hit distinct banks for both 128- and 256-byte LDS cycles.  A pair whose
// second step lies past kend fetches its first step twice (chunks 4..7
// repeat 0..3), so no fetch leaves [kbeg, kend).
__device__ __forceinline__ uint32_t gemm_swz(uint32_t r) { return ((r >> 1) & 7u) ^ ((r & 1u) << 2); }

template <bool ONE> struct GemmFeed {
    const int8_t *src;   // the lane's first source byte of a pair at K offset 0
    uint64_t pld;        // bytes per plane row
    uint32_t ring;       // LDS address of the ring
    uint32_t plane;      // plane filled by this wave: Ah, Al, Bh, Bl
    uint32_t wrow;       // first tile row of this wave
    uint32_t lchunk;     // the lane's chunk slot (even instructions)
    uint32_t kend, last_pair;

    // (fields selected with masks: a select among the kernel argument's
    // fields by a runtime index would be compiled into a private-memory table)
    __device__ __forceinline__ void init(const GemmPlanes &g, uint32_t m0, uint32_t n0, uint32_t kbeg,
                                         uint32_t kend_, const int8_t *smem, uint32_t wave, uint32_t lane) {
        ring = (uint32_t)(uintptr_t)(__attribute__((address_space(3))) const int8_t *)smem;
        plane = wave >> 1;
        wrow = (wave & 1) * 64;
        const uint64_t m_a = plane < 2 ? ~0ull : 0ull;
        pld = (g.lda & m_a) | (g.ldb & ~m_a);
        const uint64_t poff = (uint64_t)(((uint64_t)m0 & m_a) | ((uint64_t)n0 & ~m_a)) * pld +
                              (((uint64_t)g.a_k0 & m_a) | ((uint64_t)g.b_k0 & ~m_a));
        const uint64_t m_lo = (plane & 1) ? 0ull : ~0ull;
        const uint64_t p_a = ((uint64_t)(uintptr_t)g.Ah & m_lo) | ((uint64_t)(uintptr_t)g.Al & ~m_lo);
        const uint64_t p_b = ((uint64_t)(uintptr_t)g.Bh & m_lo) | ((uint64_t)(uintptr_t)g.Bl & ~m_lo);
        // the lane's row of instruction 0 and its chunk there; instruction i
        // is 8 i rows further down, where swz differs by 4 (i odd)
        const uint32_t lrow = wrow + (lane >> 3);
        lchunk = (lane & 7) ^ gemm_swz(lrow);
        src = (const int8_t *)(uintptr_t)(((p_a & m_a) | (p_b & ~m_a)) + poff) + (uint64_t)lrow * pld;
        kend = kend_;
        last_pair = kbeg + (kend_ > kbeg ? (kend_ - kbeg - 1) / (2 * BK) * (2 * BK) : 0);
    }
    // pair starting at K offset ks (past the range: the last pair, fetched
    // again, so every pair issues the same 8 instructions per wave) into
    // slot `slot`
    __device__ __forceinline__ void issue(uint32_t ks, uint32_t slot) const {
        if (ONE && !(plane & 1)) return;  // an h plane: all zero
        const uint32_t kk = ks < kend ? ks : last_pair;
        const uint32_t cmask = kk + 2 * BK <= kend ? 7u : 3u;
        const int8_t *src_e = src + kk + ((lchunk & cmask) << 4);        // even i
        const int8_t *src_o = src + kk + (((lchunk ^ 4u) & cmask) << 4);  // odd i
#pragma unroll
        for (int i = 0; i < 8; i++) {
            const int8_t *s = ((i & 1) ? src_o : src_e) + (uint64_t)(i * 8) * pld;
            const uint32_t dst = __builtin_amdgcn_readfirstlane(ring + slot * kPairBytes + plane * kPairPlane +
                                                                (wrow + i * 8) * kPairRow);
            asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, off" ::"s"(dst), "v"(s) : "memory");
        }
    }
};

struct GemmAcc {
    v4i hh[4][2], mid[4][2], ll[4][2];
};

// The products of one tile over [kbeg, kend) (kbeg < kend) into a (zeroed
// here).  On entry the tile's first two pairs have been issued by f into
// slots 0 and 1 (other memory operations may follow them); on return every
// fetch of the ring has landed and the workgroup has passed a barrier, so
// the ring may be refilled.
//
// Step j is half j & 1 of pair j / 2 (slot (j / 2) & 1).  Its fragments
// are read during step j - 1 (into the second register set, copied over
// after the MFMAs), so the LDS reads overlap the MFMAs.  At an odd step
// the next step opens a new pair: the wave waits for that pair's fetch
// (issued two steps earlier) and for its own LDS reads; after the barrier
// nobody reads the pair just finished, and its slot is refilled with the
// pair after the next.  Even steps need no barrier.
template <bool ONE, bool BIG>
__device__ __forceinline__ void gemm_mainloop(const GemmFeed<ONE> &f, uint32_t kbeg, uint32_t kend,
                                              const int8_t *smem, const LimbCombine &lc, uint32_t wave,
                                              uint32_t lane, GemmAcc &a) {
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 2; j++) {
            a.hh[i][j] = v4i{0, 0, 0, 0};
            a.mid[i][j] = v4i{0, 0, 0, 0};
            a.ll[i][j] = v4i{0, 0, 0, 0};
        }
    const uint32_t wm = wave >> 2, wn = wave & 3;
    // The wave's fragments of a step (half h of the pair in slot `slot`): A
    // row tiles (4 of 16 rows) and B column tiles (2 of 16 columns), both
    // limb planes, 16 bytes of K per lane.
    const uint32_t kc = lane >> 4;
    auto read_ops = [&](uint32_t slot, uint32_t h, v4i (&ah)[4], v4i (&al)[4], v4i (&bh)[2], v4i (&bl)[2]) {
        const int8_t *st = smem + slot * kPairBytes;
        const uint32_t gc = h * 4 + kc;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const uint32_t ra = wm * 64 + t * 16 + (lane & 15);
            const uint32_t oa = ra * kPairRow + ((gc ^ gemm_swz(ra)) << 4);
            if (!ONE) ah[t] = *(const v4i *)(st + oa);
            al[t] = *(const v4i *)(st + kPairPlane + oa);
        }
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const uint32_t rb = wn * 32 + t * 16 + (lane & 15);
            const uint32_t ob = rb * kPairRow + ((gc ^ gemm_swz(rb)) << 4);
            if (!ONE) bh[t] = *(const v4i *)(st + 2 * kPairPlane + ob);
            bl[t] = *(const v4i *)(st + 3 * kPairPlane + ob);
        }
    };
    v4i ah[4], al[4], bh[2], bl[2], nah[4], nal[4], nbh[2], nbl[2];
    uint32_t left = kKChunk / BK;  // K steps before the accumulators are folded
    asm volatile("s_waitcnt vmcnt(8)" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    read_ops(0, 0, ah, al, bh, bl);
    // (a wait the compiler sees: the loop's MFMAs then never wait for the
    // next step's LDS reads, issued just before them)
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    uint32_t j = 0;
    for (uint32_t k0 = kbeg; k0 < kend; k0 += BK, j++) {
        const bool more = k0 + BK < kend;
        if (j & 1) {
            const uint32_t q = (j + 1) >> 1;  // the pair of step j + 1
            asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
            __builtin_amdgcn_s_barrier();
            asm volatile("" ::: "memory");
            f.issue(kbeg + (q + 1) * 2 * BK, (q + 1) & 1);
            read_ops(q & 1, 0, nah, nal, nbh, nbl);  // (past the range: stale, unused)
        } else {
            read_ops((j >> 1) & 1, 1, nah, nal, nbh, nbl);
        }
        __builtin_amdgcn_sched_barrier(0);  // the reads go out before the MFMAs
#pragma unroll
        for (int i = 0; i < 4; i++)
#pragma unroll
            for (int jj = 0; jj < 2; jj++) {
                if (!ONE) {
                    a.hh[i][jj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[i], bh[jj], a.hh[i][jj], 0, 0, 0);
                    a.mid[i][jj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[i], bl[jj], a.mid[i][jj], 0, 0, 0);
                    a.mid[i][jj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[i], bh[jj], a.mid[i][jj], 0, 0, 0);
                }
                a.ll[i][jj] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[i], bl[jj], a.ll[i][jj], 0, 0, 0);
            }
        if (--left == 0 && more) {  // a K range longer than kKChunk: fold
            left = kKChunk / BK;
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int jj = 0; jj < 2; jj++)
#pragma unroll
                    for (int e = 0; e < 4; e++) {
                        a.ll[i][jj][e] =
                            (int)combine_limbs_t<ONE, BIG>(lc, a.hh[i][jj][e], a.mid[i][jj][e], a.ll[i][jj][e]);
                        a.hh[i][jj][e] = 0;
                        a.mid[i][jj][e] = 0;
                    }
        }
#pragma unroll
        for (int t = 0; t < 4; t++) {
            if (!ONE) ah[t] = nah[t];
            al[t] = nal[t];
        }
#pragma unroll
        for (int t = 0; t < 2; t++) {
            if (!ONE) bh[t] = nbh[t];
            bl[t] = nbl[t];
        }
    }
    // drain the DMA path before the ring is reused
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
}

// Epilogue of a tile whose products are in a: C[rows_s[r], n0 + c] -= the
// residue of the limb sums.  The C tile (128 rows x 32 chunks of 4 columns,
// 8 chunks per thread) is loaded first, so its latency overlaps the
// reduction of the sums; the residues then go through LDS (sOut: 64 rows of
// kOutLd u16, one half tile at a time) and C is reduced and written back
// with coalesced 8-byte accesses.  Output element (row 4 (lane / 16) + e,
// column lane % 16) of each 16 x 16 tile is held by the wave; the waves of
// row half h (wave / 4 = h) stage half h.  rows_s (the tile's C rows, see
// gemm_tile_row) must be visible to all threads on entry; callers reusing
// sOut or rows_s afterwards must synchronise first.
constexpr int kGemmHalf = (BM / 2) * (BN / 4) / kGemmThreads;  // C chunks per thread and half tile
struct GemmC {
    uint64_t v[2][kGemmHalf];
};

// The C tile's values (chunk u of half h: 4 entries of row h (BM / 2) + ch /
// (BN / 4), ch = tid + u kGemmThreads), with the row of tile row r given by
// row(r) (0xffffffff: past M).  Every load is issued: chunks outside the
// tile read C[0].
template <typename RowOf>
__device__ __forceinline__ void gemm_cload(const GemmPlanes &g, uint32_t n0, RowOf row, GemmC &c) {
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int h = 0; h < 2; h++)
#pragma unroll
        for (int u = 0; u < kGemmHalf; u++) {
            const uint32_t ch = tid + u * kGemmThreads, r = h * (BM / 2) + ch / (BN / 4);
            const uint32_t orow = row(r), col = n0 + (ch % (BN / 4)) * 4;
            const bool ok = orow != 0xffffffffu && col + 4 <= g.N;
            c.v[h][u] = *(gu64 *)(ok ? g.C + (uint64_t)orow * g.ldc + col : g.C);
        }
}

// PRE: the C tile was loaded by the caller (ahead of the products, into c);
// otherwise it is loaded here, from the rows in rows_s.
template <bool ONE, bool BIG, bool PRE = false>
__device__ __forceinline__ void gemm_epilogue(const fl::Mod &md, const LimbCombine &lc, const GemmPlanes &g,
                                              uint32_t n0, const uint32_t *rows_s, uint16_t *sOut, uint32_t wave,
                                              uint32_t lane, GemmAcc &a, GemmC &c) {
    typedef __attribute__((address_space(1))) uint64_t gu64w;
    const uint32_t tid = threadIdx.x, wm = wave >> 2, wn = wave & 3;
    constexpr int kHalf = kGemmHalf;
    if constexpr (!PRE) gemm_cload(g, n0, [&](uint32_t r) { return rows_s[r]; }, c);
    uint64_t(&cvals)[2][kHalf] = c.v;
    // the residues, in place of the ll sums
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 2; j++)
#pragma unroll
            for (int e = 0; e < 4; e++)
                a.ll[i][j][e] = (int)combine_limbs_t<ONE, BIG>(lc, a.hh[i][j][e], a.mid[i][j][e], a.ll[i][j][e]);
#pragma unroll
    for (int h = 0; h < 2; h++) {
        if (wm == (uint32_t)h) {
#pragma unroll
            for (int i = 0; i < 4; i++)
#pragma unroll
                for (int j = 0; j < 2; j++) {
                    const uint32_t col = wn * 32 + j * 16 + (lane & 15);
#pragma unroll
                    for (int e = 0; e < 4; e++)
                        sOut[(i * 16 + (lane >> 4) * 4 + e) * kOutLd + col] = (uint16_t)a.ll[i][j][e];
                }
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kHalf; u++) {
            const uint32_t ch = tid + u * kGemmThreads, rl = ch / (BN / 4), c4 = (ch % (BN / 4)) * 4;
            const uint32_t orow = rows_s[h * (BM / 2) + rl], col = n0 + c4;
            // (every C value is taken on every path, also where it is not
            // needed: a load left outstanding would make the compiler wait
            // for it inside the next tile's main loop, which reuses its
            // registers)
            const uint64_t ov = cvals[h][u];
            if (orow == 0xffffffffu || col >= g.N) {
                asm volatile("" ::"v"(ov));
                continue;
            }
            uint16_t *o = g.C + (uint64_t)orow * g.ldc + col;
            const uint64_t sv = *(const uint64_t *)(sOut + rl * kOutLd + c4);
            if (col + 4 <= g.N) {
                uint64_t nv = 0;
#pragma unroll
                for (int c = 0; c < 4; c++)
                    nv |= (uint64_t)fl::submod((uint32_t)(ov >> (16 * c)) & 0xffffu,
                                               (uint32_t)(sv >> (16 * c)) & 0xffffu, md.p) << (16 * c);
                *(gu64w *)o = nv;
            } else {
                asm volatile("" ::"v"(ov));
                for (uint32_t c = 0; col + c < g.N; c++)
                    o[c] = (uint16_t)fl::submod(o[c], (uint32_t)(sv >> (16 * c)) & 0xffffu, md.p);
            }
        }
        if (h == 0) __syncthreads();  // half 1 is staged in the same buffer
    }
}

// One tile (bx, by) by one workgroup, for kernels that take their tiles one
// at a time (smem: kGemmLds bytes; callers looping over tiles must
// synchronise between them).  Any p (two-limb operands unless ONE).
template <bool ONE = false>
__device__ __forceinline__ void mfma_gemm_tile(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                               const GemmPlanes &g, uint32_t bx, uint32_t by,
                                               int8_t *smem) {
    static_assert(kGemmOutBytes <= kGemmLds, "epilogue tile must fit the operand buffers");
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));  // wave-uniform
    // C row of each tile row, read by the epilogue after the main loop's barriers
    __shared__ uint32_t rows_s[BM];
    if (tid < BM) rows_s[tid] = gemm_tile_row(g, by * BM, tid);
    uint32_t kbeg, kend;
    gemm_tile_krange(g, bx, by, kbeg, kend);
    if (kbeg >= kend) {  // nothing to subtract
        __syncthreads();
        return;
    }
    const LimbCombine lc = limb_combine(md, bias, c16);
    // (a wait the compiler sees for the accesses still in flight, such as a
    // previous tile's write-back: the compiler then places no wait inside the
    // main loop, where it would also wait for the operand fetch)
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
    GemmFeed<ONE> f;
    f.init(g, by * BM, bx * BN, kbeg, kend, smem, wave, lane);
    f.issue(kbeg, 0);
    f.issue(kbeg + 2 * BK, 1);
    GemmAcc a;
    GemmC c;
    gemm_mainloop<ONE, false>(f, kbeg, kend, smem, lc, wave, lane, a);
    gemm_epilogue<ONE, false>(md, lc, g, bx * BN, rows_s, (uint16_t *)smem, wave, lane, a, c);
}

// Rank-k update, k <= 64 KS (Gauss-Jordan panel and block updates, TRSM near
// updates): only KS MFMA K-steps, so the kernel is bound by the
// read-modify-write of C, its epilogue and the latency of its operand loads.
// A tile is 64 RT rows x 16 NJ columns (RT = 1 or 2, NJ = 8 or 4); rows are
// taken through an optional row list (row_map, M rows: only rows with
// nonzero multipliers), the C tile is loaded first with row-contiguous
// 8-byte accesses (latency overlapping the operand loads and MFMAs),
// residues are staged through LDS and C is written back with 8-byte
// accesses.  A planes are indexed by the C row (lda bytes per row), B planes
// by the C column (ldb bytes per column).  The three limb sums are combined
// by combine_limbs (K <= 384, far inside its bounds).  sv: kRank64Ld * 64 RT u16, rows_s: 64 RT u32 in LDS;
// callers looping over tiles must synchronise between them.
// rankk_rows sets up the row block (its row list entries and its A
// fragments, kept in registers for any number of column tiles): wave w holds
// the A fragments (both limb planes, K = 64 KS) of its RT row tiles of 16,
// rows (w RT + rt) 16 + [0, 16).
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

// The C tile of column tile bx of a rank-k row block (64 RT rows x 16 NJ
// columns, kChunks 8-byte chunks per thread): its row numbers (from rows_s)
// and its values, loaded ahead of the tile's products (possibly while the
// previous tile is computed).
template <int RT, int NJ> struct RankkC {
    static constexpr int kChunks = NJ * RT;
    uint32_t crow[kChunks];
    uint64_t cv[kChunks];
};

template <int RT, int NJ>
__device__ __forceinline__ void rankk_cload(RankkC<RT, NJ> &T, const uint16_t *C, uint64_t ldc, uint32_t N,
                                            uint32_t bx, const uint32_t *rows_s) {
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    constexpr int kCpr = 4 * NJ;
    const uint32_t tid = threadIdx.x, n0 = bx * 16 * NJ;
    // every load is issued (chunks outside the tile read C[0]); the row
    // numbers are read from LDS first, all together, so the loads go out
    // back to back
#pragma unroll
    for (int u = 0; u < T.kChunks; u++) T.crow[u] = rows_s[(tid + u * 256) / kCpr];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < T.kChunks; u++) {
        const uint32_t ch = tid + u * 256, c4 = (ch % kCpr) * 4;
        const uint32_t row = T.crow[u], col = n0 + c4;
        const bool ok = row != 0xffffffffu && col + 4 <= N;
        T.cv[u] = *(gu64 *)(ok ? C + (uint64_t)row * ldc + col : C);
    }
}

// The products and the write-back of column tile bx (16 NJ columns, NJ = 8
// or 4) of the row block set up by rankk_rows, its C tile loaded (sv: 64 RT
// rows of kRank64Ld residues).  Callers looping over column tiles must
// synchronise between tiles (sv is reused).  Each B fragment feeds the RT
// row tiles of the wave.
template <int KS, int RT, int NJ>
__device__ __forceinline__ void rankk_cols_loaded(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                                  const RankkRows<KS, RT> &R, const int8_t *__restrict__ Bh,
                                                  const int8_t *__restrict__ Bl, uint32_t ldb, uint16_t *C,
                                                  uint64_t ldc, uint32_t N, uint32_t bx, uint16_t *sv,
                                                  const RankkC<RT, NJ> &T) {
    typedef __attribute__((address_space(1))) uint64_t gu64w;
    typedef __attribute__((address_space(1))) const v4i gv4i;
    constexpr int kLd = kRank64Ld;
    static_assert(NJ == 8 || NJ == 4, "128 or 64 columns per tile");
    constexpr int kCpr = 4 * NJ;        // C chunks of 4 columns per row
    constexpr int kChunks = NJ * RT;    // C chunks per thread
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t n0 = bx * 16 * NJ;
    const uint32_t *crow = T.crow;
    const uint64_t *cv = T.cv;
    const uint32_t rq = (lane >> 4) * 4, cl = lane & 15, kq = (lane >> 4) * 16;
    // B fragments of column tile j + 1 are fetched while tile j is multiplied
    v4i bh[2][KS], bl[2][KS];
#pragma unroll
    for (int s = 0; s < KS; s++) {
        const uint64_t b = (uint64_t)(n0 + cl) * ldb + s * 64 + kq;
        bh[0][s] = *(gv4i *)(Bh + b);
        bl[0][s] = *(gv4i *)(Bl + b);
    }
    const LimbCombine lc = limb_combine(md, bias, c16);
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
        const uint32_t row = crow[u], col = n0 + c4;
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


// One column tile bx (16 NJ columns, NJ = 8 or 4) of the row block set up by
// rankk_rows: C tile loaded, products, write-back.
template <int KS, int RT = 1, int NJ = 8>
__device__ __forceinline__ void rankk_cols(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                           const RankkRows<KS, RT> &R, const int8_t *__restrict__ Bh,
                                           const int8_t *__restrict__ Bl, uint32_t ldb, uint16_t *C, uint64_t ldc,
                                           uint32_t N, uint32_t bx, uint16_t *sv, const uint32_t *rows_s) {
    RankkC<RT, NJ> T;
    rankk_cload<RT, NJ>(T, C, ldc, N, bx, rows_s);
    rankk_cols_loaded<KS, RT, NJ>(md, bias, c16, R, Bh, Bl, ldb, C, ldc, N, bx, sv, T);
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
