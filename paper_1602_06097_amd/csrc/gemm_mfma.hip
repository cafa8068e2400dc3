// gemm_mfma.hip -- dense C = C - A B mod p on the int8 matrix cores (gfx950).
//
// The limb arithmetic and the tiles are in mfma_tile.h.  Operands are first
// converted to limb planes in the workspace, both stored K-contiguous (A as
// M x Kp, B transposed as N x Kp, zero padded to the tile sizes), so the GEMM
// kernel streams int8 rows with 16-byte loads and needs no bounds checks in
// its main loop.
#include "fl_internal.h"
#include "mfma_tile.h"

#include <cstdio>

namespace {

using namespace fl_mfma;

__device__ __forceinline__ void split_limbs(uint32_t x, uint32_t p, int &h, int &l) {
    fl_split_limbs(x, p, h, l);
}

// A (rows x K, row-major u16, lda) -> Ah, Al (Rp x Kp int8, K-contiguous).
// Rows >= rows or k >= K (K read from Kdev when non-NULL) are zero.
__global__ __launch_bounds__(256) void k_limbs_rows(uint32_t p, const uint16_t *__restrict__ A,
                                                    uint64_t lda, uint32_t rows, uint32_t Kh,
                                                    const uint32_t *__restrict__ Kdev,
                                                    int8_t *Ah, int8_t *Al, uint32_t Rp,
                                                    uint32_t Kp) {
    const uint32_t K = Kdev ? *Kdev : Kh;
    const uint32_t k4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    if (k4 >= Kp) return;
    for (uint32_t i = blockIdx.y; i < Rp; i += gridDim.y) {
        uint32_t hv = 0, lv = 0;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint32_t k = k4 + e;
            int h = 0, l = 0;
            if (i < rows && k < K) split_limbs(A[(uint64_t)i * lda + k], p, h, l);
            hv |= (uint32_t)(h & 0xff) << (8 * e);
            lv |= (uint32_t)(l & 0xff) << (8 * e);
        }
        *(uint32_t *)(Ah + (uint64_t)i * Kp + k4) = hv;
        *(uint32_t *)(Al + (uint64_t)i * Kp + k4) = lv;
    }
}

// B (K x cols, row-major u16, ldb) -> Bh, Bl transposed (Cp x Kp int8).
// One workgroup per 64 (K) x 64 (column) tile: rows are read as 8-byte
// chunks of four columns (entry by entry past cols or where B or ldb is not
// 8-byte aligned), the limbs are transposed through LDS, and each column's
// 64 K bytes are written as four 16-byte stores per plane.  Rows k >= K
// (K read from Kdev when non-NULL) and columns >= cols are zero.
__global__ __launch_bounds__(256) void k_limbs_cols(uint32_t p, const uint16_t *__restrict__ B,
                                                    uint64_t ldb, uint32_t cols, uint32_t Kh,
                                                    const uint32_t *__restrict__ Kdev,
                                                    int8_t *Bh, int8_t *Bl, uint32_t Kp, uint32_t *row_end) {
    constexpr uint32_t kLd = 80;  // LDS bytes per column (16-byte aligned rows)
    __shared__ __attribute__((aligned(16))) int8_t th[64 * kLd], tl[64 * kLd];
    const uint32_t K = Kdev ? *Kdev : Kh;
    const uint32_t k0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const uint32_t tid = threadIdx.x, cq = tid & 15, kr = tid >> 4;  // 16 chunks x 16 rows
    const bool vec = ((((uintptr_t)B) | (uintptr_t)(ldb * 2)) & 7) == 0;
    const uint32_t c = c0 + cq * 4;
    uint32_t last = 0;  // 1 + the last row k with a nonzero in these columns
#pragma unroll
    for (int i = 0; i < 4; i++) {
        const uint32_t kk = kr + 16 * i, k = k0 + kk;
        uint64_t v = 0;
        if (k < K) {
            const uint16_t *row = B + (uint64_t)k * ldb;
            if (vec && c + 4 <= cols) v = *(const uint64_t *)(row + c);
            else
                for (uint32_t e = 0; e < 4 && c + e < cols; e++) v |= (uint64_t)row[c + e] << (16 * e);
        }
        if (v) last = k + 1;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            int h, l;
            split_limbs((uint32_t)(v >> (16 * e)) & 0xffffu, p, h, l);
            th[(cq * 4 + e) * kLd + kk] = (int8_t)h;
            tl[(cq * 4 + e) * kLd + kk] = (int8_t)l;
        }
    }
    if (row_end) {  // per 128-column tile (one per two workgroups along x)
        last = fl_wave_max(last);
        if ((tid & 63) == 0 && last) atomicMax(&row_end[c0 / 128], last);
    }
    __syncthreads();
    const uint32_t cc = tid >> 2, seg = (tid & 3) * 16;
    const uint4 hv = *(const uint4 *)&th[cc * kLd + seg];
    const uint4 lv = *(const uint4 *)&tl[cc * kLd + seg];
    *(uint4 *)(Bh + (uint64_t)(c0 + cc) * Kp + k0 + seg) = hv;
    *(uint4 *)(Bl + (uint64_t)(c0 + cc) * Kp + k0 + seg) = lv;
}

// Tile `pid` of an nx x ny tile grid under GemmPlanes::group_m, in a launch
// of G workgroups (workgroup b takes the tiles pid = b + j G).  Tile
// numbers are dealt round-robin to the 8 XCDs (pid % 8: the XCD of the
// workgroup that takes it); they are renumbered so that every XCD receives a
// contiguous range, which is walked column tile by column tile in groups of
// gm row tiles.  Within an XCD, the W = G / 8 tiles of one round (j) are
// rotated by j, so that a workgroup's tiles in successive rounds lie in
// different rows of a group (row tiles can differ much in their K ranges).
// Every step is a bijection.
__device__ __forceinline__ void gemm_tile_of(uint32_t gm, uint32_t nx, uint32_t ny, uint32_t G, uint32_t pid,
                                             uint32_t &bx, uint32_t &by) {
    if (gm == 0) {
        bx = pid % nx;
        by = pid / nx;
        return;
    }
    const uint32_t total = nx * ny;
    const uint32_t q = total / 8, r = total % 8, x = pid % 8;
    uint32_t i = pid / 8;
    const uint32_t W = G / 8;
    if (W > 1) {
        const uint32_t c = i / W, qx = q + (x < r ? 1u : 0u);
        if ((c + 1) * W <= qx) i = c * W + (i % W + c) % W;
    }
    const uint32_t id = x * q + (x < r ? x : r) + i;
    const uint32_t per = gm * nx, group = id / per, first = group * gm;
    const uint32_t rows = ny - first < gm ? ny - first : gm;
    const uint32_t within = id - group * per;
    by = first + within % rows;
    bx = within / rows;
}

// A tile of the grid and its K range.
struct GemmTile {
    uint32_t t, bx, by, kbeg, kend;
};

// The first tile t + i G (i >= 0) whose K range is not empty (t = nx ny if
// none).  The tile t itself is probed alone (the usual case); past an empty
// one the lanes of the wave probe 64 tiles at once.  The result is uniform.
__device__ __forceinline__ GemmTile gemm_next_tile(const GemmPlanes &g, uint32_t nx, uint32_t ny, uint32_t t,
                                                   uint32_t G, uint32_t lane) {
    const uint32_t total = nx * ny;
    GemmTile r = {total, 0, 0, 0, 0};
    if (t >= total) return r;
    gemm_tile_of(g.group_m, nx, ny, G, t, r.bx, r.by);
    gemm_tile_krange(g, r.bx, r.by, r.kbeg, r.kend);
    if (r.kbeg < r.kend) {
        r.t = t;
        return r;
    }
    for (uint64_t t0 = (uint64_t)t + G; t0 < total; t0 += 64ull * G) {
        const uint64_t c = t0 + (uint64_t)lane * G;
        bool ne = false;
        uint32_t bx, by, kb, ke;
        if (c < total) {
            gemm_tile_of(g.group_m, nx, ny, G, (uint32_t)c, bx, by);
            gemm_tile_krange(g, bx, by, kb, ke);
            ne = kb < ke;
        }
        const uint64_t m = __ballot(ne);
        if (m) {
            const int src = __builtin_ctzll(m);
            r.t = (uint32_t)(t0 + (uint64_t)src * G);
            r.bx = (uint32_t)__builtin_amdgcn_readlane((int)bx, src);
            r.by = (uint32_t)__builtin_amdgcn_readlane((int)by, src);
            r.kbeg = (uint32_t)__builtin_amdgcn_readlane((int)kb, src);
            r.kend = (uint32_t)__builtin_amdgcn_readlane((int)ke, src);
            return r;
        }
    }
    return r;
}

// Persistent GEMM: gridDim.x workgroups (at most one per compute unit: the
// LDS of kGemmLdsP bytes) take the tiles blockIdx.x + i gridDim.x of the nx x
// ny grid that have a K range, in order.  As soon as a tile's products are
// done, the first two operand pairs of the workgroup's next tile are fetched
// into the ring, so the fetch overlaps the write-back of the tile (staged
// beside the ring).  The next tile is looked up while the current tile's
// first operands are in flight.  ONE: single-limb operands (p < 256); the
// launch takes ONE exactly when p < 256, so the two-limb form combines the
// limb sums with p >= 256.
template <bool ONE, bool PRE>
__global__ __launch_bounds__(kGemmThreads) void k_mfma_gemm(fl::Mod md, uint32_t bias, uint32_t c16,
                                                            GemmPlanes g, uint32_t nx, uint32_t ny) {
    __shared__ __attribute__((aligned(16))) int8_t smem[kGemmLdsP];
    __shared__ uint32_t rows_s[2][BM];  // C rows of the current tile and of the next one
    const uint32_t tid = threadIdx.x, lane = tid & 63;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(tid >> 6));  // wave-uniform
    const uint32_t G = gridDim.x, total = nx * ny;
    const LimbCombine lc = limb_combine(md, bias, c16);
    GemmTile cur = gemm_next_tile(g, nx, ny, blockIdx.x, G, lane);
    if (cur.t >= total) return;
    // (a tile's row numbers are read before its first fetch is issued: the
    // wait for them would otherwise wait for the fetch too)
    if (tid < BM) rows_s[0][tid] = gemm_tile_row(g, cur.by * BM, tid);
    GemmFeed<ONE> f;
    f.init(g, cur.by * BM, cur.bx * BN, cur.kbeg, cur.kend, smem, wave, lane);
    f.issue(cur.kbeg, 0);
    f.issue(cur.kbeg + 2 * BK, 1);
    GemmAcc a;
    for (uint32_t it = 0;; it++) {
        // A wait for every memory access in flight (the write-back of the
        // tile before; this tile's operands, issued before that write-back's
        // loads, have landed, except on the first tile) that the compiler
        // sees: with it, the compiler's model of the queue is empty, and it
        // places no wait inside the main loop (such a wait would also wait
        // for the operand fetch, issued by inline asm the compiler does not
        // count).
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        const GemmTile nxt = gemm_next_tile(g, nx, ny, cur.t + G, G, lane);
        const bool more = nxt.t < total;
        GemmC c;
        if constexpr (PRE) {  // C tile loaded now, its latency hidden by the products
            const uint32_t m0 = cur.by * BM;
            gemm_cload(g, cur.bx * BN, [&](uint32_t r) { return m0 + r < g.M ? m0 + r : 0xffffffffu; }, c);
        }
        gemm_mainloop<ONE, !ONE>(f, cur.kbeg, cur.kend, smem, lc, wave, lane, a);
        if (more) {
            // (rows_s[(it + 1) & 1] was last read by the epilogue of the tile
            // before, ahead of the main loop's barriers)
            if (tid < BM) rows_s[(it + 1) & 1][tid] = gemm_tile_row(g, nxt.by * BM, tid);
            f.init(g, nxt.by * BM, nxt.bx * BN, nxt.kbeg, nxt.kend, smem, wave, lane);
            f.issue(nxt.kbeg, 0);
            f.issue(nxt.kbeg + 2 * BK, 1);
        }
        gemm_epilogue<ONE, !ONE, PRE>(md, lc, g, cur.bx * BN, rows_s[it & 1], (uint16_t *)(smem + kGemmLds), wave,
                                         lane, a, c);
        if (!more) return;
        cur = nxt;
    }
}

// Workgroups of a GEMM launch over `tiles` tiles (GemmPlanes::max_wg): one
// per tile by default (the dispatcher then balances tiles of uneven K
// ranges); with kGemmPerCu one per compute unit (the LDS allows no more),
// each taking every G-th tile, which hides the operand fetch of a tile
// behind the write-back of the one before (short, even K ranges); any other
// value caps the count (a multiple of 8, the XCD count, when it caps).
uint32_t gemm_workgroups(uint32_t tiles, uint32_t max_wg) {
    if (max_wg == 0) return tiles;
    uint32_t G = fl_queue_grid(tiles, 1);
    if (max_wg != kGemmPerCu && G > max_wg) G = max_wg >= 8 ? max_wg / 8 * 8 : max_wg;
    return G ? G : 1;
}

hipError_t launch_gemm(uint32_t p, uint32_t nx, uint32_t ny, const fl::Mod &md, uint32_t bias, uint32_t c16,
                       const GemmPlanes &gp, hipStream_t s) {
    const dim3 grid(gemm_workgroups(nx * ny, gp.max_wg));
    // Persistent launches load the C tile ahead of the products when its rows
    // need no row map (a mapped row would be one more dependent load).
    // (Measured: TRSM band and second pass 2-3% faster; with one workgroup
    // per tile, short K ranges were 6% slower: the first step waited for C.)
    const bool pre = gp.row_map == nullptr && gp.max_wg != 0;
    if (p < 256) {
        if (pre)
            hipLaunchKernelGGL((k_mfma_gemm<true, true>), grid, dim3(kGemmThreads), 0, s, md, bias, c16, gp, nx, ny);
        else
            hipLaunchKernelGGL((k_mfma_gemm<true, false>), grid, dim3(kGemmThreads), 0, s, md, bias, c16, gp, nx, ny);
    } else {
        if (pre)
            hipLaunchKernelGGL((k_mfma_gemm<false, true>), grid, dim3(kGemmThreads), 0, s, md, bias, c16, gp, nx, ny);
        else
            hipLaunchKernelGGL((k_mfma_gemm<false, false>), grid, dim3(kGemmThreads), 0, s, md, bias, c16, gp, nx,
                               ny);
    }
    return hipGetLastError();
}

// Rank-k update, k <= 64: one 64-row x 128-column tile per workgroup; row
// blocks beyond the row count *Mdev (a device value) exit at once.
__global__ __launch_bounds__(256) void k_mfma_rank64(fl::Mod md, uint32_t bias, uint32_t c16,
                                                     const int8_t *__restrict__ Ah,
                                                     const int8_t *__restrict__ Al,
                                                     const int8_t *__restrict__ Bh,
                                                     const int8_t *__restrict__ Bl,
                                                     const uint32_t *__restrict__ Kdev,
                                                     const uint32_t *__restrict__ row_map,
                                                     const uint32_t *__restrict__ Mdev,
                                                     uint16_t *C, uint64_t ldc, uint32_t Mh,
                                                     uint32_t N) {
    __shared__ __attribute__((aligned(16))) uint16_t sv[64 * kRank64Ld];
    __shared__ uint32_t rows_s[64];
    const uint32_t M = Mdev ? *Mdev : Mh;
    if (blockIdx.y * 64 >= M || (Kdev && *Kdev == 0)) return;
    mfma_rank64_tile(md, bias, c16, Ah, Al, Bh, Bl, row_map, M, C, ldc, N, blockIdx.x, blockIdx.y, sv, rows_s);
}

inline uint32_t round_up(uint32_t x, uint32_t m) { return (x + m - 1) / m * m; }

struct MfmaWs {
    int8_t *Ah, *Al, *Bh, *Bl;
    uint32_t Mp, Np, Kp;
};

size_t mfma_layout(uint32_t M, uint32_t N, uint32_t Kmax, void *ws, MfmaWs *w) {
    WsCarve c(ws);
    MfmaWs t;
    t.Mp = round_up(M ? M : 1, BM);
    t.Np = round_up(N ? N : 1, BN);
    t.Kp = round_up(Kmax ? Kmax : 1, BK);
    t.Ah = c.take<int8_t>((size_t)t.Mp * t.Kp);
    t.Al = c.take<int8_t>((size_t)t.Mp * t.Kp);
    t.Bh = c.take<int8_t>((size_t)t.Np * t.Kp);
    t.Bl = c.take<int8_t>((size_t)t.Np * t.Kp);
    if (w) *w = t;
    return c.off;
}

}  // namespace

// Rank-k (k <= 64) update on prepared limb planes: A rows indexed by the C
// row (64 bytes each), B transposed (N_pad x 64); rows from row_map[0..*Mdev).
hipError_t fl_mfma_rank64_planes(uint32_t p, const int8_t *Ah, const int8_t *Al, const int8_t *Bh,
                                 const int8_t *Bl, const uint32_t *Kdev, const uint32_t *row_map,
                                 const uint32_t *Mdev, uint32_t Mmax, uint16_t *C, uint64_t ldc,
                                 uint32_t N, hipStream_t s, const char *site) {
    if (Mmax == 0 || N == 0) return hipSuccess;
    const fl::Mod md = fl::make_mod(p);
    const uint32_t bias = (uint32_t)((((uint64_t)1 << 31) + p - 1) / p * p);
    const uint32_t c16 = (uint32_t)((1u << 16) % p);
    dim3 g((N + 127) / 128, (Mmax + 63) / 64);
    FL_PROF(site, s, hipLaunchKernelGGL(k_mfma_rank64, g, dim3(256), 0, s, md, bias, c16, Ah, Al, Bh, Bl,
                                        Kdev, row_map, Mdev, C, ldc, Mmax, N));
    return hipGetLastError();
}

hipError_t fl_mfma_gemm_planes(uint32_t p, const GemmPlanes &gp, hipStream_t s, const char *site) {
    if (gp.M == 0 || gp.N == 0) return hipSuccess;
    const fl::Mod md = fl::make_mod(p);
    const uint32_t bias = (uint32_t)((((uint64_t)1 << 31) + p - 1) / p * p);
    const uint32_t c16 = (uint32_t)((1u << 16) % p);
    hipError_t e;
    FL_PROF(site, s, e = launch_gemm(p, (gp.N + BN - 1) / BN, (gp.M + BM - 1) / BM, md, bias, c16, gp, s));
    return e;
}

// The transposing limb conversion, for other translation units: B (K x cols,
// ld ldb) -> Bh, Bl (cols_pad x Kp); launch with grid (cols_pad/64, Kp/64),
// 256 threads.
typedef void (*fl_limbs_cols_fn)(uint32_t, const uint16_t *, uint64_t, uint32_t, uint32_t,
                                 const uint32_t *, int8_t *, int8_t *, uint32_t, uint32_t *);
fl_limbs_cols_fn fl_limbs_cols_kernel() { return k_limbs_cols; }

size_t fl_gemm_sub_mfma_ws(uint32_t M, uint32_t N, uint32_t Kmax) {
    return mfma_layout(M, N, Kmax, nullptr, nullptr);
}

// C[M x N] -= A[M x K] B[K x N] (mod p) on the matrix cores.  K = *Kdev when
// Kdev is non-NULL (then K <= Kmax), else Kmax.  Bit-identical to
// fl_gemm_sub_plain.
hipError_t fl_gemm_sub_mfma(uint32_t p, uint32_t M, uint32_t N, uint32_t Kmax, const uint32_t *Kdev,
                            const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                            uint16_t *C, uint64_t ldc, void *ws, size_t ws_bytes, hipStream_t s,
                            const char *site) {
    char site_limbs[64], site_mfma[64];
    snprintf(site_limbs, sizeof site_limbs, "%s.limbs", site ? site : "gemm");
    snprintf(site_mfma, sizeof site_mfma, "%s.mfma", site ? site : "gemm");
    if (M == 0 || N == 0 || Kmax == 0) return hipSuccess;
    MfmaWs w;
    if (mfma_layout(M, N, Kmax, ws, &w) > ws_bytes || !ws) return hipErrorInvalidValue;
    const fl::Mod md = fl::make_mod(p);
    // bias: the smallest multiple of p that is >= 2^31, so s + bias >= 0 and
    // s + bias < 2^32 for |s| < 2^31 - 2^16.
    const uint32_t bias = (uint32_t)((((uint64_t)1 << 31) + p - 1) / p * p);
    const uint32_t c16 = (uint32_t)((1u << 16) % p);
    {
        dim3 g(w.Kp / 4 / 256 + 1, w.Mp < 65535 ? w.Mp : 65535);
        FL_PROF(site_limbs, s, hipLaunchKernelGGL(k_limbs_rows, g, dim3(256), 0, s, p, A, lda, M, Kmax, Kdev,
                                                  w.Ah, w.Al, w.Mp, w.Kp));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    {
        dim3 g(w.Np / 64, w.Kp / 64);
        FL_PROF(site_limbs, s, hipLaunchKernelGGL(k_limbs_cols, g, dim3(256), 0, s, p, B, ldb, N, Kmax, Kdev,
                                                  w.Bh, w.Bl, w.Kp, (uint32_t *)nullptr));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (w.Kp == BK) {  // one K-step: rank-k update kernel
        dim3 g(w.Np / 128, w.Mp / 64);
        FL_PROF(site_mfma, s, hipLaunchKernelGGL(k_mfma_rank64, g, dim3(256), 0, s, md, bias, c16, w.Ah,
                                                 w.Al, w.Bh, w.Bl, Kdev, (const uint32_t *)nullptr,
                                                 (const uint32_t *)nullptr, C, ldc, M, N));
        return hipGetLastError();
    }
    for (uint32_t kb = 0; kb < w.Kp; kb += kKChunk) {
        const uint32_t ke = kb + kKChunk < w.Kp ? kb + kKChunk : w.Kp;
        GemmPlanes gp = {w.Ah, w.Al, w.Bh, w.Bl, w.Kp, w.Kp, 0, 0, kb, ke, Kdev, nullptr, nullptr,
                         nullptr, C, ldc, M, N};
        // groups of 4 row tiles per column tile on each XCD (measured on a
        // 16384^3 product: 12% faster than row-major tile order, 8% faster
        // than groups of 8)
        gp.group_m = 4;
        hipError_t e;
        FL_PROF(site_mfma, s, e = launch_gemm(p, w.Np / BN, w.Mp / BM, md, bias, c16, gp, s));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
