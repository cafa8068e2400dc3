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

// The tile of this workgroup under GemmPlanes::group_m.  Workgroups are
// dispatched x fastest and dealt round-robin to the 8 XCDs; the linear
// dispatch index is renumbered so that every XCD receives a contiguous
// range, which is walked column tile by column tile in groups of gm row
// tiles.  Both steps are bijections of the grid.
__device__ __forceinline__ void gemm_tile_of(uint32_t gm, uint32_t &bx, uint32_t &by) {
    const uint32_t nx = gridDim.x, ny = gridDim.y;
    bx = blockIdx.x;
    by = blockIdx.y;
    if (gm == 0) return;
    const uint32_t total = nx * ny, pid = by * nx + bx;
    const uint32_t q = total / 8, r = total % 8, x = pid % 8, i = pid / 8;
    const uint32_t id = x * q + (x < r ? x : r) + i;
    const uint32_t per = gm * nx, group = id / per, first = group * gm;
    const uint32_t rows = ny - first < gm ? ny - first : gm;
    const uint32_t within = id - group * per;
    by = first + within % rows;
    bx = within / rows;
}

// ONE: single-limb operands (p < 256).
template <bool ONE>
__global__ __launch_bounds__(kGemmThreads) void k_mfma_gemm(fl::Mod md, uint32_t bias, uint32_t c16,
                                                   GemmPlanes g) {
    __shared__ __attribute__((aligned(16))) int8_t smem[kGemmLds];
    uint32_t bx, by;
    gemm_tile_of(g.group_m, bx, by);
    mfma_gemm_tile<ONE>(md, bias, c16, g, bx, by, smem);
}

hipError_t launch_gemm(uint32_t p, dim3 grid, const fl::Mod &md, uint32_t bias, uint32_t c16, const GemmPlanes &gp,
                       hipStream_t s) {
    if (p < 256)
        hipLaunchKernelGGL(k_mfma_gemm<true>, grid, dim3(kGemmThreads), 0, s, md, bias, c16, gp);
    else
        hipLaunchKernelGGL(k_mfma_gemm<false>, grid, dim3(kGemmThreads), 0, s, md, bias, c16, gp);
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
    dim3 grid((gp.N + BN - 1) / BN, (gp.M + BM - 1) / BM);
    hipError_t e;
    FL_PROF(site, s, e = launch_gemm(p, grid, md, bias, c16, gp, s));
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
    dim3 grid(w.Np / BN, w.Mp / BM);
    for (uint32_t kb = 0; kb < w.Kp; kb += kKChunk) {
        const uint32_t ke = kb + kKChunk < w.Kp ? kb + kKChunk : w.Kp;
        GemmPlanes gp = {w.Ah, w.Al, w.Bh, w.Bl, w.Kp, w.Kp, 0, 0, kb, ke, Kdev, nullptr, nullptr,
                         nullptr, C, ldc, M, N};
        hipError_t e;
        FL_PROF(site_mfma, s, e = launch_gemm(p, grid, md, bias, c16, gp, s));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
