// gemm_mfma.hip -- dense C = C - A B mod p on the int8 matrix cores (gfx950).
//
// Every residue x in [0, p), p <= 65521, is centred into
//     r = x            if x <= 32639
//     r = x - p        otherwise            (r in [-32881, 32639])
// and split into two signed 8-bit limbs r = 256 h + l with
//     h = floor((r + 128) / 256) in [-128, 127],  l = r - 256 h in [-128, 127].
// Then  sum_k A B = 65536 S_hh + 256 (S_hl + S_lh) + S_ll  with four int8 GEMMs
// accumulated exactly in int32 (v_mfma_i32_16x16x64_i8): |h h'| <= 2^14, so a
// K-chunk of at most kKChunk = 65472 terms keeps |S_hh|, |S_ll| < 2^30 and the
// shared middle accumulator |S_hl + S_lh| < 2^31.  Each partial is biased to
// a non-negative 32-bit value (a multiple of p added), Barrett-reduced, and
// recombined with 2^16 mod p and 2^8.  No floating point anywhere.
//
// Operands are first converted to limb planes in the workspace, both stored
// K-contiguous (A as M x Kp, B transposed as N x Kp, zero padded to the tile
// sizes), so the GEMM kernel streams int8 rows with 16-byte loads and needs no
// bounds checks in its main loop.
#include "fl_internal.h"

#include <cstdio>

namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 64;
constexpr uint32_t kKChunk = 65472;  // multiple of BK, < 65536
constexpr int kLdsRow = BK + 16;     // padded LDS row (bytes) against bank conflicts
constexpr int kOutLd = BN + 4;       // u16 row stride of the epilogue tile (8-byte aligned rows)

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
__global__ __launch_bounds__(256) void k_limbs_cols(uint32_t p, const uint16_t *__restrict__ B,
                                                    uint64_t ldb, uint32_t cols, uint32_t Kh,
                                                    const uint32_t *__restrict__ Kdev,
                                                    int8_t *Bh, int8_t *Bl, uint32_t Kp) {
    __shared__ int8_t th[64][65], tl[64][65];
    const uint32_t K = Kdev ? *Kdev : Kh;
    const uint32_t k0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;  // 64 x 4
    for (uint32_t kk = ty; kk < 64; kk += 4) {
        const uint32_t k = k0 + kk, c = c0 + tx;
        int h = 0, l = 0;
        if (k < K && c < cols) split_limbs(B[(uint64_t)k * ldb + c], p, h, l);
        th[kk][tx] = (int8_t)h;
        tl[kk][tx] = (int8_t)l;
    }
    __syncthreads();
    for (uint32_t cc = ty; cc < 64; cc += 4) {
        const uint32_t c = c0 + cc;
        Bh[(uint64_t)c * Kp + k0 + tx] = th[tx][cc];
        Bl[(uint64_t)c * Kp + k0 + tx] = tl[tx][cc];
    }
}

__device__ __forceinline__ uint32_t signed_to_res(int s, const fl::Mod &md, uint32_t bias) {
    return fl::reduce32((uint32_t)s + bias, md);
}

// 256 threads = 4 waves in a 2 x 2 arrangement, 64 x 64 outputs per wave as
// 4 x 4 tiles of 16 x 16.  The next K-tile is loaded into registers while
// the current one is multiplied, so global latency overlaps the MFMAs.
__global__ __launch_bounds__(256) void k_mfma_gemm(fl::Mod md, uint32_t bias, uint32_t c16,
                                                   GemmPlanes g) {
    __shared__ __attribute__((aligned(16))) int8_t smem[4 * BM * kLdsRow];
    static_assert(BM * kOutLd * 2 <= 4 * BM * kLdsRow, "epilogue tile must fit the operand buffers");
    int8_t *sAh = smem, *sAl = smem + BM * kLdsRow;
    int8_t *sBh = smem + 2 * BM * kLdsRow, *sBl = smem + 3 * BM * kLdsRow;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t wm = wave >> 1, wn = wave & 1;
    const uint32_t m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
    uint32_t kbeg = g.kbeg, kend = g.kend;
    if (g.krange) {
        kbeg = g.krange[2 * blockIdx.y];
        kend = g.krange[2 * blockIdx.y + 1];
    }
    if (g.krange_n) {  // per column block: intersect
        const uint32_t b = g.krange_n[2 * blockIdx.x], e = g.krange_n[2 * blockIdx.x + 1];
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
    // each plane tile is 128 rows x 64 bytes = 512 chunks of 16 B; thread t
    // moves chunks t and t + 256 of each of the four planes
    const uint32_t r_lo = tid >> 2, q = (tid & 3) * 16;
    const uint64_t a_off0 = (uint64_t)(m0 + r_lo) * g.lda + g.a_k0 + q;
    const uint64_t a_off1 = (uint64_t)(m0 + r_lo + 64) * g.lda + g.a_k0 + q;
    const uint64_t b_off0 = (uint64_t)(n0 + r_lo) * g.ldb + g.b_k0 + q;
    const uint64_t b_off1 = (uint64_t)(n0 + r_lo + 64) * g.ldb + g.b_k0 + q;
    v4i pf[8];
    auto gload = [&](uint32_t k0) {
        pf[0] = *(const v4i *)(g.Ah + a_off0 + k0);
        pf[1] = *(const v4i *)(g.Al + a_off0 + k0);
        pf[2] = *(const v4i *)(g.Bh + b_off0 + k0);
        pf[3] = *(const v4i *)(g.Bl + b_off0 + k0);
        pf[4] = *(const v4i *)(g.Ah + a_off1 + k0);
        pf[5] = *(const v4i *)(g.Al + a_off1 + k0);
        pf[6] = *(const v4i *)(g.Bh + b_off1 + k0);
        pf[7] = *(const v4i *)(g.Bl + b_off1 + k0);
    };
    if (kbeg < kend) gload(kbeg);
    const uint32_t s0 = r_lo * kLdsRow + q, s1 = (r_lo + 64) * kLdsRow + q;
    for (uint32_t k0 = kbeg; k0 < kend; k0 += BK) {
        *(v4i *)(sAh + s0) = pf[0];
        *(v4i *)(sAl + s0) = pf[1];
        *(v4i *)(sBh + s0) = pf[2];
        *(v4i *)(sBl + s0) = pf[3];
        *(v4i *)(sAh + s1) = pf[4];
        *(v4i *)(sAl + s1) = pf[5];
        *(v4i *)(sBh + s1) = pf[6];
        *(v4i *)(sBl + s1) = pf[7];
        __syncthreads();
        if (k0 + BK < kend) gload(k0 + BK);
        v4i ah[4], al[4], bh[4], bl[4];
        const uint32_t kq = (lane >> 4) * 16;
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const uint32_t ra = wm * 64 + t * 16 + (lane & 15);
            const uint32_t rb = wn * 64 + t * 16 + (lane & 15);
            ah[t] = *(const v4i *)(sAh + ra * kLdsRow + kq);
            al[t] = *(const v4i *)(sAl + ra * kLdsRow + kq);
            bh[t] = *(const v4i *)(sBh + rb * kLdsRow + kq);
            bl[t] = *(const v4i *)(sBl + rb * kLdsRow + kq);
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
        __syncthreads();
    }
    if (kbeg >= kend) return;  // nothing to subtract
    // epilogue: residues of the 128 x 128 tile go through LDS (the operand
    // buffers are free now), then C is read, reduced and written back with
    // coalesced 8-byte accesses.  Output element (row 4*(lane/16) + e,
    // column lane%16) of each 16 x 16 tile is held by the wave.
    uint16_t *sOut = (uint16_t *)smem;
#pragma unroll
    for (int i = 0; i < 4; i++)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const uint32_t col = wn * 64 + j * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t row = wm * 64 + i * 16 + (lane >> 4) * 4 + e;
                const uint32_t rhh = signed_to_res(acc_hh[i][j][e], md, bias);
                const uint32_t rmid = signed_to_res(acc_mid[i][j][e], md, bias);
                const uint32_t rll = signed_to_res(acc_ll[i][j][e], md, bias);
                uint32_t v = fl::reduce32(rhh * c16 + rll, md);
                v = fl::reduce32(v + rmid * 256u, md);
                sOut[row * kOutLd + col] = (uint16_t)v;
            }
        }
    __syncthreads();
    // 128 rows x 32 chunks of 4 columns; 256 threads -> 16 chunks each, in
    // batches of 4 whose C loads are issued before their stores
#pragma unroll 1
    for (int u0 = 0; u0 < 16; u0 += 4) {
        uint64_t cvals[4];
        uint32_t orows[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint32_t ch = tid + (u0 + u) * 256;
            const uint32_t r = ch / (BN / 4), c4 = (ch % (BN / 4)) * 4;
            const uint32_t row = m0 + r, col = n0 + c4;
            cvals[u] = 0;
            orows[u] = 0xffffffffu;
            if (row < g.M && col < g.N) {
                orows[u] = g.row_map ? g.row_map[row] : row;
                if (orows[u] != 0xffffffffu && col + 4 <= g.N)
                    cvals[u] = *(const uint64_t *)(g.C + (uint64_t)orows[u] * g.ldc + col);
            }
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const uint32_t ch = tid + (u0 + u) * 256;
            const uint32_t r = ch / (BN / 4), c4 = (ch % (BN / 4)) * 4;
            const uint32_t col = n0 + c4;
            if (orows[u] == 0xffffffffu) continue;
            uint16_t *o = g.C + (uint64_t)orows[u] * g.ldc + col;
            const uint64_t sv = *(const uint64_t *)(sOut + r * kOutLd + c4);
            if (col + 4 <= g.N) {
                const uint64_t ov = cvals[u];
                uint64_t nv = 0;
#pragma unroll
                for (int c = 0; c < 4; c++)
                    nv |= (uint64_t)fl::submod((uint32_t)(ov >> (16 * c)) & 0xffffu,
                                               (uint32_t)(sv >> (16 * c)) & 0xffffu, md.p) << (16 * c);
                *(uint64_t *)o = nv;
            } else {
                for (uint32_t c = 0; col + c < g.N; c++)
                    o[c] = (uint16_t)fl::submod(o[c], (uint32_t)(sv >> (16 * c)) & 0xffffu, md.p);
            }
        }
    }
}

// Rank-k update, k <= 64 (the Gauss-Jordan panel updates): one MFMA K-step,
// so the kernel is bound by the read-modify-write of C and its epilogue.  A
// block owns 64 rows x 128 columns; rows are taken through an optional row
// list (row_map, count *Mdev: only rows with nonzero multipliers), the C tile
// is loaded first with row-contiguous 8-byte accesses (latency overlapping
// the operand loads and MFMAs), residues are staged through LDS and C is
// written back with 8-byte accesses.  A planes are indexed by the C row.
// With K <= 64, |S_hh|, |S_ll| <= 2^20 and |S_mid| <= 2^21, so
// 256 S_mid + S_ll fits 32 bits and the recombination needs three Barrett
// reductions instead of five.
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
    constexpr int kLd = 128 + 4;  // u16 row stride of the residue tile
    __shared__ __attribute__((aligned(16))) uint16_t sv[64 * kLd];
    __shared__ uint32_t rows_s[64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t m0 = blockIdx.y * 64, n0 = blockIdx.x * 128;
    const uint32_t M = Mdev ? *Mdev : Mh;
    if (m0 >= M || (Kdev && *Kdev == 0)) return;
    if (tid < 64) rows_s[tid] = (m0 + tid < M) ? (row_map ? row_map[m0 + tid] : m0 + tid) : 0xffffffffu;
    __syncthreads();
    // C tile: 64 rows x 32 chunks of 4 columns = 2048 chunks, 8 per thread
    uint64_t cv[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t ch = tid + u * 256, r = ch >> 5, c4 = (ch & 31) * 4;
        const uint32_t row = rows_s[r], col = n0 + c4;
        cv[u] = 0;
        if (row != 0xffffffffu && col + 4 <= N) cv[u] = *(const uint64_t *)(C + (uint64_t)row * ldc + col);
    }
    const uint32_t rq = (lane >> 4) * 4, cl = lane & 15, kq = (lane >> 4) * 16;
    const uint32_t arow = rows_s[wave * 16 + cl];
    v4i ah = {0, 0, 0, 0}, al = {0, 0, 0, 0};
    if (arow != 0xffffffffu) {
        ah = *(const v4i *)(Ah + (uint64_t)arow * 64 + kq);
        al = *(const v4i *)(Al + (uint64_t)arow * 64 + kq);
    }
    const uint32_t bias2 = (uint32_t)(((1u << 30) + md.p - 1) / md.p * md.p);  // >= 2^30, multiple of p
#pragma unroll
    for (int j = 0; j < 8; j++) {
        const uint64_t b = (uint64_t)(n0 + j * 16 + cl) * 64 + kq;
        const v4i bh = *(const v4i *)(Bh + b);
        const v4i bl = *(const v4i *)(Bl + b);
        v4i hh = {0, 0, 0, 0}, mid = {0, 0, 0, 0}, ll = {0, 0, 0, 0};
        hh = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah, bh, hh, 0, 0, 0);
        mid = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah, bl, mid, 0, 0, 0);
        mid = __builtin_amdgcn_mfma_i32_16x16x64_i8(al, bh, mid, 0, 0, 0);
        ll = __builtin_amdgcn_mfma_i32_16x16x64_i8(al, bl, ll, 0, 0, 0);
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint32_t rhh = signed_to_res(hh[e], md, bias);
            const uint32_t rlo = fl::reduce32((uint32_t)(mid[e] * 256 + ll[e]) + bias2, md);
            const uint32_t v = fl::reduce32(rhh * c16 + rlo, md);
            sv[(wave * 16 + rq + e) * kLd + j * 16 + cl] = (uint16_t)v;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t ch = tid + u * 256, r = ch >> 5, c4 = (ch & 31) * 4;
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
            *(uint64_t *)o = nv;
        } else {
            for (uint32_t c = 0; col + c < N; c++)
                o[c] = (uint16_t)fl::submod(o[c], (uint32_t)(s4 >> (16 * c)) & 0xffffu, md.p);
        }
    }
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
    FL_PROF(site, s, hipLaunchKernelGGL(k_mfma_gemm, grid, dim3(256), 0, s, md, bias, c16, gp));
    return hipGetLastError();
}

// The transposing limb conversion, for other translation units: B (K x cols,
// ld ldb) -> Bh, Bl (cols_pad x Kp); launch with grid (cols_pad/64, Kp/64),
// 256 threads.
typedef void (*fl_limbs_cols_fn)(uint32_t, const uint16_t *, uint64_t, uint32_t, uint32_t,
                                 const uint32_t *, int8_t *, int8_t *, uint32_t);
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
                                                  w.Bh, w.Bl, w.Kp));
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
        FL_PROF(site_mfma, s, hipLaunchKernelGGL(k_mfma_gemm, grid, dim3(256), 0, s, md, bias, c16, gp));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
