// wide.hip -- the FL reduction over 32-bit field characteristic (uint32
// residues, 2 <= p < 2^32; the uint32 version of Sec. 2), steps 2-5 and the
// second pass.  Step 1 is split.hip's, instantiated for uint32 values.
//
//   k_w_spmm      rows of a sparse w-multiline matrix (A or C) times rows of
//                 a dense matrix, subtracted from dense rows: the far update
//                 of a TRSM block (entries of A past the block) and the
//                 plain reduce Dt -= C X.  One thread per column, the row's
//                 entries broadcast to the workgroup, 64-bit sums of raw
//                 products (wide.h).
//   k_w_solve     back substitution inside a 64-row TRSM block, one thread
//                 per column, rows bottom-up.
//   k_w_panel     echelon: pivot search of a 64-column panel in one
//                 workgroup (row echelon form of the panel over the rows not
//                 yet pivots), then G = D[Q, C]^{-1} for its pivot rows Q and
//                 columns C by Gauss-Jordan on the k x k block.
//   k_w_U, k_w_L  U = G D[Q, c0:], L' = D[:, C] - [row = Q_t].
//   k_w_update    D[:, c0:] -= L' U (plain form), or
//   k_w_gemm4     the same contraction on the int8 matrix cores: four signed
//                 limbs per residue, 16 limb products per multiply-add into
//                 seven int32 diagonals; one launch per kWideKChunk K terms.
//   k_w_csr_*     the read-off of RREF(M) as canonical CSR.
#include <algorithm>

#include "fl_internal.h"
#include "wide.h"

using flw::Mod64;

namespace {

constexpr uint32_t kWBlk = 64;    // rows per TRSM block
constexpr uint32_t kWCols = 256;  // columns per workgroup of the VALU kernels
constexpr uint32_t kWPanel = 64;  // columns per echelon panel

typedef int v4i __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t lane_id() { return threadIdx.x & 63; }

// ---- dense helpers ------------------------------------------------------------

__global__ void k_w_zero(uint32_t *out, uint64_t ld, uint32_t rows, uint32_t cols) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    for (uint32_t r = blockIdx.y; r < rows; r += gridDim.y) out[(uint64_t)r * ld + c] = 0;
}

// CSR rows -> dense rows (the dense target zeroed first); one wave per row.
__global__ void k_w_scatter(uint32_t rows, const uint64_t *__restrict__ rp, const uint32_t *__restrict__ ci,
                            const uint32_t *__restrict__ v, uint32_t *out, uint64_t ld) {
    const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    for (uint64_t k = rp[r] + lane_id(); k < rp[r + 1]; k += 64) out[(uint64_t)r * ld + ci[k]] = v[k];
}

hipError_t w_zero(uint32_t *out, uint64_t ld, uint32_t rows, uint32_t cols, hipStream_t s) {
    if (!rows || !cols) return hipSuccess;
    hipLaunchKernelGGL(k_w_zero, dim3((cols + 255) / 256, std::min(rows, 4096u)), dim3(256), 0, s, out, ld, rows,
                       cols);
    return hipGetLastError();
}

// ---- sparse (multiline) x dense ----------------------------------------------
// out[row0 + y] += sum over entries (col, a) of that row with kmin <= col < kmax
// of (p - a) src[col]   (i.e. out -= A src), for the columns of this workgroup.
__global__ __launch_bounds__(256) void k_w_spmm(Mod64 md, uint32_t w, const uint64_t *__restrict__ gptr,
                                                const uint32_t *__restrict__ pos, const uint32_t *__restrict__ val,
                                                uint32_t row0, uint32_t kmin, uint32_t kmax,
                                                const uint32_t *__restrict__ src, uint64_t lds, uint32_t *out,
                                                uint64_t ldo, uint32_t ncols) {
    const uint32_t r = row0 + blockIdx.y;
    const uint32_t c = blockIdx.x * kWCols + threadIdx.x;
    const uint32_t g = r / w, q = r % w;
    uint64_t acc = 0;
    for (uint64_t k = gptr[g]; k < gptr[g + 1]; k++) {
        const uint32_t col = pos[k];
        if (col < kmin) continue;
        if (col >= kmax) break;
        const uint32_t a = val[(uint64_t)w * k + q];
        if (a == 0 || c >= ncols) continue;
        flw::macw(acc, md.p - a, src[(uint64_t)col * lds + c], md);
    }
    if (c < ncols) {
        uint32_t *o = out + (uint64_t)r * ldo + c;
        *o = flw::addw(*o, flw::reduce64(acc, md), md.p);
    }
}

// Rows [r0, r1) of X solved bottom-up with the entries of A inside the block
// (the entries past it were applied by k_w_spmm).  Each thread reads only the
// X entries of its own column, which it wrote itself.
__global__ __launch_bounds__(256) void k_w_solve(Mod64 md, uint32_t w, const uint64_t *__restrict__ gptr,
                                                 const uint32_t *__restrict__ pos, const uint32_t *__restrict__ val,
                                                 uint32_t r0, uint32_t r1, uint32_t *X, uint64_t ldx, uint32_t ncols) {
    const uint32_t c = blockIdx.x * kWCols + threadIdx.x;
    if (c >= ncols) return;
    for (uint32_t r = r1; r-- > r0;) {
        const uint32_t g = r / w, q = r % w;
        uint64_t acc = 0;
        for (uint64_t k = gptr[g]; k < gptr[g + 1]; k++) {
            const uint32_t col = pos[k];
            if (col <= r) continue;
            if (col >= r1) break;
            const uint32_t a = val[(uint64_t)w * k + q];
            if (a) flw::macw(acc, md.p - a, X[(uint64_t)col * ldx + c], md);
        }
        uint32_t *o = X + (uint64_t)r * ldx + c;
        *o = flw::addw(*o, flw::reduce64(acc, md), md.p);
    }
}

// ---- int8 four-limb GEMM: C[M x N] -= A[M x K] B[K x N] mod p -----------------
// A as four limb planes (row-major, lda bytes per row, planes a_ps bytes
// apart), B as four limb planes transposed (one row of ldb bytes per column
// of B).  Zero padding up to whole 64 x 64 tiles and K steps.  K range
// [kbeg, kend), cut at *kdev rounded up to 64 when kdev is given (planes are
// zero past it).
// 64 x 64 tile per workgroup of 4 waves (2 x 2, 32 x 32 each: 2 x 2 blocks of
// v_mfma_i32_16x16x64_i8); operand tiles staged in LDS, the next K step's
// global loads issued before the current step's MFMAs.
struct Gemm4 {
    const int8_t *A;
    uint64_t lda, a_ps;
    const int8_t *B;
    uint64_t ldb, b_ps;
    uint32_t kbeg, kend;    // this launch's K range: at most kWideKChunk terms
    const uint32_t *kdev;
    uint32_t *C;
    uint64_t ldc;
    uint32_t M, N;
};

__global__ __launch_bounds__(256) void k_w_gemm4(Mod64 md, Gemm4 g) {
    __shared__ __attribute__((aligned(16))) int8_t sA[4][64][64];
    __shared__ __attribute__((aligned(16))) int8_t sB[4][64][64];
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t wm = wave >> 1, wn = wave & 1;
    const uint32_t m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    uint32_t K = g.kend;
    if (g.kdev) {
        const uint32_t kd = (*g.kdev + 63) / 64 * 64;
        K = kd < K ? kd : K;
    }
    if (K <= g.kbeg) return;  // (uniform) nothing to subtract
    // loader: thread -> (row lr, 16-byte chunk lc) of every plane of both tiles
    const uint32_t lr = tid >> 2, lc = tid & 3;
    const uint32_t sw = (lc ^ ((lr >> 2) & 3)) * 16;  // swizzled chunk slot
    const int8_t *ga = g.A + (uint64_t)(m0 + lr) * g.lda + lc * 16;
    const int8_t *gb = g.B + (uint64_t)(n0 + lr) * g.ldb + lc * 16;
    v4i pa[4], pb[4];
    v4i acc[2][2][7];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int d = 0; d < 7; d++) acc[a][b][d] = v4i{0, 0, 0, 0};
#define W_LOAD(k0)                                                    \
    _Pragma("unroll") for (int i = 0; i < 4; i++) {                   \
        pa[i] = *(const v4i *)(ga + i * g.a_ps + (k0));               \
        pb[i] = *(const v4i *)(gb + i * g.b_ps + (k0));               \
    }
    const uint32_t kc = lane >> 4;
    W_LOAD(g.kbeg)
    for (uint32_t k0 = g.kbeg; k0 < K; k0 += 64) {
        __syncthreads();  // every wave is done with the previous step's tiles
#pragma unroll
        for (int i = 0; i < 4; i++) {
            *(v4i *)&sA[i][lr][sw] = pa[i];
            *(v4i *)&sB[i][lr][sw] = pb[i];
        }
        __syncthreads();
        if (k0 + 64 < K) { W_LOAD(k0 + 64) }
        v4i fa[2][4], fb[2][4];
#pragma unroll
        for (int t = 0; t < 2; t++) {
            const uint32_t ra = wm * 32 + t * 16 + (lane & 15), rb = wn * 32 + t * 16 + (lane & 15);
            const uint32_t oa = (kc ^ ((ra >> 2) & 3)) * 16, ob = (kc ^ ((rb >> 2) & 3)) * 16;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                fa[t][i] = *(const v4i *)&sA[i][ra][oa];
                fb[t][i] = *(const v4i *)&sB[i][rb][ob];
            }
        }
#pragma unroll
        for (int a = 0; a < 2; a++)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int i = 0; i < 4; i++)
#pragma unroll
                    for (int j = 0; j < 4; j++)
                        acc[a][b][i + j] =
                            __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[a][i], fb[b][j], acc[a][b][i + j], 0, 0, 0);
    }
#undef W_LOAD
    // output element (row 4 (lane / 16) + e, column lane % 16) of each block
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const uint32_t col = n0 + wn * 32 + b * 16 + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t row = m0 + wm * 32 + a * 16 + (lane >> 4) * 4 + e;
                if (row < g.M && col < g.N) {
                    const v4i *q = acc[a][b];
                    const uint32_t v = flw::combine7(q[0][e], q[1][e], q[2][e], q[3][e], q[4][e], q[5][e], q[6][e],
                                                     md);
                    uint32_t *o = g.C + (uint64_t)row * g.ldc + col;
                    *o = flw::subw(*o, v, md.p);
                }
            }
        }
}

// Dense rows -> four limb planes, K-contiguous: plane i, row r, byte k holds
// limb i of src[r][k] (zero for r >= rows, k >= cols, or k >= *kdev).
__global__ void k_w_limbs_rows(uint32_t p, const uint32_t *__restrict__ src, uint64_t ld, uint32_t rows,
                               uint32_t cols, const uint32_t *__restrict__ kdev, int8_t *planes, uint64_t ps,
                               uint64_t kp, uint32_t row0) {
    const uint32_t k4 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    const uint32_t r = row0 + blockIdx.y;
    if (k4 >= kp) return;
    const uint32_t kl = kdev ? std::min(cols, *kdev) : cols;
    uint32_t out[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const uint32_t k = k4 + e;
        int l[4] = {0, 0, 0, 0};
        if (r < rows && k < kl) flw::split_limbs4(src[(uint64_t)r * ld + k], p, l);
#pragma unroll
        for (int i = 0; i < 4; i++) out[i] |= (uint32_t)(l[i] & 0xff) << (8 * e);
    }
#pragma unroll
    for (int i = 0; i < 4; i++) *(uint32_t *)(planes + i * ps + (uint64_t)r * kp + k4) = out[i];
}

// Dense K x N matrix -> four limb planes transposed: plane i, row n (column
// n of src), byte k.  Zero for n >= N, k >= K or k >= *kdev.
__global__ void k_w_limbs_cols(uint32_t p, const uint32_t *__restrict__ src, uint64_t ld, uint32_t K, uint32_t N,
                               const uint32_t *__restrict__ kdev, int8_t *planes, uint64_t ps, uint64_t kp) {
    const uint32_t n = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t k4 = blockIdx.y * 4;
    if (k4 >= kp) return;
    const uint32_t kl = kdev ? std::min(K, *kdev) : K;
    uint32_t out[4] = {0, 0, 0, 0};
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const uint32_t k = k4 + e;
        int l[4] = {0, 0, 0, 0};
        if (n < N && k < kl) flw::split_limbs4(src[(uint64_t)k * ld + n], p, l);
#pragma unroll
        for (int i = 0; i < 4; i++) out[i] |= (uint32_t)(l[i] & 0xff) << (8 * e);
    }
    if (n < (uint32_t)(gridDim.x * blockDim.x))
#pragma unroll
        for (int i = 0; i < 4; i++) *(uint32_t *)(planes + i * ps + (uint64_t)n * kp + k4) = out[i];
}

uint64_t pad64(uint64_t x) { return (x + 63) / 64 * 64; }

// Four limb planes of a rows x kcols matrix, row-major (rows padded to 64,
// K to kp = pad64(kcols)).
size_t planes_bytes(uint64_t rows, uint64_t kcols) { return 4 * pad64(rows) * pad64(kcols ? kcols : 1); }

hipError_t w_limbs_rows(uint32_t p, const uint32_t *src, uint64_t ld, uint32_t rows, uint32_t cols,
                        const uint32_t *kdev, int8_t *planes, uint64_t kp, hipStream_t s) {
    const uint64_t rp = pad64(rows), ps = rp * kp;
    for (uint64_t r0 = 0; r0 < rp; r0 += 65535) {
        const unsigned ny = (unsigned)std::min<uint64_t>(rp - r0, 65535);
        hipLaunchKernelGGL(k_w_limbs_rows, dim3((unsigned)((kp / 4 + 255) / 256), ny), dim3(256), 0, s, p, src, ld,
                           rows, cols, kdev, planes, ps, kp, (uint32_t)r0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t w_limbs_cols(uint32_t p, const uint32_t *src, uint64_t ld, uint32_t K, uint32_t N, const uint32_t *kdev,
                        int8_t *planes, uint64_t kp, hipStream_t s) {
    const uint64_t np = pad64(N), ps = np * kp;
    hipLaunchKernelGGL(k_w_limbs_cols, dim3((unsigned)(np / 64), (unsigned)(kp / 4)), dim3(64), 0, s, p, src, ld,
                       K, N, kdev, planes, ps, kp);
    return hipGetLastError();
}

// C[M x N] -= A B with A (M x K) and B (K x N) given as limb planes: A
// row-major planes (M padded to 64, K bytes kp per row), B transposed planes
// (N padded to 64, kp per row).
hipError_t w_gemm4(const Mod64 &md, const int8_t *Ap, const int8_t *Bp, uint32_t M, uint32_t N, uint64_t kp,
                   const uint32_t *kdev, uint32_t *C, uint64_t ldc, hipStream_t s) {
    if (!M || !N || !kp) return hipSuccess;
    Gemm4 g;
    g.A = Ap;
    g.lda = kp;
    g.a_ps = pad64(M) * kp;
    g.B = Bp;
    g.ldb = kp;
    g.b_ps = pad64(N) * kp;
    g.kdev = kdev;
    g.C = C;
    g.ldc = ldc;
    g.M = M;
    g.N = N;
    // one launch per K chunk: each launch's int32 diagonal sums stay exact,
    // and its residues are subtracted from C before the next one starts
    for (uint64_t k0 = 0; k0 < kp; k0 += flw::kWideKChunk) {
        g.kbeg = (uint32_t)k0;
        g.kend = (uint32_t)std::min<uint64_t>(kp, k0 + flw::kWideKChunk);
        hipLaunchKernelGGL(k_w_gemm4, dim3((N + 63) / 64, (M + 63) / 64), dim3(256), 0, s, md, g);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Plain dense product C[M x N] -= A[M x K] B[K x N] (K = min(kmax, *kdev)).
__global__ __launch_bounds__(256) void k_w_gemm_plain(Mod64 md, const uint32_t *__restrict__ A, uint64_t lda,
                                                      const uint32_t *__restrict__ B, uint64_t ldb, uint32_t kmax,
                                                      const uint32_t *__restrict__ kdev, uint32_t *C, uint64_t ldc,
                                                      uint32_t N) {
    const uint32_t c = blockIdx.x * kWCols + threadIdx.x;
    const uint32_t r = blockIdx.y;
    if (c >= N) return;
    const uint32_t K = kdev ? std::min(kmax, *kdev) : kmax;
    const uint32_t *a = A + (uint64_t)r * lda;
    uint64_t acc = 0;
    for (uint32_t k = 0; k < K; k++) {
        const uint32_t x = a[k];
        if (x) flw::macw(acc, md.p - x, B[(uint64_t)k * ldb + c], md);
    }
    uint32_t *o = C + (uint64_t)r * ldc + c;
    *o = flw::addw(*o, flw::reduce64(acc, md), md.p);
}

hipError_t w_gemm_plain(const Mod64 &md, const uint32_t *A, uint64_t lda, const uint32_t *B, uint64_t ldb,
                        uint32_t M, uint32_t N, uint32_t kmax, const uint32_t *kdev, uint32_t *C, uint64_t ldc,
                        hipStream_t s) {
    if (!M || !N || !kmax) return hipSuccess;
    for (uint32_t r0 = 0; r0 < M; r0 += 65535) {
        const uint32_t mr = std::min(M - r0, 65535u);
        hipLaunchKernelGGL(k_w_gemm_plain, dim3((N + kWCols - 1) / kWCols, mr), dim3(kWCols), 0, s, md,
                           A + (uint64_t)r0 * lda, lda, B, ldb, kmax, kdev, C + (uint64_t)r0 * ldc, ldc, N);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---- argument checks ------------------------------------------------------------

fl_status check_info32(const fl_split_info *info, const fl_split_out32 *s) {
    FL_ARG(info && s, "NULL split info/output");
    FL_ARG(info->status == FL_OK, "split info carries an error status");
    FL_ARG(info->p >= 2, "split info: bad p");
    FL_ARG(info->ml_width == 1 || info->ml_width == 2 || info->ml_width == 4 || info->ml_width == 8,
           "split info: bad ml_width");
    FL_ARG(info->npiv + info->nB == info->n && info->npiv + info->mD == info->m, "split info: inconsistent sizes");
    return FL_OK;
}

hipError_t w_spmm(const Mod64 &md, uint32_t w, const uint64_t *gptr, const uint32_t *pos, const uint32_t *val,
                  uint32_t row0, uint32_t nrows, uint32_t kmin, uint32_t kmax, const uint32_t *src, uint64_t lds,
                  uint32_t *out, uint64_t ldo, uint32_t ncols, hipStream_t s) {
    for (uint32_t y = 0; y < nrows; y += 65535) {
        const uint32_t ny = std::min(nrows - y, 65535u);
        hipLaunchKernelGGL(k_w_spmm, dim3((ncols + kWCols - 1) / kWCols, ny), dim3(kWCols), 0, s, md, w, gptr, pos,
                           val, row0 + y, kmin, kmax, src, lds, out, ldo, ncols);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

// ================================ step 2 ======================================

extern "C" size_t fl_trsm32_workspace(const fl_split_info *info, fl_mode mode) {
    (void)info;
    (void)mode;
    return 0;
}

extern "C" fl_status fl_trsm32(const fl_split_info *info, const fl_split_out32 *s, uint32_t *X, uint64_t ldx,
                               fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream) {
    (void)ws;
    (void)ws_bytes;
    fl_status st = check_info32(info, s);
    if (st != FL_OK) return st;
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_trsm32: bad mode");
    const uint32_t npiv = info->npiv, nB = info->nB, w = info->ml_width;
    if (npiv == 0 || nB == 0) return FL_OK;
    FL_ARG(X && ldx >= nB, "fl_trsm32: NULL X or ldx < nB");
    const Mod64 md = flw::make_mod64(info->p);
    FL_HIP(w_zero(X, ldx, npiv, nB, stream));
    hipLaunchKernelGGL(k_w_scatter, dim3((npiv + 3) / 4), dim3(256), 0, stream, npiv, s->b_ptr, s->b_col, s->b_val,
                       X, ldx);
    FL_LAUNCH_CHECK("k_w_scatter");
    const uint32_t nblk = (npiv + kWBlk - 1) / kWBlk;
    const unsigned gx = (nB + kWCols - 1) / kWCols;
    for (uint32_t I = nblk; I-- > 0;) {
        const uint32_t r0 = I * kWBlk, r1 = std::min(r0 + kWBlk, npiv);
        if (r1 < npiv)
            FL_HIP(w_spmm(md, w, s->a_gptr, s->a_pos, s->a_val, r0, r1 - r0, r1, npiv, X, ldx, X, ldx, nB, stream));
        hipLaunchKernelGGL(k_w_solve, dim3(gx), dim3(kWCols), 0, stream, md, w, s->a_gptr, s->a_pos, s->a_val, r0,
                           r1, X, ldx, nB);
        FL_LAUNCH_CHECK("k_w_solve");
    }
    return FL_OK;
}

// ================================ step 3 ======================================

namespace {
// C's multiline entries scattered as limbs into zeroed planes (row-major,
// kp bytes per row): one wave per row.
__global__ void k_w_scatter_limbs(uint32_t p, uint32_t w, uint32_t rows, const uint64_t *__restrict__ gptr,
                                  const uint32_t *__restrict__ pos, const uint32_t *__restrict__ val, int8_t *planes,
                                  uint64_t ps, uint64_t kp) {
    const uint32_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= rows) return;
    const uint32_t g = r / w, q = r % w;
    for (uint64_t k = gptr[g] + lane_id(); k < gptr[g + 1]; k += 64) {
        const uint32_t a = val[(uint64_t)w * k + q];
        if (!a) continue;
        int l[4];
        flw::split_limbs4(a, p, l);
#pragma unroll
        for (int i = 0; i < 4; i++) planes[i * ps + (uint64_t)r * kp + pos[k]] = (int8_t)l[i];
    }
}

__global__ void k_w_zero_bytes(int8_t *p, uint64_t n16) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) *(v4i *)(p + 16 * i) = v4i{0, 0, 0, 0};
}

hipError_t w_zero_bytes(void *p, uint64_t bytes, hipStream_t s) {
    const uint64_t n16 = bytes / 16;
    if (!n16) return hipSuccess;
    hipLaunchKernelGGL(k_w_zero_bytes, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s, (int8_t *)p, n16);
    return hipGetLastError();
}
}  // namespace

extern "C" size_t fl_reduce_cd32_workspace(const fl_split_info *info, fl_mode mode) {
    if (!info || mode != FL_MFMA_I8 || !info->mD || !info->nB || !info->npiv) return 0;
    return planes_bytes(info->mD, info->npiv) + planes_bytes(info->nB, info->npiv);
}

extern "C" fl_status fl_reduce_cd32(const fl_split_info *info, const fl_split_out32 *s, const uint32_t *X,
                                    uint64_t ldx, uint32_t *Dt, uint64_t ldd, fl_mode mode, void *ws,
                                    size_t ws_bytes, hipStream_t stream) {
    fl_status st = check_info32(info, s);
    if (st != FL_OK) return st;
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_reduce_cd32: bad mode");
    const uint32_t mD = info->mD, nB = info->nB, npiv = info->npiv, w = info->ml_width;
    if (mD == 0 || nB == 0) return FL_OK;
    FL_ARG(Dt && ldd >= nB, "fl_reduce_cd32: NULL Dt or ldd < nB");
    FL_ARG(npiv == 0 || (X && ldx >= nB), "fl_reduce_cd32: NULL X or ldx < nB");
    const size_t need = fl_reduce_cd32_workspace(info, mode);
    if (need && (!ws || ws_bytes < need)) {
        fl_set_error("fl_reduce_cd32: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    const Mod64 md = flw::make_mod64(info->p);
    FL_HIP(w_zero(Dt, ldd, mD, nB, stream));
    hipLaunchKernelGGL(k_w_scatter, dim3((mD + 3) / 4), dim3(256), 0, stream, mD, s->d_ptr, s->d_col, s->d_val, Dt,
                       ldd);
    FL_LAUNCH_CHECK("k_w_scatter");
    if (npiv == 0) return FL_OK;
    if (mode == FL_PLAIN) {
        FL_HIP(w_spmm(md, w, s->c_gptr, s->c_pos, s->c_val, 0, mD, 0, npiv, X, ldx, Dt, ldd, nB, stream));
        return FL_OK;
    }
    const uint64_t kp = pad64(npiv);
    int8_t *Cp = (int8_t *)ws, *Xp = Cp + planes_bytes(mD, npiv);
    FL_HIP(w_zero_bytes(Cp, planes_bytes(mD, npiv), stream));
    hipLaunchKernelGGL(k_w_scatter_limbs, dim3((mD + 3) / 4), dim3(256), 0, stream, info->p, w, mD, s->c_gptr,
                       s->c_pos, s->c_val, Cp, pad64(mD) * kp, kp);
    FL_LAUNCH_CHECK("k_w_scatter_limbs");
    FL_HIP(w_limbs_cols(info->p, X, ldx, npiv, nB, nullptr, Xp, kp, stream));
    FL_HIP(w_gemm4(md, Cp, Xp, mD, nB, kp, nullptr, Dt, ldd, stream));
    return FL_OK;
}

// ================================ step 4 ======================================

namespace {
struct WPanel {
    uint32_t k;               // pivots found in the panel
    uint32_t rank0;           // rank before the panel
    uint32_t Q[kWPanel];      // pivot rows (in pivot column order)
    uint32_t C[kWPanel];      // pivot columns (absolute, ascending)
    uint32_t G[kWPanel * kWPanel];  // D[Q, C]^{-1}
};

struct EchWs32 {
    uint32_t *is_piv;   // [rows]
    uint32_t *W;        // [rows x 64] working copy of the panel
    uint32_t *L;        // [rows x 64] L'
    uint32_t *U;        // [64 x ldu]
    uint32_t *piv_row;  // [min(rows, cols)]
    uint32_t *T;        // [min(rows, cols) x ldu] pivot rows, gathered at the end
    WPanel *ps;
    int8_t *Lp, *Up;    // limb planes of L' and U (MFMA form)
    uint64_t ldu;
};

size_t ech32_layout(uint32_t rows, uint32_t cols, fl_mode mode, void *ws, EchWs32 *e) {
    WsCarve c(ws);
    EchWs32 t = {};
    const uint64_t r1 = rows ? rows : 1, mn = std::max<uint32_t>(std::min(rows, cols), 1);
    t.ldu = pad64(cols ? cols : 1);
    t.is_piv = c.take<uint32_t>(r1);
    t.W = c.take<uint32_t>(r1 * kWPanel);
    t.L = c.take<uint32_t>(r1 * kWPanel);
    t.U = c.take<uint32_t>((uint64_t)kWPanel * t.ldu);
    t.piv_row = c.take<uint32_t>(mn);
    t.T = c.take<uint32_t>(mn * t.ldu);
    t.ps = c.take<WPanel>(1);
    if (mode == FL_MFMA_I8) {
        t.Lp = c.take<int8_t>(planes_bytes(rows, kWPanel));
        t.Up = c.take<int8_t>(planes_bytes(cols, kWPanel));
    }
    if (e) *e = t;
    return c.off;
}

// Pivot search of panel [c0, c0 + pw) in one workgroup (1024 threads):
//  1. W = the panel's columns of every row (rows already pivots excluded);
//  2. for each column j: the lowest remaining row with W[i][j] != 0 is the
//     pivot; its panel part is made monic and column j is cleared from the
//     other remaining rows (row echelon form of the panel, Gauss);
//  3. G = D[Q, C]^{-1} by Gauss-Jordan on the k x k block of the original
//     values (invertible: W[Q, C] is that block times a unit lower
//     triangular matrix, and is itself triangular with a nonzero diagonal).
__global__ __launch_bounds__(1024) void k_w_panel(Mod64 md, uint32_t rows, uint32_t cols, uint32_t c0,
                                                  const uint32_t *__restrict__ D, uint64_t ld, uint32_t *is_piv,
                                                  uint32_t *W, WPanel *ps, uint32_t *d_rank, uint32_t *pivcol,
                                                  uint32_t *piv_row) {
    __shared__ uint32_t prow[kWPanel];
    __shared__ uint32_t s_piv, s_k;
    __shared__ uint32_t Mt[kWPanel][kWPanel + 1], Gt[kWPanel][kWPanel + 1];
    __shared__ uint32_t s_sel;
    const uint32_t tid = threadIdx.x, nt = blockDim.x;
    const uint32_t pw = std::min(kWPanel, cols - c0);
    const uint32_t p = md.p;
    for (uint32_t i = tid; i < rows; i += nt)
        for (uint32_t j = 0; j < pw; j++) W[(uint64_t)i * kWPanel + j] = is_piv[i] ? 0u : D[(uint64_t)i * ld + c0 + j];
    if (tid == 0) s_k = 0;
    __syncthreads();
    for (uint32_t j = 0; j < pw; j++) {
        if (tid == 0) s_piv = 0xffffffffu;
        __syncthreads();
        for (uint32_t i = tid; i < rows; i += nt)
            if (W[(uint64_t)i * kWPanel + j] && !is_piv[i]) {
                atomicMin(&s_piv, i);
                break;  // rows ascend within a thread
            }
        __syncthreads();
        const uint32_t piv = s_piv;
        if (piv == 0xffffffffu) continue;  // (uniform)
        if (tid < pw) {
            const uint32_t inv = flw::invw(W[(uint64_t)piv * kWPanel + j], md);
            prow[tid] = tid >= j ? flw::mulw(W[(uint64_t)piv * kWPanel + tid], inv, md) : 0u;
        }
        __syncthreads();
        for (uint32_t i = tid; i < rows; i += nt) {
            if (i == piv || is_piv[i]) continue;
            uint32_t *wi = W + (uint64_t)i * kWPanel;
            const uint32_t f = wi[j];
            if (!f) continue;
            for (uint32_t jj = j; jj < pw; jj++) wi[jj] = flw::subw(wi[jj], flw::mulw(f, prow[jj], md), p);
        }
        if (tid == 0) {
            ps->Q[s_k] = piv;
            ps->C[s_k] = c0 + j;
            is_piv[piv] = 1;  // read by no thread before the next barrier
            s_k = s_k + 1;
        }
        __syncthreads();
    }
    const uint32_t k = s_k;
    // G = D[Q, C]^{-1}: Gauss-Jordan on [D[Q, C] | I] in LDS, pivoting by row swaps
    for (uint32_t e = tid; e < k * k; e += nt) {
        const uint32_t t = e / k, u = e % k;
        Mt[t][u] = D[(uint64_t)ps->Q[t] * ld + ps->C[u]];
        Gt[t][u] = t == u ? 1u : 0u;
    }
    __syncthreads();
    for (uint32_t u = 0; u < k; u++) {
        if (tid == 0) {
            uint32_t sel = u;
            while (sel < k && Mt[sel][u] == 0) sel++;  // found: the block is invertible
            s_sel = sel < k ? sel : u;
        }
        __syncthreads();
        const uint32_t sel = s_sel;
        if (sel != u && tid < k) {
            uint32_t a = Mt[u][tid], b = Gt[u][tid];
            Mt[u][tid] = Mt[sel][tid];
            Gt[u][tid] = Gt[sel][tid];
            Mt[sel][tid] = a;
            Gt[sel][tid] = b;
        }
        __syncthreads();
        if (tid == 0) s_piv = flw::invw(Mt[u][u], md);
        __syncthreads();
        if (tid < k) {
            Mt[u][tid] = flw::mulw(Mt[u][tid], s_piv, md);
            Gt[u][tid] = flw::mulw(Gt[u][tid], s_piv, md);
        }
        __syncthreads();
        for (uint32_t e = tid; e < k * k; e += nt) {
            const uint32_t t = e / k, v = e % k;
            if (t == u) continue;
            const uint32_t f = Mt[t][u];
            if (!f) continue;
            // (column u of row t is read by the threads of row t before any writes it: f taken first)
            Gt[t][v] = flw::subw(Gt[t][v], flw::mulw(f, Gt[u][v], md), p);
        }
        __syncthreads();
        for (uint32_t e = tid; e < k * k; e += nt) {
            const uint32_t t = e / k, v = e % k;
            if (t == u || v == u) continue;
            Mt[t][v] = flw::subw(Mt[t][v], flw::mulw(Mt[t][u], Mt[u][v], md), p);
        }
        __syncthreads();
        if (tid < k && tid != u) Mt[tid][u] = 0;
        __syncthreads();
    }
    for (uint32_t e = tid; e < k * k; e += nt) ps->G[(e / k) * kWPanel + e % k] = Gt[e / k][e % k];
    if (tid == 0) {
        const uint32_t r0 = *d_rank;
        ps->k = k;
        ps->rank0 = r0;
        for (uint32_t t = 0; t < k; t++) {
            pivcol[r0 + t] = ps->C[t];
            piv_row[r0 + t] = ps->Q[t];
        }
        *d_rank = r0 + k;
    }
}

// U[t][c] = sum_s G[t][s] D[Q_s][c0 + c], t < k, for the columns right of c0.
__global__ __launch_bounds__(256) void k_w_U(Mod64 md, uint32_t ncols, uint32_t c0, const uint32_t *__restrict__ D,
                                             uint64_t ld, const WPanel *__restrict__ ps, uint32_t *U, uint64_t ldu) {
    __shared__ uint32_t G[kWPanel * kWPanel];
    const uint32_t k = ps->k;
    for (uint32_t e = threadIdx.x; e < k * kWPanel; e += blockDim.x) G[e] = ps->G[e];
    __syncthreads();
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncols || !k) return;
    uint32_t x[kWPanel];
#pragma unroll
    for (uint32_t s = 0; s < kWPanel; s++) x[s] = s < k ? D[(uint64_t)ps->Q[s] * ld + c0 + c] : 0u;
    for (uint32_t t = 0; t < k; t++) {
        uint64_t acc = 0;
#pragma unroll
        for (uint32_t s = 0; s < kWPanel; s++) flw::macw(acc, G[t * kWPanel + s], x[s], md);
        U[(uint64_t)t * ldu + c] = flw::reduce64(acc, md);
    }
}

// L'[i][t] = D[i][C_t] - [i = Q_t] (zero for t >= k), every row.
__global__ void k_w_L(uint32_t p, uint32_t rows, const uint32_t *__restrict__ D, uint64_t ld,
                      const WPanel *__restrict__ ps, uint32_t *L) {
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6), t = threadIdx.x & 63;
    if (i >= rows) return;
    const uint32_t k = ps->k;
    uint32_t v = 0;
    if (t < k) {
        v = D[(uint64_t)i * ld + ps->C[t]];
        if (ps->Q[t] == i) v = flw::subw(v, 1u % p, p);
    }
    L[(uint64_t)i * kWPanel + t] = v;
}

// D[i][c0 + c] -= sum_t L'[i][t] U[t][c] (plain form); rows whose L' is zero
// are left alone.
__global__ __launch_bounds__(256) void k_w_update(Mod64 md, uint32_t ncols, uint32_t c0, uint32_t *D, uint64_t ld,
                                                  const uint32_t *__restrict__ L, const uint32_t *__restrict__ U,
                                                  uint64_t ldu, const WPanel *__restrict__ ps) {
    __shared__ uint32_t l[kWPanel];
    __shared__ uint32_t any;
    const uint32_t i = blockIdx.y;
    const uint32_t k = ps->k;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    if (threadIdx.x < kWPanel) {
        l[threadIdx.x] = L[(uint64_t)i * kWPanel + threadIdx.x];
        if (threadIdx.x < k && l[threadIdx.x]) atomicOr(&any, 1u);
    }
    __syncthreads();
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (!any || c >= ncols) return;
    uint64_t acc = 0;
    for (uint32_t t = 0; t < k; t++)
        if (l[t]) flw::macw(acc, md.p - l[t], U[(uint64_t)t * ldu + c], md);
    uint32_t *o = D + (uint64_t)i * ld + c0 + c;
    *o = flw::addw(*o, flw::reduce64(acc, md), md.p);
}

// After the last panel: pivot rows (piv_row, in pivot order) to rows 0..r-1,
// the other rows zero.  Two passes through T.
__global__ void k_w_gather_rows(uint32_t cols, const uint32_t *__restrict__ D, uint64_t ld,
                                const uint32_t *__restrict__ d_rank, const uint32_t *__restrict__ piv_row, uint32_t *T,
                                uint64_t ldt) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const uint32_t r = *d_rank;
    for (uint32_t t = blockIdx.y; t < r; t += gridDim.y) T[(uint64_t)t * ldt + c] = D[(uint64_t)piv_row[t] * ld + c];
}
__global__ void k_w_place_rows(uint32_t rows, uint32_t cols, uint32_t *D, uint64_t ld,
                               const uint32_t *__restrict__ d_rank, const uint32_t *__restrict__ T, uint64_t ldt) {
    const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const uint32_t r = *d_rank;
    for (uint32_t i = blockIdx.y; i < rows; i += gridDim.y) D[(uint64_t)i * ld + c] = i < r ? T[(uint64_t)i * ldt + c] : 0u;
}
}  // namespace

extern "C" size_t fl_echelon_d32_workspace(uint32_t rows, uint32_t cols, fl_mode mode) {
    return ech32_layout(rows, cols, mode, nullptr, nullptr);
}

extern "C" fl_status fl_echelon_d32(uint32_t p, uint32_t rows, uint32_t cols, uint32_t *Dt, uint64_t ldd,
                                    uint32_t *d_rank, uint32_t *d_pivcol, fl_mode mode, void *ws, size_t ws_bytes,
                                    hipStream_t stream) {
    FL_ARG(p >= 2, "fl_echelon_d32: p must be >= 2");
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_echelon_d32: bad mode");
    FL_ARG(d_rank, "fl_echelon_d32: NULL d_rank");
    FL_ARG(rows < (1u << 31) && cols < (1u << 31), "fl_echelon_d32: dimensions must be < 2^31");
    FL_HIP(fl_fill_u32(d_rank, 0, 1, stream));
    if (rows == 0 || cols == 0) return FL_OK;
    FL_ARG(Dt && d_pivcol && ldd >= cols, "fl_echelon_d32: NULL array or ldd < cols");
    EchWs32 e;
    const size_t need = ech32_layout(rows, cols, mode, ws, &e);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_echelon_d32: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    const Mod64 md = flw::make_mod64(p);
    FL_HIP(fl_fill_u32(e.is_piv, 0, rows, stream));
    const uint32_t mn = std::min(rows, cols);
    const uint64_t kp = kWPanel;
    for (uint32_t c0 = 0; c0 < cols; c0 += kWPanel) {
        hipLaunchKernelGGL(k_w_panel, dim3(1), dim3(1024), 0, stream, md, rows, cols, c0, (const uint32_t *)Dt, ldd,
                           e.is_piv, e.W, e.ps, d_rank, d_pivcol, e.piv_row);
        FL_LAUNCH_CHECK("k_w_panel");
        const uint32_t nc = cols - c0;
        hipLaunchKernelGGL(k_w_U, dim3((nc + 255) / 256), dim3(256), 0, stream, md, nc, c0, (const uint32_t *)Dt, ldd,
                           (const WPanel *)e.ps, e.U, e.ldu);
        FL_LAUNCH_CHECK("k_w_U");
        hipLaunchKernelGGL(k_w_L, dim3((rows + 3) / 4), dim3(256), 0, stream, p, rows, (const uint32_t *)Dt, ldd,
                           (const WPanel *)e.ps, e.L);
        FL_LAUNCH_CHECK("k_w_L");
        if (mode == FL_MFMA_I8) {
            FL_HIP(w_limbs_rows(p, e.L, kWPanel, rows, kWPanel, nullptr, e.Lp, kp, stream));
            FL_HIP(w_limbs_cols(p, e.U, e.ldu, kWPanel, nc, nullptr, e.Up, kp, stream));
            FL_HIP(w_gemm4(md, e.Lp, e.Up, rows, nc, kp, nullptr, Dt + c0, ldd, stream));
        } else {
            for (uint32_t y = 0; y < rows; y += 65535) {
                const uint32_t ny = std::min(rows - y, 65535u);
                hipLaunchKernelGGL(k_w_update, dim3((nc + 255) / 256, ny), dim3(256), 0, stream, md, nc, c0,
                                   Dt + (uint64_t)y * ldd, ldd, (const uint32_t *)(e.L + (uint64_t)y * kWPanel),
                                   (const uint32_t *)e.U, e.ldu, (const WPanel *)e.ps);
                FL_LAUNCH_CHECK("k_w_update");
            }
        }
    }
    const unsigned gx = (cols + 255) / 256;
    hipLaunchKernelGGL(k_w_gather_rows, dim3(gx, std::min(mn, 4096u)), dim3(256), 0, stream, cols,
                       (const uint32_t *)Dt, ldd, (const uint32_t *)d_rank, (const uint32_t *)e.piv_row, e.T, e.ldu);
    FL_LAUNCH_CHECK("k_w_gather_rows");
    hipLaunchKernelGGL(k_w_place_rows, dim3(gx, std::min(rows, 4096u)), dim3(256), 0, stream, rows, cols, Dt, ldd,
                       (const uint32_t *)d_rank, (const uint32_t *)e.T, e.ldu);
    FL_LAUNCH_CHECK("k_w_place_rows");
    return FL_OK;
}

// ============================ second pass =====================================

namespace {
// L[i][t] = X[i][pivcol[t]] for t < r, zero for r <= t < kmax.
__global__ void k_w_gather_pivcols(const uint32_t *__restrict__ X, uint64_t ldx, uint32_t npiv,
                                   const uint32_t *__restrict__ d_rank, const uint32_t *__restrict__ pivcol,
                                   uint32_t kmax, uint32_t *L, uint64_t ldl) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kmax) return;
    const uint32_t r = *d_rank;
    const uint32_t c = t < r ? pivcol[t] : 0;
    for (uint32_t i = blockIdx.y; i < npiv; i += gridDim.y) L[(uint64_t)i * ldl + t] = t < r ? X[(uint64_t)i * ldx + c] : 0u;
}

struct Rref32Ws {
    uint32_t *L;
    uint64_t ldl;
    int8_t *Lp, *Rp;
    uint64_t kp;
};

size_t rref32_layout(const fl_split_info *info, fl_mode mode, void *ws, Rref32Ws *o) {
    WsCarve c(ws);
    Rref32Ws t = {};
    const uint32_t maxr = std::min(info->mD, info->nB);
    t.ldl = pad64(maxr ? maxr : 1);
    t.kp = t.ldl;
    t.L = c.take<uint32_t>((uint64_t)(info->npiv ? info->npiv : 1) * t.ldl);
    if (mode == FL_MFMA_I8) {
        t.Lp = c.take<int8_t>(planes_bytes(info->npiv, t.kp));
        t.Rp = c.take<int8_t>(planes_bytes(info->nB, t.kp));
    }
    if (o) *o = t;
    return c.off;
}
}  // namespace

extern "C" size_t fl_rref32_workspace(const fl_split_info *info, fl_mode mode) {
    return info ? rref32_layout(info, mode, nullptr, nullptr) : 0;
}

extern "C" fl_status fl_rref32(const fl_split_info *info, const fl_split_out32 *s, uint32_t *X, uint64_t ldx,
                               const uint32_t *RD, uint64_t ldd, const uint32_t *d_rank, const uint32_t *d_pivcol,
                               fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream) {
    fl_status st = check_info32(info, s);
    if (st != FL_OK) return st;
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_rref32: bad mode");
    const uint32_t npiv = info->npiv, nB = info->nB, maxr = std::min(info->mD, nB);
    if (npiv == 0 || nB == 0 || maxr == 0) return FL_OK;
    FL_ARG(X && RD && d_rank && d_pivcol && ldx >= nB && ldd >= nB, "fl_rref32: NULL array or small ld");
    Rref32Ws r;
    const size_t need = rref32_layout(info, mode, ws, &r);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_rref32: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    const Mod64 md = flw::make_mod64(info->p);
    hipLaunchKernelGGL(k_w_gather_pivcols, dim3((unsigned)((r.ldl + 255) / 256), std::min(npiv, 4096u)), dim3(256), 0,
                       stream, (const uint32_t *)X, ldx, npiv, d_rank, d_pivcol, (uint32_t)r.ldl, r.L, r.ldl);
    FL_LAUNCH_CHECK("k_w_gather_pivcols");
    if (mode == FL_MFMA_I8) {
        FL_HIP(w_limbs_rows(info->p, r.L, r.ldl, npiv, (uint32_t)r.ldl, d_rank, r.Lp, r.kp, stream));
        FL_HIP(w_limbs_cols(info->p, RD, ldd, maxr, nB, d_rank, r.Rp, r.kp, stream));
        FL_HIP(w_gemm4(md, r.Lp, r.Rp, npiv, nB, r.kp, d_rank, X, ldx, stream));
    } else {
        FL_HIP(w_gemm_plain(md, r.L, r.ldl, RD, ldd, npiv, nB, maxr, d_rank, X, ldx, stream));
    }
    return FL_OK;
}

// =============================== read-off =====================================

namespace {
// Output position of every row of RREF(M): top row a (pivot col_perm[a]) or
// Schur row b (pivot col_perm[npiv + pivcol[b]]) goes after the rows of the
// other kind whose pivot column is smaller (both lists ascend).
__device__ uint32_t count_below(const uint32_t *list, uint32_t n, uint32_t x, const uint32_t *map, uint32_t off) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        const uint32_t v = map ? map[off + list[mid]] : list[mid];
        if (v < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void row_source(uint32_t j, uint32_t npiv, uint32_t r, const uint32_t *col_perm,
                                           const uint32_t *pivcol, const uint32_t *Xp, uint64_t ldx,
                                           const uint32_t *RD, uint64_t ldd, uint32_t &out_pos, uint32_t &lead,
                                           const uint32_t *&src, bool &top) {
    top = j < npiv;
    if (top) {
        lead = col_perm[j];
        out_pos = j + count_below(pivcol, r, lead, col_perm, npiv);
        src = Xp + (uint64_t)j * ldx;
    } else {
        const uint32_t b = j - npiv;
        lead = col_perm[npiv + pivcol[b]];
        out_pos = b + count_below(col_perm, npiv, lead, nullptr, 0);
        src = RD + (uint64_t)b * ldd;
    }
}

// Nonzeros of every output row (one wave per row j of [X'; R_D]): cnt at the
// row's output position.
__global__ void k_w_csr_count(uint32_t npiv, uint32_t nB, const uint32_t *__restrict__ col_perm,
                              const uint32_t *__restrict__ Xp, uint64_t ldx, const uint32_t *__restrict__ RD,
                              uint64_t ldd, const uint32_t *__restrict__ d_rank, const uint32_t *__restrict__ pivcol,
                              uint64_t *cnt) {
    const uint32_t j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = lane_id();
    const uint32_t r = d_rank ? *d_rank : 0;
    if (j >= npiv + r) return;
    uint32_t pos, lead;
    const uint32_t *src;
    bool top;
    row_source(j, npiv, r, col_perm, pivcol, Xp, ldx, RD, ldd, pos, lead, src, top);
    uint32_t n = 0;
    for (uint32_t c = lane; c < nB; c += 64) n += src[c] != 0;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) n += __shfl_xor(n, off, 64);
    if (lane == 0) cnt[pos] = n + (top ? 1 : 0);
}

// Entries of every output row in original column order: the columns of the
// non-pivot part ascend with c (col_perm ascends on the non-pivot columns);
// a top row's unit goes before the entries whose column is larger.
__global__ void k_w_csr_emit(uint32_t npiv, uint32_t nB, const uint32_t *__restrict__ col_perm,
                             const uint32_t *__restrict__ Xp, uint64_t ldx, const uint32_t *__restrict__ RD,
                             uint64_t ldd, const uint32_t *__restrict__ d_rank, const uint32_t *__restrict__ pivcol,
                             const uint64_t *__restrict__ row_ptr, uint32_t *col, uint32_t *val) {
    const uint32_t j = blockIdx.x * 4 + (threadIdx.x >> 6), lane = lane_id();
    const uint32_t r = d_rank ? *d_rank : 0;
    if (j >= npiv + r) return;
    uint32_t pos, lead;
    const uint32_t *src;
    bool top;
    row_source(j, npiv, r, col_perm, pivcol, Xp, ldx, RD, ldd, pos, lead, src, top);
    uint64_t out = row_ptr[pos];
    bool unit = top;  // the unit is still to be placed
    for (uint32_t c0 = 0; c0 < nB; c0 += 64) {
        const uint32_t c = c0 + lane;
        const uint32_t x = c < nB ? src[c] : 0u;
        const uint32_t oc = c < nB ? col_perm[npiv + c] : 0xffffffffu;
        if (unit) {  // wave-uniform
            const uint64_t before = __ballot(x != 0 && oc < lead);
            const uint64_t any_after = __ballot(c < nB && oc > lead);
            if (any_after) {
                // the unit sits after this chunk's entries left of it
                const uint32_t nb = (uint32_t)__popcll(before);
                const uint32_t rank_in = (uint32_t)__popcll(before & ((1ull << lane) - 1));
                if (x != 0 && oc < lead) {
                    col[out + rank_in] = oc;
                    val[out + rank_in] = x;
                }
                if (lane == 0) {
                    col[out + nb] = lead;
                    val[out + nb] = 1;
                }
                out += nb + 1;
                unit = false;
                const uint64_t rest = __ballot(x != 0 && oc > lead);
                const uint32_t rk = (uint32_t)__popcll(rest & ((1ull << lane) - 1));
                if (x != 0 && oc > lead) {
                    col[out + rk] = oc;
                    val[out + rk] = x;
                }
                out += (uint32_t)__popcll(rest);
                continue;
            }
        }
        const uint64_t m = __ballot(x != 0);
        const uint32_t rk = (uint32_t)__popcll(m & ((1ull << lane) - 1));
        if (x != 0) {
            col[out + rk] = oc;
            val[out + rk] = x;
        }
        out += (uint32_t)__popcll(m);
    }
    if (unit && lane == 0) {
        col[out] = lead;
        val[out] = 1;
    }
}

struct Csr32Ws {
    uint64_t *cnt, *scantmp, *dinfo;
};
size_t csr32_layout(uint32_t npiv, uint32_t maxr, void *ws, Csr32Ws *o) {
    WsCarve c(ws);
    Csr32Ws t;
    const size_t n = (size_t)npiv + maxr + 1;
    t.cnt = c.take<uint64_t>(n);
    t.scantmp = c.take<uint64_t>(fl_scan_tmp_elems(n));
    t.dinfo = c.take<uint64_t>(4);
    if (o) *o = t;
    return c.off;
}
}  // namespace

extern "C" size_t fl_rref32_csr_workspace(const fl_split_info *info) {
    return info ? csr32_layout(info->npiv, std::min(info->mD, info->nB), nullptr, nullptr) : 0;
}

extern "C" fl_status fl_rref32_csr_size(const fl_split_info *info, const fl_split_out32 *s, const uint32_t *Xp,
                                        uint64_t ldx, const uint32_t *RD, uint64_t ldd, const uint32_t *d_rank,
                                        const uint32_t *d_pivcol, uint64_t *row_ptr, uint32_t *h_rank,
                                        uint64_t *h_nnz, void *ws, size_t ws_bytes, hipStream_t stream) {
    fl_status st = check_info32(info, s);
    if (st != FL_OK) return st;
    FL_ARG(row_ptr && h_rank && h_nnz, "fl_rref32_csr_size: NULL argument");
    const uint32_t npiv = info->npiv, nB = info->nB, maxr = std::min(info->mD, nB);
    FL_ARG(npiv == 0 || nB == 0 || (Xp && ldx >= nB), "fl_rref32_csr_size: bad X'");
    FL_ARG(maxr == 0 || (RD && d_rank && d_pivcol && ldd >= nB), "fl_rref32_csr_size: bad R_D");
    Csr32Ws c;
    const size_t need = csr32_layout(npiv, maxr, ws, &c);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_rref32_csr_size: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    const size_t n = (size_t)npiv + maxr;
    FL_HIP(fl_fill_u64(c.cnt, 0, n + 1, stream));
    if (n) {
        hipLaunchKernelGGL(k_w_csr_count, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, npiv, nB,
                           (const uint32_t *)s->col_perm, Xp, ldx, RD, ldd, maxr ? d_rank : nullptr, d_pivcol, c.cnt);
        FL_LAUNCH_CHECK("k_w_csr_count");
    }
    FL_HIP(fl_exclusive_scan_u64(c.cnt, row_ptr, n + 1, c.scantmp, c.dinfo, stream));
    uint32_t r = 0;
    uint64_t tot = 0;
    if (maxr) FL_HIP(hipMemcpyAsync(&r, d_rank, sizeof(r), hipMemcpyDeviceToHost, stream));
    FL_HIP(hipMemcpyAsync(&tot, c.dinfo, sizeof(tot), hipMemcpyDeviceToHost, stream));
    FL_HIP(hipStreamSynchronize(stream));
    *h_rank = npiv + r;
    *h_nnz = tot;
    return FL_OK;
}

extern "C" fl_status fl_rref32_to_csr(const fl_split_info *info, const fl_split_out32 *s, const uint32_t *Xp,
                                      uint64_t ldx, const uint32_t *RD, uint64_t ldd, const uint32_t *d_rank,
                                      const uint32_t *d_pivcol, const uint64_t *row_ptr, uint32_t *col, uint32_t *val,
                                      void *ws, size_t ws_bytes, hipStream_t stream) {
    (void)ws;
    (void)ws_bytes;
    fl_status st = check_info32(info, s);
    if (st != FL_OK) return st;
    const uint32_t npiv = info->npiv, nB = info->nB, maxr = std::min(info->mD, nB);
    const size_t n = (size_t)npiv + maxr;
    if (n == 0) return FL_OK;
    FL_ARG(row_ptr && col && val, "fl_rref32_to_csr: NULL argument");
    hipLaunchKernelGGL(k_w_csr_emit, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, stream, npiv, nB,
                       (const uint32_t *)s->col_perm, Xp, ldx, RD, ldd, maxr ? d_rank : nullptr, d_pivcol, row_ptr,
                       col, val);
    FL_LAUNCH_CHECK("k_w_csr_emit");
    return FL_OK;
}
