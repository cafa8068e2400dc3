// echelon.hip -- FL step 4 (paper Sec. 4.1 step 4, Sec. 4.4), read as the
// reduced row echelon form of the dense Schur complement Dt, computed by
// blocked Gauss-Jordan elimination over 64-column panels.
//
// For a panel [c0, c0+64):
//  1. k_ech_greedy<false>  one block per chunk of 1024 rows: the chunk's rows
//     that are independent on the panel columns (a greedy basis in reduced
//     form kept in LDS; every wave reduces one row against the basis with
//     v_readlane broadcasts, insertions are serialised) -> candidate rows.
//  2. k_ech_greedy<true>   one block: the same over all candidates, tracking
//     the coefficients G with  G * Dt[Q, panel] = RREF(Dt[Q, panel]),
//     Q = selected rows.  This yields the panel's pivot columns C (ascending)
//     and G = Dt[Q, C]^{-1} (rows ordered by pivot column).
//     This plays the role of the paper's parallel structured Gaussian
//     elimination (Sec. 5.1: rows reduced in parallel against the known
//     pivots, a new pivot added only by one worker at a time).
//  3. k_ech_U              U = G * Dt[Q, c0:]   (unit vectors at C)
//  4. k_ech_gather_L       L = Dt[:, C]          (multipliers, saved before
//                                                 the update overwrites them)
//  5. fl_gemm_sub_plain    Dt[:, c0:] -= L U    (every row: Gauss-Jordan
//     (or the int8 MFMA form)                   clears C above and below)
//  6. k_ech_setq           Dt[Q_t, c0:] = U_t
// After the last panel the pivot rows are gathered to rows 0..r-1 in pivot
// order and the other rows (now zero) are cleared.
#include "fl_internal.h"

hipError_t fl_gemm_sub_plain(uint32_t p, uint32_t M, uint32_t N, uint32_t Kh, const uint32_t *Kdev,
                             const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                             uint16_t *C, uint64_t ldc, hipStream_t s, const char *site);
hipError_t fl_gemm_sub_mfma(uint32_t p, uint32_t M, uint32_t N, uint32_t Kmax, const uint32_t *Kdev,
                            const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                            uint16_t *C, uint64_t ldc, void *ws, size_t ws_bytes, hipStream_t s,
                            const char *site);
size_t fl_gemm_sub_mfma_ws(uint32_t M, uint32_t N, uint32_t Kmax);

namespace {

constexpr uint32_t kPanel = 64;
constexpr uint32_t kChunk = 1024;
constexpr int kGreedyThreads = 1024;

struct PanelState {
    uint32_t k;            // pivots found in this panel
    uint32_t pad[3];
    uint32_t Qs[64];       // selected rows, by insertion slot
    uint32_t Phys[64];     // row that receives U_t
    uint32_t Ccol[64];     // absolute pivot column of U_t (ascending)
    uint16_t G[64 * 64];   // G[t][s]: U_t = sum_s G[t][s] Dt[Qs[s]]
};

struct EchWs {
    uint32_t *is_piv;   // [rows] 1 once the row is a pivot row
    uint32_t *piv_row;  // [min(rows, cols)]
    uint32_t *cand;     // [nchunks * 64]
    uint32_t *cand_cnt; // [nchunks]
    PanelState *ps;
    uint16_t *U;        // [64 x ldu]
    uint16_t *L;        // [rows x 64]
    uint16_t *T;        // [min(rows, cols) x ldu]
    void *gemm_ws;
    size_t gemm_ws_bytes;
    uint64_t ldu;
};

// Reduce the wave's vector (v: panel part, g: coefficient part, lane = column
// or slot) against basis rows [t0, t1).  The basis is in reduced form, so all
// multipliers can be read from the vector as it is on entry.
__device__ inline void reduce_against(const fl::Mod &md, uint32_t &v, uint32_t &g, uint32_t t0,
                                      uint32_t t1, const uint16_t (*Bv)[64],
                                      const uint16_t (*Bg)[64], const uint32_t *Cc, uint32_t lane,
                                      bool track) {
    uint32_t vh = 0, vl = 0, gh = 0, gl = 0;
    const uint32_t vin = v;
    for (uint32_t t = t0; t < t1; t++) {
        int cidx = __builtin_amdgcn_readfirstlane((int)Cc[t]);
        uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)vin, cidx);
        if (lam == 0) continue;
        uint32_t lh = lam >> 8, ll = lam & 0xffu;
        uint32_t b = Bv[t][lane];
        vh = fl::mad24(lh, b, vh);
        vl = fl::mad24(ll, b, vl);
        if (track) {
            uint32_t bg = Bg[t][lane];
            gh = fl::mad24(lh, bg, gh);
            gl = fl::mad24(ll, bg, gl);
        }
    }
    // at most 64 terms: no intermediate fold needed
    v = fl::submod(v, fl::fold_pair(vh, vl, md), md.p);
    if (track) g = fl::submod(g, fl::fold_pair(gh, gl, md), md.p);
}

template <bool MERGE>
__global__ __launch_bounds__(kGreedyThreads) void k_ech_greedy(
    fl::Mod md, const uint16_t *__restrict__ D, uint64_t ld, uint32_t rows, uint32_t c0,
    uint32_t pw, uint32_t *is_piv, uint32_t *cand, uint32_t *cand_cnt, uint32_t nchunks,
    PanelState *ps, uint32_t *piv_row, uint32_t *piv_col, uint32_t *d_rank) {
    __shared__ uint16_t Bv[64][64];
    __shared__ uint16_t Bg[64][64];
    __shared__ uint32_t Cc[64];
    __shared__ uint32_t Qo[64];
    __shared__ uint32_t kb_s;
    __shared__ uint32_t list_s[64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    if (threadIdx.x == 0) kb_s = 0;
    __syncthreads();

    // Work list: LOCAL = rows of chunk blockIdx.x; MERGE = candidates of all
    // chunks, in chunk order.
    const uint32_t nlists = MERGE ? nchunks : 1;
    for (uint32_t li = 0; li < nlists; li++) {
        uint32_t lo, cnt;
        if (MERGE) {
            cnt = cand_cnt[li];
            if (threadIdx.x < cnt) list_s[threadIdx.x] = cand[li * 64 + threadIdx.x];
            __syncthreads();
            lo = 0;
        } else {
            lo = blockIdx.x * kChunk;
            cnt = lo < rows ? (rows - lo < kChunk ? rows - lo : kChunk) : 0;
        }
        for (uint32_t base = 0; base < cnt; base += nw) {
            if (kb_s >= pw) break;  // panel full: every further row reduces to 0
            uint32_t item = base + wave;
            uint32_t row = 0xffffffffu;
            if (item < cnt) {
                row = MERGE ? list_s[item] : lo + item;
                if (!MERGE && is_piv[row]) row = 0xffffffffu;
            }
            const bool have = row != 0xffffffffu;
            uint32_t v = (have && lane < pw) ? D[(uint64_t)row * ld + c0 + lane] : 0;
            uint32_t g = 0;
            const uint32_t ks = kb_s;
            reduce_against(md, v, g, 0, ks, Bv, Bg, Cc, lane, MERGE);
            bool nz = have && __ballot(v != 0) != 0;
            int any = __syncthreads_or(nz ? 1 : 0);
            if (any) {
                for (uint32_t w = 0; w < nw; w++) {
                    if (w == wave && nz) {
                        const uint32_t kb = kb_s;
                        reduce_against(md, v, g, ks, kb, Bv, Bg, Cc, lane, MERGE);
                        uint64_t mask = __ballot(v != 0);
                        if (mask != 0 && kb < pw) {
                            const int c = __ffsll((long long)mask) - 1;
                            if (lane == kb) g = 1;
                            uint32_t piv = (uint32_t)__builtin_amdgcn_readlane((int)v, c);
                            uint32_t inv = fl::invmod(piv, md);
                            v = fl::mulmod(v, inv, md);
                            g = fl::mulmod(g, inv, md);
                            for (uint32_t t = 0; t < kb; t++) {
                                uint32_t f = Bv[t][c];
                                if (f) {
                                    Bv[t][lane] = (uint16_t)fl::submod(Bv[t][lane], fl::mulmod(f, v, md), md.p);
                                    Bg[t][lane] = (uint16_t)fl::submod(Bg[t][lane], fl::mulmod(f, g, md), md.p);
                                }
                            }
                            Bv[kb][lane] = (uint16_t)v;
                            Bg[kb][lane] = (uint16_t)g;
                            if (lane == 0) {
                                Cc[kb] = (uint32_t)c;
                                Qo[kb] = row;
                                kb_s = kb + 1;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
        }
        __syncthreads();
    }

    const uint32_t kb = kb_s;
    if (!MERGE) {
        if (threadIdx.x < kb) cand[blockIdx.x * 64 + threadIdx.x] = Qo[threadIdx.x];
        if (threadIdx.x == 0) cand_cnt[blockIdx.x] = kb;
        return;
    }
    if (wave != 0) return;
    // order basis rows by pivot column
    uint32_t my_t = 0;
    if (lane < kb) {
        uint32_t cj = Cc[lane];
        for (uint32_t j = 0; j < kb; j++) my_t += Cc[j] < cj ? 1 : 0;
    }
    const uint32_t rank0 = *d_rank;
    for (uint32_t j = 0; j < kb; j++) {
        uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)my_t, (int)j);
        ps->G[t * 64 + lane] = lane < kb ? Bg[j][lane] : 0;
    }
    if (lane < kb) {
        const uint32_t t = my_t;
        ps->Qs[lane] = Qo[lane];
        ps->Phys[t] = Qo[lane];
        ps->Ccol[t] = c0 + Cc[lane];
        piv_row[rank0 + t] = Qo[lane];
        piv_col[rank0 + t] = c0 + Cc[lane];
        is_piv[Qo[lane]] = 1;  // later panels skip this row
    }
    if (lane == 0) {
        ps->k = kb;
        *d_rank = rank0 + kb;
    }
}

// U[t][c] = sum_s G[t][s] Dt[Qs[s]][c] for c in [c0, cols), t < k.
__global__ __launch_bounds__(256) void k_ech_U(fl::Mod md, const uint16_t *__restrict__ D,
                                               uint64_t ld, uint32_t c0, uint32_t cols,
                                               const PanelState *__restrict__ ps, uint16_t *U,
                                               uint64_t ldu) {
    __shared__ uint16_t Gs[64 * 64];
    __shared__ uint16_t xs[64][256];
    const uint32_t k = ps->k;
    if (k == 0) return;
    for (uint32_t i = threadIdx.x; i < 64 * 64; i += blockDim.x) Gs[i] = ps->G[i];
    const uint32_t c = c0 + blockIdx.x * 256 + threadIdx.x;
    const bool ok = c < cols;
    for (uint32_t s = 0; s < k; s++) xs[s][threadIdx.x] = ok ? D[(uint64_t)ps->Qs[s] * ld + c] : 0;
    __syncthreads();
    if (!ok) return;
    for (uint32_t t = 0; t < k; t++) {
        uint32_t h = 0, l = 0;
        for (uint32_t s = 0; s < k; s++) {
            uint32_t gts = Gs[t * 64 + s];
            uint32_t x = xs[s][threadIdx.x];
            h = fl::mad24(gts >> 8, x, h);
            l = fl::mad24(gts & 0xffu, x, l);
        }
        U[(uint64_t)t * ldu + c] = (uint16_t)fl::fold_pair(h, l, md);
    }
}

// L[i][t] = Dt[i][Ccol[t]] (0 for t >= k).
__global__ __launch_bounds__(256) void k_ech_gather_L(const uint16_t *__restrict__ D, uint64_t ld,
                                                      uint32_t rows,
                                                      const PanelState *__restrict__ ps,
                                                      uint16_t *L) {
    const uint32_t t = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= rows) return;
    const uint32_t k = ps->k;
    L[(uint64_t)i * 64 + t] = t < k ? D[(uint64_t)i * ld + ps->Ccol[t]] : 0;
}

// Rows of Q receive U (after the rank-k update touched them).
__global__ __launch_bounds__(256) void k_ech_setq(uint16_t *D, uint64_t ld, uint32_t c0,
                                                  uint32_t cols, const PanelState *__restrict__ ps,
                                                  const uint16_t *__restrict__ U, uint64_t ldu) {
    const uint32_t t = blockIdx.y;
    if (t >= ps->k) return;
    const uint32_t row = ps->Phys[t];
    for (uint32_t c = c0 + blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += gridDim.x * blockDim.x)
        D[(uint64_t)row * ld + c] = U[(uint64_t)t * ldu + c];
}

// Final placement: T[t] = Dt[piv_row[t]] for t < rank, then Dt[t] = T[t] and
// the remaining rows are cleared.
__global__ __launch_bounds__(256) void k_ech_gather_rows(const uint16_t *__restrict__ D, uint64_t ld,
                                                         uint32_t cols, const uint32_t *__restrict__ piv_row,
                                                         const uint32_t *__restrict__ d_rank,
                                                         uint16_t *T, uint64_t ldt) {
    const uint32_t r = *d_rank;
    for (uint32_t t = blockIdx.y; t < r; t += gridDim.y) {
        const uint32_t src = piv_row[t];
        for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += gridDim.x * blockDim.x)
            T[(uint64_t)t * ldt + c] = D[(uint64_t)src * ld + c];
    }
}

__global__ __launch_bounds__(256) void k_ech_place_rows(uint16_t *D, uint64_t ld, uint32_t rows,
                                                        uint32_t cols,
                                                        const uint32_t *__restrict__ d_rank,
                                                        const uint16_t *__restrict__ T, uint64_t ldt) {
    const uint32_t r = *d_rank;
    for (uint32_t i = blockIdx.y; i < rows; i += gridDim.y) {
        for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += gridDim.x * blockDim.x)
            D[(uint64_t)i * ld + c] = i < r ? T[(uint64_t)i * ldt + c] : 0;
    }
}

size_t ech_layout(uint32_t rows, uint32_t cols, fl_mode mode, void *ws, EchWs *e) {
    WsCarve c(ws);
    const uint32_t mn = rows < cols ? rows : cols;
    const uint32_t nchunks = (rows + kChunk - 1) / kChunk;
    const uint64_t ldu = ((uint64_t)cols + 63) & ~(uint64_t)63;
    EchWs t;
    t.is_piv = c.take<uint32_t>(rows ? rows : 1);
    t.piv_row = c.take<uint32_t>(mn ? mn : 1);
    t.cand = c.take<uint32_t>((size_t)(nchunks ? nchunks : 1) * 64);
    t.cand_cnt = c.take<uint32_t>(nchunks ? nchunks : 1);
    t.ps = c.take<PanelState>(1);
    t.U = c.take<uint16_t>((size_t)64 * ldu);
    t.L = c.take<uint16_t>((size_t)(rows ? rows : 1) * 64);
    t.T = c.take<uint16_t>((size_t)(mn ? mn : 1) * ldu);
    t.ldu = ldu;
    t.gemm_ws_bytes = mode == FL_MFMA_I8 ? fl_gemm_sub_mfma_ws(rows, cols, 64) : 0;
    t.gemm_ws = t.gemm_ws_bytes ? (void *)c.take<char>(t.gemm_ws_bytes) : nullptr;
    if (e) *e = t;
    return c.off;
}

}  // namespace

extern "C" size_t fl_echelon_d_workspace(uint32_t rows, uint32_t cols, fl_mode mode) {
    return ech_layout(rows, cols, mode, nullptr, nullptr);
}

extern "C" fl_status fl_echelon_d(uint32_t p, uint32_t rows, uint32_t cols, uint16_t *Dt,
                                  uint64_t ldd, uint32_t *d_rank, uint32_t *d_pivcol, fl_mode mode,
                                  void *ws, size_t ws_bytes, hipStream_t stream) {
    FL_ARG(p >= 2 && p <= 65521, "fl_echelon_d: p must be in [2, 65521]");
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_echelon_d: bad mode");
    FL_ARG(d_rank, "fl_echelon_d: NULL d_rank");
    FL_ARG(rows < (1u << 31) && cols < (1u << 31), "fl_echelon_d: dimensions must be < 2^31");
    if (rows == 0 || cols == 0) {
        FL_HIP(fl_fill_u32(d_rank, 0, 1, stream));
        return FL_OK;
    }
    FL_ARG(Dt && d_pivcol, "fl_echelon_d: NULL array");
    FL_ARG(ldd >= cols && ldd % 4 == 0, "fl_echelon_d: ldd must be >= cols and a multiple of 4");
    FL_ARG(((uintptr_t)Dt & 7) == 0, "fl_echelon_d: Dt must be 8-byte aligned");
    EchWs e;
    size_t need = ech_layout(rows, cols, mode, ws, &e);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_echelon_d: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    const fl::Mod md = fl::make_mod(p);
    const uint32_t nchunks = (rows + kChunk - 1) / kChunk;
    FL_HIP(fl_fill_u32(e.is_piv, 0, rows, stream));
    FL_HIP(fl_fill_u32(d_rank, 0, 1, stream));
    const uint32_t npanels = (cols + kPanel - 1) / kPanel;
    for (uint32_t P = 0; P < npanels; P++) {
        const uint32_t c0 = P * kPanel;
        const uint32_t pw = cols - c0 < kPanel ? cols - c0 : kPanel;
        FL_PROF("echelon.greedy", stream, hipLaunchKernelGGL(k_ech_greedy<false>, dim3(nchunks), dim3(kGreedyThreads), 0, stream, md,
                           (const uint16_t *)Dt, ldd, rows, c0, pw, e.is_piv, e.cand, e.cand_cnt,
                           nchunks, e.ps, e.piv_row, d_pivcol, d_rank));
        FL_LAUNCH_CHECK("k_ech_greedy<local>");
        FL_PROF("echelon.greedy", stream, hipLaunchKernelGGL(k_ech_greedy<true>, dim3(1), dim3(kGreedyThreads), 0, stream, md,
                           (const uint16_t *)Dt, ldd, rows, c0, pw, e.is_piv, e.cand, e.cand_cnt,
                           nchunks, e.ps, e.piv_row, d_pivcol, d_rank));
        FL_LAUNCH_CHECK("k_ech_greedy<merge>");
        const uint32_t ucols = cols - c0;
        FL_PROF("echelon.U", stream,
                hipLaunchKernelGGL(k_ech_U, dim3((ucols + 255) / 256), dim3(256), 0, stream, md,
                                   (const uint16_t *)Dt, ldd, c0, cols, (const PanelState *)e.ps, e.U, e.ldu));
        FL_LAUNCH_CHECK("k_ech_U");
        hipLaunchKernelGGL(k_ech_gather_L, dim3((rows + 3) / 4), dim3(256), 0, stream,
                           (const uint16_t *)Dt, ldd, rows, (const PanelState *)e.ps, e.L);
        FL_LAUNCH_CHECK("k_ech_gather_L");
        const uint32_t *kdev = &e.ps->k;
        if (mode == FL_MFMA_I8) {
            FL_HIP(fl_gemm_sub_mfma(p, rows, ucols, kPanel, kdev, e.L, 64, e.U + c0, e.ldu,
                                    Dt + c0, ldd, e.gemm_ws, e.gemm_ws_bytes, stream, "echelon"));
        } else {
            FL_HIP(fl_gemm_sub_plain(p, rows, ucols, 0, kdev, e.L, 64, e.U + c0, e.ldu, Dt + c0,
                                     ldd, stream, "echelon.plain"));
        }
        hipLaunchKernelGGL(k_ech_setq, dim3((ucols + 255) / 256, kPanel), dim3(256), 0, stream, Dt,
                           ldd, c0, cols, (const PanelState *)e.ps, (const uint16_t *)e.U, e.ldu);
        FL_LAUNCH_CHECK("k_ech_setq");
    }
    const uint32_t mn = rows < cols ? rows : cols;
    const unsigned gx = (cols + 255) / 256 < 64 ? (cols + 255) / 256 : 64;
    hipLaunchKernelGGL(k_ech_gather_rows, dim3(gx, mn < 65535 ? mn : 65535), dim3(256), 0, stream, (const uint16_t *)Dt,
                       ldd, cols, (const uint32_t *)e.piv_row, (const uint32_t *)d_rank, e.T, e.ldu);
    FL_LAUNCH_CHECK("k_ech_gather_rows");
    const unsigned gy = rows < 65535 ? rows : 65535;
    hipLaunchKernelGGL(k_ech_place_rows, dim3(gx, gy), dim3(256), 0, stream, Dt, ldd, rows, cols,
                       (const uint32_t *)d_rank, (const uint16_t *)e.T, e.ldu);
    FL_LAUNCH_CHECK("k_ech_place_rows");
    return FL_OK;
}
