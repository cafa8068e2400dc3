// echelon.hip -- FL step 4 (paper Sec. 4.1 step 4, Sec. 4.4), read as the
// reduced row echelon form of the dense Schur complement Dt, computed by
// blocked Gauss-Jordan elimination over 64-column panels.
//
// For a panel [c0, c0+64):
//  0. k_ech_check   lists the remaining rows that are nonzero on the panel.
//  1. k_ech_probe   one block: a greedy basis of (up to 256 of) those rows
//     restricted to the panel, in reduced form in LDS.  Every wave reduces one
//     row against the basis (multipliers broadcast with v_readlane); rows
//     that stay nonzero are inserted one wave at a time.  The coefficients G
//     with  G * Dt[Q, panel] = basis  are tracked (Q = selected rows).
//     This is the paper's parallel structured Gaussian elimination (Sec. 5.1:
//     rows reduced in parallel against the known pivots, a new pivot added by
//     one worker at a time) applied to a panel.
//  2. k_ech_check   every listed row is reduced against that basis in
//     parallel; rows outside its span are listed again.
//  3. k_ech_merge   only if a row was listed: the greedy pass continues over
//     those rows.  The result: pivot columns C (ascending) of the
//     panel, rows Q, and G = Dt[Q, C]^{-1} (rows ordered by pivot column).
//  4. k_ech_U              U = G * Dt[Q, c0:]   (unit vectors at C)
//  5. k_ech_gather_L       L = Dt[:, C]          (multipliers, saved before
//                                                 the update overwrites them)
//  6. rank-k update        Dt[:, c0:] -= L U    (every row: Gauss-Jordan
//     (VALU or int8 MFMA)                       clears C above and below)
//  7. k_ech_setq           Dt[Q_t, c0:] = U_t
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
constexpr uint32_t kProbe = 256;  // rows in the probe basis pass (at least)
constexpr uint32_t kListCap = 2048;  // LDS row list: room for two 1024-row windows
constexpr int kGreedyThreads = 1024;

struct PanelState {
    uint32_t k;            // pivots found in this panel (final)
    uint32_t rank0;        // rank before this panel
    uint32_t nflag;        // rows outside the probe basis' span
    uint32_t kb;           // raw basis size (insertion order)
    uint32_t nupd;         // rows with a nonzero multiplier (listed in upd_rows)
    uint32_t pad_[3];
    uint32_t Qs[64];       // selected rows, by insertion slot
    uint32_t Phys[64];     // row that receives U_t
    uint32_t Ccol[64];     // absolute pivot column of U_t (ascending)
    uint32_t Cc[64];       // raw: relative pivot column of basis row j
    uint16_t G[64 * 64];   // G[t][s]: U_t = sum_s G[t][s] Dt[Qs[s]]
    uint16_t Bv[64 * 64];  // raw basis rows (panel part), insertion order
    uint16_t Bg[64 * 64];  // raw basis rows (coefficient part)
};

struct EchWs {
    uint32_t *is_piv;   // [rows] 1 once the row is a pivot row
    uint32_t *piv_row;  // [min(rows, cols)]
    PanelState *ps;
    uint16_t *U;        // [64 x ldu]
    uint16_t *L;        // [rows x 64]
    uint16_t *T;        // [min(rows, cols) x ldu]
    int8_t *Lh, *Ll;    // [rows x 64] limb planes of L (MFMA form)
    int8_t *Uh, *Ul;    // [(cols + 128) x 64] limb planes of U transposed (MFMA form)
    uint32_t *upd_rows; // [rows] rows with a nonzero multiplier
    uint32_t *nzlist;   // [rows] remaining rows nonzero on the panel
    uint32_t *flist;    // [rows] rows outside the probe basis' span
    uint32_t *counts;   // [3 * npanels] per panel: nonzero, flagged, update rows
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

// Append the rows with flag set (one candidate row per wave) to a global
// list: positions are claimed with one LDS atomic per row and one global
// atomic per block.  All threads of the block must call it.
__device__ void block_append(bool flag, uint32_t row, uint32_t *list, uint32_t *count) {
    __shared__ uint32_t s_n, s_base;
    const uint32_t lane = threadIdx.x & 63;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    uint32_t local = 0;
    if (flag && lane == 0) local = atomicAdd(&s_n, 1u);
    __syncthreads();
    if (threadIdx.x == 0) s_base = s_n ? atomicAdd(count, s_n) : 0;
    __syncthreads();
    if (flag && lane == 0) list[s_base + local] = row;
}

// Greedy basis of the panel rows in LDS: reduced form over the panel
// columns (Bv, pivots Cc), with the coefficients G of every basis row on the
// selected input rows Qo (Bg), so that  Bv_j = sum_s Bg_j[s] Dt[Qo[s], panel].
struct GreedyLds {
    uint16_t Bv[64][64];
    uint16_t Bg[64][64];
    uint32_t Cc[64];
    uint32_t Qo[64];
    uint32_t kb;
    uint32_t cnt;
    uint32_t list[kListCap];
};

// Process rows S.list[0..S.cnt) in order: each wave reduces one row against
// the basis; rows still nonzero are inserted one wave at a time (a new pivot
// is the first nonzero column; it is cleared from the other basis rows).
// This is the paper's parallel structured elimination (Sec. 5.1) in
// miniature: reductions in parallel, insertion of a new pivot serialised.
__device__ void greedy_rows(const fl::Mod &md, const uint16_t *__restrict__ D, uint64_t ld,
                            uint32_t c0, uint32_t pw, GreedyLds &S) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t cnt = S.cnt;
    for (uint32_t base = 0; base < cnt; base += nw) {
        if (S.kb >= pw) break;  // panel full: every further row reduces to 0
        const uint32_t item = base + wave;
        const bool have = item < cnt;
        const uint32_t row = have ? S.list[item] : 0;
        uint32_t v = (have && lane < pw) ? D[(uint64_t)row * ld + c0 + lane] : 0;
        uint32_t g = 0;
        const uint32_t ks = S.kb;
        reduce_against(md, v, g, 0, ks, S.Bv, S.Bg, S.Cc, lane, true);
        const bool nz = have && __ballot(v != 0) != 0;
        const int any = __syncthreads_or(nz ? 1 : 0);
        if (!any) continue;
        for (uint32_t w = 0; w < nw; w++) {
            if (w == wave && nz) {
                const uint32_t kb = S.kb;
                reduce_against(md, v, g, ks, kb, S.Bv, S.Bg, S.Cc, lane, true);
                const uint64_t mask = __ballot(v != 0);
                if (mask != 0 && kb < pw) {
                    const int c = __ffsll((long long)mask) - 1;
                    if (lane == kb) g = 1;
                    const uint32_t piv = (uint32_t)__builtin_amdgcn_readlane((int)v, c);
                    const uint32_t inv = fl::invmod(piv, md);
                    v = fl::mulmod(v, inv, md);
                    g = fl::mulmod(g, inv, md);
                    for (uint32_t t = 0; t < kb; t++) {
                        const uint32_t f = S.Bv[t][c];
                        if (f) {
                            S.Bv[t][lane] = (uint16_t)fl::submod(S.Bv[t][lane], fl::mulmod(f, v, md), md.p);
                            S.Bg[t][lane] = (uint16_t)fl::submod(S.Bg[t][lane], fl::mulmod(f, g, md), md.p);
                        }
                    }
                    S.Bv[kb][lane] = (uint16_t)v;
                    S.Bg[kb][lane] = (uint16_t)g;
                    if (lane == 0) {
                        S.Cc[kb] = (uint32_t)c;
                        S.Qo[kb] = row;
                        S.kb = kb + 1;
                    }
                }
            }
            __syncthreads();
        }
    }
    __syncthreads();
}

__device__ void save_raw(const GreedyLds &S, PanelState *ps) {
    for (uint32_t i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        ps->Bv[i] = S.Bv[i >> 6][i & 63];
        ps->Bg[i] = S.Bg[i >> 6][i & 63];
    }
    if (threadIdx.x < 64) {
        ps->Cc[threadIdx.x] = S.Cc[threadIdx.x];
        ps->Qs[threadIdx.x] = S.Qo[threadIdx.x];
    }
    if (threadIdx.x == 0) ps->kb = S.kb;
}

// Publish the panel result: basis rows ordered by pivot column, G, and the
// global pivot bookkeeping (rank0 = rank before this panel).
__device__ void finalize(const GreedyLds &S, PanelState *ps, uint32_t c0, uint32_t rank0,
                         uint32_t *is_piv, uint32_t *piv_row, uint32_t *piv_col, uint32_t *d_rank) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (wave != 0) return;
    const uint32_t kb = S.kb;
    uint32_t my_t = 0;
    if (lane < kb) {
        const uint32_t cj = S.Cc[lane];
        for (uint32_t j = 0; j < kb; j++) my_t += S.Cc[j] < cj ? 1 : 0;
    }
    for (uint32_t j = 0; j < kb; j++) {
        const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)my_t, (int)j);
        ps->G[t * 64 + lane] = lane < kb ? S.Bg[j][lane] : 0;
    }
    if (lane < kb) {
        const uint32_t t = my_t;
        ps->Phys[t] = S.Qo[lane];
        ps->Ccol[t] = c0 + S.Cc[lane];
        piv_row[rank0 + t] = S.Qo[lane];
        piv_col[rank0 + t] = c0 + S.Cc[lane];
        is_piv[S.Qo[lane]] = 1;  // later panels skip this row
    }
    if (lane == 0) {
        ps->k = kb;
        *d_rank = rank0 + kb;
    }
}

// Panel step 1: greedy basis of (at most kProbe of) the rows nonzero on the
// panel, taken from the list built by step 0.
__global__ __launch_bounds__(kGreedyThreads) void k_ech_probe(
    fl::Mod md, const uint16_t *__restrict__ D, uint64_t ld, uint32_t c0, uint32_t pw,
    const uint32_t *__restrict__ nzlist, const uint32_t *__restrict__ nzcount, uint32_t *is_piv,
    PanelState *ps, uint32_t *piv_row, uint32_t *piv_col, uint32_t *d_rank) {
    __shared__ GreedyLds S;
    __shared__ uint32_t rank0_s;
    const uint32_t n = *nzcount;
    const uint32_t take = n < kProbe ? n : kProbe;
    if (threadIdx.x == 0) {
        S.kb = 0;
        S.cnt = take;
        rank0_s = *d_rank;
        ps->nflag = 0;
        ps->rank0 = rank0_s;
    }
    if (threadIdx.x < take) S.list[threadIdx.x] = nzlist[threadIdx.x];
    __syncthreads();
    const uint32_t rank0 = rank0_s;
    greedy_rows(md, D, ld, c0, pw, S);
    save_raw(S, ps);
    finalize(S, ps, c0, rank0, is_piv, piv_row, piv_col, d_rank);
}

// Panel steps 0 and 2.  Step 0 (use_basis = 0): every remaining row that is
// nonzero on the panel goes to out_list.  Step 2: every row of in_list is
// reduced against the probe basis in ps; rows left nonzero (outside its span)
// go to out_list.  One wave per row, 8 rows per wave, 32 rows per block.
__global__ __launch_bounds__(256) void k_ech_check(fl::Mod md, const uint16_t *__restrict__ D,
                                                   uint64_t ld, uint32_t rows, uint32_t c0,
                                                   uint32_t pw, const uint32_t *__restrict__ is_piv,
                                                   PanelState *ps, const uint32_t *__restrict__ in_list,
                                                   const uint32_t *__restrict__ in_count,
                                                   uint32_t *out_list, uint32_t *out_count, int use_basis) {
    __shared__ uint16_t Bv[64][64];
    __shared__ uint32_t Cc[64];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t kb = use_basis ? ps->kb : 0;
    const uint32_t n = in_list ? *in_count : rows;
    if (blockIdx.x * 32 >= n) return;
    for (uint32_t i = threadIdx.x; i < kb * 64; i += blockDim.x) Bv[i >> 6][i & 63] = ps->Bv[i];
    if (threadIdx.x < 64) Cc[threadIdx.x] = use_basis ? ps->Cc[threadIdx.x] : 0;
    __syncthreads();
    for (uint32_t u = 0; u < 8; u++) {
        const uint32_t idx = (blockIdx.x * 4 + wave) * 8 + u;
        bool flag = false;
        uint32_t i = 0;
        if (idx < n) {
            i = in_list ? in_list[idx] : idx;
            if (!is_piv[i] && kb < pw) {
                uint32_t v = lane < pw ? D[(uint64_t)i * ld + c0 + lane] : 0, g = 0;
                if (kb) reduce_against(md, v, g, 0, kb, Bv, Bv, Cc, lane, false);
                flag = __ballot(v != 0) != 0;
            }
        }
        block_append(flag, i, out_list, out_count);
    }
    if (use_basis && threadIdx.x == 0) __threadfence();
}

// Panel step 3 (only when some row was flagged): continue the greedy basis
// with the flagged rows and publish the final result.
__global__ __launch_bounds__(kGreedyThreads) void k_ech_merge(
    fl::Mod md, const uint16_t *__restrict__ D, uint64_t ld, uint32_t c0, uint32_t pw,
    const uint32_t *__restrict__ flist, const uint32_t *__restrict__ fcount, uint32_t *is_piv,
    PanelState *ps, uint32_t *piv_row, uint32_t *piv_col, uint32_t *d_rank) {
    __shared__ GreedyLds S;
    const uint32_t n = *fcount;
    if (n == 0) return;
    for (uint32_t i = threadIdx.x; i < 64 * 64; i += blockDim.x) {
        S.Bv[i >> 6][i & 63] = ps->Bv[i];
        S.Bg[i >> 6][i & 63] = ps->Bg[i];
    }
    if (threadIdx.x < 64) {
        S.Cc[threadIdx.x] = ps->Cc[threadIdx.x];
        S.Qo[threadIdx.x] = ps->Qs[threadIdx.x];
    }
    if (threadIdx.x == 0) S.kb = ps->kb;
    __syncthreads();
    const uint32_t rank0 = ps->rank0;
    for (uint32_t base = 0; base < n && S.kb < pw; base += kGreedyThreads) {
        const uint32_t cnt = n - base < kGreedyThreads ? n - base : kGreedyThreads;
        if (threadIdx.x < cnt) S.list[threadIdx.x] = flist[base + threadIdx.x];
        if (threadIdx.x == 0) S.cnt = cnt;
        __syncthreads();
        greedy_rows(md, D, ld, c0, pw, S);
    }
    save_raw(S, ps);
    finalize(S, ps, c0, rank0, is_piv, piv_row, piv_col, d_rank);
}

// U[t][c] = sum_s G[t][s] Dt[Qs[s]][c] for c in [c0, cols), t < k; with
// limb planes, also U transposed as int8 limbs: Uh/Ul[(c - c0) * 64 + t]
// (zero for t >= k), the B operand of the matrix-core rank-k update.
__global__ __launch_bounds__(256) void k_ech_U(fl::Mod md, const uint16_t *__restrict__ D,
                                               uint64_t ld, uint32_t c0, uint32_t cols,
                                               const PanelState *__restrict__ ps, uint16_t *U,
                                               uint64_t ldu, int8_t *Uh, int8_t *Ul) {
    __shared__ uint16_t Gs[64 * 64];
    __shared__ uint16_t xs[64][256];
    __shared__ uint32_t qs[64];
    const uint32_t k = ps->k;
    if (k == 0) return;
    for (uint32_t i = threadIdx.x; i < 64 * 64; i += blockDim.x) Gs[i] = ps->G[i];
    if (threadIdx.x < 64) qs[threadIdx.x] = ps->Qs[threadIdx.x];
    __syncthreads();
    const uint32_t c = c0 + blockIdx.x * 256 + threadIdx.x;
    const bool ok = c < cols;
#pragma unroll 8
    for (uint32_t s = 0; s < k; s++) xs[s][threadIdx.x] = ok ? D[(uint64_t)qs[s] * ld + c] : 0;
    __syncthreads();
    if (!ok) return;
    uint32_t hw[16], lw[16];
#pragma unroll
    for (int i = 0; i < 16; i++) hw[i] = lw[i] = 0;
    for (uint32_t t = 0; t < k; t++) {
        uint32_t h = 0, l = 0;
        for (uint32_t s = 0; s < k; s++) {
            uint32_t gts = Gs[t * 64 + s];
            uint32_t x = xs[s][threadIdx.x];
            h = fl::mad24(gts >> 8, x, h);
            l = fl::mad24(gts & 0xffu, x, l);
        }
        const uint32_t u = fl::fold_pair(h, l, md);
        U[(uint64_t)t * ldu + c] = (uint16_t)u;
        if (Uh) {
            int lh, ll;
            fl_split_limbs(u, md.p, lh, ll);
#pragma unroll
            for (int i = 0; i < 16; i++)
                if ((uint32_t)i == (t >> 2)) {
                    hw[i] |= (uint32_t)(lh & 0xff) << (8 * (t & 3));
                    lw[i] |= (uint32_t)(ll & 0xff) << (8 * (t & 3));
                }
        }
    }
    if (Uh) {
        uint4 *dh = (uint4 *)(Uh + (uint64_t)(c - c0) * 64), *dl = (uint4 *)(Ul + (uint64_t)(c - c0) * 64);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            dh[i] = make_uint4(hw[4 * i], hw[4 * i + 1], hw[4 * i + 2], hw[4 * i + 3]);
            dl[i] = make_uint4(lw[4 * i], lw[4 * i + 1], lw[4 * i + 2], lw[4 * i + 3]);
        }
    }
}

// L[i][t] = Dt[i][Ccol[t]] (0 for t >= k); with limb planes, also L as
// int8 limbs (64 bytes per row) and the list of rows with a nonzero
// multiplier (rows whose update is zero are skipped by the rank-k update).
// One wave per row, 8 rows per wave.
__global__ __launch_bounds__(256) void k_ech_gather_L(const uint16_t *__restrict__ D, uint64_t ld,
                                                      uint32_t rows, const PanelState *__restrict__ ps,
                                                      uint16_t *L, uint32_t p, int8_t *Lh, int8_t *Ll,
                                                      uint32_t *upd_rows, uint32_t *upd_count) {
    __shared__ uint32_t ccol[64];
    const uint32_t t = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (blockIdx.x * 32 >= rows) return;
    const uint32_t k = ps->k;
    if (threadIdx.x < 64) ccol[threadIdx.x] = ps->Ccol[threadIdx.x];
    __syncthreads();
    for (uint32_t u = 0; u < 8; u++) {
        const uint32_t i = (blockIdx.x * 4 + wave) * 8 + u;
        bool nz = false;
        if (i < rows) {
            const uint32_t x = t < k ? D[(uint64_t)i * ld + ccol[t]] : 0;
            L[(uint64_t)i * 64 + t] = (uint16_t)x;
            if (Lh) {
                int h = 0, l = 0;
                fl_split_limbs(x, p, h, l);
                Lh[(uint64_t)i * 64 + t] = (int8_t)h;
                Ll[(uint64_t)i * 64 + t] = (int8_t)l;
                nz = __ballot(x != 0) != 0;
            }
        }
        if (Lh) block_append(nz, i, upd_rows, upd_count);
    }
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
    const uint64_t ldu = ((uint64_t)cols + 63) & ~(uint64_t)63;
    EchWs t;
    t.is_piv = c.take<uint32_t>(rows ? rows : 1);
    t.nzlist = c.take<uint32_t>(rows ? rows : 1);
    t.flist = c.take<uint32_t>(rows ? rows : 1);
    t.counts = c.take<uint32_t>(3 * (size_t)((cols + kPanel - 1) / kPanel + 1));
    t.piv_row = c.take<uint32_t>(mn ? mn : 1);
    t.ps = c.take<PanelState>(1);
    t.U = c.take<uint16_t>((size_t)64 * ldu);
    t.L = c.take<uint16_t>((size_t)(rows ? rows : 1) * 64);
    t.T = c.take<uint16_t>((size_t)(mn ? mn : 1) * ldu);
    t.ldu = ldu;
    t.gemm_ws_bytes = 0;
    t.gemm_ws = nullptr;
    t.Lh = t.Ll = t.Uh = t.Ul = nullptr;
    if (mode == FL_MFMA_I8) {
        t.Lh = c.take<int8_t>((size_t)(rows ? rows : 1) * 64);
        t.Ll = c.take<int8_t>((size_t)(rows ? rows : 1) * 64);
        t.Uh = c.take<int8_t>(((size_t)cols + 256) * 64);
        t.Ul = c.take<int8_t>(((size_t)cols + 256) * 64);
    }
    t.upd_rows = c.take<uint32_t>(rows ? rows : 1);
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
    const uint32_t npanels = (cols + kPanel - 1) / kPanel;
    FL_HIP(fl_fill_u32(e.is_piv, 0, rows, stream));
    FL_HIP(fl_fill_u32(d_rank, 0, 1, stream));
    FL_HIP(fl_fill_u32(e.counts, 0, 3 * (size_t)npanels, stream));
    const unsigned row_blocks = (rows + 31) / 32;  // 32 rows per block (8 per wave)
    for (uint32_t P = 0; P < npanels; P++) {
        const uint32_t c0 = P * kPanel;
        const uint32_t pw = cols - c0 < kPanel ? cols - c0 : kPanel;
        uint32_t *n_nz = e.counts + 3 * P, *n_flag = n_nz + 1, *n_upd = n_nz + 2;
        FL_PROF("echelon.check", stream,
                hipLaunchKernelGGL(k_ech_check, dim3(row_blocks), dim3(256), 0, stream, md, (const uint16_t *)Dt,
                                   ldd, rows, c0, pw, (const uint32_t *)e.is_piv, e.ps,
                                   (const uint32_t *)nullptr, (const uint32_t *)nullptr, e.nzlist, n_nz, 0));
        FL_LAUNCH_CHECK("k_ech_check<nonzero>");
        FL_PROF("echelon.probe", stream,
                hipLaunchKernelGGL(k_ech_probe, dim3(1), dim3(kGreedyThreads), 0, stream, md,
                                   (const uint16_t *)Dt, ldd, c0, pw, (const uint32_t *)e.nzlist,
                                   (const uint32_t *)n_nz, e.is_piv, e.ps, e.piv_row, d_pivcol, d_rank));
        FL_LAUNCH_CHECK("k_ech_probe");
        FL_PROF("echelon.check", stream,
                hipLaunchKernelGGL(k_ech_check, dim3(row_blocks), dim3(256), 0, stream, md, (const uint16_t *)Dt,
                                   ldd, rows, c0, pw, (const uint32_t *)e.is_piv, e.ps,
                                   (const uint32_t *)e.nzlist, (const uint32_t *)n_nz, e.flist, n_flag, 1));
        FL_LAUNCH_CHECK("k_ech_check<basis>");
        FL_PROF("echelon.merge", stream,
                hipLaunchKernelGGL(k_ech_merge, dim3(1), dim3(kGreedyThreads), 0, stream, md,
                                   (const uint16_t *)Dt, ldd, c0, pw, (const uint32_t *)e.flist,
                                   (const uint32_t *)n_flag, e.is_piv, e.ps, e.piv_row, d_pivcol, d_rank));
        FL_LAUNCH_CHECK("k_ech_merge");
        const uint32_t ucols = cols - c0;
        FL_PROF("echelon.U", stream,
                hipLaunchKernelGGL(k_ech_U, dim3((ucols + 255) / 256), dim3(256), 0, stream, md,
                                   (const uint16_t *)Dt, ldd, c0, cols, (const PanelState *)e.ps, e.U, e.ldu,
                                   e.Uh, e.Ul));
        FL_LAUNCH_CHECK("k_ech_U");
        FL_PROF("echelon.L", stream,
                hipLaunchKernelGGL(k_ech_gather_L, dim3(row_blocks), dim3(256), 0, stream, (const uint16_t *)Dt,
                                   ldd, rows, (const PanelState *)e.ps, e.L, p, e.Lh, e.Ll, e.upd_rows, n_upd));
        FL_LAUNCH_CHECK("k_ech_gather_L");
        const uint32_t *kdev = &e.ps->k;
        if (mode == FL_MFMA_I8) {
            FL_HIP(fl_mfma_rank64_planes(p, e.Lh, e.Ll, e.Uh, e.Ul, kdev, e.upd_rows, n_upd, rows, Dt + c0, ldd,
                                         ucols, stream, "echelon.mfma"));
        } else {
            FL_HIP(fl_gemm_sub_plain(p, rows, ucols, 0, kdev, e.L, 64, e.U + c0, e.ldu, Dt + c0,
                                     ldd, stream, "echelon.plain"));
        }
        FL_PROF("echelon.setq", stream,
                hipLaunchKernelGGL(k_ech_setq, dim3((ucols + 255) / 256, kPanel), dim3(256), 0, stream, Dt,
                                   ldd, c0, cols, (const PanelState *)e.ps, (const uint16_t *)e.U, e.ldu));
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
