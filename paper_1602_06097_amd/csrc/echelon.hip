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
#include "mfma_tile.h"
#include "valu_tile.h"

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
constexpr uint32_t kProbe = 64;  // rows in the probe basis pass (at least)
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
    // one-entry task table for the single-matrix call
    FlEchTask *task;
    uint32_t *ids;       // [1] = 0
    uint32_t *pre_rows;  // [2]
    uint32_t *pre;       // 3 x [npanels][2]
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
// panel, taken from the list built by step 0.  One workgroup per matrix.
__global__ __launch_bounds__(kGreedyThreads) void k_ech_probe(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                              const uint32_t *__restrict__ ids, uint32_t P) {
    __shared__ GreedyLds S;
    __shared__ uint32_t rank0_s;
    const FlEchTask &t = tasks[ids[blockIdx.x]];
    if (P >= t.npanels) return;
    const uint32_t c0 = P * kPanel, pw = t.cols - c0 < kPanel ? t.cols - c0 : kPanel;
    PanelState *ps = (PanelState *)t.ps;
    const uint32_t n = t.counts[3 * P];
    const uint32_t take = n < kProbe ? n : kProbe;
    if (threadIdx.x == 0) {
        S.kb = 0;
        S.cnt = take;
        rank0_s = *t.d_rank;
        ps->nflag = 0;
        ps->rank0 = rank0_s;
    }
    if (threadIdx.x < take) S.list[threadIdx.x] = t.nzlist[threadIdx.x];
    __syncthreads();
    const uint32_t rank0 = rank0_s;
    greedy_rows(md, t.D, t.ld, c0, pw, S);
    save_raw(S, ps);
    finalize(S, ps, c0, rank0, t.is_piv, t.piv_row, t.piv_col, t.d_rank);
}

// Panel steps 0 and 2.  Step 0 (use_basis = 0): every remaining row that is
// nonzero on the panel goes to the nonzero list.  Step 2: every row of that
// list is reduced against the probe basis in ps; rows left nonzero (outside
// its span) go to the flagged list.  One wave per row, 8 rows per wave, 32
// rows per workgroup.
struct CheckLds {
    uint16_t Bv[64][64];
    uint32_t Cc[64];
};

// One workgroup (32 rows) of the check of panel P for table entry ti.
__device__ void check_tile(const fl::Mod &md, const FlEchTask &t, uint32_t bx, uint32_t P, int use_basis,
                           CheckLds &L) {
    const uint32_t c0 = P * kPanel, pw = t.cols - c0 < kPanel ? t.cols - c0 : kPanel;
    const PanelState *ps = (const PanelState *)t.ps;
    const uint32_t *in_list = use_basis ? t.nzlist : nullptr;
    uint32_t *out_list = use_basis ? t.flist : t.nzlist;
    uint32_t *out_count = t.counts + 3 * P + (use_basis ? 1 : 0);
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t kb = use_basis ? ps->kb : 0;
    const uint32_t n = in_list ? t.counts[3 * P] : t.rows;
    if (bx * 32 >= n) return;
    for (uint32_t i = threadIdx.x; i < kb * 64; i += blockDim.x) L.Bv[i >> 6][i & 63] = ps->Bv[i];
    if (threadIdx.x < 64) L.Cc[threadIdx.x] = use_basis ? ps->Cc[threadIdx.x] : 0;
    __syncthreads();
    for (uint32_t u = 0; u < 8; u++) {
        const uint32_t idx = (bx * 4 + wave) * 8 + u;
        bool flag = false;
        uint32_t i = 0;
        if (idx < n) {
            i = in_list ? in_list[idx] : idx;
            if (!t.is_piv[i] && kb < pw) {
                uint32_t v = lane < pw ? t.D[(uint64_t)i * t.ld + c0 + lane] : 0, g = 0;
                if (kb) reduce_against(md, v, g, 0, kb, L.Bv, L.Bv, L.Cc, lane, false);
                flag = __ballot(v != 0) != 0;
            }
        }
        block_append(flag, i, out_list, out_count);
    }
    if (use_basis && threadIdx.x == 0) __threadfence();
}

__global__ __launch_bounds__(256) void k_ech_check(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                   const uint32_t *__restrict__ ids,
                                                   const uint32_t *__restrict__ pre_rows, uint32_t ntask,
                                                   uint32_t P, int use_basis) {
    __shared__ CheckLds L;
    const uint32_t ti = fl_task_of(pre_rows, ntask, blockIdx.x);
    const FlEchTask &t = tasks[ids[ti]];
    if (P >= t.npanels) return;
    check_tile(md, t, blockIdx.x - pre_rows[ti], P, use_basis, L);
}

// Panel step 3 (only when some row was flagged): continue the greedy basis
// with the flagged rows and publish the final result.  One workgroup per
// matrix.
__global__ __launch_bounds__(kGreedyThreads) void k_ech_merge(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                              const uint32_t *__restrict__ ids, uint32_t P) {
    __shared__ GreedyLds S;
    const FlEchTask &t = tasks[ids[blockIdx.x]];
    if (P >= t.npanels) return;
    const uint32_t n = t.counts[3 * P + 1];
    if (n == 0) return;
    const uint32_t c0 = P * kPanel, pw = t.cols - c0 < kPanel ? t.cols - c0 : kPanel;
    PanelState *ps = (PanelState *)t.ps;
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
        if (threadIdx.x < cnt) S.list[threadIdx.x] = t.flist[base + threadIdx.x];
        if (threadIdx.x == 0) S.cnt = cnt;
        __syncthreads();
        greedy_rows(md, t.D, t.ld, c0, pw, S);
    }
    save_raw(S, ps);
    finalize(S, ps, c0, rank0, t.is_piv, t.piv_row, t.piv_col, t.d_rank);
}

// U[t][c] = sum_s G[t][s] Dt[Qs[s]][c] for c in [c0, cols), t < k; with
// limb planes, also U transposed as int8 limbs: Uh/Ul[(c - c0) * 64 + t]
// (zero for t >= k), the B operand of the matrix-core rank-k update.
// 256 columns per workgroup.
struct ULds {
    uint16_t Gs[64 * 64];
    uint16_t xs[64][256];
    uint32_t qs[64];
};

// One workgroup (256 columns from c0 + 256 bx) of U for panel P.
__device__ void U_tile(const fl::Mod &md, const FlEchTask &tk, uint32_t bx, uint32_t P, ULds &S) {
    uint16_t *Gs = S.Gs;
    uint16_t(*xs)[256] = S.xs;
    uint32_t *qs = S.qs;
    const PanelState *ps = (const PanelState *)tk.ps;
    const uint32_t c0 = P * kPanel, cols = tk.cols;
    const uint16_t *D = tk.D;
    const uint64_t ld = tk.ld, ldu = tk.ldu;
    uint16_t *U = tk.U;
    int8_t *Uh = tk.Uh, *Ul = tk.Ul;
    const uint32_t k = ps->k;
    if (k == 0) return;
    for (uint32_t i = threadIdx.x; i < 64 * 64; i += blockDim.x) Gs[i] = ps->G[i];
    if (threadIdx.x < 64) qs[threadIdx.x] = ps->Qs[threadIdx.x];
    __syncthreads();
    const uint32_t c = c0 + bx * 256 + threadIdx.x;
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
// One workgroup (32 rows) of the multiplier gather of panel P.
__device__ void L_tile(uint32_t p, const FlEchTask &tk, uint32_t bx, uint32_t P, uint32_t *ccol) {
    const PanelState *ps = (const PanelState *)tk.ps;
    const uint32_t rows = tk.rows;
    const uint16_t *D = tk.D;
    const uint64_t ld = tk.ld;
    uint16_t *L = tk.L;
    int8_t *Lh = tk.Lh, *Ll = tk.Ll;
    const uint32_t t = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (bx * 32 >= rows) return;
    const uint32_t k = ps->k;
    if (threadIdx.x < 64) ccol[threadIdx.x] = ps->Ccol[threadIdx.x];
    __syncthreads();
    for (uint32_t u = 0; u < 8; u++) {
        const uint32_t i = (bx * 4 + wave) * 8 + u;
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
        if (Lh) block_append(nz, i, tk.upd_rows, tk.counts + 3 * P + 2);
    }
}

// Panel steps 4 and 5 in one launch: the first grid_u workgroups compute U
// (columns), the others gather L (rows).
__global__ __launch_bounds__(256) void k_ech_UL(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                const uint32_t *__restrict__ ids, const uint32_t *__restrict__ pre_c,
                                                uint32_t n_all, uint32_t grid_u, const uint32_t *__restrict__ pre_rows,
                                                uint32_t n_active, uint32_t P) {
    __shared__ ULds S;
    if (blockIdx.x < grid_u) {
        const uint32_t ti = fl_task_of(pre_c, n_all, blockIdx.x);
        const FlEchTask &t = tasks[ids[ti]];
        if (P >= t.npanels) return;
        U_tile(md, t, blockIdx.x - pre_c[ti], P, S);
    } else {
        const uint32_t b = blockIdx.x - grid_u;
        const uint32_t ti = fl_task_of(pre_rows, n_active, b);
        const FlEchTask &t = tasks[ids[ti]];
        if (P >= t.npanels) return;
        L_tile(md.p, t, b - pre_rows[ti], P, S.qs);
    }
}

// Rank-k update of the rows with a nonzero multiplier, int8 MFMA form: one
// 64-row x 128-column tile per workgroup (column block from the prefix, row
// block blockIdx.y of the row list; blocks beyond the list exit at once).
__global__ __launch_bounds__(256) void k_ech_update_mfma(fl::Mod md, uint32_t bias, uint32_t c16,
                                                         const FlEchTask *__restrict__ tasks,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint32_t *__restrict__ pre, uint32_t ntask,
                                                         uint32_t P) {
    __shared__ __attribute__((aligned(16))) uint16_t sv[64 * fl_mfma::kRank64Ld];
    __shared__ uint32_t rows_s[64];
    const uint32_t ti = fl_task_of(pre, ntask, blockIdx.x);
    const FlEchTask &t = tasks[ids[ti]];
    if (P >= t.npanels) return;
    const uint32_t M = t.counts[3 * P + 2];
    if (blockIdx.y * 64 >= M || ((const PanelState *)t.ps)->k == 0) return;
    const uint32_t c0 = P * kPanel;
    fl_mfma::mfma_rank64_tile(md, bias, c16, t.Lh, t.Ll, t.Uh, t.Ul, t.upd_rows, M, t.D + c0, t.ld, t.cols - c0,
                              blockIdx.x - pre[ti], blockIdx.y, sv, rows_s);
}

// Rank-k update of every row, VALU form: column block (of 256) from the
// prefix, row blocks (of 32) blockIdx.y, blockIdx.y + gridDim.y, ...
__global__ __launch_bounds__(256) void k_ech_update_valu(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint32_t *__restrict__ pre, uint32_t ntask,
                                                         uint32_t P) {
    const uint32_t ti = fl_task_of(pre, ntask, blockIdx.x);
    const FlEchTask &t = tasks[ids[ti]];
    if (P >= t.npanels) return;
    const PanelState *ps = (const PanelState *)t.ps;
    const uint32_t c0 = P * kPanel, bx = blockIdx.x - pre[ti];
    for (uint32_t by = blockIdx.y; by * 32 < t.rows; by += gridDim.y)
        fl_valu::valu_gemm_tile(md, t.rows, t.cols - c0, 0, &ps->k, t.L, 64, t.U + c0, t.ldu, t.D + c0, t.ld,
                                bx, by);
}

// Rows of Q receive U (after the rank-k update touched them): 256 columns
// per workgroup from the prefix, pivot t = blockIdx.y.
__device__ void setq_tile(const FlEchTask &tk, uint32_t bx, uint32_t t, uint32_t P) {
    const PanelState *ps = (const PanelState *)tk.ps;
    if (t >= ps->k) return;
    const uint32_t row = ps->Phys[t];
    const uint32_t c = P * kPanel + bx * 256 + threadIdx.x;
    if (c < tk.cols) tk.D[(uint64_t)row * tk.ld + c] = tk.U[(uint64_t)t * tk.ldu + c];
}

__global__ __launch_bounds__(256) void k_ech_setq(const FlEchTask *__restrict__ tasks,
                                                  const uint32_t *__restrict__ ids,
                                                  const uint32_t *__restrict__ pre, uint32_t ntask, uint32_t P) {
    const uint32_t ti = fl_task_of(pre, ntask, blockIdx.x);
    const FlEchTask &tk = tasks[ids[ti]];
    if (P >= tk.npanels) return;
    setq_tile(tk, blockIdx.x - pre[ti], blockIdx.y, P);
}

// Step 7 of panel P and step 0 of panel P+1 in one launch (they touch
// different rows: the pivot rows of P, and rows that are no pivot rows):
// the first grid_c * 64 workgroups place U, the others list the rows
// nonzero on panel P+1.
__global__ __launch_bounds__(256) void k_ech_setq_check(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                        const uint32_t *__restrict__ ids,
                                                        const uint32_t *__restrict__ pre_c, uint32_t n_all,
                                                        uint32_t grid_c, const uint32_t *__restrict__ pre_rows,
                                                        uint32_t n_next, uint32_t P) {
    __shared__ CheckLds L;
    if (blockIdx.x < grid_c * kPanel) {
        const uint32_t bx = blockIdx.x % grid_c, t = blockIdx.x / grid_c;
        const uint32_t ti = fl_task_of(pre_c, n_all, bx);
        const FlEchTask &tk = tasks[ids[ti]];
        if (P >= tk.npanels) return;
        setq_tile(tk, bx - pre_c[ti], t, P);
    } else {
        const uint32_t b = blockIdx.x - grid_c * kPanel;
        const uint32_t ti = fl_task_of(pre_rows, n_next, b);
        const FlEchTask &tk = tasks[ids[ti]];
        if (P + 1 >= tk.npanels) return;
        check_tile(md, tk, b - pre_rows[ti], P + 1, 0, L);
    }
}

// Per-panel workgroup prefixes of the column-tiled kernels (one thread per
// panel and table).
__global__ void k_ech_prefixes(const FlEchTask *__restrict__ tasks, const uint32_t *__restrict__ ids,
                               uint32_t n, uint32_t panels, uint32_t tile, uint32_t *out) {
    for (uint32_t P = blockIdx.x * blockDim.x + threadIdx.x; P < panels; P += gridDim.x * blockDim.x) {
        uint32_t *o = out + (uint64_t)P * (n + 1);
        uint32_t acc = 0;
        o[0] = 0;
        for (uint32_t i = 0; i < n; i++) {
            const uint32_t cols = tasks[ids[i]].cols, c0 = 64 * P;
            acc += cols > c0 ? (cols - c0 + tile - 1) / tile : 0;
            o[i + 1] = acc;
        }
    }
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
    const uint32_t npanels = (cols + kPanel - 1) / kPanel;
    EchWs t;
    t.is_piv = c.take<uint32_t>(rows ? rows : 1);
    t.nzlist = c.take<uint32_t>(rows ? rows : 1);
    t.flist = c.take<uint32_t>(rows ? rows : 1);
    t.counts = c.take<uint32_t>(3 * (size_t)(npanels + 1));
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
    t.task = c.take<FlEchTask>(1);
    t.ids = c.take<uint32_t>(1);
    t.pre_rows = c.take<uint32_t>(2);
    t.pre = c.take<uint32_t>(3 * 2 * (size_t)(npanels ? npanels : 1));
    if (e) *e = t;
    return c.off;
}

}  // namespace

extern "C" size_t fl_echelon_d_workspace(uint32_t rows, uint32_t cols, fl_mode mode) {
    return ech_layout(rows, cols, mode, nullptr, nullptr);
}

fl_status fl_echelon_prepare(uint32_t p, uint32_t rows, uint32_t cols, uint16_t *Dt, uint64_t ldd,
                             uint32_t *d_rank, uint32_t *d_pivcol, fl_mode mode, void *ws,
                             size_t ws_bytes, hipStream_t stream, FlEchTask *task) {
    FL_ARG(p >= 2 && p <= 65521, "fl_echelon_d: p must be in [2, 65521]");
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_echelon_d: bad mode");
    FL_ARG(d_rank, "fl_echelon_d: NULL d_rank");
    FL_ARG(rows < (1u << 31) && cols < (1u << 31), "fl_echelon_d: dimensions must be < 2^31");
    FlEchTask t = {};
    t.rows = rows;
    t.cols = cols;
    t.d_rank = d_rank;
    t.mfma = mode == FL_MFMA_I8;
    if (rows == 0 || cols == 0) {
        FL_HIP(fl_fill_u32(d_rank, 0, 1, stream));
        *task = t;
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
    const uint32_t npanels = (cols + kPanel - 1) / kPanel;
    FL_HIP(fl_fill_u32(e.is_piv, 0, rows, stream));
    FL_HIP(fl_fill_u32(d_rank, 0, 1, stream));
    FL_HIP(fl_fill_u32(e.counts, 0, 3 * (size_t)npanels, stream));
    t.D = Dt;
    t.ld = ldd;
    t.npanels = npanels;
    t.is_piv = e.is_piv;
    t.piv_row = e.piv_row;
    t.piv_col = d_pivcol;
    t.ps = e.ps;
    t.U = e.U;
    t.L = e.L;
    t.T = e.T;
    t.ldu = e.ldu;
    t.Lh = e.Lh;
    t.Ll = e.Ll;
    t.Uh = e.Uh;
    t.Ul = e.Ul;
    t.upd_rows = e.upd_rows;
    t.nzlist = e.nzlist;
    t.flist = e.flist;
    t.counts = e.counts;
    *task = t;
    return FL_OK;
}

hipError_t fl_echelon_prefixes(const FlEchTask *tasks, const FlEchLists &L, uint32_t panels,
                               uint32_t *pre_c256, uint32_t *pre_m128, uint32_t *pre_p256,
                               hipStream_t stream) {
    if (panels == 0) return hipSuccess;
    const unsigned g = (panels + 255) / 256;
    hipLaunchKernelGGL(k_ech_prefixes, dim3(g), dim3(256), 0, stream, tasks, L.ids_all, L.n_all, panels, 256u,
                       pre_c256);
    if (L.n_mfma)
        hipLaunchKernelGGL(k_ech_prefixes, dim3(g), dim3(256), 0, stream, tasks, L.ids_mfma, L.n_mfma, panels,
                           128u, pre_m128);
    if (L.n_plain)
        hipLaunchKernelGGL(k_ech_prefixes, dim3(g), dim3(256), 0, stream, tasks, L.ids_plain, L.n_plain, panels,
                           256u, pre_p256);
    return hipGetLastError();
}

hipError_t fl_echelon_batch_panel(uint32_t p, const FlEchTask *tasks, const FlEchLists &L, uint32_t P,
                                  uint32_t n_active, uint32_t grid_rows, uint32_t grid_c256,
                                  uint32_t grid_m128, uint32_t grid_p256, uint32_t mfma_rows,
                                  uint32_t n_next, uint32_t grid_rows_next, hipStream_t stream) {
    if (n_active == 0) return hipSuccess;
    const fl::Mod md = fl::make_mod(p);
    const uint32_t *c256 = L.pre_c256 + (uint64_t)P * (L.n_all + 1);
    hipError_t e;
    if (P == 0) {  // later panels are listed by the previous panel's last launch
        FL_PROF("echelon.check", stream,
                hipLaunchKernelGGL(k_ech_check, dim3(grid_rows), dim3(256), 0, stream, md, tasks, L.ids_all,
                                   L.pre_rows, n_active, P, 0));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    FL_PROF("echelon.probe", stream,
            hipLaunchKernelGGL(k_ech_probe, dim3(n_active), dim3(kGreedyThreads), 0, stream, md, tasks, L.ids_all,
                               P));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    FL_PROF("echelon.check", stream,
            hipLaunchKernelGGL(k_ech_check, dim3(grid_rows), dim3(256), 0, stream, md, tasks, L.ids_all,
                               L.pre_rows, n_active, P, 1));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    FL_PROF("echelon.merge", stream,
            hipLaunchKernelGGL(k_ech_merge, dim3(n_active), dim3(kGreedyThreads), 0, stream, md, tasks, L.ids_all,
                               P));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    FL_PROF("echelon.UL", stream,
            hipLaunchKernelGGL(k_ech_UL, dim3(grid_c256 + grid_rows), dim3(256), 0, stream, md, tasks, L.ids_all,
                               c256, L.n_all, grid_c256, L.pre_rows, n_active, P));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (grid_m128) {
        const uint32_t *m128 = L.pre_m128 + (uint64_t)P * (L.n_mfma + 1);
        FL_PROF("echelon.mfma", stream,
                hipLaunchKernelGGL(k_ech_update_mfma, dim3(grid_m128, (mfma_rows + 63) / 64), dim3(256), 0, stream, md,
                                   fl_mfma::gemm_bias(p), fl_mfma::gemm_c16(p), tasks, L.ids_mfma, m128,
                                   L.n_mfma, P));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (grid_p256) {
        const uint32_t *p256 = L.pre_p256 + (uint64_t)P * (L.n_plain + 1);
        FL_PROF("echelon.plain", stream,
                hipLaunchKernelGGL(k_ech_update_valu, dim3(grid_p256, 64), dim3(256), 0, stream, md, tasks,
                                   L.ids_plain, p256, L.n_plain, P));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (n_next) {
        FL_PROF("echelon.setq_check", stream,
                hipLaunchKernelGGL(k_ech_setq_check, dim3(grid_c256 * kPanel + grid_rows_next), dim3(256), 0, stream,
                                   md, tasks, L.ids_all, c256, L.n_all, grid_c256, L.pre_rows, n_next, P));
    } else if (grid_c256) {
        FL_PROF("echelon.setq", stream,
                hipLaunchKernelGGL(k_ech_setq, dim3(grid_c256, kPanel), dim3(256), 0, stream, tasks, L.ids_all,
                                   c256, L.n_all, P));
    }
    return hipGetLastError();
}

fl_status fl_echelon_finish(const FlEchTask &t, hipStream_t stream) {
    if (t.npanels == 0) return FL_OK;
    const uint32_t rows = t.rows, cols = t.cols;
    const uint32_t mn = rows < cols ? rows : cols;
    const unsigned gx = (cols + 255) / 256 < 64 ? (cols + 255) / 256 : 64;
    hipLaunchKernelGGL(k_ech_gather_rows, dim3(gx, mn < 65535 ? mn : 65535), dim3(256), 0, stream,
                       (const uint16_t *)t.D, t.ld, cols, (const uint32_t *)t.piv_row, (const uint32_t *)t.d_rank,
                       t.T, t.ldu);
    FL_LAUNCH_CHECK("k_ech_gather_rows");
    const unsigned gy = rows < 65535 ? rows : 65535;
    hipLaunchKernelGGL(k_ech_place_rows, dim3(gx, gy), dim3(256), 0, stream, t.D, t.ld, rows, cols,
                       (const uint32_t *)t.d_rank, (const uint16_t *)t.T, t.ldu);
    FL_LAUNCH_CHECK("k_ech_place_rows");
    return FL_OK;
}

extern "C" fl_status fl_echelon_d(uint32_t p, uint32_t rows, uint32_t cols, uint16_t *Dt,
                                  uint64_t ldd, uint32_t *d_rank, uint32_t *d_pivcol, fl_mode mode,
                                  void *ws, size_t ws_bytes, hipStream_t stream) {
    FlEchTask t;
    fl_status st = fl_echelon_prepare(p, rows, cols, Dt, ldd, d_rank, d_pivcol, mode, ws, ws_bytes, stream, &t);
    if (st != FL_OK || t.npanels == 0) return st;
    EchWs e;
    ech_layout(rows, cols, mode, ws, &e);
    // a one-entry task table
    const uint32_t zero = 0, pre_rows[2] = {0, (rows + 31) / 32};
    FL_HIP(fl_upload(e.task, &t, sizeof t, stream));
    FL_HIP(fl_upload(e.ids, &zero, 4, stream));
    FL_HIP(fl_upload(e.pre_rows, pre_rows, 8, stream));
    const uint32_t np = t.npanels;
    FlEchLists L = {};
    L.ids_all = e.ids;
    L.pre_rows = e.pre_rows;
    L.pre_c256 = e.pre;
    L.n_all = 1;
    uint32_t *pre_m = e.pre + 2 * (size_t)np, *pre_p = e.pre + 4 * (size_t)np;
    if (t.mfma) {
        L.ids_mfma = e.ids;
        L.pre_m128 = pre_m;
        L.n_mfma = 1;
    } else {
        L.ids_plain = e.ids;
        L.pre_p256 = pre_p;
        L.n_plain = 1;
    }
    FL_HIP(fl_echelon_prefixes(e.task, L, np, e.pre, pre_m, pre_p, stream));
    for (uint32_t P = 0; P < np; P++) {
        const uint32_t g256 = fl_ech_tiles(cols, P, 256), g128 = fl_ech_tiles(cols, P, 128);
        const uint32_t nn = P + 1 < np ? 1 : 0;
        FL_HIP(fl_echelon_batch_panel(p, e.task, L, P, 1, pre_rows[1], g256, t.mfma ? g128 : 0,
                                      t.mfma ? 0 : g256, rows, nn, nn ? pre_rows[1] : 0, stream));
    }
    return fl_echelon_finish(t, stream);
}
