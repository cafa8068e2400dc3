// echelon.hip -- FL step 4 (paper Sec. 4.1 step 4, Sec. 4.4), read as the
// reduced row echelon form of the dense Schur complement Dt, computed by
// blocked Gauss-Jordan elimination over 64-column panels.
//
// For a panel [c0, c0+64):
//  0. k_ech_check   lists the remaining rows that are nonzero on the panel,
//     with the first nonzero column of each.
//  1. k_ech_probe   one block: the basis of one listed row per panel
//     column that is some row's first nonzero (independent rows: their
//     leading entries form a triangular matrix), in reduced form in LDS by
//     back substitution.  The coefficients G with G * Dt[Q, panel] = basis
//     are tracked (Q = selected rows).
//  2. k_ech_check   every listed row is reduced against that basis in
//     parallel (multipliers broadcast with v_readlane); rows outside its
//     span are listed again.
//  3. k_ech_merge   only if a row was listed: a greedy pass over those rows,
//     the paper's parallel structured Gaussian elimination (Sec. 5.1: rows
//     reduced in parallel against the known pivots, a new pivot added by one
//     worker at a time, all waves clearing its column from the older basis
//     rows).  The result: pivot columns C (ascending) of the panel, rows Q,
//     and G = Dt[Q, C]^{-1} (rows ordered by pivot column).
//  4. U = G * Dt[Q, c0:bend)     over the rest of the panel's 256-column block
//  5. L' = Dt[:, C] - [row = Q_t] (multipliers with the placement of U folded
//                                  in; 4 and 5 are computed from the probe
//                                  basis in step 2's launch, and again after a
//                                  merge, only for the matrices it changed)
//  6. Dt[:, c0:bend) -= L' U      (every row with a nonzero multiplier:
//     (VALU or int8 MFMA)          Gauss-Jordan clears C above and below, and
//                                  pivot row Q_t becomes U_t)
// The columns right of the block are updated once per block of four panels
// (K = 256): U of the block for them by a recurrence over its panels, then
// the next block's columns (critical path) and the far part (second stream,
// overlapping the next block's panels).
// After the last panel the pivot rows are gathered to rows 0..r-1 in pivot
// order and the other rows (now zero) are cleared.
#include <algorithm>
#include <vector>

#include "fl_internal.h"
#include "mfma_tile.h"
#include "valu_tile.h"

hipError_t fl_gemm_sub_mfma(uint32_t p, uint32_t M, uint32_t N, uint32_t Kmax, const uint32_t *Kdev,
                            const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                            uint16_t *C, uint64_t ldc, void *ws, size_t ws_bytes, hipStream_t s,
                            const char *site);
size_t fl_gemm_sub_mfma_ws(uint32_t M, uint32_t N, uint32_t Kmax);

namespace {

constexpr uint32_t kPanel = 64;
constexpr uint32_t kBlockPanels = 4;                  // panels per block of the delayed update
constexpr uint32_t kBlock = kPanel * kBlockPanels;   // 256 columns, K of the block update
constexpr uint32_t kSlots = 2 * kBlockPanels;        // panel states kept (two blocks)
constexpr uint32_t kListCap = 2048;  // LDS row list: room for two 1024-row windows
constexpr int kGreedyThreads = 1024;

struct __attribute__((aligned(16))) PanelState {
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

static_assert(offsetof(PanelState, Bv) % 16 == 0 && offsetof(PanelState, Bg) % 16 == 0 &&
                  offsetof(PanelState, G) % 16 == 0,
              "16-byte copies of the basis planes");

struct EchWs {
    uint32_t *is_piv;   // [rows] 1 once the row is a pivot row
    uint32_t *piv_row;  // [min(rows, cols)]
    PanelState *ps;     // [kSlots]
    uint16_t *U;        // [64 x ldu] U of the current panel (its block's columns)
    uint16_t *T;        // [min(rows, cols) x ldu]
    int8_t *Uh, *Ul;    // [(cols + 256) x 64] limb planes of U transposed (MFMA form)
    uint16_t *Lb;       // [2][rows x 256] multipliers of a block's panels (block parity)
    int8_t *Lbh, *Lbl;  // [2][rows x 256] their limb planes (MFMA form)
    uint16_t *Ub;       // [2][256 x ldu] U of a block for the columns right of it (VALU form)
    int8_t *Ubh, *Ubl;  // [2][(cols + 256) x 256] its limb planes, by column (MFMA form)
    uint32_t *upd_rows; // [rows] rows with a nonzero multiplier in the current panel
    uint32_t *blk_rows; // [2][rows] rows with a nonzero multiplier in a block
    uint32_t *blk_cnt;  // [nblocks] their counts
    uint32_t *mark;     // [rows] last block (+1) that listed the row
    uint32_t *nzlead;   // [rows] first nonzero column (on the panel) of each listed row
    uint32_t *nzlist;   // [rows] remaining rows nonzero on the panel
    uint32_t *flist;    // [rows] rows outside the probe basis' span
    uint32_t *counts;   // [3 * npanels] per panel: nonzero, flagged, update rows
    uint64_t ldu;
    // one-entry task table for the single-matrix call
    FlEchTask *task;
    uint32_t *ids;       // [1] = 0
    uint32_t *pre_rows;  // [2]
    uint32_t *pre;       // prefix tables: 3 x [npanels][2], 6 x [nblocks][2]
};

// The panel states of two blocks are kept, so that a block's panels can be
// searched while the previous block's far update still reads its states.
__device__ __forceinline__ PanelState *panel_state(const FlEchTask &t, uint32_t P) {
    return (PanelState *)t.ps + (P % kSlots);
}

// The K dimension of a block's delayed update holds its panels' pivots
// packed: panel j of the block takes slots [kbase_j, kbase_j + k_j), kbase_j
// the sum of round_up(k_i, 16) over the block's earlier panels (16-slot
// granularity keeps the limb planes' 16-byte fragments aligned); the slots
// up to the next multiple of 16 are padding (zero in U).  With about 22
// pivots per panel the block needs K = 128 instead of 4 x 64.
__device__ __forceinline__ uint32_t round16(uint32_t k) { return (k + 15) & ~15u; }
__device__ __forceinline__ uint32_t panel_kbase(const FlEchTask &t, uint32_t P) {
    uint32_t base = 0;
    for (uint32_t P1 = P / kBlockPanels * kBlockPanels; P1 < P; P1++) base += round16(panel_state(t, P1)->k);
    return base;
}
// K of block B's update: the packed slots of all of its panels.
__device__ __forceinline__ uint32_t block_k(const FlEchTask &t, uint32_t B) {
    const uint32_t P0 = B * kBlockPanels, P1 = P0 + kBlockPanels < t.npanels ? P0 + kBlockPanels : t.npanels;
    uint32_t k = 0;
    for (uint32_t P = P0; P < P1; P++) k += round16(panel_state(t, P)->k);
    return k;
}

// Reduce the wave's vector (v: panel part, g: coefficient part, lane = column
// or slot) against basis rows [t0, t1).  The basis is in reduced form, so all
// multipliers can be read from the vector as it is on entry.  The pivot
// columns are read once into a register (lane t holds Cc[t]); a zero
// multiplier adds nothing, so no term is skipped (no branch in the loop).
__device__ inline void reduce_against(const fl::Mod &md, uint32_t &v, uint32_t &g, uint32_t t0,
                                      uint32_t t1, const uint16_t (*Bv)[64],
                                      const uint16_t (*Bg)[64], const uint32_t *Cc, uint32_t lane,
                                      bool track) {
    uint32_t vh = 0, vl = 0, gh = 0, gl = 0;
    const uint32_t vin = v;
    const uint32_t cc = Cc[lane];
#pragma unroll 4
    for (uint32_t t = t0; t < t1; t++) {
        const int cidx = __builtin_amdgcn_readlane((int)cc, (int)t);
        const uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)vin, cidx);
        const uint32_t lh = lam >> 8, ll = lam & 0xffu;
        const uint32_t b = Bv[t][lane];
        vh = fl::mad24(lh, b, vh);
        vl = fl::mad24(ll, b, vl);
        if (track) {
            const uint32_t bg = Bg[t][lane];
            gh = fl::mad24(lh, bg, gh);
            gl = fl::mad24(ll, bg, gl);
        }
    }
    // at most 64 terms: no intermediate fold needed
    v = fl::submod(v, fl::fold_pair(vh, vl, md), md.p);
    if (track) g = fl::submod(g, fl::fold_pair(gh, gl, md), md.p);
}

// The same for the wave's 8 rows v[0..8) (no coefficient part), interleaved so
// that the basis row and pivot column are read once per basis row.
__device__ inline void reduce_rows8(const fl::Mod &md, uint32_t (&v)[8], uint32_t kb, const uint16_t (*Bv)[64],
                                    const uint32_t *Cc, uint32_t lane) {
    uint32_t vh[8], vl[8];
#pragma unroll
    for (int u = 0; u < 8; u++) vh[u] = vl[u] = 0;
    const uint32_t cc = Cc[lane];
#pragma unroll 4
    for (uint32_t t = 0; t < kb; t++) {
        const int cidx = __builtin_amdgcn_readlane((int)cc, (int)t);
        const uint32_t b = Bv[t][lane];
#pragma unroll
        for (int u = 0; u < 8; u++) {
            const uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)v[u], cidx);
            vh[u] = fl::mad24(lam >> 8, b, vh[u]);
            vl[u] = fl::mad24(lam & 0xffu, b, vl[u]);
        }
    }
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = fl::submod(v[u], fl::fold_pair(vh[u], vl[u], md), md.p);
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

// Append up to 8 rows per wave to a global list with one global atomic per
// block: bit u of the wave-uniform mask8 lists the row held by lane u (and,
// with list2, lane u's val2 at the same position).  All threads of the
// (256-thread) block must call it.
__device__ void block_append8(uint32_t mask8, uint32_t row, uint32_t *list, uint32_t *count,
                              uint32_t *list2 = nullptr, uint32_t val2 = 0) {
    __shared__ uint32_t s_w[4], s_base;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) s_w[wave] = __popc(mask8);
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t tot = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        s_base = tot ? atomicAdd(count, tot) : 0;
    }
    __syncthreads();
    uint32_t off = s_base;
    for (uint32_t w = 0; w < wave; w++) off += s_w[w];
    if (lane < 8 && ((mask8 >> lane) & 1u)) {
        const uint32_t at = off + __popc(mask8 & ((1u << lane) - 1u));
        list[at] = row;
        if (list2) list2[at] = val2;
    }
}

// Greedy basis of the panel rows in LDS: reduced form over the panel
// columns (Bv, pivots Cc), with the coefficients G of every basis row on the
// selected input rows Qo (Bg), so that  Bv_j = sum_s Bg_j[s] Dt[Qo[s], panel].
struct __attribute__((aligned(16))) GreedyLds {
    uint16_t Bv[64][64];
    uint16_t Bg[64][64];
    uint32_t Cc[64];
    uint32_t Qo[64];
    uint32_t kb;
    uint32_t cnt;
    uint32_t nzmask[2];  // waves holding a candidate row in the batch (batch parity)
    uint32_t newc;    // pivot column of the row just inserted (64: none)
    uint32_t list[kListCap];
};

// Process rows S.list[0..S.cnt), 16 at a time (one per wave): every row is
// reduced against the basis in parallel; then, while some row of the batch
// is still nonzero, the first such row is inserted (normalised at its first
// nonzero column, the new pivot) and every wave clears the new pivot column,
// from the older basis rows (dealt round-robin) and from its own row.  The
// basis stays in reduced form, so each reduction reads the multipliers from
// the vector as it is.  This is the paper's parallel structured elimination
// (Sec. 5.1) in miniature: reductions in parallel, insertion serialised.
__device__ void greedy_rows(const fl::Mod &md, const uint16_t *__restrict__ D, uint64_t ld,
                            uint32_t c0, uint32_t pw, GreedyLds &S) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t nw = blockDim.x >> 6;
    const uint32_t cnt = S.cnt;
    if (cnt == 0) {  // nothing listed (S.list holds no row to prefetch)
        __syncthreads();
        return;
    }
    const uint32_t col = c0 + (lane < pw ? lane : 0);
    // the next batch's row is fetched while the current batch is processed
    uint32_t row_n = wave < cnt ? S.list[wave] : S.list[0];
    uint32_t v_n = D[(uint64_t)row_n * ld + col];
    // S.nzmask[r & 1]: waves with a nonzero row in round r; a slot is cleared
    // one round before it is filled, after the barriers that end its last read
    uint32_t r = 0;
    for (uint32_t base = 0; base < cnt; base += nw) {
        if (S.kb >= pw) break;  // panel full: every further row reduces to 0
        const uint32_t item = base + wave;
        const bool have = item < cnt;
        const uint32_t row = row_n;
        uint32_t v = v_n;
        if (!have || lane >= pw) v = 0;
        {
            const uint32_t nx = item + nw;
            row_n = nx < cnt ? S.list[nx] : S.list[0];
            v_n = D[(uint64_t)row_n * ld + col];
        }
        uint32_t g = 0;
        r++;
        if (threadIdx.x == 0) S.nzmask[r & 1] = 0;
        __syncthreads();
        reduce_against(md, v, g, 0, S.kb, S.Bv, S.Bg, S.Cc, lane, true);
        if (__ballot(v != 0) != 0 && lane == 0) atomicOr(&S.nzmask[r & 1], 1u << wave);
        __syncthreads();
        for (;;) {
            const uint32_t mask = S.nzmask[r & 1];
            if (mask == 0 || S.kb >= pw) break;
            if (threadIdx.x == 0) S.nzmask[(r + 1) & 1] = 0;
            if (wave == (uint32_t)__ffs((int)mask) - 1) {
                const uint32_t kb = S.kb;
                const uint32_t c = (uint32_t)__ffsll((long long)__ballot(v != 0)) - 1;
                if (lane == kb) g = 1;
                const uint32_t inv = fl::invmod((uint32_t)__builtin_amdgcn_readlane((int)v, (int)c), md);
                S.Bv[kb][lane] = (uint16_t)fl::mulmod(v, inv, md);
                S.Bg[kb][lane] = (uint16_t)fl::mulmod(g, inv, md);
                if (lane == 0) {
                    S.newc = c;
                    S.Cc[kb] = c;
                    S.Qo[kb] = row;
                    S.kb = kb + 1;
                }
                v = 0;  // this row is now basis row kb
            }
            __syncthreads();
            const uint32_t c = S.newc, kn = S.kb;
            const uint32_t nb = S.Bv[kn - 1][lane], ng = S.Bg[kn - 1][lane];
            for (uint32_t t = wave; t + 1 < kn; t += nw) {
                const uint32_t f = S.Bv[t][c];
                if (f) {
                    S.Bv[t][lane] = (uint16_t)fl::submod(S.Bv[t][lane], fl::mulmod(f, nb, md), md.p);
                    S.Bg[t][lane] = (uint16_t)fl::submod(S.Bg[t][lane], fl::mulmod(f, ng, md), md.p);
                }
            }
            const uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)v, (int)c);
            if (lam) {
                v = fl::submod(v, fl::mulmod(lam, nb, md), md.p);
                g = fl::submod(g, fl::mulmod(lam, ng, md), md.p);
            }
            r++;
            if (__ballot(v != 0) != 0 && lane == 0) atomicOr(&S.nzmask[r & 1], 1u << wave);
            __syncthreads();
        }
    }
    __syncthreads();
}

// The raw basis for check and merge: the kb rows in use of both planes
// (16-byte chunks; rows past kb are never read), their pivot columns and
// their rows.
__device__ void save_raw(const GreedyLds &S, PanelState *ps) {
    const uint32_t nch = S.kb * 8;  // 16-byte chunks per plane
    for (uint32_t i = threadIdx.x; i < 2 * nch; i += blockDim.x) {
        const bool gpl = i >= nch;
        const uint32_t c = gpl ? i - nch : i;
        const uint4 v = ((const uint4 *)(gpl ? &S.Bg[0][0] : &S.Bv[0][0]))[c];
        ((uint4 *)(gpl ? ps->Bg : ps->Bv))[c] = v;
    }
    if (threadIdx.x < 64) {
        ps->Cc[threadIdx.x] = S.Cc[threadIdx.x];
        ps->Qs[threadIdx.x] = S.Qo[threadIdx.x];
    }
    if (threadIdx.x == 0) ps->kb = S.kb;
}

// Publish the panel result: basis rows ordered by pivot column, G, and the
// global pivot bookkeeping (rank0 = rank before this panel).
// All threads of the block call it (the rows of G are dealt to the waves).
__device__ void finalize(const GreedyLds &S, PanelState *ps, uint32_t c0, uint32_t rank0,
                         uint32_t *is_piv, uint32_t *piv_row, uint32_t *piv_col, uint32_t *d_rank) {
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t kb = S.kb;
    uint32_t my_t = 0;  // lane j < kb: the position of basis row j by pivot column
    if (lane < kb) {
        const uint32_t cj = S.Cc[lane];
        for (uint32_t j = 0; j < kb; j++) my_t += S.Cc[j] < cj ? 1 : 0;
    }
    for (uint32_t j = wave; j < kb; j += nw) {
        const uint32_t t = (uint32_t)__builtin_amdgcn_readlane((int)my_t, (int)j);
        ps->G[t * 64 + lane] = lane < kb ? S.Bg[j][lane] : 0;
    }
    if (wave != 0) return;
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

// Panel step 1: the probe basis, from one representative row per leading
// column of the rows nonzero on the panel (listed, with their first nonzero
// column, by step 0).  One workgroup per matrix.
//
// Rows with different first nonzero columns are independent, so the
// representatives need no elimination search: sorted by first nonzero column
// (descending), their panel parts form a matrix whose restriction T to the
// leading columns is lower triangular, and the reduced basis is T^-1 times
// the rows (coefficients: T^-1 itself).  Any listed row may represent its
// leading column (the panel's final basis, after check and merge, spans all
// of its rows whichever are picked), so the pick is a plain LDS store.
//
// The back substitution runs over groups of kProbeGroup slots.  A row's
// entries at the leading columns of the groups after its own are never
// changed by reduction against the earlier groups' finished rows (those are
// zero left of their own, larger, leading columns), so the solve of each
// group among itself commutes with the reductions against the earlier
// groups: first every group is solved among itself (one wave per group, all
// groups at once, in registers: a row's multipliers are read from it as it
// is on entry, the group's finished rows being in reduced form), then the
// groups are finished in order, each reducing every later slot (all waves,
// one barrier per group).  Every pivot's inverse is known from the start,
// since the leading entries never change.  In the matrices of the method the
// representatives span most of the panel; check and merge add what is
// missing.
constexpr uint32_t kProbeGroup = 8;
constexpr uint32_t kLeadLoads = 16;  // lead entries in flight per thread

__global__ __launch_bounds__(kGreedyThreads) void k_ech_probe(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                              const uint32_t *__restrict__ ids, uint32_t P) {
    typedef __attribute__((address_space(1))) const uint32_t gu32;
    __shared__ GreedyLds S;
    __shared__ uint32_t rank0_s;
    __shared__ uint32_t s_rep[kPanel];  // a listed row per leading column
    const FlEchTask &t = tasks[ids[blockIdx.x]];
    if (P >= t.npanels) return;
    const uint32_t c0 = P * kPanel, pw = t.cols - c0 < kPanel ? t.cols - c0 : kPanel;
    PanelState *ps = panel_state(t, P);
    const uint32_t n = t.counts[3 * P];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if (threadIdx.x < kPanel) s_rep[threadIdx.x] = ~0u;
    __syncthreads();
    // a listed row of every leading column: a chunk of lead entries and list
    // rows is loaded before any is used (the loads overlap); the first store
    // seen wins (a store after it overwrites with another valid row)
    const gu32 *lead = (const gu32 *)t.nzlead, *list = (const gu32 *)t.nzlist;
    for (uint32_t base = 0; base < n; base += kLeadLoads * blockDim.x) {
        uint32_t l[kLeadLoads], r[kLeadLoads];
#pragma unroll
        for (uint32_t u = 0; u < kLeadLoads; u++) {
            const uint32_t i = base + u * blockDim.x + threadIdx.x;
            l[u] = lead[i < n ? i : 0];
            r[u] = list[i < n ? i : 0];
        }
#pragma unroll
        for (uint32_t u = 0; u < kLeadLoads; u++) {
            const uint32_t i = base + u * blockDim.x + threadIdx.x;
            if (i < n && s_rep[l[u]] == ~0u) s_rep[l[u]] = r[u];
        }
    }
    __syncthreads();
    // slots by leading column, descending (lane 0 takes column 63)
    if (wave == 0) {
        const uint32_t c = kPanel - 1 - lane;
        const uint32_t at = s_rep[c];
        const uint64_t have = __ballot(at != ~0u);
        if (at != ~0u) {
            const uint32_t s = (uint32_t)__popcll(have & ((1ull << lane) - 1));
            S.Cc[s] = c;
            S.Qo[s] = at;
        }
        if (lane == 0) {
            S.kb = (uint32_t)__popcll(have);
            rank0_s = *t.d_rank;
            ps->nflag = 0;
            ps->rank0 = rank0_s;
        }
    }
    __syncthreads();
    const uint32_t kr = S.kb;
    // the representatives' panel parts (one wave per row) and unit coefficients
    for (uint32_t s = wave; s < kr; s += nw) {
        S.Bv[s][lane] = lane < pw ? t.D[(uint64_t)S.Qo[s] * t.ld + c0 + lane] : 0;
        S.Bg[s][lane] = lane == s ? 1 : 0;
    }
    __syncthreads();
    const uint32_t ng = (kr + kProbeGroup - 1) / kProbeGroup;
    static_assert(kGreedyThreads / 64 >= kPanel / kProbeGroup, "one wave per group");
    if (wave < ng) {
        // group `wave` among itself: rows j = slot g0 + j in registers,
        // finished in order
        const uint32_t g0 = wave * kProbeGroup, g1 = g0 + kProbeGroup < kr ? g0 + kProbeGroup : kr;
        const uint32_t ccv = S.Cc[lane];  // lane t: Cc[t]
        // lane s of the group: inverse of slot s's leading entry
        const uint32_t inv = lane >= g0 && lane < g1 ? fl::invmod(S.Bv[lane][ccv], md) : 0;
        uint32_t v[kProbeGroup], g[kProbeGroup];
#pragma unroll
        for (uint32_t j = 0; j < kProbeGroup; j++) {
            v[j] = g0 + j < g1 ? S.Bv[g0 + j][lane] : 0;
            g[j] = g0 + j < g1 ? S.Bg[g0 + j][lane] : 0;
        }
#pragma unroll
        for (uint32_t j = 0; j < kProbeGroup; j++) {
            if (g0 + j >= g1) break;
            uint32_t hv = 0, lv = 0, hg = 0, lg = 0;
#pragma unroll
            for (uint32_t u = 0; u < j; u++) {
                const int cidx = __builtin_amdgcn_readlane((int)ccv, (int)(g0 + u));
                const uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)v[j], cidx);
                hv = fl::mad24(lam >> 8, v[u], hv);
                lv = fl::mad24(lam & 0xffu, v[u], lv);
                hg = fl::mad24(lam >> 8, g[u], hg);
                lg = fl::mad24(lam & 0xffu, g[u], lg);
            }
            const uint32_t is = (uint32_t)__builtin_amdgcn_readlane((int)inv, (int)(g0 + j));
            v[j] = fl::mulmod(fl::submod(v[j], fl::fold_pair(hv, lv, md), md.p), is, md);
            g[j] = fl::mulmod(fl::submod(g[j], fl::fold_pair(hg, lg, md), md.p), is, md);
        }
#pragma unroll
        for (uint32_t j = 0; j < kProbeGroup; j++) {
            if (g0 + j < g1) {
                S.Bv[g0 + j][lane] = (uint16_t)v[j];
                S.Bg[g0 + j][lane] = (uint16_t)g[j];
            }
        }
    }
    __syncthreads();
    // group h is finished: every later slot is reduced against it
    for (uint32_t h = 0; h + 1 < ng; h++) {
        const uint32_t g0 = h * kProbeGroup, g1 = g0 + kProbeGroup;
        for (uint32_t s = g1 + wave; s < kr; s += nw) {
            uint32_t v = S.Bv[s][lane], g = S.Bg[s][lane];
            reduce_against(md, v, g, g0, g1, S.Bv, S.Bg, S.Cc, lane, true);
            S.Bv[s][lane] = (uint16_t)v;
            S.Bg[s][lane] = (uint16_t)g;
        }
        __syncthreads();
    }
    const uint32_t rank0 = rank0_s;
    save_raw(S, ps);
    finalize(S, ps, c0, rank0, t.is_piv, t.piv_row, t.piv_col, t.d_rank);
}

// Panel steps 0 and 2.  Step 0 (use_basis = 0): every remaining row that is
// nonzero on the panel goes to the nonzero list.  Step 2: every row of that
// list is reduced against the probe basis in ps; rows left nonzero (outside
// its span) go to the flagged list.  One wave per row, 8 rows per wave, 32
// rows per workgroup.
struct __attribute__((aligned(16))) CheckLds {
    uint16_t Bv[64][64];
    uint32_t Cc[64];
};

// One workgroup (32 rows) of the check of panel P for table entry ti.  The
// wave's 8 row ids, pivot flags and panel rows are fetched with independent
// loads, reduced together, and listed with one append per workgroup.
__device__ void check_tile(const fl::Mod &md, const FlEchTask &t, uint32_t bx, uint32_t P, int use_basis,
                           CheckLds &L) {
    const uint32_t c0 = P * kPanel, pw = t.cols - c0 < kPanel ? t.cols - c0 : kPanel;
    const PanelState *ps = panel_state(t, P);
    const uint32_t *in_list = use_basis ? t.nzlist : nullptr;
    uint32_t *out_list = use_basis ? t.flist : t.nzlist;
    uint32_t *out_count = t.counts + 3 * P + (use_basis ? 1 : 0);
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t kb = use_basis ? ps->kb : 0;
    const uint32_t n = in_list ? t.counts[3 * P] : t.rows;
    if (bx * 32 >= n) return;
    // basis rows: kb * 64 halfwords = kb * 8 16-byte chunks (at most 512)
    {
        const uint4 *src = (const uint4 *)ps->Bv;
        uint4 *dst = (uint4 *)&L.Bv[0][0];
        const uint32_t nv = kb * 8, i0 = threadIdx.x, i1 = threadIdx.x + 256;
        uint4 a = make_uint4(0, 0, 0, 0), b = a;
        if (i0 < nv) a = src[i0];
        if (i1 < nv) b = src[i1];
        if (i0 < nv) dst[i0] = a;
        if (i1 < nv) dst[i1] = b;
    }
    if (threadIdx.x < 64) L.Cc[threadIdx.x] = use_basis ? ps->Cc[threadIdx.x] : 0;
    // lane u < 8: row id and liveness of the wave's row u
    const uint32_t idx0 = (bx * 4 + wave) * 8;
    uint32_t my_row = 0, my_live = 0;
    if (lane < 8 && idx0 + lane < n) {
        my_row = in_list ? in_list[idx0 + lane] : idx0 + lane;
        my_live = (kb < pw && !t.is_piv[my_row]) ? 1u : 0u;
    }
    const uint32_t col = c0 + (lane < pw ? lane : 0);
    uint32_t v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t row = (uint32_t)__builtin_amdgcn_readlane((int)my_row, u);
        v[u] = t.D[(uint64_t)row * t.ld + col];  // row 0 stands in for rows not live
    }
    uint32_t live = 0;
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const bool lv = __builtin_amdgcn_readlane((int)my_live, u) != 0;
        live |= lv ? 1u << u : 0u;
        if (!lv || lane >= pw) v[u] = 0;
    }
    __syncthreads();
    if (kb && live) reduce_rows8(md, v, kb, L.Bv, L.Cc, lane);
    uint32_t mask = 0, my_lead = 0;
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint64_t nz = __ballot(v[u] != 0);
        mask |= nz != 0 ? 1u << u : 0u;
        if (lane == (uint32_t)u) my_lead = nz ? (uint32_t)__ffsll((long long)nz) - 1 : 0;
    }
    // step 0 also records each listed row's first nonzero column
    block_append8(mask & live, my_row, out_list, out_count, use_basis ? nullptr : t.nzlead, my_lead);
    // (no fence: the lists are read by later launches on the same stream)
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
// with the flagged rows and publish the final result.  Run by one whole
// workgroup (any number of waves).
__device__ void merge_panel(const fl::Mod &md, const FlEchTask &t, uint32_t P, GreedyLds &S) {
    const uint32_t n = t.counts[3 * P + 1];
    const uint32_t c0 = P * kPanel, pw = t.cols - c0 < kPanel ? t.cols - c0 : kPanel;
    PanelState *ps = panel_state(t, P);
    // the raw basis: 2 x 512 16-byte chunks
    for (uint32_t i = threadIdx.x; i < 1024; i += blockDim.x) {
        const uint4 *src = (const uint4 *)(i < 512 ? ps->Bv : ps->Bg);
        uint4 *dst = (uint4 *)(i < 512 ? &S.Bv[0][0] : &S.Bg[0][0]);
        dst[i & 511] = src[i & 511];
    }
    if (threadIdx.x < 64) {
        S.Cc[threadIdx.x] = ps->Cc[threadIdx.x];
        S.Qo[threadIdx.x] = ps->Qs[threadIdx.x];
    }
    if (threadIdx.x == 0) S.kb = ps->kb;
    __syncthreads();
    const uint32_t rank0 = ps->rank0;
    for (uint32_t base = 0; base < n && S.kb < pw; base += blockDim.x) {
        const uint32_t cnt = n - base < blockDim.x ? n - base : blockDim.x;
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
// 64 columns per workgroup, lane = column: every wave holds the column's k
// entries of the selected rows in registers (independent loads) and computes
// the rows t = wave, wave + 4, ... (G read from LDS 8 entries at a time;
// G[t][s] = 0 for s >= k, so the sums run over whole groups of 8); the limb
// planes are assembled in LDS.
struct __attribute__((aligned(16))) ULds {
    uint16_t Gs[64 * 64];
    uint16_t Us[64][64];
    uint32_t qs[128];  // U: selected rows; L: pivot columns and rows
};

// One workgroup (64 columns from c0 + lo + 64 bx, below c0 + hi) of U for
// panel P.
__device__ void U_tile(const fl::Mod &md, const FlEchTask &tk, uint32_t bx, uint32_t P, ULds &S, uint32_t lo,
                       uint32_t hi) {
    uint16_t *Gs = S.Gs;
    uint32_t *qs = S.qs;
    const PanelState *ps = panel_state(tk, P);
    const uint32_t c0 = P * kPanel;
    const uint32_t cols = hi < tk.cols - c0 ? c0 + hi : tk.cols;
    const uint32_t cbase = c0 + lo + bx * 64;
    if (cbase >= cols) return;
    const uint16_t *D = tk.D;
    const uint64_t ld = tk.ld, ldu = tk.ldu;
    uint16_t *U = tk.U;
    int8_t *Uh = tk.Uh, *Ul = tk.Ul;
    const uint32_t k = ps->k;
    if (k == 0) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    {
        const uint4 *g4 = (const uint4 *)ps->G;
        uint4 *s4 = (uint4 *)Gs;
        const uint4 a = g4[threadIdx.x], b = g4[threadIdx.x + 256];
        s4[threadIdx.x] = a;
        s4[threadIdx.x + 256] = b;
    }
    if (threadIdx.x < 64) qs[threadIdx.x] = ps->Qs[threadIdx.x];
    __syncthreads();
    const uint32_t c = cbase + lane;
    const bool ok = c < cols;
    const uint32_t cc = ok ? c : cbase;  // a valid column for idle lanes
    uint32_t x[64];
#pragma unroll
    for (int s16 = 0; s16 < 4; s16++) {
        if ((uint32_t)s16 * 16 < k) {
#pragma unroll
            for (int j = 0; j < 16; j++) {
                const uint32_t s = s16 * 16 + j < k ? s16 * 16 + j : k - 1;
                x[s16 * 16 + j] = D[(uint64_t)qs[s] * ld + cc];
            }
        } else {
#pragma unroll
            for (int j = 0; j < 16; j++) x[s16 * 16 + j] = 0;
        }
    }
    for (uint32_t t = wave; t < 64; t += 4) {
        uint32_t u = 0;
        if (t < k) {
            uint32_t h = 0, l = 0;
            const uint4 *gr = (const uint4 *)(Gs + t * 64);
#pragma unroll
            for (int s8 = 0; s8 < 8; s8++) {
                if ((uint32_t)s8 * 8 < k) {
                    const uint4 gv = gr[s8];
                    const uint32_t gw[4] = {gv.x, gv.y, gv.z, gv.w};
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        const uint32_t gts = (gw[j >> 1] >> (16 * (j & 1))) & 0xffffu;
                        h = fl::mad24(gts >> 8, x[s8 * 8 + j], h);
                        l = fl::mad24(gts & 0xffu, x[s8 * 8 + j], l);
                    }
                }
            }
            u = fl::fold_pair(h, l, md);
            if (ok) U[(uint64_t)t * ldu + c] = (uint16_t)u;
        }
        S.Us[t][lane] = (uint16_t)u;
    }
    if (!Uh) return;
    __syncthreads();
    if (!ok) return;
    // wave w: bytes [16 w, 16 w + 16) of the column's 64
    uint32_t hw[4] = {0, 0, 0, 0}, lw[4] = {0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 16; i++) {
        int lh, ll;
        fl_split_limbs(S.Us[wave * 16 + i][lane], md.p, lh, ll);
        hw[i >> 2] |= (uint32_t)(lh & 0xff) << (8 * (i & 3));
        lw[i >> 2] |= (uint32_t)(ll & 0xff) << (8 * (i & 3));
    }
    *(uint4 *)(Uh + (uint64_t)(c - c0) * 64 + wave * 16) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
    *(uint4 *)(Ul + (uint64_t)(c - c0) * 64 + wave * 16) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
}

// L'[i][t] = Dt[i][Ccol[t]] - [i = Phys[t]] (0 for t >= k): the multipliers
// of panel P with the placement of U folded in (a pivot row t first loses
// its whole panel combination, Dt[Q_t] - Dt[Q_t, C] U = 0, then gains U_t),
// stored at the panel's packed slots of the block buffer Lb (256 per row;
// slots kbase .. kbase + 63 are written, the next panel's overwrite the
// tail) and, with limb
// planes, as int8 limbs.  MFMA form: the rows with a nonzero multiplier are
// listed for the panel's update, and the first time in the block also for
// the block's update.  One workgroup (32 rows): one wave per 8 rows, lane t =
// multiplier t, the 8 loads issued together, one list append per workgroup.
__device__ void L_tile(uint32_t p, const FlEchTask &tk, uint32_t bx, uint32_t P, uint32_t *ccol,
                       uint32_t *phys) {
    const PanelState *ps = panel_state(tk, P);
    const uint32_t rows = tk.rows;
    const uint16_t *D = tk.D;
    const uint64_t ld = tk.ld;
    const uint32_t b = P / kBlockPanels, slot = panel_kbase(tk, P);
    const uint64_t half = (uint64_t)(b & 1) * rows * kBlock;
    uint16_t *Lb = tk.Lb + half;
    int8_t *Lh = tk.Lbh ? tk.Lbh + half : nullptr, *Ll = tk.Lbl ? tk.Lbl + half : nullptr;
    const uint32_t t = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (bx * 32 >= rows) return;
    const uint32_t k = ps->k;
    if (k == 0) return;
    if (threadIdx.x < 64) {
        ccol[threadIdx.x] = ps->Ccol[threadIdx.x];
        phys[threadIdx.x] = ps->Phys[threadIdx.x];
    }
    __syncthreads();
    const uint32_t col = t < k ? ccol[t] : P * kPanel;  // a valid column for t >= k
    const uint32_t ph = t < k ? phys[t] : 0xffffffffu;
    const uint32_t i0 = (bx * 4 + wave) * 8;
    uint32_t x[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t i = i0 + u < rows ? i0 + u : rows - 1;
        x[u] = D[(uint64_t)i * ld + col];
    }
    uint32_t mask = 0;
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t i = i0 + u;
        if (t >= k) x[u] = 0;
        else if (ph == i) x[u] = fl::submod(x[u], 1, p);
        if (i < rows) {
            Lb[(uint64_t)i * kBlock + slot + t] = (uint16_t)x[u];
            if (Lh) {
                int h = 0, l = 0;
                fl_split_limbs(x[u], p, h, l);
                Lh[(uint64_t)i * kBlock + slot + t] = (int8_t)h;
                Ll[(uint64_t)i * kBlock + slot + t] = (int8_t)l;
                mask |= (__ballot(x[u] != 0) != 0) ? 1u << u : 0u;
            }
        }
    }
    if (!Lh) return;
    block_append8(mask, i0 + t, tk.upd_rows, tk.counts + 3 * P + 2);
    bool first = false;
    if (t < 8 && ((mask >> t) & 1u)) first = atomicMax(&tk.mark[i0 + t], b + 1) < b + 1;
    const uint32_t fmask = (uint32_t)__ballot(first) & 0xffu;
    __syncthreads();  // block_append8's shared words are reused
    block_append8(fmask, i0 + t, tk.blk_rows + (uint64_t)(b & 1) * rows, tk.blk_cnt + b);
}

// Panel steps 4 and 5 in one launch: the first grid_u workgroups compute U
// over the rest of the panel's block (four workgroups of 64 columns per
// matrix), the others gather L' (rows).
// One workgroup of steps 4 + 5 from the probe basis: the first grid_u
// workgroups of the launch compute U, the next (pre_rows) L'.
__device__ __forceinline__ void UL_tile(const fl::Mod &md, const FlEchTask *__restrict__ tasks,
                                        const uint32_t *__restrict__ ids, const uint32_t *__restrict__ pre_c,
                                        uint32_t n_c, uint32_t grid_u, const uint32_t *__restrict__ pre_rows,
                                        uint32_t n_active, uint32_t P, uint32_t bid, ULds &S) {
    if (bid < grid_u) {
        const uint32_t ti = fl_task_of(pre_c, n_c, bid / kBlockPanels);
        const FlEchTask &t = tasks[ids[ti]];
        if (P >= t.npanels) return;
        const uint32_t c0 = P * kPanel, bend = (P / kBlockPanels + 1) * kBlock;
        U_tile(md, t, bid % kBlockPanels, P, S, 0, bend - c0);
    } else {
        const uint32_t b = bid - grid_u;
        const uint32_t ti = fl_task_of(pre_rows, n_active, b);
        const FlEchTask &t = tasks[ids[ti]];
        if (P >= t.npanels) return;
        L_tile(md.p, t, b - pre_rows[ti], P, S.qs, S.qs + 64);
    }
}

// Step 3, only for the matrices whose check flagged rows (almost never): one
// workgroup per matrix merges the flagged rows into the basis, then computes
// U and L' again from the final basis, tile after tile (its row list
// restarts), so that no further launch waits on the critical path.
__global__ __launch_bounds__(256) void k_ech_merge(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                   const uint32_t *__restrict__ ids, uint32_t P) {
    __shared__ union {
        GreedyLds g;
        ULds u;
    } S;
    const FlEchTask &t = tasks[ids[blockIdx.x]];
    if (P >= t.npanels || t.counts[3 * P + 1] == 0) return;
    merge_panel(md, t, P, S.g);
    if (threadIdx.x == 0) t.counts[3 * P + 2] = 0;
    __syncthreads();  // (also: S.g is reused)
    const uint32_t c0 = P * kPanel, bend = (P / kBlockPanels + 1) * kBlock;
    for (uint32_t bx = 0; bx < kBlockPanels; bx++) {
        U_tile(md, t, bx, P, S.u, 0, bend - c0);
        __syncthreads();
    }
    for (uint32_t bx = 0; bx * 32 < t.rows; bx++) {
        L_tile(md.p, t, bx, P, S.u.qs, S.u.qs + 64);
        __syncthreads();
    }
}

// Step 2 (the check against the probe basis: workgroups from grid_ul on) and
// steps 4 + 5 with the probe basis (before them) in one launch.  Almost
// always no row is flagged and the probe basis is final; otherwise the merge
// kernel redoes U and L' for the matrices concerned.
__global__ __launch_bounds__(256) void k_ech_check_UL(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                      const uint32_t *__restrict__ ids,
                                                      const uint32_t *__restrict__ pre_c, uint32_t n_c,
                                                      uint32_t grid_u, const uint32_t *__restrict__ pre_rows,
                                                      uint32_t n_active, uint32_t grid_rows, uint32_t P) {
    __shared__ union {
        ULds u;
        CheckLds c;
    } S;
    const uint32_t grid_ul = grid_u + grid_rows;
    if (blockIdx.x < grid_ul) {
        UL_tile(md, tasks, ids, pre_c, n_c, grid_u, pre_rows, n_active, P, blockIdx.x, S.u);
    } else {
        const uint32_t b = blockIdx.x - grid_ul;
        const uint32_t ti = fl_task_of(pre_rows, n_active, b);
        const FlEchTask &t = tasks[ids[ti]];
        if (P >= t.npanels) return;
        check_tile(md, t, b - pre_rows[ti], P, 1, S.c);
    }
}

// Panel P's update of the rest of its block, int8 MFMA form: rows with a
// nonzero multiplier, one 64-row x 128-column tile per workgroup (two column
// tiles per matrix: workgroup x = 2 slot + tile; row block blockIdx.y;
// blocks beyond the list or the block exit at once).
__global__ __launch_bounds__(256) void k_ech_update_mfma(fl::Mod md, uint32_t bias, uint32_t c16,
                                                         const FlEchTask *__restrict__ tasks,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint32_t *__restrict__ pre, uint32_t ntask,
                                                         uint32_t P) {
    __shared__ __attribute__((aligned(16))) uint16_t sv[64 * fl_mfma::kRank64Ld];
    __shared__ uint32_t rows_s[64];
    // four 64-column tiles per matrix (the panel's block has at most 256
    // columns from the panel on): more workgroups in flight on this
    // latency-bound step
    const uint32_t ti = fl_task_of(pre, ntask, blockIdx.x >> 2), bx = blockIdx.x & 3;
    const FlEchTask &t = tasks[ids[ti]];
    if (P >= t.npanels) return;
    const uint32_t M = t.counts[3 * P + 2];
    if (blockIdx.y * 64 >= M || panel_state(t, P)->k == 0) return;
    const uint32_t c0 = P * kPanel, b = P / kBlockPanels, bend = (b + 1) * kBlock;
    const uint32_t N = (bend < t.cols ? bend : t.cols) - c0;
    if (bx * 64 >= N) return;
    const uint64_t half = (uint64_t)(b & 1) * t.rows * kBlock, slot = panel_kbase(t, P);
    fl_mfma::mfma_rankk_tile<1, 4>(md, bias, c16, t.Lbh + half + slot, t.Lbl + half + slot, kBlock, t.Uh, t.Ul,
                                   64, t.upd_rows, M, t.D + c0, t.ld, N, bx, blockIdx.y, sv, rows_s);
}

// The same, VALU form: every row, one 256-column tile per matrix, row blocks
// (of 32) blockIdx.y, blockIdx.y + gridDim.y, ...
__global__ __launch_bounds__(256) void k_ech_update_valu(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                         const uint32_t *__restrict__ ids,
                                                         const uint32_t *__restrict__ pre, uint32_t ntask,
                                                         uint32_t P) {
    const uint32_t ti = fl_task_of(pre, ntask, blockIdx.x);
    const FlEchTask &t = tasks[ids[ti]];
    if (P >= t.npanels) return;
    const PanelState *ps = panel_state(t, P);
    const uint32_t c0 = P * kPanel, b = P / kBlockPanels, bend = (b + 1) * kBlock;
    const uint32_t N = (bend < t.cols ? bend : t.cols) - c0;
    const uint16_t *A = t.Lb + (uint64_t)(b & 1) * t.rows * kBlock + panel_kbase(t, P);
    for (uint32_t by = blockIdx.y; by * 32 < t.rows; by += gridDim.y)
        fl_valu::valu_gemm_tile(md, t.rows, N, 0, &ps->k, A, kBlock, t.U + c0, t.ldu, t.D + c0, t.ld, 0, by);
}

// U of block b for the columns right of it.  With D0 = Dt at the start of
// the block (the columns right of it are untouched by the block's panels)
// and R_j = D0[Q_j] the selected rows of panel j of the block:
//   U_j = G_j (R_j - sum_{j' < j} L'_j'[Q_j] U_j')
// (the rows of panel j as the earlier panels of the block left them, then
// panel j's combination).  One workgroup per 64 columns, lane = column:
// wave w computes the entries s = w, w + 4, ... of the bracket, then the
// rows t = w, w + 4, ... of U_j; the U rows of the block are kept in LDS.
// Output: Ubh/Ubl (256 bytes per column, by absolute column) or Ub (rows
// 64 j + t, u16).
struct __attribute__((aligned(16))) UblkLds {
    uint16_t Us[kBlock][64];
    uint16_t Xs[64][64];
    uint32_t qs[kBlockPanels][64];  // the panels' selected rows (16-wave form)
};

template <int NT>
__global__ __launch_bounds__(NT) void k_ech_ublk(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                 const uint32_t *__restrict__ ids,
                                                 const uint32_t *__restrict__ pre, uint32_t ntask, uint32_t B,
                                                 uint32_t lo, uint32_t span) {
    constexpr uint32_t NW = NT / 64;  // waves: entries s and rows t are dealt round-robin
    __shared__ UblkLds S;
    const uint32_t ti = fl_task_of(pre, ntask, blockIdx.x);
    const FlEchTask &t = tasks[ids[ti]];
    const uint32_t P0 = B * kBlockPanels;
    if (P0 >= t.npanels) return;
    const uint32_t start = (B + 1) * kBlock + lo;
    const uint32_t end = span < t.cols - start ? start + span : t.cols;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t wave = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const uint32_t c = start + (blockIdx.x - pre[ti]) * 64 + lane;
    const bool ok = c < end;
    const uint32_t cc = ok ? c : start;  // a valid column for idle lanes
    const uint16_t *Lb = t.Lb + (uint64_t)(B & 1) * t.rows * kBlock;
    {
        uint4 *z = (uint4 *)&S.Us[0][0];
        for (uint32_t i = threadIdx.x; i < kBlock * 64 * 2 / 16; i += NT) z[i] = make_uint4(0, 0, 0, 0);
    }
    __syncthreads();
    const uint32_t nj = t.npanels - P0 < kBlockPanels ? t.npanels - P0 : kBlockPanels;
    uint32_t kj[kBlockPanels], kb[kBlockPanels];  // pivots and packed K base of each panel
#pragma unroll
    for (uint32_t j = 0; j < kBlockPanels; j++) kj[j] = j < nj ? panel_state(t, P0 + j)->k : 0;
    kb[0] = 0;
#pragma unroll
    for (uint32_t j = 1; j < kBlockPanels; j++) kb[j] = kb[j - 1] + ((kj[j - 1] + 15) & ~15u);
    if constexpr (NW == 16) {
        // Every load of the four stages depends only on the panel states, so
        // all are issued up front, in two rounds: the panels' selected rows
        // (into LDS) with the rows of G (registers), then each entry's value
        // and multipliers; the stages then run on registers and LDS only.
        // Entry s of stage j and row tt of U_j: s, tt = wave + 16 i, i < 4.
        constexpr uint32_t kE = 64 / NW;
        for (uint32_t i = threadIdx.x; i < kBlockPanels * 64; i += NT) {
            const uint32_t j = i >> 6, s = i & 63;
            S.qs[j][s] = s < kj[j] ? panel_state(t, P0 + j)->Qs[s] : 0;
        }
        uint32_t gq[kBlockPanels][kE];
#pragma unroll
        for (uint32_t j = 0; j < kBlockPanels; j++)
#pragma unroll
            for (uint32_t i = 0; i < kE; i++) {
                const uint32_t tt = wave + NW * i;
                gq[j][i] = tt < kj[j] ? panel_state(t, P0 + j)->G[tt * 64 + lane] : 0;
            }
        __syncthreads();
        // stage j's multipliers on the j earlier panels: cf[j (j - 1) / 2 * kE + i j + jj]
        uint32_t xq[kBlockPanels][kE], cf[kE * kBlockPanels * (kBlockPanels - 1) / 2];
#pragma unroll
        for (uint32_t j = 0; j < kBlockPanels; j++)
#pragma unroll
            for (uint32_t i = 0; i < kE; i++) {
                const uint32_t s = wave + NW * i;
                const uint32_t q = S.qs[j][s < kj[j] ? s : 0];  // row 0 stands in for absent entries
                xq[j][i] = t.D[(uint64_t)q * t.ld + cc];
#pragma unroll
                for (uint32_t jj = 0; jj < j; jj++)
                    cf[j * (j - 1) / 2 * kE + i * j + jj] = Lb[(uint64_t)q * kBlock + kb[jj] + lane];
            }
#pragma unroll
        for (uint32_t j = 0; j < kBlockPanels; j++) {
            const uint32_t k = kj[j];
            if (k == 0) continue;
#pragma unroll
            for (uint32_t i = 0; i < kE; i++) {
                const uint32_t s = wave + NW * i;
                if (s >= k) break;
                uint32_t h = 0, l = 0;
#pragma unroll
                for (uint32_t jj = 0; jj < j; jj++) {
                    const uint32_t cfv = cf[j * (j - 1) / 2 * kE + i * j + jj];
#pragma unroll 8
                    for (uint32_t tt = 0; tt < kj[jj]; tt++) {
                        const uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)cfv, (int)tt);
                        const uint32_t u = S.Us[jj * kPanel + tt][lane];
                        h = fl::mad24(lam >> 8, u, h);
                        l = fl::mad24(lam & 0xffu, u, l);
                    }
                }
                S.Xs[s][lane] = (uint16_t)fl::submod(xq[j][i], fl::fold_pair(h, l, md), md.p);
            }
            __syncthreads();
#pragma unroll
            for (uint32_t i = 0; i < kE; i++) {
                const uint32_t tt = wave + NW * i;
                if (tt >= k) break;
                uint32_t h = 0, l = 0;
#pragma unroll 8
                for (uint32_t s2 = 0; s2 < k; s2++) {
                    const uint32_t gv = (uint32_t)__builtin_amdgcn_readlane((int)gq[j][i], (int)s2);
                    const uint32_t xv = S.Xs[s2][lane];
                    h = fl::mad24(gv >> 8, xv, h);
                    l = fl::mad24(gv & 0xffu, xv, l);
                }
                S.Us[j * kPanel + tt][lane] = (uint16_t)fl::fold_pair(h, l, md);
            }
            __syncthreads();
        }
    } else {
#pragma unroll
    for (uint32_t j = 0; j < kBlockPanels; j++) {
        const PanelState *ps = panel_state(t, P0 + j);
        const uint32_t k = kj[j];
        if (k == 0) continue;
        // bracket entries s = wave + 4 i: row q's entry and its multipliers
        // on the earlier panels (lane tt holds L'_jj[q][tt]), fetched one
        // entry ahead
        uint32_t s = wave, q = s < k ? ps->Qs[s] : 0;
        uint32_t x_n = t.D[(uint64_t)q * t.ld + cc], cf_n[kBlockPanels - 1];
#pragma unroll
        for (uint32_t jj = 0; jj < kBlockPanels - 1; jj++)
            cf_n[jj] = jj < j ? Lb[(uint64_t)q * kBlock + kb[jj] + lane] : 0;
        for (; s < k; s += NW) {
            const uint32_t x = x_n;
            uint32_t cf[kBlockPanels - 1];
#pragma unroll
            for (uint32_t jj = 0; jj < kBlockPanels - 1; jj++) cf[jj] = cf_n[jj];
            if (s + NW < k) {
                const uint32_t qn = ps->Qs[s + NW];
                x_n = t.D[(uint64_t)qn * t.ld + cc];
#pragma unroll
                for (uint32_t jj = 0; jj < kBlockPanels - 1; jj++)
                    if (jj < j) cf_n[jj] = Lb[(uint64_t)qn * kBlock + kb[jj] + lane];
            }
            uint32_t h = 0, l = 0;
#pragma unroll
            for (uint32_t jj = 0; jj < kBlockPanels - 1; jj++) {
                if (jj >= j) break;
                for (uint32_t tt = 0; tt < kj[jj]; tt++) {
                    const uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)cf[jj], (int)tt);
                    const uint32_t u = S.Us[jj * kPanel + tt][lane];
                    h = fl::mad24(lam >> 8, u, h);
                    l = fl::mad24(lam & 0xffu, u, l);
                }
            }
            // at most 192 terms of 2^8 x 2^16: no intermediate fold needed
            S.Xs[s][lane] = (uint16_t)fl::submod(x, fl::fold_pair(h, l, md), md.p);
        }
        __syncthreads();
        // rows tt = wave + 4 i of U_j (lane s holds G_j[tt][s]), one row ahead
        uint32_t g_n = wave < k ? ps->G[wave * 64 + lane] : 0;
        for (uint32_t tt = wave; tt < k; tt += NW) {
            const uint32_t gr = g_n;
            if (tt + NW < k) g_n = ps->G[(tt + NW) * 64 + lane];
            uint32_t h = 0, l = 0;
            for (uint32_t s2 = 0; s2 < k; s2++) {
                const uint32_t gv = (uint32_t)__builtin_amdgcn_readlane((int)gr, (int)s2), xv = S.Xs[s2][lane];
                h = fl::mad24(gv >> 8, xv, h);
                l = fl::mad24(gv & 0xffu, xv, l);
            }
            S.Us[j * kPanel + tt][lane] = (uint16_t)fl::fold_pair(h, l, md);
        }
        __syncthreads();
    }
    }
    if (!ok || wave >= 4) return;
    // packed K position x -> the row of S.Us holding it (kBlock: padding,
    // zero): panel j's pivot x - kb[j] when kb[j] <= x < kb[j] + kj[j]
    auto urow = [&](uint32_t x) {
        uint32_t r = kBlock;
#pragma unroll
        for (uint32_t j = 0; j < kBlockPanels; j++)
            if (x >= kb[j] && x < kb[j] + kj[j]) r = j * kPanel + (x - kb[j]);
        return r;
    };
    if (t.Ubh) {
        // wave w: bytes [64 w, 64 w + 64) of the column's 256-byte rows
        const uint64_t off = (uint64_t)(B & 1) * (t.cols + kBlock) * kBlock + (uint64_t)c * kBlock + wave * 64;
        uint32_t hw[16], lw[16];
#pragma unroll
        for (int i = 0; i < 16; i++) {
            hw[i] = lw[i] = 0;
#pragma unroll
            for (int e = 0; e < 4; e++) {
                int lh, ll;
                const uint32_t r = urow(wave * 64 + 4 * i + e);
                fl_split_limbs(r < kBlock ? S.Us[r][lane] : 0u, md.p, lh, ll);
                hw[i] |= (uint32_t)(lh & 0xff) << (8 * e);
                lw[i] |= (uint32_t)(ll & 0xff) << (8 * e);
            }
        }
        uint4 *dh = (uint4 *)(t.Ubh + off), *dl = (uint4 *)(t.Ubl + off);
#pragma unroll
        for (int i = 0; i < 4; i++) {
            dh[i] = make_uint4(hw[4 * i], hw[4 * i + 1], hw[4 * i + 2], hw[4 * i + 3]);
            dl[i] = make_uint4(lw[4 * i], lw[4 * i + 1], lw[4 * i + 2], lw[4 * i + 3]);
        }
    } else {
        uint16_t *Ub = t.Ub + (uint64_t)(B & 1) * kBlock * t.ldu;
        for (uint32_t x = wave; x < kBlock; x += 4) {
            const uint32_t r = urow(x);
            Ub[(uint64_t)x * t.ldu + c] = r < kBlock ? S.Us[r][lane] : 0;
        }
    }
}

// Block B's rank-256 update of columns [start, end) (start = 256 (B + 1) +
// lo), int8 MFMA form: the rows listed for the block, tiles of 64 RT rows x
// 16 NJ columns.  A workgroup owns one row block (blockIdx.x) and walks the
// column tiles blockIdx.y, blockIdx.y + gridDim.y, ... (`gcols` in all, from
// the prefix), keeping the row block's multiplier fragments in registers.
// One pass of the block update over the matrices whose block needs K
// steps of 64 in (KS_MIN, KS] (the block's packed K rounded up); the others
// are skipped (the kernel runs a pass for at most two steps, then one for
// more, so that both kinds cost one launch and the registers of one pass).
template <int RT, int NJ, int KS, int KS_MIN>
__device__ __forceinline__ void blk_update_pass(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                                const FlEchTask *__restrict__ tasks,
                                                const uint32_t *__restrict__ ids, const uint32_t *__restrict__ pre,
                                                uint32_t ntask, uint32_t gcols, uint32_t B, uint32_t lo,
                                                uint32_t span, uint16_t *sv, uint32_t *rows_s) {
    constexpr uint32_t kRows = 64 * RT;  // rows of a workgroup's block
    fl_mfma::RankkRows<KS, RT> R;
    fl_mfma::RankkC<RT, NJ> T;   // (KS <= 2) the C tile of column tile pf, loaded ahead
    uint32_t pf = 0xffffffffu;
    uint32_t cur = 0xffffffffu;  // task whose row block is loaded
    for (uint32_t cy = blockIdx.y; cy < gcols; cy += gridDim.y) {
        const uint32_t ti = fl_task_of(pre, ntask, cy);
        const FlEchTask &t = tasks[ids[ti]];
        if (B * kBlockPanels >= t.npanels) continue;
        const uint32_t M = t.blk_cnt[B];
        if (blockIdx.x * kRows >= M) continue;
        {
            const uint32_t steps = (block_k(t, B) + 63) / 64;
            if (steps > KS || steps <= KS_MIN) continue;
        }
        const uint32_t start = (B + 1) * kBlock + lo;
        const uint32_t end = span < t.cols - start ? start + span : t.cols;
        if (ti != cur) {
            const uint64_t lhalf = (uint64_t)(B & 1) * t.rows * kBlock;
            __syncthreads();  // rows_s of the previous task is still read
            fl_mfma::rankk_rows<KS, RT>(t.Lbh + lhalf, t.Lbl + lhalf, kBlock,
                                                  t.blk_rows + (uint64_t)(B & 1) * t.rows, M, blockIdx.x, rows_s, R);
            cur = ti;
        }
        const uint64_t uoff = (uint64_t)(B & 1) * (t.cols + kBlock) * kBlock + (uint64_t)start * kBlock;
        if constexpr (KS <= 2) {
            // the C tile of this workgroup's next column tile of the same
            // matrix (same rows) is loaded while this one is computed
            if (pf != cy) fl_mfma::rankk_cload<RT, NJ>(T, t.D + start, t.ld, end - start, cy - pre[ti], rows_s);
            const uint32_t nx = cy + gridDim.y;
            const bool more = nx < gcols && fl_task_of(pre, ntask, nx) == ti;
            fl_mfma::RankkC<RT, NJ> Tn;
            if (more) fl_mfma::rankk_cload<RT, NJ>(Tn, t.D + start, t.ld, end - start, nx - pre[ti], rows_s);
            fl_mfma::rankk_cols_loaded<KS, RT, NJ>(md, bias, c16, R, t.Ubh + uoff, t.Ubl + uoff, kBlock, t.D + start,
                                                   t.ld, end - start, cy - pre[ti], sv, T);
            if (more) {
                T = Tn;
                pf = nx;
            }
        } else {
            fl_mfma::rankk_cols<KS, RT, NJ>(md, bias, c16, R, t.Ubh + uoff, t.Ubl + uoff, kBlock, t.D + start, t.ld,
                                            end - start, cy - pre[ti], sv, rows_s);
        }
        __syncthreads();  // sv is reused by the next tile
    }
}

template <int RT, int NJ>
__global__ __launch_bounds__(256) void k_ech_update_blk_mfma(fl::Mod md, uint32_t bias, uint32_t c16,
                                                             const FlEchTask *__restrict__ tasks,
                                                             const uint32_t *__restrict__ ids,
                                                             const uint32_t *__restrict__ pre, uint32_t ntask,
                                                             uint32_t gcols, uint32_t B, uint32_t lo, uint32_t span) {
    __shared__ __attribute__((aligned(16))) uint16_t sv[64 * RT * fl_mfma::kRank64Ld];
    __shared__ uint32_t rows_s[64 * RT];
    blk_update_pass<RT, NJ, 2, 0>(md, bias, c16, tasks, ids, pre, ntask, gcols, B, lo, span, sv, rows_s);
    __syncthreads();  // rows_s and sv are reused
    blk_update_pass<RT, NJ, kBlockPanels, 2>(md, bias, c16, tasks, ids, pre, ntask, gcols, B, lo, span, sv,
                                             rows_s);
}

// The same, VALU form: every row, 256-column tiles from the prefix, row
// blocks (of 32) blockIdx.y, blockIdx.y + gridDim.y, ...
__global__ __launch_bounds__(256) void k_ech_update_blk_valu(fl::Mod md, const FlEchTask *__restrict__ tasks,
                                                             const uint32_t *__restrict__ ids,
                                                             const uint32_t *__restrict__ pre, uint32_t ntask,
                                                             uint32_t B, uint32_t lo, uint32_t span) {
    const uint32_t ti = fl_task_of(pre, ntask, blockIdx.x);
    const FlEchTask &t = tasks[ids[ti]];
    if (B * kBlockPanels >= t.npanels) return;
    const uint32_t start = (B + 1) * kBlock + lo;
    const uint32_t end = span < t.cols - start ? start + span : t.cols;
    const uint16_t *A = t.Lb + (uint64_t)(B & 1) * t.rows * kBlock;
    const uint16_t *Ub = t.Ub + (uint64_t)(B & 1) * kBlock * t.ldu + start;
    for (uint32_t by = blockIdx.y; by * 32 < t.rows; by += gridDim.y)
        fl_valu::valu_gemm_tile(md, t.rows, end - start, kBlock, nullptr, A, kBlock, Ub, t.ldu, t.D + start,
                                t.ld, blockIdx.x - pre[ti], by);
}

// Prefix tables: entry [i][x + 1] = workgroups of matrices ids[0..x] for panel
// or block i, each counting ceil(min(cols - c, span) / tile) tiles over
// [c, c + span), c = stride i + off (0 when cols <= c).
__global__ void k_ech_prefixes(const FlEchTask *__restrict__ tasks, const uint32_t *__restrict__ ids,
                               uint32_t n, uint32_t count, uint32_t stride, uint32_t off, uint32_t span,
                               uint32_t tile, uint32_t *out) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        uint32_t *o = out + (uint64_t)i * (n + 1);
        uint32_t acc = 0;
        o[0] = 0;
        for (uint32_t x = 0; x < n; x++) {
            const uint64_t cols = tasks[ids[x]].cols, c = (uint64_t)stride * i + off;
            if (cols > c) {
                const uint64_t w = cols - c < span ? cols - c : span;
                acc += (uint32_t)((w + tile - 1) / tile);
            }
            o[x + 1] = acc;
        }
    }
}

// Rows are moved as 8-byte chunks of four entries (D and T rows start
// 8-byte aligned: ld and ldt are multiples of 4), the cols % 4 entries past
// the last chunk one by one.
__global__ __launch_bounds__(256) void k_ech_gather_rows(const uint16_t *__restrict__ D, uint64_t ld,
                                                         uint32_t cols, const uint32_t *__restrict__ piv_row,
                                                         const uint32_t *__restrict__ d_rank,
                                                         uint16_t *T, uint64_t ldt) {
    const uint32_t r = *d_rank, nq = cols / 4;
    for (uint32_t t = blockIdx.y; t < r; t += gridDim.y) {
        const uint32_t src = piv_row[t];
        const uint64_t *s8 = (const uint64_t *)(D + (uint64_t)src * ld);
        uint64_t *d8 = (uint64_t *)(T + (uint64_t)t * ldt);
        for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) d8[q] = s8[q];
        if (blockIdx.x == 0 && threadIdx.x < cols - nq * 4)
            T[(uint64_t)t * ldt + nq * 4 + threadIdx.x] = D[(uint64_t)src * ld + nq * 4 + threadIdx.x];
    }
}

__global__ __launch_bounds__(256) void k_ech_place_rows(uint16_t *D, uint64_t ld, uint32_t rows,
                                                        uint32_t cols,
                                                        const uint32_t *__restrict__ d_rank,
                                                        const uint16_t *__restrict__ T, uint64_t ldt) {
    const uint32_t r = *d_rank, nq = cols / 4;
    for (uint32_t i = blockIdx.y; i < rows; i += gridDim.y) {
        uint64_t *d8 = (uint64_t *)(D + (uint64_t)i * ld);
        const uint64_t *s8 = (const uint64_t *)(T + (uint64_t)i * ldt);
        for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x)
            d8[q] = i < r ? s8[q] : 0;
        if (blockIdx.x == 0 && threadIdx.x < cols - nq * 4)
            D[(uint64_t)i * ld + nq * 4 + threadIdx.x] = i < r ? T[(uint64_t)i * ldt + nq * 4 + threadIdx.x] : 0;
    }
}

size_t ech_layout(uint32_t rows, uint32_t cols, fl_mode mode, void *ws, EchWs *e) {
    WsCarve c(ws);
    const uint32_t mn = rows < cols ? rows : cols;
    const uint64_t ldu = ((uint64_t)cols + 63) & ~(uint64_t)63;
    const uint32_t npanels = (cols + kPanel - 1) / kPanel;
    const uint32_t nblocks = (npanels + kBlockPanels - 1) / kBlockPanels;
    const size_t r1 = rows ? rows : 1;
    EchWs t;
    t.is_piv = c.take<uint32_t>(r1);
    t.nzlist = c.take<uint32_t>(r1);
    t.flist = c.take<uint32_t>(r1);
    t.counts = c.take<uint32_t>(3 * (size_t)(npanels + 1));
    t.piv_row = c.take<uint32_t>(mn ? mn : 1);
    t.ps = c.take<PanelState>(kSlots);
    // tiles read up to 4 columns past a row's last one: one spare row
    t.U = c.take<uint16_t>((size_t)65 * ldu);
    t.T = c.take<uint16_t>((size_t)(mn ? mn : 1) * ldu);
    t.Lb = c.take<uint16_t>(2 * r1 * kBlock);
    t.ldu = ldu;
    t.Uh = t.Ul = t.Lbh = t.Lbl = t.Ubh = t.Ubl = nullptr;
    t.Ub = nullptr;
    if (mode == FL_MFMA_I8) {
        t.Uh = c.take<int8_t>(((size_t)cols + 256) * 64);
        t.Ul = c.take<int8_t>(((size_t)cols + 256) * 64);
        t.Lbh = c.take<int8_t>(2 * r1 * kBlock);
        t.Lbl = c.take<int8_t>(2 * r1 * kBlock);
        t.Ubh = c.take<int8_t>(2 * ((size_t)cols + kBlock) * kBlock);
        t.Ubl = c.take<int8_t>(2 * ((size_t)cols + kBlock) * kBlock);
    } else {
        t.Ub = c.take<uint16_t>((2 * (size_t)kBlock + 1) * ldu);
    }
    t.upd_rows = c.take<uint32_t>(r1);
    t.blk_rows = c.take<uint32_t>(2 * r1);
    t.blk_cnt = c.take<uint32_t>(nblocks ? nblocks : 1);
    t.mark = c.take<uint32_t>(r1);
    t.nzlead = c.take<uint32_t>(r1);
    t.task = c.take<FlEchTask>(1);
    t.ids = c.take<uint32_t>(1);
    t.pre_rows = c.take<uint32_t>(2);
    t.pre = c.take<uint32_t>(2 * (3 * (size_t)(npanels ? npanels : 1) + 6 * (size_t)(nblocks ? nblocks : 1)));
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
    const uint32_t nblocks = (npanels + kBlockPanels - 1) / kBlockPanels;
    FL_HIP(fl_fill_u32(e.is_piv, 0, rows, stream));
    FL_HIP(fl_fill_u32(e.mark, 0, rows, stream));
    FL_HIP(fl_fill_u32(e.blk_cnt, 0, nblocks, stream));
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
    t.T = e.T;
    t.ldu = e.ldu;
    t.Uh = e.Uh;
    t.Ul = e.Ul;
    t.Lb = e.Lb;
    t.Ub = e.Ub;
    t.Lbh = e.Lbh;
    t.Lbl = e.Lbl;
    t.Ubh = e.Ubh;
    t.Ubl = e.Ubl;
    t.upd_rows = e.upd_rows;
    t.blk_rows = e.blk_rows;
    t.blk_cnt = e.blk_cnt;
    t.mark = e.mark;
    t.nzlead = e.nzlead;
    t.nzlist = e.nzlist;
    t.flist = e.flist;
    t.counts = e.counts;
    *task = t;
    return FL_OK;
}

hipError_t fl_echelon_prefixes(const FlEchTask *tasks, const FlEchLists &L, uint32_t panels, uint32_t blocks,
                               hipStream_t stream) {
    const uint32_t one = 1u << 31, all = 0xffffffffu;  // a tile wider than any matrix; no cap
    struct Tab {
        const uint32_t *ids;
        uint32_t n, count, stride, off, span, tile;
        uint32_t *out;
    } const tab[9] = {
        {L.ids_all, L.n_all, panels, kPanel, 0, all, one, L.pre_n_all},
        {L.ids_mfma, L.n_mfma, panels, kPanel, 0, all, one, L.pre_n_mfma},
        {L.ids_plain, L.n_plain, panels, kPanel, 0, all, one, L.pre_n_plain},
        {L.ids_all, L.n_all, blocks, kBlock, kBlock, kBlock, 64, L.pre_bn_all},
        {L.ids_mfma, L.n_mfma, blocks, kBlock, kBlock, kBlock, 64, L.pre_bn_mfma},
        {L.ids_plain, L.n_plain, blocks, kBlock, kBlock, kBlock, 256, L.pre_bn_plain},
        {L.ids_all, L.n_all, blocks, kBlock, 2 * kBlock, all, 64, L.pre_bf_all},
        {L.ids_mfma, L.n_mfma, blocks, kBlock, 2 * kBlock, all, 128, L.pre_bf_mfma},
        {L.ids_plain, L.n_plain, blocks, kBlock, 2 * kBlock, all, 256, L.pre_bf_plain}};
    for (const Tab &t : tab)
        if (t.n && t.count)
            hipLaunchKernelGGL(k_ech_prefixes, dim3((t.count + 255) / 256), dim3(256), 0, stream, tasks, t.ids, t.n,
                               t.count, t.stride, t.off, t.span, t.tile, t.out);
    return hipGetLastError();
}

// Far-part kernels reserve this much LDS per workgroup (the rest of what
// they use as dynamic shared memory), so that at most 2 of them share a
// compute unit: the main stream's kernels (the pivot search is a single
// 1024-thread workgroup on the critical path) then get a unit as soon as a
// far workgroup on it finishes, instead of queueing behind a chip filled
// with thousands of far workgroups.
constexpr uint32_t kFarLds = 64 * 1024;
// Column tiles walked by one workgroup of the block update: at most this
// many workgroups per row block.  Many short workgroups rather than few long
// ones: the main stream's kernels get a compute unit whenever a far
// workgroup finishes, so short far workgroups keep the critical path moving
// (and balance the far kernel's own tail).
constexpr uint32_t kBlkColGroups = 64;

template <class K>
uint32_t far_dyn_lds(K kernel) {
    hipFuncAttributes a;
    if (hipFuncGetAttributes(&a, (const void *)kernel) != hipSuccess || a.sharedSizeBytes >= kFarLds) return 0;
    return kFarLds - (uint32_t)a.sharedSizeBytes;
}

// Block B's update of the columns [256 (B + 1) + lo, + span) on stream s:
// U of the block for those columns, then the rank-256 update.
hipError_t block_update(const fl::Mod &md, uint32_t p, const FlEchTask *tasks, const FlEchLists &L, uint32_t B,
                        uint32_t lo, uint32_t span, uint32_t g_all, uint32_t g_mfma, uint32_t g_plain,
                        uint32_t mfma_rows, const uint32_t *pa, const uint32_t *pm, const uint32_t *pp,
                        bool far, uint32_t far_groups, hipStream_t s) {
    static const uint32_t dyn_u = far_dyn_lds(k_ech_ublk<512>), dyn_m = far_dyn_lds((k_ech_update_blk_mfma<2, 8>)),
                          dyn_v = far_dyn_lds(k_ech_update_blk_valu);
    hipError_t e;
    if (!g_all) return hipSuccess;
    // 16 waves per 64 columns on the critical path (the entries of the
    // bracket and the rows of U dealt to the waves); the far part takes 8
    // (and the LDS reservation), which leaves every unit room for the main
    // stream's waves
    if (far)
        FL_PROF("echelon.ublk_far", s,
                hipLaunchKernelGGL(k_ech_ublk<512>, dim3(g_all), dim3(512), dyn_u, s, md, tasks, L.ids_all, pa,
                                   L.n_all, B, lo, span));
    else
        FL_PROF("echelon.ublk", s,
                hipLaunchKernelGGL(k_ech_ublk<1024>, dim3(g_all), dim3(1024), 0, s, md, tasks, L.ids_all, pa,
                                   L.n_all, B, lo, span));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the far part takes 32 rows per wave, so each B fragment feeds two row
    // tiles; the next block's update (256 columns, latency bound) takes 16
    // rows per wave and 64-column tiles, four times the workgroups
    if (g_mfma && far) {
        FL_PROF("echelon.blk_mfma_far", s,
                hipLaunchKernelGGL((k_ech_update_blk_mfma<2, 8>),
                                   dim3((mfma_rows + 127) / 128, std::min(g_mfma, far_groups)), dim3(256), dyn_m, s,
                                   md, fl_mfma::gemm_bias(p), fl_mfma::gemm_c16(p), tasks, L.ids_mfma, pm, L.n_mfma,
                                   g_mfma, B, lo, span));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if (g_mfma) {
        FL_PROF("echelon.blk_mfma", s,
                hipLaunchKernelGGL((k_ech_update_blk_mfma<1, 4>),
                                   dim3((mfma_rows + 63) / 64, std::min(g_mfma, kBlkColGroups)), dim3(256), 0, s, md,
                                   fl_mfma::gemm_bias(p), fl_mfma::gemm_c16(p), tasks, L.ids_mfma, pm, L.n_mfma,
                                   g_mfma, B, lo, span));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (g_plain) {
        FL_PROF(far ? "echelon.blk_plain_far" : "echelon.blk_plain", s,
                hipLaunchKernelGGL(k_ech_update_blk_valu, dim3(g_plain, 64), dim3(256), far ? dyn_v : 0, s, md,
                                   tasks, L.ids_plain, pp, L.n_plain, B, lo, span));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fl_echelon_batch_panel(uint32_t p, const FlEchTask *tasks, const FlEchLists &L, uint32_t P,
                                  const FlEchGrid &g, const FlEchBlockGrid *blk, hipStream_t stream,
                                  FlEchAux &aux) {
    if (g.n_active == 0) return hipSuccess;
    const fl::Mod md = fl::make_mod(p);
    auto at = [](const uint32_t *pre, uint32_t i, uint32_t n) { return pre + (uint64_t)i * (n + 1); };
    const uint32_t mfma_y = (g.mfma_rows + 63) / 64;
    hipError_t e;
    // pivot search: nonzero listing (panel 0 only: later panels are listed at
    // the end of the previous one), probe basis, check, merge
    if (P == 0) {
        FL_PROF("echelon.check", stream,
                hipLaunchKernelGGL(k_ech_check, dim3(g.grid_rows), dim3(256), 0, stream, md, tasks, L.ids_all,
                                   L.pre_rows, g.n_active, P, 0));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    FL_PROF("echelon.probe", stream,
            hipLaunchKernelGGL(k_ech_probe, dim3(g.n_active), dim3(kGreedyThreads), 0, stream, md, tasks, L.ids_all,
                               P));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the check, with U over the rest of the block and L' from the probe
    // basis; when a row was flagged: the merge, then U and L' again
    FL_PROF("echelon.check_UL", stream,
            hipLaunchKernelGGL(k_ech_check_UL, dim3(kBlockPanels * g.n_active + 2 * g.grid_rows), dim3(256), 0,
                               stream, md, tasks, L.ids_all, at(L.pre_n_all, P, L.n_all), L.n_all,
                               kBlockPanels * g.n_active, L.pre_rows, g.n_active, g.grid_rows, P));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    FL_PROF("echelon.merge", stream,
            hipLaunchKernelGGL(k_ech_merge, dim3(g.n_active), dim3(256), 0, stream, md, tasks, L.ids_all, P));
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (g.n_mfma) {
        FL_PROF("echelon.mfma", stream,
                hipLaunchKernelGGL(k_ech_update_mfma, dim3(4 * g.n_mfma, mfma_y), dim3(256), 0, stream, md,
                                   fl_mfma::gemm_bias(p), fl_mfma::gemm_c16(p), tasks, L.ids_mfma,
                                   at(L.pre_n_mfma, P, L.n_mfma), L.n_mfma, P));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (g.n_plain) {
        FL_PROF("echelon.plain", stream,
                hipLaunchKernelGGL(k_ech_update_valu, dim3(g.n_plain, 64), dim3(256), 0, stream, md, tasks,
                                   L.ids_plain, at(L.pre_n_plain, P, L.n_plain), L.n_plain, P));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (blk) {
        const uint32_t B = P / kBlockPanels;
        // the previous block's far part wrote the columns read and updated now
        if (aux.far_pending) {
            if ((e = hipStreamWaitEvent(stream, aux.ev_far, 0)) != hipSuccess) return e;
            aux.far_pending = false;
        }
        // The far part (columns past the next block) needs only the block's
        // panels, not the next block's update (disjoint columns), so the
        // second stream starts it first.  (The wait above was enqueued before
        // ev_far is recorded again.)
        if (blk->bf_all) {
            if ((e = hipEventRecord(aux.ev_near, stream)) != hipSuccess) return e;
            if ((e = hipStreamWaitEvent(aux.far, aux.ev_near, 0)) != hipSuccess) return e;
            if ((e = block_update(md, p, tasks, L, B, kBlock, 0xffffffffu, blk->bf_all, blk->bf_mfma,
                                  blk->bf_plain, blk->mfma_rows, at(L.pre_bf_all, B, L.n_all),
                                  at(L.pre_bf_mfma, B, L.n_mfma), at(L.pre_bf_plain, B, L.n_plain), true,
                                  aux.far_groups ? aux.far_groups : kBlkColGroups, aux.far)) != hipSuccess)
                return e;
            if ((e = hipEventRecord(aux.ev_far, aux.far)) != hipSuccess) return e;
            aux.far_pending = true;
        }
        if ((e = block_update(md, p, tasks, L, B, 0, kBlock, blk->bn_all, blk->bn_mfma, blk->bn_plain,
                              blk->mfma_rows, at(L.pre_bn_all, B, L.n_all), at(L.pre_bn_mfma, B, L.n_mfma),
                              at(L.pre_bn_plain, B, L.n_plain), false, kBlkColGroups, stream)) != hipSuccess)
            return e;
    }
    if (g.n_next) {
        FL_PROF("echelon.check", stream,
                hipLaunchKernelGGL(k_ech_check, dim3(g.grid_rows_next), dim3(256), 0, stream, md, tasks, L.ids_all,
                                   L.pre_rows, g.n_next, P + 1, 0));
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t fl_echelon_join(hipStream_t stream, FlEchAux &aux) {
    if (!aux.far_pending) return hipSuccess;
    aux.far_pending = false;
    return hipStreamWaitEvent(stream, aux.ev_far, 0);
}

fl_status fl_echelon_finish(const FlEchTask &t, hipStream_t stream) {
    if (t.npanels == 0) return FL_OK;
    const uint32_t rows = t.rows, cols = t.cols;
    const uint32_t mn = rows < cols ? rows : cols;
    // 8-byte chunks of four columns, at most 16 workgroups of 256 per row
    // (at least one: it also moves the cols % 4 last entries)
    const unsigned gq = (cols / 4 + 255) / 256, gx = gq < 1 ? 1 : gq < 16 ? gq : 16;
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
    FlEchAux aux = {};
    FL_CHECK_ST(fl_aux_stream(0, &aux.far, &aux.ev_near, &aux.ev_far));
    EchWs e;
    ech_layout(rows, cols, mode, ws, &e);
    // a one-entry task table
    const uint32_t zero = 0, pre_rows[2] = {0, (rows + 31) / 32};
    FL_HIP(fl_upload(e.task, &t, sizeof t, stream));
    FL_HIP(fl_upload(e.ids, &zero, 4, stream));
    FL_HIP(fl_upload(e.pre_rows, pre_rows, 8, stream));
    const uint32_t np = t.npanels, nb = (np + kBlockPanels - 1) / kBlockPanels;
    FlEchLists L = {};
    L.ids_all = e.ids;
    L.pre_rows = e.pre_rows;
    L.n_all = 1;
    uint32_t *q = e.pre;
    auto take = [&q](uint32_t count) {
        uint32_t *r = q;
        q += 2 * (size_t)count;
        return r;
    };
    L.pre_n_all = take(np);
    L.pre_bn_all = take(nb);
    L.pre_bf_all = take(nb);
    uint32_t *pn = take(np), *pbn = take(nb), *pbf = take(nb);
    if (t.mfma) {
        L.ids_mfma = e.ids;
        L.n_mfma = 1;
        L.pre_n_mfma = pn;
        L.pre_bn_mfma = pbn;
        L.pre_bf_mfma = pbf;
    } else {
        L.ids_plain = e.ids;
        L.n_plain = 1;
        L.pre_n_plain = pn;
        L.pre_bn_plain = pbn;
        L.pre_bf_plain = pbf;
    }
    FL_HIP(fl_echelon_prefixes(e.task, L, np, nb, stream));
    for (uint32_t P = 0; P < np; P++) {
        FlEchGrid g = {};
        g.n_active = 1;
        g.grid_rows = pre_rows[1];
        g.n_mfma = t.mfma ? 1 : 0;
        g.n_plain = t.mfma ? 0 : 1;
        g.mfma_rows = rows;
        g.n_next = P + 1 < np ? 1 : 0;
        g.grid_rows_next = g.n_next ? pre_rows[1] : 0;
        FlEchBlockGrid bg = {};
        const bool end = P % kBlockPanels == kBlockPanels - 1 || P + 1 == np;
        if (end) {
            const uint64_t bend = (uint64_t)(P / kBlockPanels + 1) * kBlock;
            bg.bn_all = fl_ech_tiles(cols, bend, kBlock, 64);
            bg.bf_all = fl_ech_tiles(cols, bend + kBlock, ~0ull, 64);
            const uint32_t bn = fl_ech_tiles(cols, bend, kBlock, t.mfma ? 64 : 256);
            const uint32_t bf = fl_ech_tiles(cols, bend + kBlock, ~0ull, t.mfma ? 128 : 256);
            (t.mfma ? bg.bn_mfma : bg.bn_plain) = bn;
            (t.mfma ? bg.bf_mfma : bg.bf_plain) = bf;
            bg.mfma_rows = rows;
        }
        FL_HIP(fl_echelon_batch_panel(p, e.task, L, P, g, end ? &bg : nullptr, stream, aux));
    }
    FL_HIP(fl_echelon_join(stream, aux));
    return fl_echelon_finish(t, stream);
}
