// trsm.hip -- FL step 2 (X = A^{-1} B, paper Sec. 4.1 step 2) and the sparse
// form of FL step 3 (Dt = D - C X, Sec. 4.1 step 3), both built on one
// kernel: a w-multiline row group times a dense matrix (Sec. 4.2: the w rows
// of a multiline share one pass over the positions, so each row of X that is
// read serves all w rows -- the GPU analogue of the paper's multiline AXPY).
//
// TRSM schedule: rows of A are cut into blocks of kTrsmBlock rows; blocks
// are solved from the bottom up.  For block [r0, r1):
//   k_ml_spmm  (update)  X[r0:r1] -= A[r0:r1, r1:] X[r1:]   -- fully parallel
//                        over (multiline group, 256-column tile)
//   k_trsm_solve         back substitution inside the block, one wave per
//                        64-column stripe, the block's finished rows kept in
//                        LDS; each multiline group is solved with the 2x2 /
//                        wxw triangular correction between its own rows.
// Arithmetic: coefficients are split a = 256 a_h + a_l and multiplied with
// 24-bit multiply-adds into two 32-bit accumulators, folded mod p at most
// every 256 terms (see fl_internal.h for the bound).
#include "fl_internal.h"
#include "mfma_tile.h"

namespace {

constexpr uint32_t kTrsmBlock = kFlTrsmBlock;  // rows per TRSM block (multiple of 8)
constexpr int kTile = 256;            // columns per wave in k_ml_spmm (4 per lane)

// ---- CSR rows -> dense rows (out zeroed beforehand) ------------------------------
__global__ __launch_bounds__(256) void k_csr_scatter(uint32_t rows, const uint64_t *__restrict__ rp,
                                                     const uint32_t *__restrict__ ci,
                                                     const uint16_t *__restrict__ v, uint16_t *out,
                                                     uint64_t ld) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= rows) return;
    uint16_t *row = out + (uint64_t)i * ld;
    for (uint64_t k = rp[i] + lane; k < rp[i + 1]; k += 64) row[ci[k]] = v[k];
}

// ---- metadata of one multiline position, broadcast from lane j --------------------
template <int W> struct MlVals;
template <> struct MlVals<1> {
    uint32_t v;
    __device__ void load(const uint16_t *val, uint64_t k) { v = val[k]; }
    __device__ uint16_t raw(int q) const { (void)q; return (uint16_t)v; }
    __device__ uint32_t get(int j, int q) const {
        (void)q;
        return (uint32_t)__builtin_amdgcn_readlane((int)v, j);
    }
};
template <> struct MlVals<2> {
    uint32_t v;
    __device__ void load(const uint16_t *val, uint64_t k) { v = *(const uint32_t *)(val + 2 * k); }
    __device__ uint16_t raw(int q) const { return (uint16_t)(q ? v >> 16 : v); }
    __device__ uint32_t get(int j, int q) const {
        uint32_t s = (uint32_t)__builtin_amdgcn_readlane((int)v, j);
        return q ? s >> 16 : s & 0xffffu;
    }
};
template <> struct MlVals<4> {
    uint32_t v0, v1;
    __device__ void load(const uint16_t *val, uint64_t k) {
        uint64_t x = *(const uint64_t *)(val + 4 * k);
        v0 = (uint32_t)x; v1 = (uint32_t)(x >> 32);
    }
    __device__ uint16_t raw(int q) const {
        const uint32_t s = q < 2 ? v0 : v1;
        return (uint16_t)((q & 1) ? s >> 16 : s);
    }
    __device__ uint32_t get(int j, int q) const {
        uint32_t s = (uint32_t)__builtin_amdgcn_readlane((int)(q < 2 ? v0 : v1), j);
        return (q & 1) ? s >> 16 : s & 0xffffu;
    }
};
template <> struct MlVals<8> {
    uint32_t v[4];
    __device__ void load(const uint16_t *val, uint64_t k) {
        uint4 x = *(const uint4 *)(val + 8 * k);
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
    }
    __device__ uint16_t raw(int q) const { return (uint16_t)((q & 1) ? v[q >> 1] >> 16 : v[q >> 1]); }
    __device__ uint32_t get(int j, int q) const {
        uint32_t s = (uint32_t)__builtin_amdgcn_readlane((int)v[q >> 1], j);
        return (q & 1) ? s >> 16 : s & 0xffffu;
    }
};

// First index k in [kb, ke) with pos[k] >= lo (pos ascending), wave-cooperative.
__device__ __forceinline__ uint64_t first_at_least(const uint32_t *__restrict__ pos, uint64_t kb,
                                                   uint64_t ke, uint32_t lo) {
    const uint32_t lane = threadIdx.x & 63;
    uint64_t k = kb;
    while (k < ke) {
        uint64_t kk = k + lane;
        bool below = kk < ke && pos[kk] < lo;
        uint64_t mask = __ballot(below);
        if (mask != ~(uint64_t)0) return k + __popcll(mask);
        k += 64;
    }
    return ke;
}

// out[g*W+q][c] = out[...][c] - sum_{k: pos[k] >= pos_lo} val[W*k+q] * X[pos[k]][c]  (mod p)
// for groups g in [g0, g0 + ngroups), rows < row_limit, columns < ncols.
// One wave per (group, 256-column tile); blockIdx.y picks 4 consecutive groups.
template <int W>
__device__ __forceinline__ void ml_spmm_tile(const fl::Mod &md, const uint64_t *__restrict__ gptr,
                                             const uint32_t *__restrict__ pos,
                                             const uint16_t *__restrict__ val, uint32_t g0,
                                             uint32_t ngroups, uint32_t row_limit, uint32_t pos_lo,
                                             const uint16_t *X, uint64_t ldx, uint16_t *out,
                                             uint64_t ldo, uint32_t ncols, uint32_t bx, uint32_t by) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t gi = by * 4 + (threadIdx.x >> 6);
    if (gi >= ngroups) return;
    const uint32_t g = g0 + gi;
    const uint32_t c0 = bx * kTile + lane * 4;
    const bool colok = c0 < ncols;
    uint64_t kb = gptr[g], ke = gptr[g + 1];
    if (pos_lo) kb = first_at_least(pos, kb, ke, pos_lo);
    if (kb >= ke) return;  // nothing to subtract

    uint32_t ah[W][4], al[W][4];
#pragma unroll
    for (int q = 0; q < W; q++)
#pragma unroll
        for (int c = 0; c < 4; c++) ah[q][c] = al[q][c] = 0;

    uint32_t terms = 0;
    for (uint64_t k = kb; k < ke; k += 64) {
        const int batch = (int)((ke - k) < 64 ? (ke - k) : 64);
        uint32_t mypos = 0;
        MlVals<W> mv;
        if ((int)lane < batch) {
            mypos = pos[k + lane];
            mv.load(val, k + lane);
        }
        int j = 0;
        for (; j + 4 <= batch; j += 4) {
            uint64_t xv[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                uint32_t pj = (uint32_t)__builtin_amdgcn_readlane((int)mypos, j + u);
                xv[u] = colok ? *(const uint64_t *)(X + (uint64_t)pj * ldx + c0) : 0;
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                uint32_t x[4] = {(uint32_t)xv[u] & 0xffffu, (uint32_t)(xv[u] >> 16) & 0xffffu,
                                 (uint32_t)(xv[u] >> 32) & 0xffffu, (uint32_t)(xv[u] >> 48)};
#pragma unroll
                for (int q = 0; q < W; q++) {
                    uint32_t a = mv.get(j + u, q);
                    uint32_t a_h = a >> 8, a_l = a & 0xffu;
#pragma unroll
                    for (int c = 0; c < 4; c++) {
                        ah[q][c] = fl::mad24(a_h, x[c], ah[q][c]);
                        al[q][c] = fl::mad24(a_l, x[c], al[q][c]);
                    }
                }
            }
        }
        for (; j < batch; j++) {
            uint32_t pj = (uint32_t)__builtin_amdgcn_readlane((int)mypos, j);
            uint64_t xv = colok ? *(const uint64_t *)(X + (uint64_t)pj * ldx + c0) : 0;
            uint32_t x[4] = {(uint32_t)xv & 0xffffu, (uint32_t)(xv >> 16) & 0xffffu,
                             (uint32_t)(xv >> 32) & 0xffffu, (uint32_t)(xv >> 48)};
#pragma unroll
            for (int q = 0; q < W; q++) {
                uint32_t a = mv.get(j, q);
                uint32_t a_h = a >> 8, a_l = a & 0xffu;
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    ah[q][c] = fl::mad24(a_h, x[c], ah[q][c]);
                    al[q][c] = fl::mad24(a_l, x[c], al[q][c]);
                }
            }
        }
        terms += (uint32_t)batch;
        if (terms > FL_FOLD_TERMS - 64) {
#pragma unroll
            for (int q = 0; q < W; q++)
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    al[q][c] = fl::fold_pair(ah[q][c], al[q][c], md);
                    ah[q][c] = 0;
                }
            terms = 0;
        }
    }
    if (!colok) return;
#pragma unroll
    for (int q = 0; q < W; q++) {
        const uint32_t row = g * W + q;
        if (row >= row_limit) break;
        uint16_t *o = out + (uint64_t)row * ldo + c0;
        uint32_t s[4];
#pragma unroll
        for (int c = 0; c < 4; c++) s[c] = fl::fold_pair(ah[q][c], al[q][c], md);
        if (c0 + 4 <= ncols) {
            uint64_t ov = *(const uint64_t *)o;
            uint64_t nv = 0;
#pragma unroll
            for (int c = 0; c < 4; c++)
                nv |= (uint64_t)fl::submod((uint32_t)(ov >> (16 * c)) & 0xffffu, s[c], md.p) << (16 * c);
            *(uint64_t *)o = nv;
        } else {
            for (int c = 0; c < 4 && c0 + c < ncols; c++) o[c] = (uint16_t)fl::submod(o[c], s[c], md.p);
        }
    }
}

template <int W>
__global__ __launch_bounds__(256) void k_ml_spmm(fl::Mod md, const uint64_t *__restrict__ gptr,
                                                 const uint32_t *__restrict__ pos,
                                                 const uint16_t *__restrict__ val, uint32_t g0,
                                                 uint32_t ngroups, uint32_t row_limit,
                                                 uint32_t pos_lo, const uint16_t *X, uint64_t ldx,
                                                 uint16_t *out, uint64_t ldo, uint32_t ncols) {
    ml_spmm_tile<W>(md, gptr, pos, val, g0, ngroups, row_limit, pos_lo, X, ldx, out, ldo, ncols, blockIdx.x,
                    blockIdx.y);
}

// For every multiline group g of A: nin[g] = number of its entries inside
// the group (positions < (g+1)w, the w x w triangle), nnear[g] = number of
// entries before the first position >= r1 of its TRSM block.  One wave per
// group, computed once per TRSM.
__global__ __launch_bounds__(256) void k_trsm_bounds(uint32_t w, uint32_t npiv, uint32_t ngroups,
                                                     const uint64_t *__restrict__ gptr,
                                                     const uint32_t *__restrict__ pos, uint32_t *nin,
                                                     uint32_t *nnear) {
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= ngroups) return;
    const uint32_t I = (g * w) / kTrsmBlock;
    const uint32_t r1 = (I + 1) * kTrsmBlock < npiv ? (I + 1) * kTrsmBlock : npiv;
    const uint64_t kb = gptr[g], ke = gptr[g + 1];
    const uint64_t kin = first_at_least(pos, kb, ke, (g + 1) * w);
    const uint64_t kfar = first_at_least(pos, kin, ke, r1);
    if ((threadIdx.x & 63) == 0) {
        nin[g] = (uint32_t)(kin - kb);
        nnear[g] = (uint32_t)(kfar - kb);
    }
}

constexpr uint32_t kNearCap = 2048;  // staged intra+near entries per block

// Entry j of group gi: from the LDS copy (STAGED) or from global memory.
template <int W, bool STAGED> struct Entries {
    const uint32_t *s_pos;
    const uint16_t *s_val;
    const uint32_t *s_off;
    const uint64_t *s_kb;
    const uint32_t *pos;
    const uint16_t *val;
    __device__ uint32_t p(uint32_t gi, uint32_t j) const {
        return STAGED ? s_pos[s_off[gi] + j] : pos[s_kb[gi] + j];
    }
    __device__ uint32_t v(uint32_t gi, uint32_t j, int q) const {
        return STAGED ? s_val[(s_off[gi] + j) * W + q] : val[(uint64_t)W * (s_kb[gi] + j) + q];
    }
};

// Solve the block's groups from the bottom up on the LDS tile blk.
template <int W, bool STAGED>
__device__ void solve_groups(const fl::Mod &md, const Entries<W, STAGED> &E, uint16_t (*blk)[64],
                             const uint32_t *s_nin, const uint32_t *s_off, uint32_t gfirst,
                             uint32_t ng, uint32_t r0, uint32_t r1, uint32_t lane) {
    for (uint32_t gi = ng; gi-- > 0;) {
        const uint32_t gr0 = (gfirst + gi) * W;
        const uint32_t nin = s_nin[gi], nend = s_off[gi + 1] - s_off[gi];
        uint32_t ah[W], al[W];
#pragma unroll
        for (int q = 0; q < W; q++) ah[q] = al[q] = 0;
        uint32_t terms = 0;
        uint32_t j = nin;
        // 8 entries at a time: their reads are independent and overlap
        for (; j + 8 <= nend; j += 8) {
            uint32_t pj[8], x[8], a[8][W];
#pragma unroll
            for (int u = 0; u < 8; u++) {
                pj[u] = E.p(gi, j + u);
#pragma unroll
                for (int q = 0; q < W; q++) a[u][q] = E.v(gi, j + u, q);
            }
#pragma unroll
            for (int u = 0; u < 8; u++) x[u] = blk[pj[u] - r0][lane];
#pragma unroll
            for (int u = 0; u < 8; u++)
#pragma unroll
                for (int q = 0; q < W; q++) {
                    ah[q] = fl::mad24(a[u][q] >> 8, x[u], ah[q]);
                    al[q] = fl::mad24(a[u][q] & 0xffu, x[u], al[q]);
                }
            terms += 8;
            if (terms > FL_FOLD_TERMS - 8) {
#pragma unroll
                for (int q = 0; q < W; q++) {
                    al[q] = fl::fold_pair(ah[q], al[q], md);
                    ah[q] = 0;
                }
                terms = 0;
            }
        }
        for (; j < nend; j++) {
            const uint32_t x = blk[E.p(gi, j) - r0][lane];
#pragma unroll
            for (int q = 0; q < W; q++) {
                const uint32_t a = E.v(gi, j, q);
                ah[q] = fl::mad24(a >> 8, x, ah[q]);
                al[q] = fl::mad24(a & 0xffu, x, al[q]);
            }
        }
        // T_q = X[row] - near sum, then the triangular correction inside the group
        uint32_t tq[W];
#pragma unroll
        for (int q = 0; q < W; q++) {
            const uint32_t row = gr0 + q;
            const uint32_t cur = row < r1 ? blk[row - r0][lane] : 0;
            tq[q] = fl::submod(cur, fl::fold_pair(ah[q], al[q], md), md.p);
        }
#pragma unroll
        for (int q = W - 1; q >= 0; q--) {
            const uint32_t row = gr0 + q;
            if (row < r1) {
                // subtract a[q][jj] * v[jj] for jj > q (rows of the group already final)
                for (uint32_t e = 0; e < nin; e++) {
                    const uint32_t qq = E.p(gi, e) - gr0;
                    const uint32_t a = E.v(gi, e, q);
#pragma unroll
                    for (int jj = q + 1; jj < W; jj++)
                        if (qq == (uint32_t)jj && a) tq[q] = fl::submod(tq[q], fl::mulmod(a, tq[jj], md), md.p);
                }
                blk[row - r0][lane] = (uint16_t)tq[q];
            }
        }
    }
}

// Back substitution inside one TRSM block [r0, r1): one wave per 64-column
// stripe (one column per lane).  The block's intra-group and near entries of
// A (positions < r1) and the block's rows of X (after the far update) are
// staged in LDS with independent, vectorised loads; rows are then finished
// from the bottom up in LDS, each multiline group with the w x w triangular
// correction between its own rows.  Entries at positions >= r1 were applied
// by the preceding update launch.
template <int W>
__device__ __forceinline__ void trsm_solve_tile(const fl::Mod &md, const uint64_t *__restrict__ gptr,
                                                const uint32_t *__restrict__ pos,
                                                const uint16_t *__restrict__ val,
                                                const uint32_t *__restrict__ nin_a,
                                                const uint32_t *__restrict__ nnear_a, uint32_t r0,
                                                uint32_t r1, uint16_t *X, uint64_t ldx, uint32_t ncols,
                                                int8_t *Xth, int8_t *Xtl, uint64_t kp, uint32_t bx) {
    constexpr uint32_t kG = kTrsmBlock / W;
    __shared__ __attribute__((aligned(16))) uint16_t blk[kTrsmBlock][64];
    __shared__ uint32_t s_off[kG + 1];
    __shared__ uint32_t s_nin[kG];
    __shared__ uint64_t s_kb[kG];
    __shared__ uint32_t s_pos[kNearCap];
    __shared__ uint16_t s_val[kNearCap * W];
    const uint32_t lane = threadIdx.x;
    const uint32_t c0 = bx * 64;
    const uint32_t c = c0 + lane;
    const bool colok = c < ncols;
    const uint32_t gfirst = r0 / W, glast = (r1 + W - 1) / W, ng = glast - gfirst;
    const uint32_t nrow = r1 - r0;
    // group metadata and offsets of the staged entries
    for (uint32_t gi = lane; gi < ng; gi += 64) {
        s_kb[gi] = gptr[gfirst + gi];
        s_nin[gi] = nin_a[gfirst + gi];
        s_off[gi + 1] = nnear_a[gfirst + gi];
    }
    // X tile: 128 rows x 64 columns; lane l moves 4 columns (8 bytes) of rows
    // l/16, l/16 + 4, ... (16 lanes per row)
    const uint32_t tr = lane >> 4, tc = (lane & 15) * 4;
    const bool vec = c0 + tc + 4 <= ncols;
    if (vec) {
        // all 32 loads in flight before the first LDS store
        constexpr int kR = kTrsmBlock / 4;
        uint64_t tv[kR];
#pragma unroll
        for (int k = 0; k < kR; k++) {
            const uint32_t r = tr + 4 * k;
            tv[k] = r < nrow ? *(const uint64_t *)(X + (uint64_t)(r0 + r) * ldx + c0 + tc) : 0;
        }
#pragma unroll
        for (int k = 0; k < kR; k++)
            if (tr + 4 * k < nrow) *(uint64_t *)&blk[tr + 4 * k][tc] = tv[k];
    } else {
        for (uint32_t r = tr; r < nrow; r += 4) {
            const uint16_t *src = X + (uint64_t)(r0 + r) * ldx + c0 + tc;
            for (uint32_t k = 0; k < 4; k++) blk[r][tc + k] = c0 + tc + k < ncols ? src[k] : 0;
        }
    }
    __syncthreads();
    if (lane == 0) {
        s_off[0] = 0;
        for (uint32_t gi = 0; gi < ng; gi++) s_off[gi + 1] += s_off[gi];
    }
    __syncthreads();
    const uint32_t total = s_off[ng];
    if (total <= kNearCap) {
        // one lane per group: its entries are contiguous in A; 8 loads per
        // round in flight
        for (uint32_t gi = lane; gi < ng; gi += 64) {
            const uint32_t cnt = s_off[gi + 1] - s_off[gi], o = s_off[gi];
            const uint64_t kb = s_kb[gi];
            for (uint32_t j0 = 0; j0 < cnt; j0 += 8) {
                uint32_t pv[8];
                MlVals<W> vv[8];
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (j0 + u < cnt) {
                        pv[u] = pos[kb + j0 + u];
                        vv[u].load(val, kb + j0 + u);
                    }
#pragma unroll
                for (int u = 0; u < 8; u++)
                    if (j0 + u < cnt) {
                        s_pos[o + j0 + u] = pv[u];
#pragma unroll
                        for (int q = 0; q < W; q++) s_val[(o + j0 + u) * W + q] = vv[u].raw(q);
                    }
            }
        }
        __syncthreads();
        Entries<W, true> E{s_pos, s_val, s_off, s_kb, pos, val};
        solve_groups<W, true>(md, E, blk, s_nin, s_off, gfirst, ng, r0, r1, lane);
    } else {
        Entries<W, false> E{s_pos, s_val, s_off, s_kb, pos, val};
        solve_groups<W, false>(md, E, blk, s_nin, s_off, gfirst, ng, r0, r1, lane);
    }
    __syncthreads();
    for (uint32_t r = tr; r < nrow; r += 4) {
        uint16_t *dst = X + (uint64_t)(r0 + r) * ldx + c0 + tc;
        if (vec) *(uint64_t *)dst = *(const uint64_t *)&blk[r][tc];
        else
            for (uint32_t k = 0; k < 4; k++)
                if (c0 + tc + k < ncols) dst[k] = blk[r][tc + k];
    }
    // MFMA form: the finished rows, as transposed int8 limb planes (column c
    // of X is row c of the planes, K-contiguous), for the updates of the
    // blocks above
    if (Xth && colok) {
        int8_t *dh = Xth + (uint64_t)c * kp + r0, *dl = Xtl + (uint64_t)c * kp + r0;
        const uint32_t nrow = r1 - r0;
        for (uint32_t i0 = 0; i0 < nrow; i0 += 16) {
            uint32_t hw[4] = {0, 0, 0, 0}, lw[4] = {0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < 16; k++) {
                int h = 0, l = 0;
                if (i0 + k < nrow) fl_split_limbs(blk[i0 + k][lane], md.p, h, l);
                hw[k >> 2] |= (uint32_t)(h & 0xff) << (8 * (k & 3));
                lw[k >> 2] |= (uint32_t)(l & 0xff) << (8 * (k & 3));
            }
            if (i0 + 16 <= nrow) {
                *(uint4 *)(dh + i0) = make_uint4(hw[0], hw[1], hw[2], hw[3]);
                *(uint4 *)(dl + i0) = make_uint4(lw[0], lw[1], lw[2], lw[3]);
            } else {
                for (uint32_t k = 0; i0 + k < nrow; k++) {
                    dh[i0 + k] = (int8_t)((hw[k >> 2] >> (8 * (k & 3))) & 0xff);
                    dl[i0 + k] = (int8_t)((lw[k >> 2] >> (8 * (k & 3))) & 0xff);
                }
            }
        }
    }
}

template <int W>
__global__ __launch_bounds__(64) void k_trsm_solve(fl::Mod md, const uint64_t *__restrict__ gptr,
                                                   const uint32_t *__restrict__ pos,
                                                   const uint16_t *__restrict__ val,
                                                   const uint32_t *__restrict__ nin_a,
                                                   const uint32_t *__restrict__ nnear_a, uint32_t r0,
                                                   uint32_t r1, uint16_t *X, uint64_t ldx,
                                                   uint32_t ncols, int8_t *Xth, int8_t *Xtl,
                                                   uint64_t kp) {
    trsm_solve_tile<W>(md, gptr, pos, val, nin_a, nnear_a, r0, r1, X, ldx, ncols, Xth, Xtl, kp, blockIdx.x);
}

// ---- many TRSMs at once: step `step` solves block nblk - 1 - step of every
// matrix in the task table (matrices with fewer blocks are finished) --------

// Superblocks: kFlTrsmSuper consecutive blocks counted from the bottom
// (block nblk - 1 starts the first).  The far update of a superblock takes
// the A columns at and beyond its end R1 for all its rows in one GEMM; block
// I's K range there, relative to R1, is [0, r1 + round_up(kext, 64) - R1)
// (empty when negative); the columns between the block and R1 are the
// block's near update, after the blocks below it in the superblock.  The
// single-matrix call splits the far GEMM by K: the columns of the superblock
// just below (critical path), and the columns past it, which are solved one
// superblock earlier and are issued then on a second stream.
__device__ __host__ inline uint32_t trsm_super_end(uint32_t I, uint32_t nblk, uint32_t npiv) {
    const uint32_t s = nblk - 1 - I;                          // step of block I
    const uint32_t bottom = nblk - 1 - s / kFlTrsmSuper * kFlTrsmSuper;  // the superblock's first block
    const uint32_t e = (bottom + 1) * kTrsmBlock;
    return e < npiv ? e : npiv;
}

// Rows [r0, r1) of the task's block for this step; false if none.
__device__ __forceinline__ bool step_block(const FlTrsmTask &t, uint32_t step, uint32_t &I, uint32_t &r0,
                                           uint32_t &r1) {
    if (step >= t.nblk) return false;
    I = t.nblk - 1 - step;
    r0 = I * kTrsmBlock;
    r1 = r0 + kTrsmBlock < t.npiv ? r0 + kTrsmBlock : t.npiv;
    return true;
}

template <int W>
__global__ __launch_bounds__(64) void k_trsm_solve_b(fl::Mod md, const FlTrsmTask *__restrict__ tasks,
                                                     const uint32_t *__restrict__ ids,
                                                     const uint32_t *__restrict__ prefix, uint32_t n,
                                                     uint32_t step, FlQueue q) {
    uint32_t task;
    for (bool ok = fl_queue_take(q, task, true); ok; ok = fl_queue_take(q, task, false)) {
        const uint32_t i = fl_task_of(prefix, n, task);
        const FlTrsmTask &t = tasks[ids[i]];
        uint32_t I, r0, r1;
        if (!step_block(t, step, I, r0, r1)) continue;
        trsm_solve_tile<W>(md, t.gptr, t.pos, t.val, t.nin, t.nnear, r0, r1, t.X, t.ldx, t.nB, t.Xh, t.Xl, t.kp,
                           task - prefix[i]);
    }
}

// Far update of the step's block, VALU form: workgroup (bx, by) of the task as
// in k_ml_spmm, flattened as by * ceil(nB / 256) + bx.
template <int W>
__global__ __launch_bounds__(256) void k_trsm_update_b(fl::Mod md, const FlTrsmTask *__restrict__ tasks,
                                                       const uint32_t *__restrict__ ids,
                                                       const uint32_t *__restrict__ prefix, uint32_t n,
                                                       uint32_t step, FlQueue q) {
    uint32_t task;
    for (bool ok = fl_queue_take(q, task, true); ok; ok = fl_queue_take(q, task, false)) {
        const uint32_t i = fl_task_of(prefix, n, task);
        const FlTrsmTask &t = tasks[ids[i]];
        uint32_t I, r0, r1;
        if (!step_block(t, step, I, r0, r1) || r1 >= t.npiv) continue;
        const uint32_t local = task - prefix[i], ct = (t.nB + kTile - 1) / kTile;
        const uint32_t g0 = r0 / W, ng = (r1 + W - 1) / W - g0;
        // (per-wave early exits inside the tile: it has no barrier)
        ml_spmm_tile<W>(md, t.gptr, t.pos, t.val, g0, ng, r1, r1, t.X, t.ldx, t.X, t.ldx, t.nB, local % ct,
                        local / ct);
    }
}

// Update of the step's block, int8-MFMA form, by superblocks: at the first
// step of a superblock, its far update (all its rows, A columns from its end
// R1 on: up to kFlTrsmSuper row tiles); at the other steps, the block's near
// update (A columns [r1, R1): the blocks solved since).  Workgroups per
// matrix: ceil(nB / 128) column tiles x kFlTrsmSuper row tiles, local index
// = row tile * column tiles + column tile.
__global__ __launch_bounds__(fl_mfma::kGemmThreads) void k_trsm_update_mfma_b(fl::Mod md, uint32_t bias, uint32_t c16,
                                                            const FlTrsmTask *__restrict__ tasks,
                                                            const uint32_t *__restrict__ ids,
                                                            const uint32_t *__restrict__ prefix,
                                                            uint32_t n, uint32_t step, FlQueue q) {
    __shared__ __attribute__((aligned(16))) int8_t smem[fl_mfma::kGemmLds];
    uint32_t task;
    for (bool ok = fl_queue_take(q, task, true); ok; ok = fl_queue_take(q, task, false)) {
        const uint32_t i = fl_task_of(prefix, n, task);
        const FlTrsmTask &t = tasks[ids[i]];
        uint32_t I, r0, r1;
        if (!step_block(t, step, I, r0, r1)) continue;
        const uint32_t ct = (t.nB + 127) / 128, local = task - prefix[i];
        const uint32_t bx = local % ct, by = local / ct;
        const uint32_t R1 = trsm_super_end(I, t.nblk, t.npiv);
        if (step % kFlTrsmSuper == 0) {
            const uint32_t top = I >= kFlTrsmSuper - 1 ? I - (kFlTrsmSuper - 1) : 0;
            if (R1 >= t.npiv || top + by > I) continue;
            const uint32_t rt = top * kTrsmBlock;
            const GemmPlanes g = {t.Ah + (uint64_t)rt * t.kp, t.Al + (uint64_t)rt * t.kp, t.Xh, t.Xl, t.kp, t.kp, R1,
                                  R1, 0, (uint32_t)(t.kp - R1), nullptr, t.krange + 2 * top, nullptr, nullptr,
                                  t.X + (uint64_t)rt * t.ldx, t.ldx, R1 - rt, t.nB, 0, t.xkend};
            fl_mfma::mfma_gemm_tile(md, bias, c16, g, bx, by, smem);
        } else {
            if (by != 0) continue;
            // (R1 - r1 is a multiple of 128 unless R1 = npiv, where the band
            // past R1 is zero)
            const GemmPlanes g = {t.Ah + (uint64_t)r0 * t.kp, t.Al + (uint64_t)r0 * t.kp, t.Xh, t.Xl, t.kp, t.kp, r1,
                                  r1, 0, (R1 - r1 + 63) / 64 * 64, t.kext + I, nullptr, nullptr, nullptr,
                                  t.X + (uint64_t)r0 * t.ldx, t.ldx, r1 - r0, t.nB, 0, t.xkend};
            fl_mfma::mfma_gemm_tile(md, bias, c16, g, bx, 0, smem);
        }
    }
}


// ---- int8-MFMA form: block solves as products with the block inverses ----
// The diagonal block T = A[r0:r1, r0:r1] of every block is unit upper
// triangular; its inverse is computed once for all blocks together (the
// back substitution applied to the identity, every block in parallel).
// The solve of a block at its step is then X[r0:r1] = T^-1 R (R: the block's
// rows after the far and near updates), computed as R - (I - T^-1) R on the
// matrix cores.

// Y: identity in every 128 x 128 block (rows past npiv zero).
__global__ __launch_bounds__(256) void k_trsm_eye(uint32_t npiv, uint32_t rows, uint16_t *Y) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)rows * kTrsmBlock) return;
    const uint32_t r = (uint32_t)(i / kTrsmBlock), c = (uint32_t)(i % kTrsmBlock);
    Y[i] = (r < npiv && c == r % kTrsmBlock) ? 1 : 0;
}

// Back substitution of every block on its identity: block blockIdx.x / 2,
// 64-column half blockIdx.x % 2.
template <int W>
__global__ __launch_bounds__(64) void k_trsm_inv(fl::Mod md, const uint64_t *__restrict__ gptr,
                                                 const uint32_t *__restrict__ pos, const uint16_t *__restrict__ val,
                                                 const uint32_t *__restrict__ nin_a,
                                                 const uint32_t *__restrict__ nnear_a, uint32_t npiv, uint16_t *Y) {
    const uint32_t I = blockIdx.x / 2, r0 = I * kTrsmBlock;
    const uint32_t r1 = r0 + kTrsmBlock < npiv ? r0 + kTrsmBlock : npiv;
    trsm_solve_tile<W>(md, gptr, pos, val, nin_a, nnear_a, r0, r1, Y, kTrsmBlock, kTrsmBlock, nullptr, nullptr, 0,
                       blockIdx.x % 2);
}

// Th/Tl = limbs of (I - Y) (zero rows past npiv).
__global__ __launch_bounds__(256) void k_trsm_inv_planes(uint32_t p, uint32_t npiv, uint32_t rows,
                                                         const uint16_t *__restrict__ Y, int8_t *Th, int8_t *Tl) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (uint64_t)rows * kTrsmBlock) return;
    const uint32_t r = (uint32_t)(i / kTrsmBlock), c = (uint32_t)(i % kTrsmBlock);
    int h = 0, l = 0;
    if (r < npiv) {
        const uint32_t y = Y[i], e = c == r % kTrsmBlock ? 1u : 0u;
        fl_split_limbs(e >= y ? e - y : e + p - y, p, h, l);
    }
    Th[i] = (int8_t)h;
    Tl[i] = (int8_t)l;
}

// Solve of block [r0, r1) for 64 columns per workgroup: R (the block's X
// rows) is staged in LDS and transposed to int8 limbs there (the B operand,
// 128 bytes of K per column); wave w computes rows [32 w, 32 w + 32) of
// (I - T^-1) R with K = 128; X = R - that, written back with the transposed
// limb planes of the finished rows (for the updates of the blocks above).
struct __attribute__((aligned(16))) ApplyLds {
    uint16_t R[kTrsmBlock][64];
    int8_t Bh[64][kTrsmBlock];
    int8_t Bl[64][kTrsmBlock];
};

// The block's near update inside its solve: R[0:nrow) -= A[r0:r1, r1:r1 + 64 KS]
// X[r1:r1 + 64 KS] for the workgroup's 64 columns, from the limb planes
// (A row-major, X transposed, kp bytes per row / column), on R in LDS.  Wave
// w computes rows [32 w, 32 w + 32) as two 16-row tiles, column tile j (16
// columns) at a time with the next tile's X fragments in flight; every
// output is owned by one lane.  K <= 384 terms: the limb sums stay far
// inside combine_limbs' bounds.
template <int KS>
__device__ __forceinline__ void trsm_near_lds(const fl::Mod &md, const fl_mfma::LimbCombine &lc,
                                              const int8_t *__restrict__ Ah, const int8_t *__restrict__ Al,
                                              const int8_t *__restrict__ Xh, const int8_t *__restrict__ Xl,
                                              uint64_t kp, uint32_t r0, uint32_t r1, uint32_t c0, uint32_t nB,
                                              uint16_t (*R)[64]) {
    using fl_mfma::v4i;
    typedef __attribute__((address_space(1))) const v4i gv4i;
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nrow = r1 - r0;
    const uint32_t cl = lane & 15, kq = (lane >> 4) * 16, rq = (lane >> 4) * 4;
    v4i ah[2][KS], al[2][KS];
#pragma unroll
    for (int rt = 0; rt < 2; rt++) {
        const uint32_t row = wave * 32 + rt * 16 + cl;
        const uint64_t o = (uint64_t)(r0 + (row < nrow ? row : 0)) * kp + r1 + kq;
#pragma unroll
        for (int s = 0; s < KS; s++) {
            ah[rt][s] = row < nrow ? *(gv4i *)(Ah + o + s * 64) : v4i{0, 0, 0, 0};
            al[rt][s] = row < nrow ? *(gv4i *)(Al + o + s * 64) : v4i{0, 0, 0, 0};
        }
    }
    v4i bh[2][KS], bl[2][KS];
#pragma unroll
    for (int s = 0; s < KS; s++) {
        const uint64_t o = (uint64_t)(c0 + cl) * kp + r1 + s * 64 + kq;
        bh[0][s] = *(gv4i *)(Xh + o);
        bl[0][s] = *(gv4i *)(Xl + o);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int cur = j & 1, nxt = cur ^ 1;
        if (j + 1 < 4) {
#pragma unroll
            for (int s = 0; s < KS; s++) {
                const uint64_t o = (uint64_t)(c0 + (j + 1) * 16 + cl) * kp + r1 + s * 64 + kq;
                bh[nxt][s] = *(gv4i *)(Xh + o);
                bl[nxt][s] = *(gv4i *)(Xl + o);
            }
        }
        v4i hh[2], mid[2], ll[2];
#pragma unroll
        for (int rt = 0; rt < 2; rt++) hh[rt] = mid[rt] = ll[rt] = v4i{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < KS; s++)
#pragma unroll
            for (int rt = 0; rt < 2; rt++) {
                hh[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[rt][s], bh[cur][s], hh[rt], 0, 0, 0);
                mid[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[rt][s], bl[cur][s], mid[rt], 0, 0, 0);
                mid[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[rt][s], bh[cur][s], mid[rt], 0, 0, 0);
                ll[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[rt][s], bl[cur][s], ll[rt], 0, 0, 0);
            }
        const uint32_t col = j * 16 + cl;
#pragma unroll
        for (int rt = 0; rt < 2; rt++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t row = wave * 32 + rt * 16 + rq + e;
                const uint32_t v = fl_mfma::combine_limbs(lc, hh[rt][e], mid[rt][e], ll[rt][e]);
                if (row < nrow && c0 + col < nB) R[row][col] = (uint16_t)fl::submod(R[row][col], v, md.p);
            }
    }
}

// KS > 0: the near update of the block (A columns [r1, r1 + 64 KS)) is
// applied to R in LDS first (see trsm_near_lds); column tiles whose X rows
// past r1 are all zero skip it.
template <int KS = 0>
__device__ __forceinline__ void trsm_apply_tile(const fl::Mod &md, uint32_t bias, uint32_t c16,
                                                const int8_t *__restrict__ Th, const int8_t *__restrict__ Tl,
                                                uint32_t r0, uint32_t r1, uint16_t *X, uint64_t ldx, uint32_t nB,
                                                int8_t *Xh, int8_t *Xl, uint64_t kp, uint32_t *xkend, uint32_t bx,
                                                ApplyLds &S, const int8_t *Ah = nullptr, const int8_t *Al = nullptr) {
    using fl_mfma::v4i;
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    typedef __attribute__((address_space(1))) const v4i gv4i;
    const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t nrow = r1 - r0, c0 = bx * 64;
    const fl_mfma::LimbCombine lc = fl_mfma::limb_combine(md, bias, c16);
    // R: 128 rows x 16 chunks of 4 columns, 8 chunks per thread (rows past the
    // block or columns past nB read as zero)
    uint64_t rv[8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t ch = tid + u * 256, r = ch >> 4, c4 = (ch & 15) * 4;
        const bool ok = r < nrow && c0 + c4 + 4 <= nB;
        rv[u] = *(gu64 *)(ok ? X + (uint64_t)(r0 + r) * ldx + c0 + c4 : X);
        if (!ok) {
            rv[u] = 0;
            if (r < nrow)
                for (uint32_t k = 0; k < 4 && c0 + c4 + k < nB; k++)
                    rv[u] |= (uint64_t)X[(uint64_t)(r0 + r) * ldx + c0 + c4 + k] << (16 * k);
        }
    }
    // A fragments: rows 32 w + 16 rt + (lane & 15), K bytes 64 s + 16 (lane >> 4)
    // (after the near update when there is one: fewer registers live there)
    const uint32_t cl = lane & 15, kq = (lane >> 4) * 16, rq = (lane >> 4) * 4;
    v4i ah[2][2], al[2][2];
    auto load_t = [&]() {
#pragma unroll
        for (int rt = 0; rt < 2; rt++)
#pragma unroll
            for (int s = 0; s < 2; s++) {
                const uint64_t o = (uint64_t)(r0 + wave * 32 + rt * 16 + cl) * kTrsmBlock + s * 64 + kq;
                ah[rt][s] = *(gv4i *)(Th + o);
                al[rt][s] = *(gv4i *)(Tl + o);
            }
    };
    if (KS == 0) load_t();
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t ch = tid + u * 256, r = ch >> 4, c4 = (ch & 15) * 4;
        *(uint64_t *)&S.R[r][c4] = rv[u];
    }
    __syncthreads();
    if constexpr (KS > 0) {
        // (uniform per workgroup) rows past r1 of X are zero in these columns
        if (!(xkend && xkend[c0 / 128] <= r1)) {
            trsm_near_lds<KS>(md, lc, Ah, Al, Xh, Xl, kp, r0, r1, c0, nB, S.R);
            __syncthreads();
        }
        load_t();
    }
    // transpose to limbs: thread -> (column, 16-row group), two per thread
#pragma unroll
    for (int u = 0; u < 2; u++) {
        const uint32_t task = tid + u * 256, c = task & 63, g = task >> 6;
        uint32_t hw[4] = {0, 0, 0, 0}, lw[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 16; k++) {
            int h, l;
            fl_split_limbs(S.R[g * 16 + k][c], md.p, h, l);
            hw[k >> 2] |= (uint32_t)(h & 0xff) << (8 * (k & 3));
            lw[k >> 2] |= (uint32_t)(l & 0xff) << (8 * (k & 3));
        }
        *(uint4 *)&S.Bh[c][g * 16] = make_uint4(hw[0], hw[1], hw[2], hw[3]);
        *(uint4 *)&S.Bl[c][g * 16] = make_uint4(lw[0], lw[1], lw[2], lw[3]);
    }
    __syncthreads();
    // per 16-column group j: K = 128 in two steps, then X = R - (I - T^-1) R
    // in place in LDS (each output is read and written by its own lane only)
#pragma unroll
    for (int j = 0; j < 4; j++) {
        v4i acc_hh[2], acc_mid[2], acc_ll[2];
#pragma unroll
        for (int rt = 0; rt < 2; rt++) acc_hh[rt] = acc_mid[rt] = acc_ll[rt] = v4i{0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < 2; s++) {
            const v4i bh = *(const v4i *)&S.Bh[j * 16 + cl][s * 64 + kq];
            const v4i bl = *(const v4i *)&S.Bl[j * 16 + cl][s * 64 + kq];
#pragma unroll
            for (int rt = 0; rt < 2; rt++) {
                acc_hh[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[rt][s], bh, acc_hh[rt], 0, 0, 0);
                acc_mid[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ah[rt][s], bl, acc_mid[rt], 0, 0, 0);
                acc_mid[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[rt][s], bh, acc_mid[rt], 0, 0, 0);
                acc_ll[rt] = __builtin_amdgcn_mfma_i32_16x16x64_i8(al[rt][s], bl, acc_ll[rt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int rt = 0; rt < 2; rt++)
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const uint32_t v = fl_mfma::combine_limbs(lc, acc_hh[rt][e], acc_mid[rt][e], acc_ll[rt][e]);
                uint16_t &o = S.R[wave * 32 + rt * 16 + rq + e][j * 16 + cl];
                o = (uint16_t)fl::submod(o, v, md.p);
            }
    }
    __syncthreads();
    uint32_t last = 0;  // 1 + the last row of the block with a nonzero in these columns
#pragma unroll
    for (int u = 0; u < 8; u++) {
        const uint32_t ch = tid + u * 256, r = ch >> 4, c4 = (ch & 15) * 4;
        if (r >= nrow || c0 + c4 >= nB) continue;
        uint16_t *o = X + (uint64_t)(r0 + r) * ldx + c0 + c4;
        const uint64_t v = *(const uint64_t *)&S.R[r][c4];  // zero past nB
        if (v) last = r0 + r + 1;
        if (c0 + c4 + 4 <= nB) *(uint64_t *)o = v;
        else
            for (uint32_t k = 0; c0 + c4 + k < nB; k++) o[k] = S.R[r][c4 + k];
    }
    if (xkend) {
        last = fl_wave_max(last);
        if (lane == 0 && last) atomicMax(&xkend[c0 / 128], last);
    }
    // transposed limb planes of the finished rows: column c, rows r0 + 16 g ..
#pragma unroll
    for (int u = 0; u < 2; u++) {
        const uint32_t task = tid + u * 256, c = task & 63, g = task >> 6;
        if (c0 + c >= nB || g * 16 >= nrow) continue;
        uint32_t hw[4] = {0, 0, 0, 0}, lw[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < 16; k++) {
            int h = 0, l = 0;
            if (g * 16 + k < nrow) fl_split_limbs(S.R[g * 16 + k][c], md.p, h, l);
            hw[k >> 2] |= (uint32_t)(h & 0xff) << (8 * (k & 3));
            lw[k >> 2] |= (uint32_t)(l & 0xff) << (8 * (k & 3));
        }
        int8_t *dh = Xh + (uint64_t)(c0 + c) * kp + r0 + g * 16, *dl = Xl + (uint64_t)(c0 + c) * kp + r0 + g * 16;
        if (g * 16 + 16 <= nrow) {
            *(uint4 *)dh = make_uint4(hw[0], hw[1], hw[2], hw[3]);
            *(uint4 *)dl = make_uint4(lw[0], lw[1], lw[2], lw[3]);
        } else {
            for (uint32_t k = 0; g * 16 + k < nrow; k++) {
                dh[k] = (int8_t)((hw[k >> 2] >> (8 * (k & 3))) & 0xff);
                dl[k] = (int8_t)((lw[k >> 2] >> (8 * (k & 3))) & 0xff);
            }
        }
    }
}

__global__ __launch_bounds__(256) void k_trsm_apply(fl::Mod md, uint32_t bias, uint32_t c16,
                                                    const int8_t *__restrict__ Th, const int8_t *__restrict__ Tl,
                                                    uint32_t r0, uint32_t r1, uint16_t *X, uint64_t ldx, uint32_t nB,
                                                    int8_t *Xh, int8_t *Xl, uint64_t kp, uint32_t *xkend) {
    __shared__ ApplyLds S;
    trsm_apply_tile(md, bias, c16, Th, Tl, r0, r1, X, ldx, nB, Xh, Xl, kp, xkend, blockIdx.x, S);
}

// The near update of block [r0, r1) (A columns [r1, r1 + 64 KS), the blocks
// of its superblock solved since its far update) and its solve in one
// launch: both are local to the workgroup's 64 columns.
template <int KS>
__global__ __launch_bounds__(256) void k_trsm_near_apply(fl::Mod md, uint32_t bias, uint32_t c16,
                                                         const int8_t *__restrict__ Th,
                                                         const int8_t *__restrict__ Tl, const int8_t *Ah,
                                                         const int8_t *Al, uint32_t r0, uint32_t r1, uint16_t *X,
                                                         uint64_t ldx, uint32_t nB, int8_t *Xh, int8_t *Xl,
                                                         uint64_t kp, uint32_t *xkend) {
    __shared__ ApplyLds S;
    trsm_apply_tile<KS>(md, bias, c16, Th, Tl, r0, r1, X, ldx, nB, Xh, Xl, kp, xkend, blockIdx.x, S, Ah, Al);
}

// The same for many matrices: the step's block of every MFMA-form matrix,
// 64-column tiles from the prefix.
__global__ __launch_bounds__(256) void k_trsm_apply_b(fl::Mod md, uint32_t bias, uint32_t c16,
                                                      const FlTrsmTask *__restrict__ tasks,
                                                      const uint32_t *__restrict__ ids,
                                                      const uint32_t *__restrict__ prefix, uint32_t n, uint32_t step,
                                                      FlQueue q) {
    __shared__ ApplyLds S;
    uint32_t task;
    for (bool ok = fl_queue_take(q, task, true); ok; ok = fl_queue_take(q, task, false)) {
        const uint32_t i = fl_task_of(prefix, n, task);
        const FlTrsmTask &t = tasks[ids[i]];
        uint32_t I, r0, r1;
        if (!step_block(t, step, I, r0, r1)) continue;
        trsm_apply_tile(md, bias, c16, t.Th, t.Tl, r0, r1, t.X, t.ldx, t.nB, t.Xh, t.Xl, t.kp, t.xkend,
                        task - prefix[i], S);
    }
}

// ---- int8-MFMA form of the TRSM: far part of every block as a limb GEMM ----

// kext[I] = (last A column used by block I's rows) + 1 - r1, or 0.
__global__ void k_trsm_kext(uint32_t w, uint32_t npiv, uint32_t nblk, const uint64_t *__restrict__ gptr,
                            const uint32_t *__restrict__ pos, uint32_t *kext) {
    const uint32_t I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nblk) return;
    const uint32_t r0 = I * kTrsmBlock;
    const uint32_t r1 = r0 + kTrsmBlock < npiv ? r0 + kTrsmBlock : npiv;
    uint32_t kend = r1;
    for (uint32_t g = r0 / w; g < (r1 + w - 1) / w; g++) {
        const uint64_t b = gptr[g], e = gptr[g + 1];
        if (e > b) {
            const uint32_t last = pos[e - 1] + 1;
            kend = last > kend ? last : kend;
        }
    }
    kext[I] = kend - r1;
}

__global__ void k_trsm_krange(uint32_t npiv, uint32_t nblk, const uint32_t *__restrict__ kext, uint32_t *krange) {
    const uint32_t I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nblk) return;
    const uint32_t r1 = (I + 1) * kTrsmBlock < npiv ? (I + 1) * kTrsmBlock : npiv;
    const uint32_t R1 = trsm_super_end(I, nblk, npiv);
    const uint32_t end = r1 + (kext[I] + 63) / 64 * 64;
    krange[2 * I] = 0;
    krange[2 * I + 1] = end > R1 ? end - R1 : 0;
}

// Zero the band [r1, r1 + round_up(max(kext, R1 - r1), 64)) of the A limb
// planes for every row of block blockIdx.x (row blockIdx.y within the block).
__global__ __launch_bounds__(256) void k_trsm_zero_band(uint32_t npiv, const uint32_t *__restrict__ kext,
                                                        int8_t *Ah, int8_t *Al, uint64_t kp) {
    const uint32_t I = blockIdx.x, row = I * kTrsmBlock + blockIdx.y;
    if (row >= npiv) return;
    const uint32_t r1 = (I + 1) * kTrsmBlock < npiv ? (I + 1) * kTrsmBlock : npiv;
    // the near update of the block reads up to round_up(R1 - r1, 64)
    const uint32_t R1 = trsm_super_end(I, (npiv + kTrsmBlock - 1) / kTrsmBlock, npiv);
    const uint32_t kf = (kext[I] + 63) / 64 * 64, kn = (R1 - r1 + 63) / 64 * 64;
    const uint32_t kb = kf > kn ? kf : kn;
    int8_t *h = Ah + (uint64_t)row * kp + r1, *l = Al + (uint64_t)row * kp + r1;
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (uint32_t k = threadIdx.x * 16; k < kb; k += blockDim.x * 16) {
        *(uint4 *)(h + k) = z;
        *(uint4 *)(l + k) = z;
    }
}

// Far entries (column >= r1 of the row's block) of A -> dense limb planes.
__global__ __launch_bounds__(256) void k_trsm_scatter_far(uint32_t w, uint32_t p, uint32_t npiv,
                                                          uint32_t ngroups,
                                                          const uint64_t *__restrict__ gptr,
                                                          const uint32_t *__restrict__ pos,
                                                          const uint16_t *__restrict__ val,
                                                          int8_t *Ah, int8_t *Al, uint64_t kp) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= ngroups) return;
    const uint32_t I = (g * w) / kTrsmBlock;
    const uint32_t r1 = (I + 1) * kTrsmBlock < npiv ? (I + 1) * kTrsmBlock : npiv;
    for (uint64_t k = gptr[g] + lane; k < gptr[g + 1]; k += 64) {
        const uint32_t c = pos[k];
        if (c < r1) continue;
        for (uint32_t q = 0; q < w; q++) {
            const uint32_t row = g * w + q;
            if (row >= npiv) break;
            int h, l;
            fl_split_limbs(val[(uint64_t)w * k + q], p, h, l);
            Ah[(uint64_t)row * kp + c] = (int8_t)h;
            Al[(uint64_t)row * kp + c] = (int8_t)l;
        }
    }
}

template <int W>
hipError_t launch_ml_spmm(const fl::Mod &md, const uint64_t *gptr, const uint32_t *pos,
                          const uint16_t *val, uint32_t g0, uint32_t ngroups, uint32_t row_limit,
                          uint32_t pos_lo, const uint16_t *X, uint64_t ldx, uint16_t *out,
                          uint64_t ldo, uint32_t ncols, hipStream_t s) {
    if (ngroups == 0 || ncols == 0) return hipSuccess;
    dim3 grid((ncols + kTile - 1) / kTile, (ngroups + 3) / 4);
    hipLaunchKernelGGL(k_ml_spmm<W>, grid, dim3(256), 0, s, md, gptr, pos, val, g0, ngroups,
                       row_limit, pos_lo, X, ldx, out, ldo, ncols);
    return hipGetLastError();
}

hipError_t ml_spmm(uint32_t w, const fl::Mod &md, const uint64_t *gptr, const uint32_t *pos,
                   const uint16_t *val, uint32_t g0, uint32_t ngroups, uint32_t row_limit,
                   uint32_t pos_lo, const uint16_t *X, uint64_t ldx, uint16_t *out, uint64_t ldo,
                   uint32_t ncols, hipStream_t s) {
    switch (w) {
    case 1: return launch_ml_spmm<1>(md, gptr, pos, val, g0, ngroups, row_limit, pos_lo, X, ldx, out, ldo, ncols, s);
    case 2: return launch_ml_spmm<2>(md, gptr, pos, val, g0, ngroups, row_limit, pos_lo, X, ldx, out, ldo, ncols, s);
    case 4: return launch_ml_spmm<4>(md, gptr, pos, val, g0, ngroups, row_limit, pos_lo, X, ldx, out, ldo, ncols, s);
    default: return launch_ml_spmm<8>(md, gptr, pos, val, g0, ngroups, row_limit, pos_lo, X, ldx, out, ldo, ncols, s);
    }
}

hipError_t trsm_solve(uint32_t w, const fl::Mod &md, const uint64_t *gptr, const uint32_t *pos,
                      const uint16_t *val, const uint32_t *nin, const uint32_t *nnear, uint32_t r0,
                      uint32_t r1, uint16_t *X, uint64_t ldx, uint32_t ncols, hipStream_t s,
                      int8_t *Xth, int8_t *Xtl, uint64_t kp) {
    dim3 grid((ncols + 63) / 64);
    switch (w) {
    case 1: hipLaunchKernelGGL(k_trsm_solve<1>, grid, dim3(64), 0, s, md, gptr, pos, val, nin, nnear, r0, r1, X, ldx, ncols, Xth, Xtl, kp); break;
    case 2: hipLaunchKernelGGL(k_trsm_solve<2>, grid, dim3(64), 0, s, md, gptr, pos, val, nin, nnear, r0, r1, X, ldx, ncols, Xth, Xtl, kp); break;
    case 4: hipLaunchKernelGGL(k_trsm_solve<4>, grid, dim3(64), 0, s, md, gptr, pos, val, nin, nnear, r0, r1, X, ldx, ncols, Xth, Xtl, kp); break;
    default: hipLaunchKernelGGL(k_trsm_solve<8>, grid, dim3(64), 0, s, md, gptr, pos, val, nin, nnear, r0, r1, X, ldx, ncols, Xth, Xtl, kp); break;
    }
    return hipGetLastError();
}

struct TrsmWs {
    int8_t *Ah, *Al, *Xh, *Xl;
    uint16_t *Y;        // [nblk * 128 x 128] inverses of the diagonal blocks
    int8_t *Th, *Tl;    // [nblk * 128 x 128] limb planes of I - (block inverse)
    uint32_t *kext, *krange;
    uint32_t *nin, *nnear;
    uint32_t *xkend;    // [ceil(nB / 128)] see FlTrsmTask::xkend
    uint64_t kp;
};

size_t trsm_layout(const fl_split_info *info, fl_mode mode, void *ws, TrsmWs *t) {
    WsCarve c(ws);
    TrsmWs r = {};
    if (info->npiv && info->nB) {
        const uint32_t w = info->ml_width ? info->ml_width : 1;
        const uint32_t ngroups = (info->npiv + w - 1) / w;
        r.nin = c.take<uint32_t>(ngroups);
        r.nnear = c.take<uint32_t>(ngroups);
    }
    if (mode == FL_MFMA_I8 && info->npiv && info->nB) {
        const uint64_t mp = ((uint64_t)info->npiv + 127) / 128 * 128;
        const uint64_t np = ((uint64_t)info->nB + 127) / 128 * 128;
        r.kp = ((uint64_t)info->npiv + 63) / 64 * 64 + 64;
        r.Ah = c.take<int8_t>(mp * r.kp);
        r.Al = c.take<int8_t>(mp * r.kp);
        r.Xh = c.take<int8_t>(np * r.kp);
        r.Xl = c.take<int8_t>(np * r.kp);
        r.kext = c.take<uint32_t>((info->npiv + kTrsmBlock - 1) / kTrsmBlock);
        r.krange = c.take<uint32_t>(2 * (size_t)((info->npiv + kTrsmBlock - 1) / kTrsmBlock));
        r.Y = c.take<uint16_t>(mp * kTrsmBlock);
        r.Th = c.take<int8_t>(mp * kTrsmBlock);
        r.Tl = c.take<int8_t>(mp * kTrsmBlock);
        r.xkend = c.take<uint32_t>(np / 128);
    }
    if (t) *t = r;
    return c.off;
}

hipError_t csr_to_dense(uint32_t rows, uint32_t cols, const uint64_t *rp, const uint32_t *ci,
                        const uint16_t *v, uint16_t *out, uint64_t ld, hipStream_t s) {
    if (rows == 0) return hipSuccess;
    hipError_t e = fl_zero_rows_u16(out, ld, rows, cols, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_csr_scatter, dim3((rows + 3) / 4), dim3(256), 0, s, rows, rp, ci, v, out, ld);
    return hipGetLastError();
}

fl_status check_split_info(const fl_split_info *info, const fl_split_out *s) {
    FL_ARG(info && s, "NULL split info/output");
    FL_ARG(info->status == FL_OK, "split info carries an error status");
    FL_ARG(info->p >= 2 && info->p <= 65521, "split info: bad p");
    FL_ARG(info->ml_width == 1 || info->ml_width == 2 || info->ml_width == 4 || info->ml_width == 8,
           "split info: bad ml_width");
    FL_ARG(info->npiv + info->nB == info->n && info->npiv + info->mD == info->m,
           "split info: inconsistent sizes");
    return FL_OK;
}

}  // namespace

// Exposed to the other translation units of the library.
hipError_t fl_ml_spmm(uint32_t w, uint32_t p, const uint64_t *gptr, const uint32_t *pos,
                      const uint16_t *val, uint32_t g0, uint32_t ngroups, uint32_t row_limit,
                      uint32_t pos_lo, const uint16_t *X, uint64_t ldx, uint16_t *out,
                      uint64_t ldo, uint32_t ncols, hipStream_t s, const char *site) {
    hipError_t e;
    FL_PROF(site, s, e = ml_spmm(w, fl::make_mod(p), gptr, pos, val, g0, ngroups, row_limit, pos_lo,
                                 X, ldx, out, ldo, ncols, s));
    return e;
}
hipError_t fl_csr_to_dense(uint32_t rows, uint32_t cols, const uint64_t *rp, const uint32_t *ci,
                           const uint16_t *v, uint16_t *out, uint64_t ld, hipStream_t s) {
    return csr_to_dense(rows, cols, rp, ci, v, out, ld, s);
}
fl_status fl_check_split(const fl_split_info *info, const fl_split_out *s) {
    return check_split_info(info, s);
}

extern "C" size_t fl_trsm_workspace(const fl_split_info *info, fl_mode mode) {
    if (!info) return 0;
    return trsm_layout(info, mode, nullptr, nullptr);
}

// The limb planes of X that an MFMA-form fl_trsm leaves in its workspace
// (written by the block solves, read by the far and near updates).
extern "C" fl_status fl_trsm_planes(const fl_split_info *info, const void *ws, size_t ws_bytes,
                                    const int8_t **Xh, const int8_t **Xl, uint64_t *ldp,
                                    const uint32_t **row_end) {
    FL_ARG(info && Xh && Xl && ldp, "fl_trsm_planes: NULL argument");
    FL_ARG(info->npiv && info->nB, "fl_trsm_planes: empty X (npiv or nB is 0)");
    TrsmWs tw;
    const size_t need = trsm_layout(info, FL_MFMA_I8, const_cast<void *>(ws), &tw);
    FL_ARG(ws && ws_bytes >= need, "fl_trsm_planes: workspace smaller than fl_trsm_workspace(info, FL_MFMA_I8)");
    *Xh = tw.Xh;
    *Xl = tw.Xl;
    *ldp = tw.kp;
    if (row_end) *row_end = tw.xkend;
    return FL_OK;
}

fl_status fl_trsm_prepare(const fl_split_info *info, const fl_split_out *s, uint16_t *X, uint64_t ldx,
                          fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream, FlTrsmTask *task) {
    fl_status st = check_split_info(info, s);
    if (st != FL_OK) return st;
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_trsm: bad mode");
    const uint32_t npiv = info->npiv, nB = info->nB, w = info->ml_width;
    FlTrsmTask t = {};
    t.npiv = npiv;
    t.nB = nB;
    t.X = X;
    t.ldx = ldx;
    t.mfma = mode == FL_MFMA_I8;
    t.gptr = s->a_gptr;
    t.pos = s->a_pos;
    t.val = s->a_val;
    if (npiv == 0 || nB == 0) {
        *task = t;  // nblk = 0: nothing to do
        return FL_OK;
    }
    FL_ARG(X, "fl_trsm: NULL X");
    FL_ARG(ldx >= nB && ldx % 4 == 0, "fl_trsm: ldx must be >= nB and a multiple of 4");
    FL_ARG(((uintptr_t)X & 7) == 0, "fl_trsm: X must be 8-byte aligned");
    TrsmWs tw;
    const size_t need = trsm_layout(info, mode, ws, &tw);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_trsm: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    hipError_t e0;
    FL_PROF("trsm.densify", stream, e0 = csr_to_dense(npiv, nB, s->b_ptr, s->b_col, s->b_val, X, ldx, stream));
    FL_HIP(e0);
    const uint32_t nblk = (npiv + kTrsmBlock - 1) / kTrsmBlock;
    const uint32_t ngroups = (npiv + w - 1) / w;
    FL_PROF("trsm.bounds", stream,
            hipLaunchKernelGGL(k_trsm_bounds, dim3((ngroups + 3) / 4), dim3(256), 0, stream, w, npiv, ngroups,
                               (const uint64_t *)s->a_gptr, (const uint32_t *)s->a_pos, tw.nin, tw.nnear));
    FL_LAUNCH_CHECK("k_trsm_bounds");
    if (t.mfma) {
        FL_PROF("trsm.tiles", stream, {
            hipLaunchKernelGGL(k_trsm_kext, dim3((nblk + 255) / 256), dim3(256), 0, stream, w, npiv,
                               nblk, (const uint64_t *)s->a_gptr, (const uint32_t *)s->a_pos, tw.kext);
            hipLaunchKernelGGL(k_trsm_krange, dim3((nblk + 255) / 256), dim3(256), 0, stream, npiv, nblk,
                               (const uint32_t *)tw.kext, tw.krange);
            hipLaunchKernelGGL(k_trsm_zero_band, dim3(nblk, kTrsmBlock), dim3(256), 0, stream, npiv,
                               (const uint32_t *)tw.kext, tw.Ah, tw.Al, tw.kp);
            hipLaunchKernelGGL(k_trsm_scatter_far, dim3((ngroups + 3) / 4), dim3(256), 0, stream, w,
                               info->p, npiv, ngroups, (const uint64_t *)s->a_gptr,
                               (const uint32_t *)s->a_pos, (const uint16_t *)s->a_val, tw.Ah, tw.Al, tw.kp);
        });
        FL_LAUNCH_CHECK("trsm tiles");
        FL_HIP(fl_fill_u32(tw.xkend, 0, (nB + 127) / 128, stream));
        const uint32_t rows = nblk * kTrsmBlock;
        const unsigned ge = (unsigned)(((uint64_t)rows * kTrsmBlock + 255) / 256);
        const fl::Mod md = fl::make_mod(info->p);
        FL_PROF("trsm.inverse", stream, {
            hipLaunchKernelGGL(k_trsm_eye, dim3(ge), dim3(256), 0, stream, npiv, rows, tw.Y);
            switch (w) {
            case 1: hipLaunchKernelGGL(k_trsm_inv<1>, dim3(2 * nblk), dim3(64), 0, stream, md, s->a_gptr, s->a_pos, s->a_val, tw.nin, tw.nnear, npiv, tw.Y); break;
            case 2: hipLaunchKernelGGL(k_trsm_inv<2>, dim3(2 * nblk), dim3(64), 0, stream, md, s->a_gptr, s->a_pos, s->a_val, tw.nin, tw.nnear, npiv, tw.Y); break;
            case 4: hipLaunchKernelGGL(k_trsm_inv<4>, dim3(2 * nblk), dim3(64), 0, stream, md, s->a_gptr, s->a_pos, s->a_val, tw.nin, tw.nnear, npiv, tw.Y); break;
            default: hipLaunchKernelGGL(k_trsm_inv<8>, dim3(2 * nblk), dim3(64), 0, stream, md, s->a_gptr, s->a_pos, s->a_val, tw.nin, tw.nnear, npiv, tw.Y); break;
            }
            hipLaunchKernelGGL(k_trsm_inv_planes, dim3(ge), dim3(256), 0, stream, info->p, npiv, rows,
                               (const uint16_t *)tw.Y, tw.Th, tw.Tl);
        });
        FL_LAUNCH_CHECK("trsm inverse");
    }
    t.nblk = nblk;
    t.nin = tw.nin;
    t.nnear = tw.nnear;
    t.Ah = tw.Ah;
    t.Al = tw.Al;
    t.Xh = tw.Xh;
    t.Xl = tw.Xl;
    t.kext = tw.kext;
    t.krange = tw.krange;
    t.Th = tw.Th;
    t.Tl = tw.Tl;
    t.kp = tw.kp;
    t.xkend = tw.xkend;
    *task = t;
    return FL_OK;
}

hipError_t fl_trsm_batch_launch(int kind, uint32_t p, uint32_t w, const FlTrsmTask *tasks,
                                const uint32_t *ids, const uint32_t *prefix, uint32_t n, uint32_t total,
                                uint32_t step, uint32_t *counter, uint32_t per_cu, hipStream_t stream) {
    if (n == 0 || total == 0) return hipSuccess;
    const fl::Mod md = fl::make_mod(p);
    // persistent launch over the step's tiles of every matrix, or one
    // workgroup per tile
    const FlQueue q = {per_cu && counter ? counter : nullptr, total};
    const uint32_t grid = q.counter ? fl_queue_grid(total, per_cu) : total;
    if (kind == 3) {
        hipLaunchKernelGGL(k_trsm_apply_b, dim3(grid), dim3(256), 0, stream, md, fl_mfma::gemm_bias(p),
                           fl_mfma::gemm_c16(p), tasks, ids, prefix, n, step, q);
    } else if (kind == 2) {
        switch (w) {
        case 1: hipLaunchKernelGGL(k_trsm_solve_b<1>, dim3(grid), dim3(64), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        case 2: hipLaunchKernelGGL(k_trsm_solve_b<2>, dim3(grid), dim3(64), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        case 4: hipLaunchKernelGGL(k_trsm_solve_b<4>, dim3(grid), dim3(64), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        default: hipLaunchKernelGGL(k_trsm_solve_b<8>, dim3(grid), dim3(64), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        }
    } else if (step == 0) {
        return hipSuccess;  // the bottom blocks have nothing below them
    } else if (kind == 1) {
        hipLaunchKernelGGL(k_trsm_update_mfma_b, dim3(grid), dim3(fl_mfma::kGemmThreads), 0, stream, md, fl_mfma::gemm_bias(p),
                           fl_mfma::gemm_c16(p), tasks, ids, prefix, n, step, q);
    } else {
        switch (w) {
        case 1: hipLaunchKernelGGL(k_trsm_update_b<1>, dim3(grid), dim3(256), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        case 2: hipLaunchKernelGGL(k_trsm_update_b<2>, dim3(grid), dim3(256), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        case 4: hipLaunchKernelGGL(k_trsm_update_b<4>, dim3(grid), dim3(256), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        default: hipLaunchKernelGGL(k_trsm_update_b<8>, dim3(grid), dim3(256), 0, stream, md, tasks, ids, prefix, n, step, q); break;
        }
    }
    return hipGetLastError();
}

extern "C" fl_status fl_trsm(const fl_split_info *info, const fl_split_out *s, uint16_t *X,
                             uint64_t ldx, fl_mode mode, void *ws, size_t ws_bytes,
                             hipStream_t stream) {
    FlTrsmTask t;
    fl_status st = fl_trsm_prepare(info, s, X, ldx, mode, ws, ws_bytes, stream, &t);
    if (st != FL_OK || t.nblk == 0) return st;
    const fl::Mod md = fl::make_mod(info->p);
    const uint32_t npiv = t.npiv, nB = t.nB, w = info->ml_width;
    // MFMA form: the far update of a superblock is split by K.  The terms
    // from the superblock just below it are the critical path (main stream);
    // the terms from the rows below that are ready one superblock earlier and
    // run on a second stream, overlapping the superblock below's solve.
    hipStream_t far_s = nullptr;
    hipEvent_t ev_ready = nullptr, ev_far = nullptr;
    if (t.mfma) FL_CHECK_ST(fl_aux_stream(1, &far_s, &ev_ready, &ev_far));
    bool far_pending = false;
    for (uint32_t I = t.nblk; I-- > 0;) {
        const uint32_t r0 = I * kTrsmBlock;
        const uint32_t r1 = r0 + kTrsmBlock < npiv ? r0 + kTrsmBlock : npiv;
        uint32_t near_ks = 0;  // MFMA form: K steps of the near update, done in the solve's launch
        if (r1 < npiv) {
            hipError_t e;
            if (t.mfma) {
                const uint32_t step = t.nblk - 1 - I, R1 = trsm_super_end(I, t.nblk, npiv);
                e = hipSuccess;
                if (step % kFlTrsmSuper == 0) {
                    // superblock [rt, R1) (not the bottom one: it has 512 rows
                    // unless it is the top one); every row at or past R1 is solved
                    const uint32_t top = I >= kFlTrsmSuper - 1 ? I - (kFlTrsmSuper - 1) : 0;
                    const uint32_t rt = top * kTrsmBlock;
                    const uint32_t R2 = R1 + kFlTrsmSuper * kTrsmBlock < npiv ? R1 + kFlTrsmSuper * kTrsmBlock : npiv;
                    // wait for its terms from rows at or past R2 (second stream)
                    if (far_pending) {
                        FL_HIP(hipStreamWaitEvent(stream, ev_far, 0));
                        far_pending = false;
                    }
                    // its terms from the superblock [R1, R2) below it
                    GemmPlanes gp = {t.Ah + (uint64_t)rt * t.kp, t.Al + (uint64_t)rt * t.kp, t.Xh, t.Xl, t.kp,
                                     t.kp, R1, R1, 0, (R2 - R1 + 63) / 64 * 64, nullptr, t.krange + 2 * top, nullptr,
                                     nullptr, X + (uint64_t)rt * ldx, ldx, R1 - rt, nB};
                    gp.group_m = kFlTrsmSuper;  // the superblock's row tiles share each B column tile
                    gp.kcap_n = t.xkend;        // column tiles where those rows of X are zero: skipped
                    gp.max_wg = kGemmPerCu;     // short K ranges: fetch overlapping write-back
                    FL_HIP(fl_mfma_gemm_planes(info->p, gp, stream, "trsm.update.mfma"));
                    // the superblock above [ru, rt): its terms from rows at or past R1,
                    // issued after the critical-path GEMM, which then does not queue behind it
                    if (top > 0) {
                        const uint32_t topu = top >= kFlTrsmSuper ? top - kFlTrsmSuper : 0;
                        const uint32_t ru = topu * kTrsmBlock;
                        FL_HIP(hipEventRecord(ev_ready, stream));
                        FL_HIP(hipStreamWaitEvent(far_s, ev_ready, 0));
                        GemmPlanes gf = {t.Ah + (uint64_t)ru * t.kp, t.Al + (uint64_t)ru * t.kp, t.Xh, t.Xl, t.kp,
                                         t.kp, rt, rt, R1 - rt, (uint32_t)(t.kp - rt), nullptr, t.krange + 2 * topu,
                                         nullptr, nullptr, X + (uint64_t)ru * ldx, ldx, rt - ru, nB};
                        gf.group_m = kFlTrsmSuper;
                        gf.kcap_n = t.xkend;
                        // 32 compute units stay free for the solves of the
                        // superblock below, which run meanwhile (measured on
                        // 256: 1 ms faster than all units, equal to 64 free)
                        gf.max_wg = fl_cu_count() > 96 ? fl_cu_count() - 32 : kGemmPerCu;
                        FL_HIP(fl_mfma_gemm_planes(info->p, gf, far_s, "trsm.update.far"));
                        FL_HIP(hipEventRecord(ev_far, far_s));
                        far_pending = true;
                    }
                } else {  // near update: the blocks of the superblock solved since
                    near_ks = (R1 - r1 + 63) / 64;
                }
            } else {
                const uint32_t g0 = r0 / w, g1 = (r1 + w - 1) / w;
                FL_PROF("trsm.update", stream,
                        e = ml_spmm(w, md, s->a_gptr, s->a_pos, s->a_val, g0, g1 - g0, r1, r1, X, ldx, X,
                                    ldx, nB, stream));
            }
            FL_HIP(e);
        }
        hipError_t e;
        if (t.mfma) {
            const uint32_t bias = fl_mfma::gemm_bias(info->p), c16 = fl_mfma::gemm_c16(info->p);
            const dim3 grid((nB + 63) / 64);
            const int8_t *Th = t.Th, *Tl = t.Tl;
            if (near_ks == 0) {
                FL_PROF("trsm.apply", stream,
                        hipLaunchKernelGGL(k_trsm_apply, grid, dim3(256), 0, stream, md, bias, c16, Th, Tl, r0, r1,
                                           X, ldx, nB, t.Xh, t.Xl, t.kp, t.xkend));
            } else {
#define FL_NEAR_APPLY(K)                                                                                        \
    case K:                                                                                                     \
        FL_PROF("trsm.near_apply", stream,                                                                      \
                hipLaunchKernelGGL(k_trsm_near_apply<K>, grid, dim3(256), 0, stream, md, bias, c16, Th, Tl,     \
                                   (const int8_t *)t.Ah, (const int8_t *)t.Al, r0, r1, X, ldx, nB, t.Xh, t.Xl, \
                                   t.kp, t.xkend));                                                             \
        break;
                switch (near_ks) {
                    FL_NEAR_APPLY(1)
                    FL_NEAR_APPLY(2)
                    FL_NEAR_APPLY(3)
                    FL_NEAR_APPLY(4)
                    FL_NEAR_APPLY(5)
                    FL_NEAR_APPLY(6)
                default: FL_HIP(hipErrorInvalidValue);
                }
#undef FL_NEAR_APPLY
            }
            e = hipGetLastError();
        } else {
            FL_PROF("trsm.solve", stream,
                    e = trsm_solve(w, md, s->a_gptr, s->a_pos, s->a_val, t.nin, t.nnear, r0, r1, X, ldx, nB, stream,
                                   nullptr, nullptr, t.kp));
        }
        FL_HIP(e);
    }
    if (far_pending) FL_HIP(hipStreamWaitEvent(stream, ev_far, 0));
    return FL_OK;
}
