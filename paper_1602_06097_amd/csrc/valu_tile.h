// valu_tile.h -- dense C = C - A B mod p on the vector ALUs (one tile).
//
// The dense contractions of the reduction (the rank-k trailing updates of the
// Gauss-Jordan elimination of the Schur complement, the second FL pass, and
// the dense form of C X) all have this shape.  One wave computes 8 rows x 256
// columns (4 columns per lane).  The K dimension is walked in chunks of 64:
// lane t holds A[row][k0 + t] for the wave's 8 rows, and each step broadcasts
// one coefficient per row with v_readlane while every lane loads 4 residues of
// one row of B.  Products use the split-coefficient 24-bit multiply-add with
// folding at most every 256 terms.
#pragma once

#include "fl_internal.h"

namespace fl_valu {

constexpr int kRowsPerWave = 8;
constexpr int kColsPerWave = 256;

// Workgroup (bx, by): rows [(4 by + wave) * 8, +8) x columns [256 bx, +256).
// Optional zero-skipping (both NULL: the whole K range):
//   krange_n  per 128-column tile of B a range [b, e) of K holding every row
//             of B with a nonzero in those columns (b >= e: none);
//   kfirst    per row of A the first k with A[row][k] != 0 (0xffffffff: none).
__device__ __forceinline__ void valu_gemm_tile(const fl::Mod &md, uint32_t M, uint32_t N, uint32_t Kh,
                                               const uint32_t *__restrict__ Kdev,
                                               const uint16_t *__restrict__ A, uint64_t lda,
                                               const uint16_t *__restrict__ B, uint64_t ldb,
                                               uint16_t *C, uint64_t ldc, uint32_t bx, uint32_t by,
                                               const uint32_t *__restrict__ krange_n = nullptr,
                                               const uint32_t *__restrict__ kfirst = nullptr) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t row0 = (by * 4 + (threadIdx.x >> 6)) * kRowsPerWave;
    if (row0 >= M) return;
    const uint32_t K = Kdev ? *Kdev : Kh;
    if (K == 0) return;
    uint32_t kbeg = 0, kend = K;
    if (krange_n) {  // the (one or two) 128-column tiles of this 256-column tile
        const uint32_t t0 = 2 * bx, nt = (N + 127) / 128;
        uint32_t b = 0xffffffffu, e = 0;
        for (uint32_t t = t0; t < t0 + 2 && t < nt; t++) {
            const uint32_t tb = krange_n[2 * t], te = krange_n[2 * t + 1];
            if (tb < te) {
                b = tb < b ? tb : b;
                e = te > e ? te : e;
            }
        }
        kbeg = b > kbeg ? b : kbeg;
        kend = e < kend ? e : kend;
    }
    if (kfirst) {  // the wave's rows are zero in A before their first nonzero
        uint32_t f = 0xffffffffu;
        for (uint32_t r = 0; r < kRowsPerWave && row0 + r < M; r++) f = kfirst[row0 + r] < f ? kfirst[row0 + r] : f;
        kbeg = f > kbeg ? f : kbeg;
    }
    if (kbeg >= kend) return;  // (wave-uniform) nothing to subtract
    const uint32_t c0 = bx * kColsPerWave + lane * 4;
    const bool colok = c0 < N;
    uint32_t ah[kRowsPerWave][4], al[kRowsPerWave][4];
#pragma unroll
    for (int r = 0; r < kRowsPerWave; r++)
#pragma unroll
        for (int c = 0; c < 4; c++) ah[r][c] = al[r][c] = 0;
    uint32_t terms = 0;
    for (uint32_t k0 = kbeg; k0 < kend; k0 += 64) {
        const uint32_t chunk = kend - k0 < 64 ? kend - k0 : 64;
        uint32_t a[kRowsPerWave];
#pragma unroll
        for (int r = 0; r < kRowsPerWave; r++)
            a[r] = (row0 + r < M && lane < chunk) ? A[(uint64_t)(row0 + r) * lda + k0 + lane] : 0;
        uint32_t t = 0;
        for (; t + 2 <= chunk; t += 2) {
            uint64_t bv[2];
#pragma unroll
            for (int u = 0; u < 2; u++)
                bv[u] = colok ? *(const uint64_t *)(B + (uint64_t)(k0 + t + u) * ldb + c0) : 0;
#pragma unroll
            for (int u = 0; u < 2; u++) {
                uint32_t x[4] = {(uint32_t)bv[u] & 0xffffu, (uint32_t)(bv[u] >> 16) & 0xffffu,
                                 (uint32_t)(bv[u] >> 32) & 0xffffu, (uint32_t)(bv[u] >> 48)};
#pragma unroll
                for (int r = 0; r < kRowsPerWave; r++) {
                    uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)a[r], (int)(t + u));
                    uint32_t lh = lam >> 8, ll = lam & 0xffu;
#pragma unroll
                    for (int c = 0; c < 4; c++) {
                        ah[r][c] = fl::mad24(lh, x[c], ah[r][c]);
                        al[r][c] = fl::mad24(ll, x[c], al[r][c]);
                    }
                }
            }
        }
        for (; t < chunk; t++) {
            uint64_t bv = colok ? *(const uint64_t *)(B + (uint64_t)(k0 + t) * ldb + c0) : 0;
            uint32_t x[4] = {(uint32_t)bv & 0xffffu, (uint32_t)(bv >> 16) & 0xffffu,
                             (uint32_t)(bv >> 32) & 0xffffu, (uint32_t)(bv >> 48)};
#pragma unroll
            for (int r = 0; r < kRowsPerWave; r++) {
                uint32_t lam = (uint32_t)__builtin_amdgcn_readlane((int)a[r], (int)t);
                uint32_t lh = lam >> 8, ll = lam & 0xffu;
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    ah[r][c] = fl::mad24(lh, x[c], ah[r][c]);
                    al[r][c] = fl::mad24(ll, x[c], al[r][c]);
                }
            }
        }
        terms += chunk;
        if (terms > FL_FOLD_TERMS - 64) {
#pragma unroll
            for (int r = 0; r < kRowsPerWave; r++)
#pragma unroll
                for (int c = 0; c < 4; c++) {
                    al[r][c] = fl::fold_pair(ah[r][c], al[r][c], md);
                    ah[r][c] = 0;
                }
            terms = 0;
        }
    }
    if (!colok) return;
#pragma unroll
    for (int r = 0; r < kRowsPerWave; r++) {
        if (row0 + r >= M) break;
        uint16_t *o = C + (uint64_t)(row0 + r) * ldc + c0;
        uint32_t s[4];
#pragma unroll
        for (int c = 0; c < 4; c++) s[c] = fl::fold_pair(ah[r][c], al[r][c], md);
        if (c0 + 4 <= N) {
            uint64_t ov = *(const uint64_t *)o;
            uint64_t nv = 0;
#pragma unroll
            for (int c = 0; c < 4; c++)
                nv |= (uint64_t)fl::submod((uint32_t)(ov >> (16 * c)) & 0xffffu, s[c], md.p) << (16 * c);
            *(uint64_t *)o = nv;
        } else {
            for (int c = 0; c < 4 && c0 + c < N; c++) o[c] = (uint16_t)fl::submod(o[c], s[c], md.p);
        }
    }
}

}  // namespace fl_valu
