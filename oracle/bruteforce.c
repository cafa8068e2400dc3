/*
 * bruteforce.c -- Gauss-Jordan elimination mod p directly on a dense copy of
 * the whole input matrix M, with no splicing into A, B, C, D.
 *
 * TEST INFRASTRUCTURE ONLY (loaded by the test suite).  Independent of both
 * fl_oracle.c and the device library: it exists to pin the FL oracle through
 * the uniqueness of the reduced row echelon form over a field -- whatever
 * order of operations reaches it, RREF(M) is the same matrix.
 *
 * To differ from the oracle's own Gauss-Jordan on purpose it picks the *last*
 * remaining row holding a nonzero in the current column as the pivot row, and
 * it inverts by Fermat's little theorem instead of the extended Euclidean
 * algorithm.
 */
#include <stdint.h>
#include <stdlib.h>

static uint32_t bf_pow(uint32_t a, uint32_t e, uint32_t p)
{
    uint64_t r = 1, b = a % p;
    while (e) {
        if (e & 1) r = (r * b) % p;
        b = (b * b) % p;
        e >>= 1;
    }
    return (uint32_t)r;
}

/* In-place RREF of the dense m x n matrix W (row-major, int32 residues).
 * Rows 0..rank-1 end up sorted by pivot column.  Returns the rank. */
static uint32_t bf_gauss_jordan(uint32_t m, uint32_t n, int32_t *W, uint32_t p)
{
    uint32_t rank = 0;
    for (uint32_t c = 0; c < n && rank < m; c++) {
        int64_t piv = -1;
        for (int64_t i = (int64_t)m - 1; i >= (int64_t)rank; i--)
            if (W[(uint64_t)i * n + c] != 0) { piv = i; break; }
        if (piv < 0) continue;
        int32_t *pr = W + (uint64_t)piv * n, *rr = W + (uint64_t)rank * n;
        for (uint32_t k = 0; k < n; k++) { int32_t t = pr[k]; pr[k] = rr[k]; rr[k] = t; }
        int64_t inv = bf_pow((uint32_t)rr[c], p - 2, p);
        for (uint32_t k = 0; k < n; k++) rr[k] = (int32_t)((rr[k] * inv) % p);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)m; i++) {
            int32_t *ri = W + (uint64_t)i * n;
            int64_t f = ri[c];
            if (i == (int64_t)rank || f == 0) continue;
            for (uint32_t k = 0; k < n; k++) {
                int64_t x = ((int64_t)ri[k] - f * rr[k]) % (int64_t)p;
                ri[k] = (int32_t)(x < 0 ? x + p : x);
            }
        }
        rank++;
    }
    return rank;
}

/*
 * RREF(M) of a CSR matrix, returned as CSR (rows = rank, sorted by pivot
 * column, columns ascending, no zeros).  Call once with oci == NULL to get
 * the nonzero count and rank (row pointers filled if orp != NULL), then again
 * with buffers.  Returns nnz; *rank_out receives the rank.
 */
uint64_t bf_rref_csr(uint32_t m, uint32_t n, const uint64_t *rp, const uint32_t *ci,
                     const uint16_t *v, uint32_t p, uint32_t *rank_out,
                     uint64_t *orp, uint32_t *oci, uint16_t *ov)
{
    int32_t *W = calloc((uint64_t)m * n + 1, sizeof(int32_t));
    for (uint32_t i = 0; i < m; i++)
        for (uint64_t e = rp[i]; e < rp[i + 1]; e++) W[(uint64_t)i * n + ci[e]] = v[e];
    uint32_t rank = bf_gauss_jordan(m, n, W, p);
    uint64_t nnz = 0;
    if (orp) orp[0] = 0;
    for (uint32_t i = 0; i < rank; i++) {
        for (uint32_t k = 0; k < n; k++) {
            int32_t x = W[(uint64_t)i * n + k];
            if (!x) continue;
            if (oci) { oci[nnz] = k; ov[nnz] = (uint16_t)x; }
            nnz++;
        }
        if (orp) orp[i + 1] = nnz;
    }
    free(W);
    *rank_out = rank;
    return nnz;
}
