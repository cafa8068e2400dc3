/*
 * fl_oracle_wide.c -- the plain CPU reference of the FL reduction for 32-bit
 * field characteristic: coefficients stored as uint32 residues, p prime,
 * 2 <= p < 2^32 (the paper's Sec. 2 lists such a uint32 version beside the
 * uint16 one for p < 2^16).
 *
 * TEST INFRASTRUCTURE ONLY, like fl_oracle.c: only the test suite and the
 * benchmark's CPU baseline load it; it shares no code with the device
 * library.
 *
 * The steps and readings are those of fl_oracle.c (Sec. 3.1 splicing,
 * Sec. 4.1 steps 2-5, the second pass, the read-off); only the arithmetic
 * differs: a product of two residues needs up to 64 bits, so every product
 * is reduced with `%` at once and sums are kept as residues (no delayed
 * reduction at all).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { OW_OK = 0, OW_BAD_P = 1, OW_BAD_ROWPTR = 2, OW_COL_RANGE = 3,
       OW_COL_ORDER = 4, OW_BAD_VALUE = 5 };

/* a * b mod p and a + b mod p for residues a, b < p < 2^32 */
static uint32_t mulm(uint32_t a, uint32_t b, uint32_t p) { return (uint32_t)(((uint64_t)a * b) % p); }
static uint32_t addm(uint32_t a, uint32_t b, uint32_t p) { return (uint32_t)(((uint64_t)a + b) % p); }

/* Modular inverse by the extended Euclidean algorithm (a != 0, p prime). */
uint32_t ow_inv(uint32_t a, uint32_t p)
{
    int64_t t = 0, newt = 1, r = p, newr = a % p;
    while (newr != 0) {
        int64_t q = r / newr, tmp;
        tmp = t - q * newt; t = newt; newt = tmp;
        tmp = r - q * newr; r = newr; newr = tmp;
    }
    if (t < 0) t += p;
    return (uint32_t)t;
}

/* Input checks: columns < n and strictly increasing per row, values in
 * [1, p-1], p >= 2. */
int ow_validate(uint32_t m, uint32_t n, const uint64_t *rp, const uint32_t *ci,
                const uint32_t *v, uint32_t p)
{
    if (p < 2) return OW_BAD_P;
    if (rp[0] != 0) return OW_BAD_ROWPTR;
    for (uint32_t i = 0; i < m; i++) {
        if (rp[i + 1] < rp[i]) return OW_BAD_ROWPTR;
        for (uint64_t k = rp[i]; k < rp[i + 1]; k++) {
            if (ci[k] >= n) return OW_COL_RANGE;
            if (k > rp[i] && ci[k] <= ci[k - 1]) return OW_COL_ORDER;
            if (v[k] == 0 || v[k] >= p) return OW_BAD_VALUE;
        }
    }
    return OW_OK;
}

/* FL step 1, splicing (Sec. 3.1, Sec. 4.1 step 1), with the readings of
 * fl_oracle.c: candidate = first nonzero; pivot row = fewest nonzeros, then
 * lowest index; pivot columns ascending then the others; pivot rows by
 * pivot column, then the others in input order; pivot rows made monic.
 * Returns npiv. */
uint32_t ow_split(uint32_t m, uint32_t n, const uint64_t *rp, const uint32_t *ci,
                  const uint32_t *v, uint32_t p,
                  uint32_t *col_perm, uint32_t *row_perm,
                  uint64_t *Arp, uint32_t *Aci, uint32_t *Av,
                  uint64_t *Brp, uint32_t *Bci, uint32_t *Bv,
                  uint64_t *Crp, uint32_t *Cci, uint32_t *Cv,
                  uint64_t *Drp, uint32_t *Dci, uint32_t *Dv)
{
    int64_t *best = malloc(sizeof(int64_t) * (n ? n : 1));
    uint32_t *newcol = malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t *is_pivrow = calloc(m ? m : 1, 1);
    for (uint32_t c = 0; c < n; c++) best[c] = -1;
    for (uint32_t i = 0; i < m; i++) {
        uint64_t len = rp[i + 1] - rp[i];
        if (len == 0) continue;
        uint32_t lead = ci[rp[i]];
        int64_t b = best[lead];
        if (b < 0 || len < rp[b + 1] - rp[b]) best[lead] = i;
    }
    uint32_t npiv = 0;
    for (uint32_t c = 0; c < n; c++)
        if (best[c] >= 0) npiv++;
    uint32_t kp = 0, kn = npiv;
    for (uint32_t c = 0; c < n; c++) {
        if (best[c] >= 0) { newcol[c] = kp; col_perm[kp++] = c; }
        else              { newcol[c] = kn; col_perm[kn++] = c; }
    }
    uint32_t r = 0;
    for (uint32_t k = 0; k < npiv; k++) {
        uint32_t i = (uint32_t)best[col_perm[k]];
        row_perm[r++] = i;
        is_pivrow[i] = 1;
    }
    for (uint32_t i = 0; i < m; i++)
        if (!is_pivrow[i]) row_perm[r++] = i;
    Arp[0] = Brp[0] = Crp[0] = Drp[0] = 0;
    uint64_t na = 0, nb = 0, nc = 0, nd = 0;
    for (uint32_t k = 0; k < m; k++) {
        uint32_t i = row_perm[k];
        int top = k < npiv;
        uint32_t scale = top ? ow_inv(v[rp[i]], p) : 1;
        for (uint64_t e = rp[i]; e < rp[i + 1]; e++) {
            uint32_t c = newcol[ci[e]];
            uint32_t x = mulm(v[e], scale, p);
            if (top && c < npiv)  { Aci[na] = c;        Av[na++] = x; }
            else if (top)         { Bci[nb] = c - npiv; Bv[nb++] = x; }
            else if (c < npiv)    { Cci[nc] = c;        Cv[nc++] = x; }
            else                  { Dci[nd] = c - npiv; Dv[nd++] = x; }
        }
        if (top) { Arp[k + 1] = na; Brp[k + 1] = nb; }
        else     { Crp[k - npiv + 1] = nc; Drp[k - npiv + 1] = nd; }
    }
    free(best); free(newcol); free(is_pivrow);
    return npiv;
}

/* FL step 2 (Sec. 4.1): X = A^{-1} B by back substitution from the last
 * pivot row up, X_i = B_i - sum_{j > i} A_ij X_j.  Returns 1 if A is not
 * unit upper triangular. */
int ow_trsm(uint32_t npiv, uint32_t nB, const uint64_t *Arp, const uint32_t *Aci,
            const uint32_t *Av, const uint64_t *Brp, const uint32_t *Bci,
            const uint32_t *Bv, uint32_t p, uint32_t *X, uint64_t ldx)
{
    for (int64_t i = (int64_t)npiv - 1; i >= 0; i--) {
        if (Arp[i + 1] == Arp[i] || Aci[Arp[i]] != (uint32_t)i || Av[Arp[i]] != 1) return 1;
        uint32_t *xi = X + (uint64_t)i * ldx;
        for (uint32_t c = 0; c < nB; c++) xi[c] = 0;
        for (uint64_t e = Brp[i]; e < Brp[i + 1]; e++) xi[Bci[e]] = Bv[e];
        for (uint64_t e = Arp[i] + 1; e < Arp[i + 1]; e++) {
            uint32_t lam = p - Av[e];           /* subtract A_ij X_j */
            const uint32_t *xj = X + (uint64_t)Aci[e] * ldx;
            for (uint32_t c = 0; c < nB; c++) xi[c] = addm(xi[c], mulm(lam, xj[c], p), p);
        }
    }
    return 0;
}

/* FL step 3 (Sec. 4.1): Dt = D - C X, dense mD x nB.  Rows independent. */
void ow_reduce(uint32_t mD, uint32_t nB, const uint64_t *Crp, const uint32_t *Cci,
               const uint32_t *Cv, const uint64_t *Drp, const uint32_t *Dci,
               const uint32_t *Dv, const uint32_t *X, uint64_t ldx, uint32_t p,
               uint32_t *Dt, uint64_t ldd)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)mD; i++) {
        uint32_t *di = Dt + (uint64_t)i * ldd;
        for (uint32_t c = 0; c < nB; c++) di[c] = 0;
        for (uint64_t e = Drp[i]; e < Drp[i + 1]; e++) di[Dci[e]] = Dv[e];
        for (uint64_t e = Crp[i]; e < Crp[i + 1]; e++) {
            uint32_t lam = p - Cv[e];
            const uint32_t *xj = X + (uint64_t)Cci[e] * ldx;
            for (uint32_t c = 0; c < nB; c++) di[c] = addm(di[c], mulm(lam, xj[c], p), p);
        }
    }
}

/* FL step 4, read as the reduced row echelon form of the dense Schur
 * complement: textbook Gauss-Jordan (first remaining nonzero row of each
 * column is the pivot, made monic, eliminated from every other row).  In
 * place; returns the rank, pivot columns in pivcols. */
uint32_t ow_rref_dense(uint32_t rows, uint32_t cols, uint32_t *R, uint64_t ld,
                       uint32_t p, uint32_t *pivcols)
{
    uint32_t rank = 0;
    for (uint32_t c = 0; c < cols && rank < rows; c++) {
        uint32_t piv = rows;
        for (uint32_t i = rank; i < rows; i++)
            if (R[(uint64_t)i * ld + c]) { piv = i; break; }
        if (piv == rows) continue;
        uint32_t *pr = R + (uint64_t)piv * ld, *rr = R + (uint64_t)rank * ld;
        if (piv != rank)
            for (uint32_t k = 0; k < cols; k++) { uint32_t t = pr[k]; pr[k] = rr[k]; rr[k] = t; }
        uint32_t inv = ow_inv(rr[c], p);
        for (uint32_t k = c; k < cols; k++) rr[k] = mulm(rr[k], inv, p);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)rows; i++) {
            uint32_t *ri = R + (uint64_t)i * ld;
            if ((uint32_t)i == rank || ri[c] == 0) continue;
            uint32_t lam = p - ri[c];
            for (uint32_t k = c; k < cols; k++) ri[k] = addm(ri[k], mulm(lam, rr[k], p), p);
        }
        pivcols[rank++] = c;
    }
    return rank;
}

/* The second FL pass (end of Sec. 4.1): X'_i = X_i - sum_t X_i[P_D[t]] D'_t,
 * in place on X. */
void ow_second_pass(uint32_t npiv, uint32_t nB, uint32_t *X, uint64_t ldx,
                    uint32_t r, const uint32_t *RD, uint64_t ldr,
                    const uint32_t *pivcols, uint32_t p)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)npiv; i++) {
        uint32_t *xi = X + (uint64_t)i * ldx;
        uint32_t *lam = malloc(sizeof(uint32_t) * (r ? r : 1));
        for (uint32_t t = 0; t < r; t++) lam[t] = xi[pivcols[t]];
        for (uint32_t t = 0; t < r; t++) {
            if (lam[t] == 0) continue;
            uint32_t l = p - lam[t];
            const uint32_t *rt = RD + (uint64_t)t * ldr;
            for (uint32_t c = 0; c < nB; c++) xi[c] = addm(xi[c], mulm(l, rt[c], p), p);
        }
        free(lam);
    }
}

/* FL step 5 (Sec. 4.1): the reduced form [Id X'; 0 D'] read off in original
 * column order as CSR, rows sorted by pivot column, columns ascending, no
 * zeros.  Call with NULL outputs for the nonzero count (returned). */
uint64_t ow_assemble(uint32_t n, uint32_t npiv, uint32_t nB, const uint32_t *col_perm,
                     const uint32_t *X, uint64_t ldx, uint32_t r, const uint32_t *RD,
                     uint64_t ldr, const uint32_t *pivcols,
                     uint64_t *orp, uint32_t *oci, uint32_t *ov)
{
    uint32_t total = npiv + r, a = 0, b = 0;
    uint64_t nnz = 0;
    (void)n;
    if (orp) orp[0] = 0;
    for (uint32_t row = 0; row < total; row++) {
        int take_top;
        if (a == npiv) take_top = 0;
        else if (b == r) take_top = 1;
        else take_top = col_perm[a] < col_perm[npiv + pivcols[b]];
        const uint32_t *src = take_top ? X + (uint64_t)a * ldx : RD + (uint64_t)b * ldr;
        uint64_t start = nnz;
        if (take_top) {
            if (oci) { oci[nnz] = col_perm[a]; ov[nnz] = 1; }
            nnz++;
        }
        for (uint32_t c = 0; c < nB; c++) {
            if (!src[c]) continue;
            if (oci) { oci[nnz] = col_perm[npiv + c]; ov[nnz] = src[c]; }
            nnz++;
        }
        if (oci)  /* keep the row sorted by original column */
            for (uint64_t k = start + 1; k < nnz; k++) {
                uint32_t cc = oci[k], vv = ov[k];
                uint64_t j = k;
                while (j > start && oci[j - 1] > cc) { oci[j] = oci[j - 1]; ov[j] = ov[j - 1]; j--; }
                oci[j] = cc; ov[j] = vv;
            }
        if (take_top) a++; else b++;
        if (orp) orp[row + 1] = nnz;
    }
    return nnz;
}
