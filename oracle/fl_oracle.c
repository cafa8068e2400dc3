/*
 * fl_oracle.c -- plain, slow, obviously correct CPU reference of the
 * Faugere-Lachartre (FL) reduction over F_p, as the GBLA paper frames it
 * (Boyer, Eder, Faugere, Lachartre, Martani, arXiv 1602.06097).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code, header
 * or table with the device library and includes none of its files.
 *
 * Arithmetic: canonical residues in [0, p), p prime, 2 <= p <= 65521.  Sums
 * are accumulated exactly in uint64_t and reduced with `%`; subtraction of
 * lambda*r is done as adding (p - lambda)*r.  No Barrett reduction, no limbs,
 * no multilines in the arithmetic -- those are device-side design choices.
 *
 * Every function cites the passage of the paper it follows.  Where the paper
 * is silent or garbled the reading used is stated next to the code.
 *
 * Matrices: CSR with uint64 row pointers, uint32 column indices (strictly
 * increasing in each row) and uint16 values; dense matrices row-major uint16.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Error codes of or_validate (the test suite maps them to the library's). */
enum { OR_OK = 0, OR_BAD_P = 1, OR_BAD_ROWPTR = 2, OR_COL_RANGE = 3,
       OR_COL_ORDER = 4, OR_BAD_VALUE = 5 };

/* Modular inverse by the extended Euclidean algorithm (a != 0, p prime). */
uint32_t or_inv(uint32_t a, uint32_t p)
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

/*
 * Input checks (Sec. 3.2: Format 1 is CSR; Sec. 2: coefficients are uint16
 * residues for p < 2^16).  Columns must be < n and strictly increasing within
 * a row; values must lie in [1, p-1] (explicit zeros are rejected).
 */
int or_validate(uint32_t m, uint32_t n, const uint64_t *rp, const uint32_t *ci,
                const uint16_t *v, uint32_t p)
{
    if (p < 2 || p > 65521) return OR_BAD_P;
    if (rp[0] != 0) return OR_BAD_ROWPTR;
    for (uint32_t i = 0; i < m; i++) {
        if (rp[i + 1] < rp[i]) return OR_BAD_ROWPTR;
        for (uint64_t k = rp[i]; k < rp[i + 1]; k++) {
            if (ci[k] >= n) return OR_COL_RANGE;
            if (k > rp[i] && ci[k] <= ci[k - 1]) return OR_COL_ORDER;
            if (v[k] == 0 || v[k] >= p) return OR_BAD_VALUE;
        }
    }
    return OR_OK;
}

/*
 * FL step 1, splicing (Sec. 3.1 and Sec. 4.1 step 1, Table "fl-splices").
 *
 * Readings:
 *  - the pivoting candidate of a row is its first nonzero entry; a column is
 *    a pivot column iff it holds the pivoting candidate of some row;
 *  - among the candidates of one column the pivot row is the row with the
 *    fewest nonzeros ("keep A as sparse as possible"), ties broken by the
 *    lower input row index;
 *  - new column order: pivot columns ascending, then the other columns
 *    ascending (so A is upper triangular); new row order: pivot rows by their
 *    pivot column, then the other rows in input order (empty rows included);
 *  - pivot rows are made monic (multiplied by the inverse of their leading
 *    coefficient); the other rows are left untouched.
 *
 * Outputs (caller-allocated, upper bounds m+1 / nnz):
 *   col_perm[n]: new column position -> original column;
 *   row_perm[m]: new row position    -> original row;
 *   A (npiv x npiv, incl. its unit diagonal), B (npiv x nB), C (mD x npiv),
 *   D (mD x nB) in CSR over the new column indices (B, D shifted by npiv).
 * Returns npiv.
 */
uint32_t or_split(uint32_t m, uint32_t n, const uint64_t *rp, const uint32_t *ci,
                  const uint16_t *v, uint32_t p,
                  uint32_t *col_perm, uint32_t *row_perm,
                  uint64_t *Arp, uint32_t *Aci, uint16_t *Av,
                  uint64_t *Brp, uint32_t *Bci, uint16_t *Bv,
                  uint64_t *Crp, uint32_t *Cci, uint16_t *Cv,
                  uint64_t *Drp, uint32_t *Dci, uint16_t *Dv)
{
    int64_t *best = malloc(sizeof(int64_t) * (n ? n : 1));
    uint32_t *newcol = malloc(sizeof(uint32_t) * (n ? n : 1));
    uint8_t *is_pivrow = calloc(m ? m : 1, 1);
    for (uint32_t c = 0; c < n; c++) best[c] = -1;

    /* pivot row of each pivot column: fewest nonzeros, then lowest index */
    for (uint32_t i = 0; i < m; i++) {
        uint64_t len = rp[i + 1] - rp[i];
        if (len == 0) continue;
        uint32_t lead = ci[rp[i]];
        int64_t b = best[lead];
        if (b < 0 || len < rp[b + 1] - rp[b]) best[lead] = i;
    }

    /* column permutation: pivot columns first, both classes ascending */
    uint32_t npiv = 0;
    for (uint32_t c = 0; c < n; c++)
        if (best[c] >= 0) npiv++;
    uint32_t kp = 0, kn = npiv;
    for (uint32_t c = 0; c < n; c++) {
        if (best[c] >= 0) { newcol[c] = kp; col_perm[kp++] = c; }
        else              { newcol[c] = kn; col_perm[kn++] = c; }
    }

    /* row permutation: pivot rows by pivot column, then the rest in order */
    uint32_t r = 0;
    for (uint32_t k = 0; k < npiv; k++) {
        uint32_t i = (uint32_t)best[col_perm[k]];
        row_perm[r++] = i;
        is_pivrow[i] = 1;
    }
    for (uint32_t i = 0; i < m; i++)
        if (!is_pivrow[i]) row_perm[r++] = i;

    /* scatter into A|B (pivot rows, made monic) and C|D (other rows) */
    Arp[0] = Brp[0] = Crp[0] = Drp[0] = 0;
    uint64_t na = 0, nb = 0, nc = 0, nd = 0;
    for (uint32_t k = 0; k < m; k++) {
        uint32_t i = row_perm[k];
        int top = k < npiv;
        uint32_t scale = 1;
        if (top) scale = or_inv(v[rp[i]], p);
        for (uint64_t e = rp[i]; e < rp[i + 1]; e++) {
            uint32_t c = newcol[ci[e]];
            uint16_t x = (uint16_t)(((uint64_t)v[e] * scale) % p);
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

/*
 * n-multiline vectors (Sec. 4.2, the multiline Definition and its worked
 * Example).  Rows g*w .. g*w+w-1 of a CSR matrix form group g; `pos` lists,
 * ascending, every column where at least one of the w rows is nonzero, and
 * `val` stores the w entries of each such column consecutively (zeros
 * allowed).  Rows past the end of the matrix count as empty.
 * Outputs: gptr[ngroups+1] (offsets into pos; val offsets are w times these).
 */
void or_multiline(uint32_t rows, uint32_t cols, const uint64_t *rp,
                  const uint32_t *ci, const uint16_t *v, uint32_t w,
                  uint64_t *gptr, uint32_t *pos, uint16_t *val)
{
    uint32_t ngroups = (rows + w - 1) / w;
    int64_t *slot = malloc(sizeof(int64_t) * (cols ? cols : 1));
    for (uint32_t c = 0; c < cols; c++) slot[c] = -1;
    uint64_t len = 0;
    gptr[0] = 0;
    for (uint32_t g = 0; g < ngroups; g++) {
        uint32_t r0 = g * w, r1 = r0 + w < rows ? r0 + w : rows;
        /* mark the union of columns, then list it in ascending order */
        uint8_t any = 0;
        for (uint32_t i = r0; i < r1; i++)
            for (uint64_t e = rp[i]; e < rp[i + 1]; e++) { slot[ci[e]] = 0; any = 1; }
        uint64_t start = len;
        if (any)
            for (uint32_t c = 0; c < cols; c++)
                if (slot[c] == 0) { slot[c] = (int64_t)len; pos[len++] = c; }
        for (uint64_t k = start; k < len; k++)
            for (uint32_t q = 0; q < w; q++) val[k * w + q] = 0;
        for (uint32_t i = r0; i < r1; i++)
            for (uint64_t e = rp[i]; e < rp[i + 1]; e++)
                val[(uint64_t)slot[ci[e]] * w + (i - r0)] = v[e];
        for (uint64_t k = start; k < len; k++) slot[pos[k]] = -1;
        gptr[g + 1] = len;
    }
    free(slot);
}

/*
 * FL step 2, TRSM (Sec. 4.1 step 2): X = A^{-1} B with A unit upper
 * triangular, by back substitution from the last pivot row up:
 *   X_i = B_i - sum_{j > i} A_ij X_j.
 * X is dense npiv x nB (row stride ldx).  Returns 0, or 1 if A is not unit
 * upper triangular.
 */
int or_trsm(uint32_t npiv, uint32_t nB, const uint64_t *Arp, const uint32_t *Aci,
            const uint16_t *Av, const uint64_t *Brp, const uint32_t *Bci,
            const uint16_t *Bv, uint32_t p, uint16_t *X, uint64_t ldx)
{
    uint64_t *acc = malloc(sizeof(uint64_t) * (nB ? nB : 1));
    for (int64_t i = (int64_t)npiv - 1; i >= 0; i--) {
        if (Arp[i + 1] == Arp[i] || Aci[Arp[i]] != (uint32_t)i || Av[Arp[i]] != 1) {
            free(acc);
            return 1;
        }
        for (uint32_t c = 0; c < nB; c++) acc[c] = 0;
        for (uint64_t e = Brp[i]; e < Brp[i + 1]; e++) acc[Bci[e]] = Bv[e];
        for (uint64_t e = Arp[i] + 1; e < Arp[i + 1]; e++) {
            uint64_t lam = p - Av[e];           /* subtract A_ij X_j */
            const uint16_t *xj = X + (uint64_t)Aci[e] * ldx;
            for (uint32_t c = 0; c < nB; c++) acc[c] += lam * xj[c];
        }
        uint16_t *xi = X + (uint64_t)i * ldx;
        for (uint32_t c = 0; c < nB; c++) xi[c] = (uint16_t)(acc[c] % p);
    }
    free(acc);
    return 0;
}

/*
 * FL step 3, AXPY (Sec. 4.1 step 3): reduce C to zero with Id and apply the
 * same operations to D:  Dt = D - C X  with X = A^{-1} B.  Dense output
 * mD x nB (row stride ldd).  Rows are independent.
 */
void or_reduce(uint32_t mD, uint32_t nB, const uint64_t *Crp, const uint32_t *Cci,
               const uint16_t *Cv, const uint64_t *Drp, const uint32_t *Dci,
               const uint16_t *Dv, const uint16_t *X, uint64_t ldx, uint32_t p,
               uint16_t *Dt, uint64_t ldd)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)mD; i++) {
        uint64_t *acc = malloc(sizeof(uint64_t) * (nB ? nB : 1));
        for (uint32_t c = 0; c < nB; c++) acc[c] = 0;
        for (uint64_t e = Drp[i]; e < Drp[i + 1]; e++) acc[Dci[e]] = Dv[e];
        for (uint64_t e = Crp[i]; e < Crp[i + 1]; e++) {
            uint64_t lam = p - Cv[e];
            const uint16_t *xj = X + (uint64_t)Cci[e] * ldx;
            for (uint32_t c = 0; c < nB; c++) acc[c] += lam * xj[c];
        }
        for (uint32_t c = 0; c < nB; c++) Dt[(uint64_t)i * ldd + c] = (uint16_t)(acc[c] % p);
        free(acc);
    }
}

/*
 * The "new order of operations" (Sec. 4.3, the algorithm "Reduction of C and
 * D"): for each row of C/D, walk the columns of C left to right and, whenever
 * the (already partly reduced) dense C row is nonzero at column j, subtract
 * lambda times row j of A from the C row and lambda times row j of B from the
 * D row.  No TRSM is needed; the result equals D - C A^{-1} B.  The AXPY of
 * the paper is read as d <- d - lambda*r.
 */
void or_reduce_neworder(uint32_t npiv, uint32_t mD, uint32_t nB,
                        const uint64_t *Arp, const uint32_t *Aci, const uint16_t *Av,
                        const uint64_t *Brp, const uint32_t *Bci, const uint16_t *Bv,
                        const uint64_t *Crp, const uint32_t *Cci, const uint16_t *Cv,
                        const uint64_t *Drp, const uint32_t *Dci, const uint16_t *Dv,
                        uint32_t p, uint16_t *Dt, uint64_t ldd)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < (int64_t)mD; i++) {
        uint32_t *dc = calloc(npiv ? npiv : 1, sizeof(uint32_t));
        uint32_t *dd = calloc(nB ? nB : 1, sizeof(uint32_t));
        for (uint64_t e = Crp[i]; e < Crp[i + 1]; e++) dc[Cci[e]] = Cv[e];
        for (uint64_t e = Drp[i]; e < Drp[i + 1]; e++) dd[Dci[e]] = Dv[e];
        for (uint32_t j = 0; j < npiv; j++) {
            if (dc[j] == 0) continue;
            uint64_t lam = p - dc[j];
            for (uint64_t e = Arp[j]; e < Arp[j + 1]; e++)
                dc[Aci[e]] = (uint32_t)((dc[Aci[e]] + lam * Av[e]) % p);
            for (uint64_t e = Brp[j]; e < Brp[j + 1]; e++)
                dd[Bci[e]] = (uint32_t)((dd[Bci[e]] + lam * Bv[e]) % p);
        }
        for (uint32_t c = 0; c < nB; c++) Dt[(uint64_t)i * ldd + c] = (uint16_t)dd[c];
        free(dc); free(dd);
    }
}

/*
 * FL step 4 (Sec. 4.1 step 4), read as the reduced row echelon form of the
 * dense Schur complement: textbook Gauss-Jordan, columns left to right; the
 * first remaining row with a nonzero entry becomes the pivot row, is made
 * monic and is eliminated from every other row.  In place: rows 0..rank-1
 * hold RREF(R) (pivots ascending), the remaining rows are zero.
 * pivcols[0..rank) receives the pivot columns.  Returns the rank.
 */
uint32_t or_rref_dense(uint32_t rows, uint32_t cols, uint16_t *R, uint64_t ld,
                       uint32_t p, uint32_t *pivcols)
{
    uint32_t rank = 0;
    for (uint32_t c = 0; c < cols && rank < rows; c++) {
        uint32_t piv = rows;
        for (uint32_t i = rank; i < rows; i++)
            if (R[(uint64_t)i * ld + c]) { piv = i; break; }
        if (piv == rows) continue;
        uint16_t *pr = R + (uint64_t)piv * ld, *rr = R + (uint64_t)rank * ld;
        if (piv != rank)
            for (uint32_t k = 0; k < cols; k++) { uint16_t t = pr[k]; pr[k] = rr[k]; rr[k] = t; }
        uint64_t inv = or_inv(rr[c], p);
        for (uint32_t k = c; k < cols; k++) rr[k] = (uint16_t)((rr[k] * inv) % p);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < (int64_t)rows; i++) {
            uint16_t *ri = R + (uint64_t)i * ld;
            if ((uint32_t)i == rank || ri[c] == 0) continue;
            uint64_t lam = p - ri[c];
            for (uint32_t k = c; k < cols; k++) ri[k] = (uint16_t)((ri[k] + lam * rr[k]) % p);
        }
        pivcols[rank++] = c;
    }
    return rank;
}

/*
 * Second FL pass towards the reduced form (end of Sec. 4.1: run the
 * reduction again on the right part [A^{-1}B ; D']).  With D' = RREF(Dt) of
 * rank r and pivot columns P_D, every row of X = A^{-1}B is reduced by the
 * rows of D':   X'_i = X_i - sum_t X_i[P_D[t]] * D'_t.
 * In place on X (npiv x nB); D' rows 0..r-1 of RD (stride ldr).
 */
void or_second_pass(uint32_t npiv, uint32_t nB, uint16_t *X, uint64_t ldx,
                    uint32_t r, const uint16_t *RD, uint64_t ldr,
                    const uint32_t *pivcols, uint32_t p)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < (int64_t)npiv; i++) {
        uint16_t *xi = X + (uint64_t)i * ldx;
        uint64_t *acc = malloc(sizeof(uint64_t) * (nB ? nB : 1));
        uint32_t *lam = malloc(sizeof(uint32_t) * (r ? r : 1));
        for (uint32_t c = 0; c < nB; c++) acc[c] = xi[c];
        for (uint32_t t = 0; t < r; t++) lam[t] = xi[pivcols[t]];
        for (uint32_t t = 0; t < r; t++) {
            if (lam[t] == 0) continue;
            uint64_t l = p - lam[t];
            const uint16_t *rt = RD + (uint64_t)t * ldr;
            for (uint32_t c = 0; c < nB; c++) acc[c] += l * rt[c];
        }
        for (uint32_t c = 0; c < nB; c++) xi[c] = (uint16_t)(acc[c] % p);
        free(acc); free(lam);
    }
}

/*
 * FL step 5 (Sec. 4.1 step 5): undo the column permutation and read off the
 * result.  The reduced form in permuted columns is
 *     [ Id  X' ]   (npiv rows, pivot k at permuted column k)
 *     [ 0   D' ]   (r rows, pivot P_D[t] at permuted column npiv + P_D[t])
 * Output: CSR in original column order, rows sorted by their pivot column,
 * columns ascending, no zero entries.  Sizes: call with out pointers NULL to
 * get the nonzero count (returned), then again to fill.
 */
uint64_t or_assemble(uint32_t n, uint32_t npiv, uint32_t nB, const uint32_t *col_perm,
                     const uint16_t *X, uint64_t ldx, uint32_t r, const uint16_t *RD,
                     uint64_t ldr, const uint32_t *pivcols,
                     uint64_t *orp, uint32_t *oci, uint16_t *ov)
{
    /* merge the two pivot lists by original column */
    uint32_t total = npiv + r, a = 0, b = 0;
    uint64_t nnz = 0;
    if (orp) orp[0] = 0;
    for (uint32_t row = 0; row < total; row++) {
        int take_top;
        if (a == npiv) take_top = 0;
        else if (b == r) take_top = 1;
        else take_top = col_perm[a] < col_perm[npiv + pivcols[b]];
        /* gather (original column, value) pairs; both parts are ascending in
         * original order because col_perm is ascending on each class */
        uint32_t first = take_top ? col_perm[a] : 0;
        const uint16_t *src = take_top ? X + (uint64_t)a * ldx : RD + (uint64_t)b * ldr;
        uint64_t start = nnz;
        if (take_top) {
            if (oci) { oci[nnz] = first; ov[nnz] = 1; }
            nnz++;
        }
        for (uint32_t c = 0; c < nB; c++) {
            if (!src[c]) continue;
            if (oci) { oci[nnz] = col_perm[npiv + c]; ov[nnz] = src[c]; }
            nnz++;
        }
        /* the unit of a top row may not be first in original order only if
         * X' had an entry left of it; keep the row sorted in every case */
        if (oci)
            for (uint64_t k = start + 1; k < nnz; k++) {
                uint32_t cc = oci[k]; uint16_t vv = ov[k]; uint64_t j = k;
                while (j > start && oci[j - 1] > cc) { oci[j] = oci[j - 1]; ov[j] = ov[j - 1]; j--; }
                oci[j] = cc; ov[j] = vv;
            }
        if (take_top) a++; else b++;
        if (orp) orp[row + 1] = nnz;
    }
    return nnz;
}
