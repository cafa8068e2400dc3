/*
 * fl.h -- C ABI of the MI355X (gfx950) Faugere-Lachartre reduction library.
 *
 * The library implements the FL reduction of a sparse matrix M over F_p,
 * p prime, 2 <= p <= 65521, stored as uint16 residues, following the GBLA
 * paper (Boyer, Eder, Faugere, Lachartre, Martani, arXiv 1602.06097),
 * Sec. 4.1 ("The reduction by Faugere and Lachartre"):
 *
 *   step 1  fl_split      splice M into [A B; C D] by pivot columns
 *   step 2  fl_trsm       X = A^{-1} B                      (the TRSM)
 *   step 3  fl_reduce_cd  Dt = D - C X                       (the AXPY step)
 *   step 4  fl_echelon_d  RREF of Dt: rank r, pivot columns P_D
 *   step 5  fl_rref       second pass X' = X - X[:,P_D] RREF(Dt), then
 *                         fl_rref_csr_size / fl_rref_to_csr read off RREF(M)
 *                         in original column order (column rearrangement).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every array argument is a DEVICE pointer, allocated and owned by the
 *    caller; the library allocates no device memory and keeps no pointer
 *    after the enqueued work completes.  Pointers to the fl_split_info and
 *    fl_split_out structs themselves, and h_* arguments, are HOST pointers.
 *  - Work is enqueued on the caller's `stream` (0 = the null stream).  Only
 *    fl_split and fl_rref_csr_size synchronise that stream (once each, to
 *    return sizes to the host).
 *  - Residues are canonical: every value is in [0, p).
 *  - Dense matrices are row-major uint16 with a leading dimension (row
 *    stride, in elements) `ld` that must satisfy ld >= cols and ld % 4 == 0;
 *    base pointers must be 8-byte aligned.  Columns in [cols, ld) are
 *    padding: they are read but never written, and never affect results.
 *  - Workspace: every call that needs scratch memory takes `ws`/`ws_bytes`
 *    (device memory, no alignment beyond 256 bytes required); the matching
 *    fl_*_workspace() function returns the required size.
 *  - Errors: host-checkable problems (NULL pointers, p out of range, bad
 *    dimensions, ld too small or misaligned, ml_width not in {1,2,4,8},
 *    workspace too small) return immediately with nothing enqueued.  Data
 *    errors in M are detected by fl_split's validation pass and reported at
 *    its synchronisation; later calls assume validated, split data.  HIP
 *    runtime failures return FL_ERR_HIP; fl_last_error() then holds the HIP
 *    error string (thread-local).  p must be prime; this is not checked.
 */
#ifndef FL_H
#define FL_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FL_OK = 0,
    FL_ERR_ARG = 1,            /* invalid argument (host-checked)            */
    FL_ERR_WORKSPACE = 2,      /* ws_bytes smaller than fl_*_workspace()     */
    FL_ERR_DATA_ROWPTR = 3,    /* row_ptr[0] != 0, decreasing, or != nnz     */
    FL_ERR_DATA_COL_RANGE = 4, /* a column index >= n                        */
    FL_ERR_DATA_COL_ORDER = 5, /* columns of a row not strictly increasing   */
    FL_ERR_DATA_VALUE = 6,     /* a value == 0 or >= p                       */
    FL_ERR_HIP = 7             /* HIP runtime error, see fl_last_error()     */
} fl_status;

/* Arithmetic form of the dense contractions.  Both give bit-identical
 * results.  FL_PLAIN: 32-bit VALU multiply-adds with delayed reduction.
 * FL_MFMA_I8: centred residues split into two signed 8-bit limbs (one limb,
 * the symmetric residue, for p < 256), products on the int8 matrix cores
 * with exact int32 accumulation, recombined and reduced mod p. */
typedef enum { FL_PLAIN = 0, FL_MFMA_I8 = 1 } fl_mode;

/* Sparse input (Sec. 3.2, Format 1 is this CSR layout).  Device pointers. */
typedef struct {
    uint32_t rows, cols;
    uint64_t nnz;
    const uint64_t *row_ptr; /* [rows + 1], row_ptr[0] = 0, row_ptr[rows] = nnz */
    const uint32_t *col;     /* [nnz], strictly increasing within each row       */
    const uint16_t *val;     /* [nnz], in [1, p-1]                               */
} fl_csr;

/*
 * Outputs of fl_split (device buffers, caller-allocated with the capacities
 * given, which depend only on m, n, nnz(M) and ml_width w -- the pivot count
 * is not known in advance).
 *
 * A and C are stored as w-multiline vectors (Sec. 4.2, the multiline
 * Definition): rows are grouped w at a time (group g = rows g*w .. g*w+w-1);
 * pos[gptr[g] .. gptr[g+1]) lists, ascending, every column where one of the
 * group's rows is nonzero, and val[w*k + q] is row q's entry at pos[k]
 * (zero allowed).  A holds only the strictly upper part of the unit upper
 * triangular npiv x npiv block (its unit diagonal is implicit).  B and D are
 * CSR.  Column indices of A, C are in [0, npiv); of B, D in [0, n - npiv).
 */
typedef struct {
    uint32_t *row_perm;  /* [m]  new row position -> input row               */
    uint32_t *col_perm;  /* [n]  new column position -> input column         */
    uint64_t *a_gptr;    /* [ceil(m/w) + 1]                                   */
    uint32_t *a_pos;     /* [nnz]                                             */
    uint16_t *a_val;     /* [w * nnz]                                         */
    uint64_t *b_ptr;     /* [m + 1]                                           */
    uint32_t *b_col;     /* [nnz]                                             */
    uint16_t *b_val;     /* [nnz]                                             */
    uint64_t *c_gptr;    /* [ceil(m/w) + 1]                                   */
    uint32_t *c_pos;     /* [nnz]                                             */
    uint16_t *c_val;     /* [w * nnz]                                         */
    uint64_t *d_ptr;     /* [m + 1]                                           */
    uint32_t *d_col;     /* [nnz]                                             */
    uint16_t *d_val;     /* [nnz]                                             */
} fl_split_out;

/* Sizes returned by fl_split (host struct). */
typedef struct {
    uint32_t p, m, n, ml_width;
    uint32_t npiv;        /* number of pivot columns = rows of A and B        */
    uint32_t nB;          /* n - npiv                                          */
    uint32_t mD;          /* m - npiv                                          */
    uint32_t status;      /* fl_status of the validation pass                  */
    uint64_t nnz;         /* nnz(M)                                            */
    uint64_t nnzA;        /* strictly upper entries of A                       */
    uint64_t nnzB, nnzC, nnzD;
    uint64_t lenA, lenC;  /* multiline lengths: gptr[last] of A and C          */
} fl_split_info;

/* ---- step 1 --------------------------------------------------------------
 * fl_split -- Sec. 3.1 (pivoting candidates, pivot columns, pivot-row
 * selection keeping A sparse) and Sec. 4.1 step 1 (the splice [A B; C D]).
 *   - validates M (columns < n and strictly increasing, values in [1, p-1],
 *     row_ptr monotone from 0 to nnz);
 *   - the pivoting candidate of a row is its first entry; pivot columns are
 *     the columns holding a candidate;
 *   - pivot row of a pivot column: the candidate row with the fewest
 *     nonzeros, ties to the lowest input row index;
 *   - column order: pivot columns ascending, then the others ascending;
 *     row order: pivot rows by pivot column, then the other rows (including
 *     empty rows) in input order;
 *   - pivot rows are scaled by the inverse of their leading coefficient
 *     (a no-op for monic rows); other rows are copied unchanged.
 * ml_width w in {1, 2, 4, 8} is the multiline width of A and C.
 * Synchronises `stream` once and fills *h_info.  Returns the validation
 * status (FL_ERR_DATA_*) if M is malformed; outputs are then undefined. */
fl_status fl_split(const fl_csr *M, uint32_t p, uint32_t ml_width, const fl_split_out *out,
                   fl_split_info *h_info, void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_split_workspace(uint32_t m, uint32_t n, uint64_t nnz, uint32_t ml_width);

/* ---- step 2 --------------------------------------------------------------
 * fl_trsm -- Sec. 4.1 step 2: X = A^{-1} B mod p, A unit upper triangular,
 * by back substitution over blocks of 128 rows from the bottom up, using the
 * multiline rows of A (Sec. 4.2: one read of a row of X serves the w rows of
 * a multiline).  X: dense npiv x nB (ld = ldx).  B is read from s->b_*.
 * FL_PLAIN: the part of each block's rows that refers to finished rows below
 * the block is applied by the multiline sparse-times-dense kernel on the
 * vector ALUs, and each block is solved by a back substitution on the vector
 * ALUs.  FL_MFMA_I8: A's band is expanded into dense int8 limb planes in the
 * workspace; the part beyond each superblock of four blocks is applied by
 * limb GEMMs on the matrix cores (the columns of the superblock below it on
 * `stream`, the columns past those one superblock earlier on a second stream
 * of the library's that `stream` then waits for), the part inside it by a
 * rank-k product per block, and each block is solved as a product with its
 * (precomputed) inverse.  Both forms give the same, unique X; all work is
 * ordered before later work on `stream`. */
fl_status fl_trsm(const fl_split_info *info, const fl_split_out *s, uint16_t *X, uint64_t ldx,
                  fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_trsm_workspace(const fl_split_info *info, fl_mode mode);

/* fl_trsm_planes -- where an FL_MFMA_I8 fl_trsm leaves the int8 limb planes
 * of X in its workspace ws (ws_bytes >= fl_trsm_workspace(info, FL_MFMA_I8)):
 * the centred residue of X[k][c] (X[k][c], or X[k][c] - p above 32639;
 * for p < 256 above (p - 1) / 2, with Xh zero) is
 * 256 Xh[c * ldp + k] + Xl[c * ldp + k] (the limb form of the matrix-core
 * products), for k < npiv, c < nB; the planes hold round_up(nB, 128) columns.  Pointers into ws, no copy; their
 * contents are those of the last fl_trsm that used ws in the FL_MFMA_I8 form
 * and stay valid until ws is reused.  *row_end (may be NULL) receives, per
 * 128-column tile j of X, 1 + the last row of X with a nonzero in columns
 * [128 j, 128 j + 128) (0: none), device u32[round_up(nB, 128) / 128].
 * Errors: FL_ERR_ARG for NULL arguments, npiv or nB of 0, or a workspace
 * that is too small. */
fl_status fl_trsm_planes(const fl_split_info *info, const void *ws, size_t ws_bytes, const int8_t **Xh,
                         const int8_t **Xl, uint64_t *ldp, const uint32_t **row_end);

/* ---- step 3 --------------------------------------------------------------
 * fl_reduce_cd -- Sec. 4.1 step 3: Dt = D - C X mod p (C reduced to zero by
 * the identity, the same operations applied to D).  Dt: dense mD x nB
 * (ld = ldd).  FL_PLAIN multiplies the sparse multiline rows of C; FL_MFMA_I8
 * multiplies C as a dense int8-limb operand on the matrix cores. */
fl_status fl_reduce_cd(const fl_split_info *info, const fl_split_out *s, const uint16_t *X,
                       uint64_t ldx, uint16_t *Dt, uint64_t ldd, fl_mode mode, void *ws,
                       size_t ws_bytes, hipStream_t stream);
size_t fl_reduce_cd_workspace(const fl_split_info *info, fl_mode mode);

/* fl_reduce_cd_planes -- fl_reduce_cd in the FL_MFMA_I8 form with X given by
 * its int8 limb planes (as fl_trsm_planes returns them: column c of X at
 * Xh/Xl + c * ldp, round_up(nB, 128) columns, ldp >= round_up(npiv, 64),
 * ldp a multiple of 16, both planes 16-byte aligned), so that X is not
 * converted again; the planes are only read.  Same Dt as fl_reduce_cd, bit
 * for bit.  Workspace: fl_reduce_cd_planes_workspace(info) bytes (smaller
 * than fl_reduce_cd's: no planes of X).  row_end (device, may be NULL): per
 * 128-column tile of X an upper bound on 1 + its last row with a nonzero
 * there, as fl_trsm_planes returns it; the product skips the rows past it.
 * Errors as fl_reduce_cd. */
fl_status fl_reduce_cd_planes(const fl_split_info *info, const fl_split_out *s, const int8_t *Xh,
                              const int8_t *Xl, uint64_t ldp, const uint32_t *row_end, uint16_t *Dt,
                              uint64_t ldd, void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_reduce_cd_planes_workspace(const fl_split_info *info);

/* ---- step 4 --------------------------------------------------------------
 * fl_echelon_d -- Sec. 4.1 step 4 / Sec. 4.4, read as the REDUCED row
 * echelon form of the dense rows x cols matrix Dt, in place: on return rows
 * 0..r-1 hold RREF(Dt) with pivot columns ascending, rows r.. are zero,
 * *d_rank = r and d_pivcol[0..r) the pivot columns (device outputs;
 * d_pivcol capacity min(rows, cols)).  Blocked Gauss-Jordan over column
 * panels: pivot search in the panel, then a rank-k update of all other rows. */
fl_status fl_echelon_d(uint32_t p, uint32_t rows, uint32_t cols, uint16_t *Dt, uint64_t ldd,
                       uint32_t *d_rank, uint32_t *d_pivcol, fl_mode mode, void *ws,
                       size_t ws_bytes, hipStream_t stream);
size_t fl_echelon_d_workspace(uint32_t rows, uint32_t cols, fl_mode mode);

/* ---- step 5 --------------------------------------------------------------
 * fl_rref -- end of Sec. 4.1: the FL reduction run a second time on the
 * right part [A^{-1}B ; D'], which for D' = RREF(Dt) amounts to
 *     X' = X - X[:, P_D] * RREF(Dt)   (in place on X; X'[:, P_D] = 0).
 * Then [Id X'; 0 RREF(Dt)] is RREF(M) in the permuted column order.
 * RD: the output of fl_echelon_d (ld = ldd); d_rank/d_pivcol as returned. */
fl_status fl_rref(const fl_split_info *info, const fl_split_out *s, uint16_t *X, uint64_t ldx,
                  const uint16_t *RD, uint64_t ldd, const uint32_t *d_rank,
                  const uint32_t *d_pivcol, fl_mode mode, void *ws, size_t ws_bytes,
                  hipStream_t stream);
size_t fl_rref_workspace(const fl_split_info *info, fl_mode mode);

/* Sec. 4.1 step 5 (column rearrangement and read-off) as canonical CSR of
 * RREF(M) in the ORIGINAL column order: one row per pivot (rank = npiv + r
 * rows), rows sorted by pivot column, columns ascending, no zero entries,
 * leading entry 1.
 * fl_rref_csr_size writes row_ptr[rank + 1] (device, capacity
 * npiv + min(mD, nB) + 1), synchronises `stream` and returns the rank and
 * the nonzero count through h_rank / h_nnz.
 * fl_rref_to_csr then fills col[nnz] and val[nnz] (device) given row_ptr.
 * Xp and RD as fl_rref leaves them: ldx, ldd multiples of 4 and both
 * 8-byte aligned (FL_ERR_ARG otherwise). */
fl_status fl_rref_csr_size(const fl_split_info *info, const fl_split_out *s, const uint16_t *Xp,
                           uint64_t ldx, const uint16_t *RD, uint64_t ldd,
                           const uint32_t *d_rank, const uint32_t *d_pivcol, uint64_t *row_ptr,
                           uint32_t *h_rank, uint64_t *h_nnz, void *ws, size_t ws_bytes,
                           hipStream_t stream);
fl_status fl_rref_to_csr(const fl_split_info *info, const fl_split_out *s, const uint16_t *Xp,
                         uint64_t ldx, const uint16_t *RD, uint64_t ldd, const uint32_t *d_rank,
                         const uint32_t *d_pivcol, const uint64_t *row_ptr, uint32_t *col,
                         uint16_t *val, void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_rref_csr_workspace(const fl_split_info *info);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): fl_rref_csr_size
 * with its count/scan scratch in a static device array of
 * fl_rref_csr_noalloc_scratch_bytes() = 16 MiB per GPU, held until the
 * process ends, instead of a caller workspace.  Same arguments and results
 * as fl_rref_csr_size otherwise.  Allocates nothing (no hipMalloc/hipFree, no
 * allocating library call); the first call on a device looks up the array's
 * device address.  FL_ERR_ARG when npiv + min(mD, nB) + 1 rows need more
 * scratch than that (about 2.09 million rows).  Every call on one GPU uses the
 * same array: calls that overlap on one GPU (different streams or threads)
 * race, and must be ordered by the caller. */
fl_status fl_rref_csr_size_noalloc(const fl_split_info *info, const fl_split_out *s, const uint16_t *Xp,
                                   uint64_t ldx, const uint16_t *RD, uint64_t ldd,
                                   const uint32_t *d_rank, const uint32_t *d_pivcol, uint64_t *row_ptr,
                                   uint32_t *h_rank, uint64_t *h_nnz, hipStream_t stream);
size_t fl_rref_csr_noalloc_scratch_bytes(void);

/* Sec. 4.3 (new order of operations): the same Dt = D - C A^{-1} B as
 * fl_trsm + fl_reduce_cd, without forming X = A^{-1} B -- for callers that
 * need only the echelon form of D and the rank of M.  C is reduced by A
 * (its multipliers C' = C A^{-1} come from the blocked TRSM run on the
 * transpose of A with the columns of C as right-hand sides, pivot order
 * reversed) and Dt = D - C' B.  Dt: dense mD x nB (ld = ldd >= nB, ldd % 4
 * == 0, 8-byte aligned), fully overwritten.  Bit-identical to fl_reduce_cd in
 * both modes.  nnz(A) and nnz(C) must be below 2^31. */
fl_status fl_reduce_neworder(const fl_split_info *info, const fl_split_out *s, uint16_t *Dt,
                             uint64_t ldd, fl_mode mode, void *ws, size_t ws_bytes,
                             hipStream_t stream);
size_t fl_reduce_neworder_workspace(const fl_split_info *info, fl_mode mode);

/* ---- dense contraction ------------------------------------------------------
 * fl_matmul_sub -- the dense form of the step-3 contraction:
 *     Dm = Dm - Cm * Xm mod p,  Cm: M x K (ld ldc), Xm: K x N (ld ldx),
 *     Dm: M x N (ld ldd), all dense uint16 residues, in place on Dm.
 * Used when C is dense; bit-identical in both modes. */
fl_status fl_matmul_sub(uint32_t p, uint32_t M, uint32_t N, uint32_t K, const uint16_t *Cm,
                        uint64_t ldc, const uint16_t *Xm, uint64_t ldx, uint16_t *Dm,
                        uint64_t ldd, fl_mode mode, void *ws, size_t ws_bytes,
                        hipStream_t stream);
size_t fl_matmul_sub_workspace(uint32_t M, uint32_t N, uint32_t K, fl_mode mode);

/* ---- batched form -------------------------------------------------------------
 * An F4 run produces a sequence of matrices of very uneven sizes (Sec. 6.2
 * and its tables); one small matrix cannot fill the GPU, and Sec. 5.2 found
 * the cost of scheduling many small tasks decisive on CPUs.  The batched form
 * reduces `count` independent matrices M_0..M_{count-1} over one F_p:
 *
 *   fl_batch_plan   splits every matrix (fl_split) on `stream`, with ONE host
 *                   synchronisation for the whole batch, and returns a host
 *                   plan object that fixes every size, the arena layout and
 *                   each matrix's arithmetic form;
 *   fl_batch_run    enqueues steps 2-5 of every matrix (fl_trsm ..
 *                   read-off) with no host synchronisation, spread over
 *                   `streams` concurrent branches forked from and joined
 *                   back into `stream`; capturable;
 *   fl_batch_graph_build / fl_batch_graph_launch
 *                   capture fl_batch_run into a hipGraph once and replay it
 *                   (each replay recomputes every result from the split);
 *   fl_batch_autotune
 *                   times candidate configurations (multiline width, branch
 *                   count, MFMA size threshold, work-queue width, far-update
 *                   column groups) on the given batch and remembers the best
 *                   one for batches of the same shape.
 *
 * Memory: the caller allocates two device arenas: the split arena
 * (fl_batch_split_workspace, known from the CSR shapes alone; it holds every
 * matrix's fl_split outputs and must stay alive as long as the plan) and the
 * run arena (fl_batch_run_workspace(plan): dense X and Dt of every matrix,
 * per-branch workspaces, the CSR outputs at their upper bound
 * (npiv + min(mD, nB)) * (nB + 1) entries, and the summary table).  Both are
 * 256-byte aligned device memory.  The plan object itself is host memory
 * owned by the library until fl_batch_free.
 *
 * Results: after the run (or a graph replay) completes, fl_batch_summary's
 * device table holds per matrix {rank of M, nnz of RREF(M), status, 0}
 * (uint64 each), and fl_batch_matrix gives the device pointers of matrix i's
 * CSR of RREF(M) (same canonical form as fl_rref_to_csr).  A matrix whose
 * split found a data error is skipped by the run; its status is the error
 * code and its rank and nnz are 0.  Results are bit-identical to the
 * single-matrix entry points for every configuration. */
typedef struct {
    uint32_t ml_width;         /* 1, 2, 4 or 8; 0 = default (2) */
    uint32_t streams;          /* concurrent branches, 1..16; 0 = default (8) */
    uint64_t mfma_min_entries; /* a matrix runs its dense steps (TRSM band updates,
                                  C X, echelon updates, second pass) on int8 MFMA
                                  when (npiv + mD) * nB >= this; 0 = default (2^22);
                                  UINT64_MAX = always the VALU form */
    uint32_t queue_per_cu;     /* the stepped launches of the TRSM (one per block
                                  step for all matrices) run as persistent
                                  work-queue launches with this many workgroups
                                  per compute unit, which take the step's tiles
                                  of every matrix from an atomic counter;
                                  0 = default (2), FL_BATCH_DIRECT = one
                                  workgroup per tile instead */
    uint32_t far_groups;       /* workgroups along the columns of the echelon
                                  step's far block updates (each walks that
                                  many-th column tile); 0 = default (128) */
} fl_batch_config;
#define FL_BATCH_DIRECT 0xFFFFu

typedef struct fl_batch fl_batch;   /* opaque host object */

typedef struct {
    uint64_t *row_ptr;   /* [rank_max + 1], device */
    uint32_t *col;       /* [nnz_cap], device */
    uint16_t *val;       /* [nnz_cap], device */
    uint64_t nnz_cap;
    uint32_t rank_max;   /* npiv + min(mD, nB) */
    uint32_t npiv, mD, nB;
    fl_mode mode;        /* arithmetic form chosen for this matrix */
    fl_status status;    /* the matrix's split status */
} fl_batch_matrix;

/* Bytes of the split arena for this batch at multiline width ml_width. */
size_t fl_batch_split_workspace(const fl_csr *Ms, uint32_t count, uint32_t ml_width);
/* cfg may be NULL: the configuration fl_batch_autotune found for a batch of
 * this shape, else the defaults.  Errors: FL_ERR_ARG (bad arguments, count
 * 0), FL_ERR_WORKSPACE (split arena too small), FL_ERR_HIP.  Per-matrix data
 * errors do not fail the plan (see fl_batch_matrix.status). */
fl_status fl_batch_plan(const fl_csr *Ms, uint32_t count, uint32_t p, const fl_batch_config *cfg,
                        void *split_arena, size_t split_bytes, fl_batch **plan,
                        hipStream_t stream);
size_t fl_batch_run_workspace(const fl_batch *plan);
fl_status fl_batch_run(fl_batch *plan, void *run_arena, size_t run_bytes, hipStream_t stream);
/* Captures fl_batch_run(plan, run_arena, ...) on `stream` into a graph kept in
 * the plan (replacing an earlier one).  Nothing is executed.  With the null
 * stream (which cannot be captured) the capture uses a stream of the plan,
 * after synchronising the null stream. */
fl_status fl_batch_graph_build(fl_batch *plan, void *run_arena, size_t run_bytes,
                               hipStream_t stream);
fl_status fl_batch_graph_launch(fl_batch *plan, hipStream_t stream);
/* Device pointer of the summary table (count x 4 uint64) in run_arena. */
uint64_t *fl_batch_summary(const fl_batch *plan, void *run_arena);
fl_status fl_batch_matrix_info(const fl_batch *plan, uint32_t i, void *run_arena,
                               fl_batch_matrix *out);
void fl_batch_get_config(const fl_batch *plan, fl_batch_config *out);
/* Runs each candidate (plan + run, eagerly, timed with HIP events after one
 * warm-up) in the given arenas; candidates that do not fit are skipped.
 * Writes the fastest to *best (and its time to *best_ms) and records it for
 * fl_batch_plan(cfg = NULL) on batches of the same shape (count, p, and the
 * rounded log2 of the total nonzeros and of the largest row count).  The
 * split arena must be sized for ml_width 4. */
fl_status fl_batch_autotune(const fl_csr *Ms, uint32_t count, uint32_t p, void *split_arena,
                            size_t split_bytes, void *run_arena, size_t run_bytes,
                            fl_batch_config *best, double *best_ms, hipStream_t stream);
void fl_batch_free(fl_batch *plan);

/* ---- matrix files (Sec. 3.2) ------------------------------------------------------
 * Format 1: m, n, p (u32), nnz (u64), data (u16 x nnz), cols (u32 x nnz), rows
 *   (u32 x m, row lengths) -- CSR with row lengths.
 * Format 2: b (u32: element type of pdata, bit 0 signed, bits 1-2 log2 of the
 *   byte width, higher bits a version), m, n (u32), p, nnz (u64), rows (u32 x m),
 *   polmap (u32 x m), k (u64), colid (u64 x k: a run of s > 1 consecutive
 *   columns from f is the pair f, s; a single column f is f | 2^31), pnb
 *   (u32), pnnz (u64), prow (u32 x pnb, polynomial sizes), pdata (pnnz
 *   elements); row i's coefficients are those of polynomial polmap[i].
 * fl_file_layout_parse reads the header of a file image in HOST memory,
 * checks that the file holds every section and that the sizes agree (row
 * lengths add up to nnz; Format 2: polynomial sizes add up to pnnz, every row
 * names a polynomial of its own length), and returns the byte offset of each
 * section.  Errors: FL_ERR_ARG with a message.
 * fl_file_decode builds the CSR of M on the device from the sections copied
 * to device memory (d_sections: Format 1 {data, cols, rows}, Format 2 {rows,
 * polmap, colid, prow, pdata}).  Format 1: writes row_ptr[m + 1] only (data
 * and cols ARE val and col).  Format 2: writes row_ptr[m + 1], col[nnz],
 * val[nnz] (coefficients reduced mod p).  *d_status (device) receives 0, or a
 * bit mask: 1 a run without its length, 2 runs beyond nnz or n, 4 a row whose
 * polynomial is missing or of another length.  Column order, range and zero
 * values are checked later by fl_split's validation. */
typedef struct {
    uint32_t format;            /* 1 or 2 */
    uint32_t m, n;
    uint64_t p, nnz;
    uint32_t b, elem_bytes, elem_signed, version;   /* Format 2 */
    uint64_t k, pnb, pnnz;                          /* Format 2 */
    uint64_t off_data, off_cols, off_rows;          /* byte offsets in the file */
    uint64_t off_polmap, off_colid, off_prow, off_pdata;
    uint64_t bytes;             /* size implied by the header */
} fl_file_layout;
fl_status fl_file_layout_parse(const void *file, uint64_t bytes, uint32_t format, fl_file_layout *out);
size_t fl_file_decode_workspace(const fl_file_layout *layout);
fl_status fl_file_decode(const fl_file_layout *layout, const void *const *d_sections, uint64_t *row_ptr,
                         uint32_t *col, uint16_t *val, uint32_t *d_status, void *ws, size_t ws_bytes,
                         hipStream_t stream);

/* ==== 32-bit field characteristic ==========================================
 * Sec. 2 lists, beside the uint16 coefficients for p < 2^16, a version for
 * 32-bit field characteristic with uint32 coefficients.  The calls below
 * run the same five steps with the same readings over uint32 residues,
 * p prime, 2 <= p < 2^32 (p's primality is not checked).  Arithmetic:
 * 64-bit products reduced by Barrett (mu = floor((2^64 - 1) / p)), sums of
 * raw products in 64 bits with 2^64 mod p folded back on wrap-around.
 * FL_PLAIN runs every step on the vector ALUs.  FL_MFMA_I8 runs the dense
 * contractions (the reduce with C as a dense operand, the echelon step's
 * rank-k updates, the second pass) on the int8 matrix cores: a residue is
 * centred to r = x (x <= 2139062143) or x - p and written as four balanced
 * signed bytes; the 16 limb products per multiply-add are summed into seven
 * int32 diagonals over K chunks of at most 32,704 terms (4 * 2^14 * K <
 * 2^31), then combined mod p.  The TRSM is the sparse back substitution of
 * Sec. 4.1 step 2 on the vector ALUs in both forms.  Results are
 * bit-identical across forms.  Conventions (device pointers owned by the
 * caller, workspaces, errors, single syncs) are those of the uint16 calls;
 * dense matrices are row-major uint32 with leading dimension >= their
 * column count. */
typedef struct {
    uint32_t rows, cols;
    uint64_t nnz;
    const uint64_t *row_ptr; /* [rows + 1]                                    */
    const uint32_t *col;     /* [nnz], strictly increasing within each row    */
    const uint32_t *val;     /* [nnz], in [1, p-1]                            */
} fl_csr32;

/* fl_split_out with uint32 values (same capacities). */
typedef struct {
    uint32_t *row_perm, *col_perm;
    uint64_t *a_gptr;
    uint32_t *a_pos;
    uint32_t *a_val;     /* [w * nnz] */
    uint64_t *b_ptr;
    uint32_t *b_col;
    uint32_t *b_val;     /* [nnz]     */
    uint64_t *c_gptr;
    uint32_t *c_pos;
    uint32_t *c_val;     /* [w * nnz] */
    uint64_t *d_ptr;
    uint32_t *d_col;
    uint32_t *d_val;     /* [nnz]     */
} fl_split_out32;

/* Step 1 (Sec. 3.1, Sec. 4.1 step 1) over uint32 residues; the layout,
 * rules, workspace (fl_split_workspace) and the single sync are those of
 * fl_split.  FL_ERR_ARG for p < 2. */
fl_status fl_split32(const fl_csr32 *M, uint32_t p, uint32_t ml_width, const fl_split_out32 *out,
                     fl_split_info *h_info, void *ws, size_t ws_bytes, hipStream_t stream);
/* Step 2 (Sec. 4.1): X = A^{-1} B, dense npiv x nB (ldx >= nB), by back
 * substitution over 64-row blocks: the entries of A past a block are
 * applied as one sparse update of the block's rows, then the block is
 * solved row by row. */
fl_status fl_trsm32(const fl_split_info *info, const fl_split_out32 *s, uint32_t *X, uint64_t ldx,
                    fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_trsm32_workspace(const fl_split_info *info, fl_mode mode);
/* Step 3 (Sec. 4.1): Dt = D - C X, dense mD x nB (ldd >= nB). */
fl_status fl_reduce_cd32(const fl_split_info *info, const fl_split_out32 *s, const uint32_t *X, uint64_t ldx,
                         uint32_t *Dt, uint64_t ldd, fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_reduce_cd32_workspace(const fl_split_info *info, fl_mode mode);
/* Step 4 (Sec. 4.1 step 4, Sec. 4.4), read as the reduced row echelon form
 * of the dense rows x cols matrix Dt, in place (rows 0..r-1 = RREF, pivots
 * ascending in d_pivcol, the other rows zero, *d_rank = r): blocked
 * Gauss-Jordan over 64-column panels (pivot search in one workgroup, then
 * a rank-k update of every row, k <= 64). */
fl_status fl_echelon_d32(uint32_t p, uint32_t rows, uint32_t cols, uint32_t *Dt, uint64_t ldd,
                         uint32_t *d_rank, uint32_t *d_pivcol, fl_mode mode, void *ws, size_t ws_bytes,
                         hipStream_t stream);
size_t fl_echelon_d32_workspace(uint32_t rows, uint32_t cols, fl_mode mode);
/* Second pass (end of Sec. 4.1): X <- X - X[:, P_D] R_D in place. */
fl_status fl_rref32(const fl_split_info *info, const fl_split_out32 *s, uint32_t *X, uint64_t ldx,
                    const uint32_t *RD, uint64_t ldd, const uint32_t *d_rank, const uint32_t *d_pivcol,
                    fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_rref32_workspace(const fl_split_info *info, fl_mode mode);
/* Step 5 (Sec. 4.1): the canonical CSR of RREF(M) in the original column
 * order with uint32 values, in two calls as fl_rref_csr_size /
 * fl_rref_to_csr (the first synchronises and returns rank and nonzeros). */
fl_status fl_rref32_csr_size(const fl_split_info *info, const fl_split_out32 *s, const uint32_t *Xp,
                             uint64_t ldx, const uint32_t *RD, uint64_t ldd, const uint32_t *d_rank,
                             const uint32_t *d_pivcol, uint64_t *row_ptr, uint32_t *h_rank, uint64_t *h_nnz,
                             void *ws, size_t ws_bytes, hipStream_t stream);
fl_status fl_rref32_to_csr(const fl_split_info *info, const fl_split_out32 *s, const uint32_t *Xp,
                           uint64_t ldx, const uint32_t *RD, uint64_t ldd, const uint32_t *d_rank,
                           const uint32_t *d_pivcol, const uint64_t *row_ptr, uint32_t *col, uint32_t *val,
                           void *ws, size_t ws_bytes, hipStream_t stream);
size_t fl_rref32_csr_workspace(const fl_split_info *info);

/* ---- helpers ----------------------------------------------------------------- */
const char *fl_status_string(fl_status s);
const char *fl_last_error(void);   /* thread-local; "" if none */
/* Version string of the device library ("fl-gfx950 <semver>"). */
const char *fl_version(void);

/* Device self-check of the modular reductions used by the kernels: for each
 * prime in p_list and every x in [0, 2^32), compares the 32-bit reduction of
 * x with x % p, the fold of an accumulator pair (256 x + y, y = x times an
 * odd constant mod 2^32) with 64-bit division, the product of the
 * residues (x mod 2^16) mod p and (x >> 16) mod p, and the recombination of
 * the three int32 limb sums of the int8 MFMA contractions (65536 S_hh +
 * 256 S_mid + S_ll mod p) on a 2^32-point grid over the whole range those
 * sums can take, its corners included; returns the number of mismatches
 * through d_mismatch (device, one uint64 per prime).
 * Diagnostic only. */
fl_status fl_check_modp(const uint32_t *h_p_list, uint32_t count, uint64_t *d_mismatch,
                        hipStream_t stream);

/* Launch profiler (diagnostic).  While enabled, the library records HIP
 * events on the launch stream around its hot kernels (the multiline SpMM, the
 * TRSM block solve, the dense GEMMs, the echelon panel kernels);
 * fl_prof_report waits for them and writes a JSON object
 * {"<site>": {"count": N, "total_ms": T}, ...} into buf (at most len bytes,
 * NUL-terminated) and returns the length it needs including the NUL.
 * fl_prof_reset drops the records.  Not thread-safe across concurrent calls
 * on different streams beyond record bookkeeping. */
void fl_prof_enable(int on);
void fl_prof_reset(void);
size_t fl_prof_report(char *buf, size_t len);

#ifdef __cplusplus
}
#endif
#endif /* FL_H */
