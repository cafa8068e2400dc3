// fl_internal.h -- shared device/host helpers of the gfx950 FL library.
//
// Modular arithmetic model (all exact, no floating point):
//  * residues are uint16 in [0, p), p <= 65521;
//  * reduction of a 32-bit value uses Barrett with mu = floor(2^32 / p):
//    q = umulhi(x, mu) is floor(x/p) or floor(x/p) - 1 for every x < 2^32
//    (x/p - q < x/2^32 + 1 < 2), so one conditional subtraction finishes;
//  * multiply-accumulate of a coefficient a against many residues x keeps two
//    32-bit accumulators, splitting a = 256*a_h + a_l (a_h, a_l < 256): each
//    product a_h*x, a_l*x < 2^24 fits the 24-bit multiplier, and 256 such
//    products plus a residue stay below 2^32 (256*255*65535 + 65535 < 2^32),
//    so accumulators are folded at least every 256 terms.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include "../../include/fl.h"

#define FL_FOLD_TERMS 256u

namespace fl {

struct Mod {
    uint32_t p;
    uint32_t mu;  // floor(2^32 / p)
};

__host__ __device__ inline Mod make_mod(uint32_t p) {
    Mod m;
    m.p = p;
    m.mu = (uint32_t)(((uint64_t)1 << 32) / p);
    return m;
}

__device__ __forceinline__ uint32_t reduce32(uint32_t x, const Mod &m) {
    uint32_t q = __umulhi(x, m.mu);
    uint32_t r = x - q * m.p;
    return r >= m.p ? r - m.p : r;
}

// (a * b) mod p for residues a, b < 2^16 (the product, below 2^32, is the
// low word of the full-rate 24-bit multiply).
__device__ __forceinline__ uint32_t mulmod(uint32_t a, uint32_t b, const Mod &m) {
    return reduce32(__umul24(a, b), m);
}

// (a - b) mod p for residues.
__device__ __forceinline__ uint32_t submod(uint32_t a, uint32_t b, uint32_t p) {
    return a >= b ? a - b : a + p - b;
}

__device__ __forceinline__ uint32_t addmod(uint32_t a, uint32_t b, uint32_t p) {
    uint32_t s = a + b;
    return s >= p ? s - p : s;
}

// 24-bit multiply-add: a, b < 2^24.
__device__ __forceinline__ uint32_t mad24(uint32_t a, uint32_t b, uint32_t c) {
    return __umul24(a, b) + c;
}

// Fold a split accumulator pair (hi counts 256x) into one residue:
// 256 hi + lo = 256 (hi mod p) + (lo mod p) (mod p), and
// 256 (hi mod p) + (lo mod p) < 2^24 + 2^16, so a third reduction finishes.
// The first two reductions are independent.
__device__ __forceinline__ uint32_t fold_pair(uint32_t hi, uint32_t lo, const Mod &m) {
    const uint32_t rh = reduce32(hi, m), rl = reduce32(lo, m);
    return reduce32((rh << 8) + rl, m);
}

// Modular inverse by Fermat's little theorem (x != 0, p prime).
__device__ inline uint32_t invmod(uint32_t x, const Mod &m) {
    uint32_t r = 1, b = x, e = m.p - 2;
    while (e) {
        if (e & 1) r = mulmod(r, b, m);
        b = mulmod(b, b, m);
        e >>= 1;
    }
    return r;
}

}  // namespace fl

// ---- host-side error plumbing -------------------------------------------------
void fl_set_error(const char *msg);
fl_status fl_hip_fail(hipError_t e, const char *where);

#define FL_HIP(call)                                                    \
    do {                                                                \
        hipError_t e_ = (call);                                         \
        if (e_ != hipSuccess) return fl_hip_fail(e_, #call);            \
    } while (0)

#define FL_LAUNCH_CHECK(where)                                          \
    do {                                                                \
        hipError_t e_ = hipGetLastError();                              \
        if (e_ != hipSuccess) return fl_hip_fail(e_, where);            \
    } while (0)

#define FL_ARG(cond, msg)                                               \
    do {                                                                \
        if (!(cond)) { fl_set_error(msg); return FL_ERR_ARG; }          \
    } while (0)

// Workspace carving: 256-byte aligned slices.
struct WsCarve {
    char *base;
    size_t off;
    explicit WsCarve(void *b) : base((char *)b), off(0) {}
    template <class T> T *take(size_t count) {
        size_t bytes = (count * sizeof(T) + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += bytes;
        return p;
    }
};

// Exclusive scans on the device (three-phase: tile reduce, scan of tile sums,
// tile scan).  `tmp` must hold fl_scan_tmp_elems(n) elements.  out may alias in.
size_t fl_scan_tmp_elems(size_t n);
hipError_t fl_exclusive_scan_u64(const uint64_t *in, uint64_t *out, size_t n, uint64_t *tmp,
                                 uint64_t *total_out, hipStream_t s);

// Fill a device buffer with a 32-bit / 16-bit pattern by a kernel (kept out
// of hipMemsetAsync so that calls stay safe under stream capture).
hipError_t fl_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t fl_fill_u64(uint64_t *p, uint64_t v, size_t n, hipStream_t s);
hipError_t fl_zero_rows_u16(uint16_t *p, uint64_t ld, uint32_t rows, uint32_t cols, hipStream_t s);

// Launch profiler (see fl_prof_* in fl.h): returns a token for fl_prof_end,
// or -1 when profiling is off.
int fl_prof_begin(const char *site, hipStream_t s);
void fl_prof_end(int tok, hipStream_t s);
// Switches the profiler on or off; returns the previous state.
bool fl_prof_set(bool on);

// Bracket one launch statement with profiler events (no-op when disabled).
// Returns a non-OK fl_status from the enclosing function.
#define FL_CHECK_ST(call)                      \
    do {                                       \
        fl_status st_ = (call);                \
        if (st_ != FL_OK) return st_;          \
    } while (0)

#define FL_PROF(site, stream, ...)                                      \
    do {                                                                \
        int tok_ = fl_prof_begin(site, stream);                         \
        __VA_ARGS__;                                                    \
        fl_prof_end(tok_, stream);                                      \
    } while (0)

// One int8-limb-plane GEMM on the matrix cores (gemm_mfma.hip):
//   C[rows x N] -= A B   with A row m (k = 0..) at Ah/Al + m*lda + a_k0 + k and
//   B column n at Bh/Bl + n*ldb + b_k0 + k (B transposed), k in [kbeg, kend)
//   (multiples of 64; kend capped by round_up(*klen_dev, 64) when given);
//   optional per-128-row-block ranges krange[2*mb..2*mb+1], per-128-column-
//   block ranges krange_n[2*nb..2*nb+1] (intersected; all-zero blocks of the
//   operands are skipped), and output row map (~0u = no output row).
// A must have round_up(M, 128) readable rows, B round_up(N, 128).
// group_m: 0 = tiles in grid order; g > 0 = each XCD takes a contiguous
// range of tiles, walked column by column in groups of g row tiles (the
// row tiles that share a B column tile run together on one XCD's L2).
struct GemmPlanes {
    const int8_t *Ah, *Al, *Bh, *Bl;
    uint64_t lda, ldb;
    uint32_t a_k0, b_k0;
    uint32_t kbeg, kend;
    const uint32_t *klen_dev;
    const uint32_t *krange;
    const uint32_t *krange_n;
    const uint32_t *row_map;
    uint16_t *C;
    uint64_t ldc;
    uint32_t M, N;
    uint32_t group_m;
    // optional, per 128-column tile: an exclusive upper bound on the rows of
    // B (absolute K index, before b_k0 is subtracted) that hold a nonzero in
    // that tile's columns; K blocks past it are skipped
    const uint32_t *kcap_n;
    // workgroups of the launch: 0 = one per tile; kGemmPerCu = one per
    // compute unit, each taking several tiles in turn; otherwise at most
    // this many
    uint32_t max_wg;
};
constexpr uint32_t kGemmPerCu = 0xffffffffu;
hipError_t fl_mfma_gemm_planes(uint32_t p, const GemmPlanes &g, hipStream_t s, const char *site);
// C[M x N] -= A[M x K] B[K x N] (mod p) on the vector ALUs (gemm_plain.hip),
// K = *Kdev when Kdev is given; krange_n / kfirst: optional zero-skipping
// ranges of B's column tiles and A's rows (valu_tile.h).
hipError_t fl_gemm_sub_plain(uint32_t p, uint32_t M, uint32_t N, uint32_t Kh, const uint32_t *Kdev,
                             const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                             uint16_t *C, uint64_t ldc, hipStream_t s, const char *site,
                             const uint32_t *krange_n = nullptr, const uint32_t *kfirst = nullptr);
// A second stream and two events for work that overlaps the caller's stream,
// one set per host thread, device and slot (< 4), kept until the process ends.
fl_status fl_aux_stream(uint32_t slot, hipStream_t *s, hipEvent_t *a, hipEvent_t *b);
// Rank-k (k <= 64) update C[row_map[i], :N] -= A[row_map[i]] B^T for
// i < *Mdev (<= Mmax); A planes: 64 bytes per C row; B planes: N_pad x 64.
hipError_t fl_mfma_rank64_planes(uint32_t p, const int8_t *Ah, const int8_t *Al, const int8_t *Bh,
                                 const int8_t *Bl, const uint32_t *Kdev, const uint32_t *row_map,
                                 const uint32_t *Mdev, uint32_t Mmax, uint16_t *C, uint64_t ldc,
                                 uint32_t N, hipStream_t s, const char *site);
// Maximum of v over the 64 lanes of the wave (every lane receives it).
__device__ __forceinline__ uint32_t fl_wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, off, 64);
        v = o > v ? o : v;
    }
    return v;
}

// Residue x -> signed int8 limbs (h, l) with centred r = 256 h + l = x mod p:
// r = x if x <= t, else x - p, with t = 32639, or t = (p - 1) / 2 for
// p < 256 (then r is the symmetric residue in [-127, 127]: a single limb,
// h = 0).  The threshold is a select on p, so no branch enters loops.
__device__ __forceinline__ void fl_split_limbs(uint32_t x, uint32_t p, int &h, int &l) {
    const uint32_t t = p < 256 ? (p - 1) >> 1 : 32639u;
    const int r = x <= t ? (int)x : (int)x - (int)p;
    h = (r + 128) >> 8;  // arithmetic shift: floor
    l = r - (h << 8);
}

// fl_split without its sync: enqueue everything (size words to dinfo_out, 8
// u64, when non-NULL), then turn the synced size words into fl_split_info.
fl_status fl_split_enqueue(const fl_csr *M, uint32_t p, uint32_t ml_width, const fl_split_out *o,
                           void *ws, size_t ws_bytes, uint64_t *dinfo_out, hipStream_t stream);
fl_status fl_split_finish(const fl_csr *M, uint32_t p, uint32_t ml_width, const uint64_t hinf[8],
                          fl_split_info *h_info);
// fl_rref_csr_size + fl_rref_to_csr without a host sync; col/val hold the
// upper bound (npiv + min(mD, nB)) * (nB + 1) entries.
fl_status fl_rref_csr_enqueue(const fl_split_info *info, const fl_split_out *s, const uint16_t *Xp,
                              uint64_t ldx, const uint16_t *RD, uint64_t ldd,
                              const uint32_t *d_rank, const uint32_t *d_pivcol, uint64_t *row_ptr,
                              uint32_t *col, uint16_t *val, void *ws, size_t ws_bytes,
                              hipStream_t stream);

// ---- many problems per launch --------------------------------------------------
// A launch that serves several problems gives problem i the workgroups
// [prefix[i], prefix[i+1]) of its 1-D grid; fl_task_of finds i for workgroup
// bx (binary search over the n entries; prefix[0] = 0, ascending).
__device__ __forceinline__ uint32_t fl_task_of(const uint32_t *__restrict__ prefix, uint32_t n,
                                               uint32_t bx) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (prefix[mid] <= bx) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The tasks of one workgroup.  With counter == NULL a launch maps workgroup
// x to task x (one task each).  Otherwise the launch is persistent: a fixed
// number of workgroups (about as many as stay resident) take task indices
// from the atomic *counter until it passes `total`, so tiles of all problems
// are dealt dynamically to whichever workgroup is free.  The counter of each
// launch starts at zero (cleared by a fill kernel, so graph replays work);
// no workgroup ever waits for another.  Used as
//     uint32_t task;
//     for (bool ok = fl_queue_take(q, task, true); ok; ok = fl_queue_take(q, task, false)) { ... }
// where the body ends a task with `continue` (never a bare return: every
// thread must come back for the next take).
struct FlQueue {
    uint32_t *counter;
    uint32_t total;
};
__device__ __forceinline__ bool fl_queue_take(const FlQueue &q, uint32_t &task, bool first) {
    if (!q.counter) {  // (uniform) one task per workgroup
        task = blockIdx.x;
        return first;
    }
    __shared__ uint32_t s_task;
    __syncthreads();  // the previous task is done with LDS and with s_task
    if (threadIdx.x == 0) s_task = atomicAdd(q.counter, 1u);
    __syncthreads();
    task = s_task;
    return task < q.total;
}
// Workgroups of a persistent launch: `per_cu` per compute unit, at most
// `total`; counter NULL (one workgroup per task) when per_cu is 0.
uint32_t fl_queue_grid(uint32_t total, uint32_t per_cu);
// Compute units of the current device.
uint32_t fl_cu_count();

// Copies `bytes` from host memory into device memory through kernel
// arguments (1 KiB per launch), so that the copy can be captured in a graph
// without referring to host memory at replay time.
hipError_t fl_upload(void *dst, const void *src, size_t bytes, hipStream_t s);

// One matrix's TRSM as the step kernels see it (device-side table entry).
struct FlTrsmTask {
    const uint64_t *gptr;   // A multiline groups
    const uint32_t *pos;
    const uint16_t *val;
    const uint32_t *nin, *nnear;
    uint16_t *X;
    uint64_t ldx;
    uint32_t npiv, nB, nblk, mfma;
    int8_t *Ah, *Al, *Xh, *Xl;  // int8-MFMA form only
    int8_t *Th, *Tl;            // limbs of I - (diagonal block)^-1, per block (int8-MFMA form)
    const uint32_t *kext, *krange;
    uint64_t kp;
    // per 128-column tile of X: 1 + the last solved row with a nonzero there
    // (0: none yet), raised by every block solve (int8-MFMA form)
    uint32_t *xkend;
};
constexpr uint32_t kFlTrsmBlock = 128;
constexpr uint32_t kFlTrsmSuper = 4;  // blocks per superblock of the MFMA-form update
// fl_trsm's set-up (dense B into X, group bounds, MFMA band planes) for one
// matrix, enqueued on `stream`; *task receives its table entry.
fl_status fl_trsm_prepare(const fl_split_info *info, const fl_split_out *s, uint16_t *X, uint64_t ldx,
                          fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream, FlTrsmTask *task);
// Step `step` (block nblk - 1 - step of each listed matrix): the far update
// (kind 0: VALU, 1: int8 MFMA; no-op at step 0), the block solve (kind 2: by
// back substitution) or the MFMA-form block solve (kind 3: product with the
// block inverse),
// over tasks[ids[0..n)] with workgroup prefix `prefix` and `grid` workgroups.
// Workgroups per matrix: solve and MFMA-form solve ceil(nB / 64); VALU update
// ceil(nB / 256) * (128 / w / 4); MFMA update ceil(nB / 128) * kFlTrsmSuper.
hipError_t fl_trsm_batch_launch(int kind, uint32_t p, uint32_t w, const FlTrsmTask *tasks,
                                const uint32_t *ids, const uint32_t *prefix, uint32_t n, uint32_t grid,
                                uint32_t step, uint32_t *counter, uint32_t per_cu, hipStream_t stream);

// One matrix's Gauss-Jordan elimination of the Schur complement as the panel
// kernels see it (device-side table entry).
struct FlEchTask {
    uint16_t *D;
    uint64_t ld;
    uint32_t rows, cols, npanels, mfma;
    uint32_t *is_piv, *piv_row, *piv_col, *d_rank;
    void *ps;               // panel states
    uint16_t *U, *T;
    uint64_t ldu;
    int8_t *Uh, *Ul;        // int8-MFMA form only
    uint16_t *Lb, *Ub;      // block multipliers; block U (VALU form)
    int8_t *Lbh, *Lbl, *Ubh, *Ubl;  // their limb planes (int8-MFMA form only)
    uint32_t *upd_rows, *blk_rows, *blk_cnt, *mark, *nzlist, *flist, *counts, *nzlead;
};
// Device tables for a panel loop over several matrices: ids sorted by panel
// count (descending); workgroup prefixes for the column-tiled kernels (n + 1
// entries per panel or block, matrices already finished count 0).
// Panels are grouped in blocks of four (256 columns).  A panel updates only
// the columns of its block; at the end of a block, the block's update of the
// columns right of it is applied as one rank-256 update, the next block's
// 256 columns first (they are on the critical path), the rest on a second
// stream while the next block's panels are searched.
struct FlEchLists {
    const uint32_t *ids_all, *ids_mfma, *ids_plain;
    const uint32_t *pre_rows;  // [n_all + 1]: ceil(rows / 32)
    // per panel: one workgroup per matrix with more than P panels
    uint32_t *pre_n_all, *pre_n_mfma, *pre_n_plain;
    // per block b (bend = 256 (b + 1)): tiles of 64 / 128 / 256 columns over
    // the next block [bend, bend + 256) and over the far part [bend + 256, cols)
    uint32_t *pre_bn_all, *pre_bn_mfma, *pre_bn_plain;
    uint32_t *pre_bf_all, *pre_bf_mfma, *pre_bf_plain;
    uint32_t n_all, n_mfma, n_plain;
};
constexpr uint32_t kFlEchBlock = 256;  // columns per block
// fl_echelon_d's set-up for one matrix (clears its bookkeeping on `stream`);
// *task receives its table entry (npanels = 0 when there is nothing to do).
fl_status fl_echelon_prepare(uint32_t p, uint32_t rows, uint32_t cols, uint16_t *Dt, uint64_t ldd,
                             uint32_t *d_rank, uint32_t *d_pivcol, fl_mode mode, void *ws,
                             size_t ws_bytes, hipStream_t stream, FlEchTask *task);
// Fills the prefix tables of `lists` (device; `panels` panels, `blocks`
// blocks) from the task table.
hipError_t fl_echelon_prefixes(const FlEchTask *tasks, const FlEchLists &lists, uint32_t panels,
                               uint32_t blocks, hipStream_t stream);
// Host mirror of the prefix tables' totals: tiles of `tile` columns over
// [start, start + span) of a matrix with `cols` columns.
inline uint32_t fl_ech_tiles(uint32_t cols, uint64_t start, uint64_t span, uint32_t tile) {
    if (cols <= start) return 0;
    const uint64_t w = cols - start < span ? cols - start : span;
    return (uint32_t)((w + tile - 1) / tile);
}
// Workgroup counts of panel P (host side).
struct FlEchGrid {
    uint32_t n_active, grid_rows;     // leading ids_all entries with more than P panels; their row blocks
    uint32_t n_mfma, n_plain;         // MFMA / VALU-form matrices with more than P panels
    uint32_t mfma_rows;               // largest row count among the active MFMA-form matrices
    uint32_t n_next, grid_rows_next;  // the same as n_active, grid_rows for panel P + 1
};
// Workgroup counts of the update at the end of a block (host side): prefix
// totals of the six block tables, and the largest row count among the
// MFMA-form matrices with columns right of the block.
struct FlEchBlockGrid {
    uint32_t bn_all, bn_mfma, bn_plain, bf_all, bf_mfma, bf_plain, mfma_rows;
};
// The second stream of a panel loop and its two events; far_pending is set
// while far-part work recorded on `far` has not yet been waited for.
struct FlEchAux {
    hipStream_t far;
    hipEvent_t ev_near, ev_far;
    bool far_pending;
    uint32_t far_groups;  // workgroups along the columns of a far block update (0: 128)
};
// Panel P of every listed matrix on `stream`; when P ends a block (blk
// non-NULL), also the block's update of the columns right of it, its far
// part on aux.far.
hipError_t fl_echelon_batch_panel(uint32_t p, const FlEchTask *tasks, const FlEchLists &lists, uint32_t P,
                                   const FlEchGrid &g, const FlEchBlockGrid *blk, hipStream_t stream,
                                   FlEchAux &aux);
// Makes `stream` wait for the far part of the last block.
hipError_t fl_echelon_join(hipStream_t stream, FlEchAux &aux);
// Moves the pivot rows of one matrix to the top in pivot order, clears the rest.
fl_status fl_echelon_finish(const FlEchTask &t, hipStream_t stream);
