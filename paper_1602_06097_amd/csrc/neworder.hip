// neworder.hip -- the new order of operations (paper Sec. 4.3): the Schur
// complement Dt = D - C A^{-1} B without forming X = A^{-1} B.
//
// The paper reduces each row of C by the rows of A (Algorithm "Reduction of C
// and D"), keeps the multipliers (the row of C' = C A^{-1}) and then reduces D
// by B with them.  Here the multipliers of all rows come from one triangular
// solve and the reduction of D is one contraction:
//
//   C' A = C   <=>   (J A^T J) (J C'^T) = J C^T
//
// with J the reversal of the pivot order, so J A^T J is unit upper
// triangular: the rows of C' are obtained by the same blocked TRSM as X
// (fl_trsm), run on the transpose of A with the columns of C as its
// right-hand sides.  Then Dt = D - C' B, with B's rows taken in the same
// reversed order, on the int8 matrix cores (or the vector ALUs).
//
// Transposes are built as (row << 32 | column) keys sorted on the device.
#include <hipcub/hipcub.hpp>

#include "fl_internal.h"

hipError_t fl_csr_to_dense(uint32_t rows, uint32_t cols, const uint64_t *rp, const uint32_t *ci,
                           const uint16_t *v, uint16_t *out, uint64_t ld, hipStream_t s);
fl_status fl_check_split(const fl_split_info *info, const fl_split_out *s);
typedef void (*fl_limbs_cols_fn)(uint32_t, const uint16_t *, uint64_t, uint32_t, uint32_t,
                                 const uint32_t *, int8_t *, int8_t *, uint32_t, uint32_t *);
fl_limbs_cols_fn fl_limbs_cols_kernel();

namespace {

constexpr uint32_t kKChunk = 65472;  // int32 accumulation bound of the limb GEMM (multiple of 64)

// Nonzero entries of a w-multiline matrix -> (key, value) of the reversed
// transpose: entry (row, col) goes to row npiv-1-col and column
// rev_cols ? npiv-1-row : row.  One wave per group.
__global__ __launch_bounds__(256) void k_ml_transpose_keys(uint32_t w, uint32_t rows, uint32_t ngroups,
                                                           const uint64_t *__restrict__ gptr,
                                                           const uint32_t *__restrict__ pos,
                                                           const uint16_t *__restrict__ val, uint32_t npiv,
                                                           int rev_cols, uint64_t *keys, uint16_t *vals,
                                                           unsigned long long *count) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= ngroups) return;
    for (uint64_t k = gptr[g] + lane; k < gptr[g + 1]; k += 64) {
        const uint32_t col = pos[k];
        for (uint32_t q = 0; q < w; q++) {
            const uint32_t row = g * w + q;
            if (row >= rows) break;
            const uint16_t v = val[(uint64_t)w * k + q];
            if (!v) continue;
            const uint64_t at = atomicAdd(count, 1ull);
            const uint32_t trow = npiv - 1 - col, tcol = rev_cols ? npiv - 1 - row : row;
            keys[at] = ((uint64_t)trow << 32) | tcol;
            vals[at] = v;
        }
    }
}

// Sorted keys -> CSR: row_ptr[r] = first entry of row r (rows of the sorted
// run), col = low half of the key.
__global__ __launch_bounds__(256) void k_csr_from_sorted(uint64_t n, uint32_t nrows,
                                                         const uint64_t *__restrict__ keys, uint64_t *row_ptr,
                                                         uint32_t *col) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e > n) return;
    const uint32_t r = e < n ? (uint32_t)(keys[e] >> 32) : nrows;
    const uint32_t prev = e == 0 ? 0 : (uint32_t)(keys[e - 1] >> 32) + 1;
    for (uint32_t rr = prev; rr <= r && rr <= nrows; rr++)
        if (e == 0 || rr > (uint32_t)(keys[e - 1] >> 32)) row_ptr[rr] = e;
    if (e < n) col[e] = (uint32_t)keys[e];
}

// B's entries -> transposed limb planes with the reversed pivot order:
// plane row c, byte npiv-1-j holds the limbs of B[j][c]; per 128-column tile
// the range of those bytes that hold entries (atomic min / max).
__global__ __launch_bounds__(256) void k_b_planes(uint32_t p, uint32_t npiv, const uint64_t *__restrict__ rp,
                                                  const uint32_t *__restrict__ ci, const uint16_t *__restrict__ v,
                                                  int8_t *Bh, int8_t *Bl, uint64_t kp, uint32_t *tmin,
                                                  uint32_t *tmax) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= npiv) return;
    const uint32_t kk = npiv - 1 - j;
    for (uint64_t e = rp[j] + lane; e < rp[j + 1]; e += 64) {
        const uint32_t c = ci[e];
        int h, l;
        fl_split_limbs(v[e], p, h, l);
        Bh[(uint64_t)c * kp + kk] = (int8_t)h;
        Bl[(uint64_t)c * kp + kk] = (int8_t)l;
        atomicMin(&tmin[c / 128], kk);
        atomicMax(&tmax[c / 128], kk);
    }
}

// K range [floor64(min), ceil64(max + 1)) per column tile, empty if no entry.
__global__ void k_krange_n(uint32_t ntiles, const uint32_t *__restrict__ tmin, const uint32_t *__restrict__ tmax,
                           uint32_t *krange) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    const uint32_t lo = tmin[t], hi = tmax[t];
    if (lo > hi) {
        krange[2 * t] = krange[2 * t + 1] = 0;
    } else {
        krange[2 * t] = lo / 64 * 64;
        krange[2 * t + 1] = (hi + 64) / 64 * 64;
    }
}

// VALU form: C'[r][j] = Xc[npiv-1-j][r] as a dense row-major matrix.
__global__ __launch_bounds__(256) void k_transpose_rev(uint32_t npiv, uint32_t mD, const uint16_t *__restrict__ Xc,
                                                       uint64_t ldx, uint16_t *Cp, uint64_t ldc) {
    __shared__ uint16_t t[64][65];
    const uint32_t k0 = blockIdx.y * 64, r0 = blockIdx.x * 64;
    const uint32_t tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (uint32_t kk = ty; kk < 64; kk += 4) {
        const uint32_t k = k0 + kk, r = r0 + tx;
        t[kk][tx] = k < npiv && r < mD ? Xc[(uint64_t)k * ldx + r] : 0;
    }
    __syncthreads();
    for (uint32_t rr = ty; rr < 64; rr += 4) {
        const uint32_t r = r0 + rr, k = k0 + tx;
        if (r < mD && k < npiv) Cp[(uint64_t)r * ldc + (npiv - 1 - k)] = t[tx][rr];
    }
}

inline uint64_t ld64(uint32_t c) { return c ? ((uint64_t)c + 63) / 64 * 64 : 64; }

struct NoWs {
    uint64_t *akeys[2], *ckeys[2];
    uint16_t *avals[2], *cvals[2];
    void *sort_tmp;
    size_t sort_bytes;
    uint64_t *a_ptr, *c_ptr;       // reversed transposes as CSR
    uint32_t *a_col, *c_col;
    unsigned long long *counter;   // [2]
    uint16_t *Xc;                  // npiv x ldxc: J C'^T
    uint64_t ldxc;
    void *trsm_ws;
    size_t trsm_bytes;
    // MFMA form
    int8_t *Ch, *Cl, *Bh, *Bl;
    uint64_t kp;
    uint32_t *tmin, *tmax, *krange_n;
    uint32_t ntiles;
    // VALU form
    uint16_t *Cp, *Bd;
    uint64_t ldcp, ldbd;
};

size_t sort_tmp_bytes(uint64_t n) {
    size_t b = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, b, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                             (const uint16_t *)nullptr, (uint16_t *)nullptr, (int)(n ? n : 1), 0,
                                             64, (hipStream_t)0);
    return b;
}

// The transposed problem as a split: A' = J A^T J (unit upper, w = 1),
// B' = J C^T (CSR), npiv' = npiv, nB' = mD, no C', D'.
void transposed_split(const fl_split_info *info, const NoWs &t, fl_split_info *ti, fl_split_out *to) {
    fl_split_info i = {};
    i.p = info->p;
    i.m = info->npiv;
    i.n = info->npiv + info->mD;
    i.ml_width = 1;
    i.npiv = info->npiv;
    i.nB = info->mD;
    i.mD = 0;
    i.status = FL_OK;
    i.nnzA = info->nnzA;
    i.nnzB = info->nnzC;
    i.lenA = info->nnzA;
    *ti = i;
    fl_split_out o = {};
    o.a_gptr = t.a_ptr;
    o.a_pos = t.a_col;
    o.a_val = t.avals[1];
    o.b_ptr = t.c_ptr;
    o.b_col = t.c_col;
    o.b_val = t.cvals[1];
    o.c_gptr = t.a_ptr;  // unused (no C rows), must be non-NULL
    o.d_ptr = t.c_ptr;
    *to = o;
}

size_t no_layout(const fl_split_info *info, fl_mode mode, void *ws, NoWs *out) {
    WsCarve c(ws);
    NoWs t = {};
    const uint64_t npiv = info->npiv, mD = info->mD, nB = info->nB;
    const uint64_t na = info->nnzA ? info->nnzA : 1, nc = info->nnzC ? info->nnzC : 1;
    for (int k = 0; k < 2; k++) {
        t.akeys[k] = c.take<uint64_t>(na);
        t.avals[k] = c.take<uint16_t>(na);
        t.ckeys[k] = c.take<uint64_t>(nc);
        t.cvals[k] = c.take<uint16_t>(nc);
    }
    t.sort_bytes = std::max(sort_tmp_bytes(na), sort_tmp_bytes(nc));
    t.sort_tmp = c.take<char>(t.sort_bytes);
    t.a_ptr = c.take<uint64_t>(npiv + 1);
    t.c_ptr = c.take<uint64_t>(npiv + 1);
    t.a_col = c.take<uint32_t>(na);
    t.c_col = c.take<uint32_t>(nc);
    t.counter = c.take<unsigned long long>(2);
    t.ldxc = ld64((uint32_t)mD);
    t.Xc = c.take<uint16_t>((npiv ? npiv : 1) * t.ldxc);
    fl_split_info ti;
    fl_split_out to;
    transposed_split(info, t, &ti, &to);
    t.trsm_bytes = fl_trsm_workspace(&ti, mode);
    t.trsm_ws = c.take<char>(t.trsm_bytes);
    if (mode == FL_MFMA_I8) {
        const uint64_t mp = (mD + 127) / 128 * 128, np = (nB + 127) / 128 * 128;
        t.kp = (npiv + 63) / 64 * 64;
        if (!t.kp) t.kp = 64;
        t.ntiles = (uint32_t)(np / 128);
        t.Ch = c.take<int8_t>(mp * t.kp);
        t.Cl = c.take<int8_t>(mp * t.kp);
        t.Bh = c.take<int8_t>(np * t.kp);
        t.Bl = c.take<int8_t>(np * t.kp);
        t.tmin = c.take<uint32_t>(t.ntiles ? t.ntiles : 1);
        t.tmax = c.take<uint32_t>(t.ntiles ? t.ntiles : 1);
        t.krange_n = c.take<uint32_t>(2 * (size_t)(t.ntiles ? t.ntiles : 1));
    } else {
        t.ldcp = ld64((uint32_t)npiv);
        t.ldbd = ld64((uint32_t)nB);
        t.Cp = c.take<uint16_t>((mD ? mD : 1) * t.ldcp);
        t.Bd = c.take<uint16_t>((npiv ? npiv : 1) * t.ldbd);
    }
    if (out) *out = t;
    return c.off;
}

// Sorted reversed transpose of a multiline matrix into CSR (ptr, col, vals[1]).
fl_status transpose_ml(uint32_t w, uint32_t rows, const uint64_t *gptr, const uint32_t *pos, const uint16_t *val,
                       uint32_t npiv, int rev_cols, uint64_t n, uint64_t *keys[2], uint16_t *vals[2],
                       unsigned long long *counter, void *tmp, size_t tmp_bytes, uint64_t *ptr, uint32_t *col,
                       hipStream_t s) {
    FL_HIP(fl_fill_u64((uint64_t *)counter, 0, 1, s));
    const uint32_t ngroups = (rows + w - 1) / w;
    if (ngroups && n) {
        hipLaunchKernelGGL(k_ml_transpose_keys, dim3((ngroups + 3) / 4), dim3(256), 0, s, w, rows, ngroups, gptr,
                           pos, val, npiv, rev_cols, keys[0], vals[0], counter);
        FL_LAUNCH_CHECK("k_ml_transpose_keys");
        size_t b = tmp_bytes;
        FL_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, b, keys[0], keys[1], vals[0], vals[1], (int)n, 0, 64, s));
    }
    hipLaunchKernelGGL(k_csr_from_sorted, dim3((unsigned)((n + 1 + 255) / 256)), dim3(256), 0, s, n, npiv,
                       (const uint64_t *)keys[1], ptr, col);
    FL_LAUNCH_CHECK("k_csr_from_sorted");
    return FL_OK;
}

}  // namespace

extern "C" size_t fl_reduce_neworder_workspace(const fl_split_info *info, fl_mode mode) {
    if (!info) return 0;
    return no_layout(info, mode, nullptr, nullptr);
}

extern "C" fl_status fl_reduce_neworder(const fl_split_info *info, const fl_split_out *s, uint16_t *Dt,
                                        uint64_t ldd, fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream) {
    fl_status st = fl_check_split(info, s);
    if (st != FL_OK) return st;
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_reduce_neworder: bad mode");
    const uint32_t npiv = info->npiv, mD = info->mD, nB = info->nB, p = info->p, w = info->ml_width;
    if (mD == 0 || nB == 0) return FL_OK;
    FL_ARG(Dt && ldd >= nB && ldd % 4 == 0 && ((uintptr_t)Dt & 7) == 0,
           "fl_reduce_neworder: bad Dt (NULL, ldd < nB, ldd % 4, or misaligned)");
    FL_ARG(info->nnzA < (1ull << 31) && info->nnzC < (1ull << 31),
           "fl_reduce_neworder: A and C must have fewer than 2^31 entries");
    NoWs t;
    const size_t need = no_layout(info, mode, ws, &t);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_reduce_neworder: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    FL_HIP(fl_csr_to_dense(mD, nB, s->d_ptr, s->d_col, s->d_val, Dt, ldd, stream));
    if (npiv == 0) return FL_OK;
    // J A^T J (strictly upper, rows of A become columns) and J C^T
    st = transpose_ml(w, npiv, s->a_gptr, s->a_pos, s->a_val, npiv, 1, info->nnzA, t.akeys, t.avals, t.counter,
                      t.sort_tmp, t.sort_bytes, t.a_ptr, t.a_col, stream);
    if (st != FL_OK) return st;
    st = transpose_ml(w, mD, s->c_gptr, s->c_pos, s->c_val, npiv, 0, info->nnzC, t.ckeys, t.cvals,
                      t.counter + 1, t.sort_tmp, t.sort_bytes, t.c_ptr, t.c_col, stream);
    if (st != FL_OK) return st;
    // J C'^T by the blocked TRSM
    fl_split_info ti;
    fl_split_out to;
    transposed_split(info, t, &ti, &to);
    st = fl_trsm(&ti, &to, t.Xc, t.ldxc, mode, t.trsm_ws, t.trsm_bytes, stream);
    if (st != FL_OK) return st;
    // Dt -= C' B
    if (mode == FL_MFMA_I8) {
        const uint64_t mp = ((uint64_t)mD + 127) / 128 * 128;
        FL_PROF("neworder.limbs", stream,
                hipLaunchKernelGGL(fl_limbs_cols_kernel(), dim3((unsigned)(mp / 64), (unsigned)(t.kp / 64)), dim3(256),
                                   0, stream, p, (const uint16_t *)t.Xc, t.ldxc, mD, npiv, (const uint32_t *)nullptr,
                                   t.Ch, t.Cl, (uint32_t)t.kp, (uint32_t *)nullptr));
        FL_LAUNCH_CHECK("neworder limbs");
        const uint64_t np = (uint64_t)t.ntiles * 128;
        FL_HIP(fl_fill_u32((uint32_t *)t.Bh, 0, np * t.kp / 4, stream));
        FL_HIP(fl_fill_u32((uint32_t *)t.Bl, 0, np * t.kp / 4, stream));
        FL_HIP(fl_fill_u32(t.tmin, ~0u, t.ntiles, stream));
        FL_HIP(fl_fill_u32(t.tmax, 0, t.ntiles, stream));
        hipLaunchKernelGGL(k_b_planes, dim3((npiv + 3) / 4), dim3(256), 0, stream, p, npiv,
                           (const uint64_t *)s->b_ptr, (const uint32_t *)s->b_col, (const uint16_t *)s->b_val, t.Bh,
                           t.Bl, t.kp, t.tmin, t.tmax);
        FL_LAUNCH_CHECK("k_b_planes");
        hipLaunchKernelGGL(k_krange_n, dim3((t.ntiles + 255) / 256), dim3(256), 0, stream, t.ntiles,
                           (const uint32_t *)t.tmin, (const uint32_t *)t.tmax, t.krange_n);
        FL_LAUNCH_CHECK("k_krange_n");
        for (uint64_t kb = 0; kb < t.kp; kb += kKChunk) {
            const uint64_t ke = kb + kKChunk < t.kp ? kb + kKChunk : t.kp;
            GemmPlanes gp = {t.Ch, t.Cl, t.Bh, t.Bl, t.kp, t.kp, 0, 0, (uint32_t)kb, (uint32_t)ke, nullptr,
                             nullptr, t.krange_n, nullptr, Dt, ldd, mD, nB};
            gp.group_m = 4;  // groups of 4 row tiles per column tile on each XCD
            FL_HIP(fl_mfma_gemm_planes(p, gp, stream, "neworder.mfma"));
        }
    } else {
        hipLaunchKernelGGL(k_transpose_rev, dim3((mD + 63) / 64, (npiv + 63) / 64), dim3(256), 0, stream, npiv, mD,
                           (const uint16_t *)t.Xc, t.ldxc, t.Cp, t.ldcp);
        FL_LAUNCH_CHECK("k_transpose_rev");
        FL_HIP(fl_csr_to_dense(npiv, nB, s->b_ptr, s->b_col, s->b_val, t.Bd, t.ldbd, stream));
        FL_HIP(fl_gemm_sub_plain(p, mD, nB, npiv, nullptr, t.Cp, t.ldcp, t.Bd, t.ldbd, Dt, ldd, stream,
                                 "neworder.plain"));
    }
    return FL_OK;
}
