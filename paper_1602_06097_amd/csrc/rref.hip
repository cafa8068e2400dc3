// rref.hip -- the second FL pass (end of paper Sec. 4.1: run the reduction
// again on [A^{-1}B ; D']) and FL step 5 (column rearrangement / read-off).
//
// With R_D = RREF(Dt) of rank r and pivot columns P_D, the second pass is
//     X' = X - X[:, P_D] R_D :
//   k_gather_pivcols   L = X[:, P_D]   (npiv x r, saved before X is updated)
//   dense GEMM         X -= L R_D      (VALU or int8 MFMA form)
// Then [Id X'; 0 R_D] is the reduced row echelon form of M under col_perm,
// read off as canonical CSR in the original column order:
//   k_csr_count        nonzeros of every output row, stored at the row's
//                      position in pivot-column order; exclusive scan
//   k_csr_emit         one wave per output row: pivot 1, then the nonzeros of
//                      the X' or R_D row (both ascending in original order),
//                      staged in LDS up to 256 entries at a time for coalesced stores.
#include <mutex>
#include <string>

#include "fl_internal.h"

hipError_t fl_gemm_sub_mfma(uint32_t p, uint32_t M, uint32_t N, uint32_t Kmax, const uint32_t *Kdev,
                            const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                            uint16_t *C, uint64_t ldc, void *ws, size_t ws_bytes, hipStream_t s,
                            const char *site);
size_t fl_gemm_sub_mfma_ws(uint32_t M, uint32_t N, uint32_t Kmax);
typedef void (*fl_limbs_cols_fn)(uint32_t, const uint16_t *, uint64_t, uint32_t, uint32_t,
                                 const uint32_t *, int8_t *, int8_t *, uint32_t, uint32_t *);
fl_limbs_cols_fn fl_limbs_cols_kernel();
fl_status fl_check_split(const fl_split_info *info, const fl_split_out *s);

namespace {

// L[i][t] = X[i][pivcol[t]] for t < r (L row stride ldl).
__global__ __launch_bounds__(256) void k_gather_pivcols(const uint16_t *__restrict__ X, uint64_t ldx,
                                                        uint32_t npiv,
                                                        const uint32_t *__restrict__ d_rank,
                                                        const uint32_t *__restrict__ pivcol,
                                                        uint16_t *L, uint64_t ldl, uint32_t *tfirst) {
    const uint32_t r = *d_rank;
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = t < r;  // (every lane takes part in the wave minimum)
    const uint32_t c = act ? pivcol[t] : 0;
    for (uint32_t i = blockIdx.y; i < npiv; i += gridDim.y) {
        const uint32_t x = act ? X[(uint64_t)i * ldx + c] : 0;
        if (act) L[(uint64_t)i * ldl + t] = (uint16_t)x;
        if (tfirst) {  // first pivot index t with X[i][q_t] != 0
            const uint32_t first = ~fl_wave_max(x ? ~t : 0u);
            if ((threadIdx.x & 63) == 0 && first != 0xffffffffu) atomicMin(&tfirst[i], first);
        }
    }
}

// MFMA form: L = X[:, P_D] directly as int8 limb planes (Kp bytes per row,
// zero for t >= r).
// Four K entries per thread (kp is a multiple of 64): the limbs of each row
// are written four bytes at a time.
__global__ __launch_bounds__(256) void k_gather_pivcols_limbs(uint32_t p, const uint16_t *__restrict__ X,
                                                              uint64_t ldx, uint32_t npiv,
                                                              const uint32_t *__restrict__ d_rank,
                                                              const uint32_t *__restrict__ pivcol,
                                                              int8_t *Lh, int8_t *Ll, uint64_t kp,
                                                              uint32_t *tfirst) {
    const uint32_t r = *d_rank;
    const uint32_t t0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
    const bool act = t0 < kp;  // (every lane takes part in the wave minimum below)
    uint32_t c[4];
#pragma unroll
    for (int e = 0; e < 4; e++) c[e] = act && t0 + e < r ? pivcol[t0 + e] : 0;
    for (uint32_t i = blockIdx.y; i < npiv; i += gridDim.y) {
        uint32_t x[4];
#pragma unroll
        for (int e = 0; e < 4; e++) x[e] = act ? X[(uint64_t)i * ldx + c[e]] : 0;
        uint32_t hw = 0, lw = 0, first = 0xffffffffu;
#pragma unroll
        for (int e = 3; e >= 0; e--) {
            int h = 0, l = 0;
            if (t0 + e < r) {
                fl_split_limbs(x[e], p, h, l);
                if (x[e]) first = t0 + e;
            }
            hw |= (uint32_t)(h & 0xff) << (8 * e);
            lw |= (uint32_t)(l & 0xff) << (8 * e);
        }
        if (act) {
            *(uint32_t *)(Lh + (uint64_t)i * kp + t0) = hw;
            *(uint32_t *)(Ll + (uint64_t)i * kp + t0) = lw;
        }
        if (tfirst) {  // first pivot index t with X[i][q_t] != 0
            first = ~fl_wave_max(~first);
            if ((threadIdx.x & 63) == 0 && first != 0xffffffffu) atomicMin(&tfirst[i], first);
        }
    }
}

// Per 128-row tile of L = X[:, P_D]: K range [first nonzero t of its rows,
// rounded down to 64; kp) (empty when all its rows are zero there).
__global__ void k_tile_kbeg(uint32_t npiv, uint32_t mtiles, const uint32_t *__restrict__ tfirst, uint32_t kp,
                            uint32_t *krange) {
    const uint32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= mtiles) return;
    uint32_t b = 0xffffffffu;
    for (uint32_t i = m * 128; i < m * 128 + 128 && i < npiv; i++) b = tfirst[i] < b ? tfirst[i] : b;
    krange[2 * m] = b == 0xffffffffu ? kp : b / 64 * 64;
    krange[2 * m + 1] = kp;
}

// For every row t < r of R_D: the 128-column output tiles its nonzeros span
// (from its pivot column to its last nonzero); per tile, the smallest and
// largest such t.  All-zero (tile, t-range) blocks of the product are skipped.
__global__ __launch_bounds__(256) void k_rd_tile_ranges(const uint16_t *__restrict__ RD, uint64_t ldd,
                                                        uint32_t nB, const uint32_t *__restrict__ d_rank,
                                                        const uint32_t *__restrict__ pivcol,
                                                        uint32_t *tmin, uint32_t *tmax) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t t = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= *d_rank) return;
    const uint32_t q = pivcol[t];
    const uint16_t *row = RD + (uint64_t)t * ldd;
    uint32_t last = q;
    for (uint32_t c0 = q; c0 < nB; c0 += 64) {
        const uint32_t c = c0 + lane;
        const uint64_t m = __ballot(c < nB && row[c] != 0);
        if (m) last = c0 + 63 - __clzll(m);
    }
    for (uint32_t tile = q / 128 + lane; tile <= last / 128; tile += 64) {
        atomicMin(&tmin[tile], t);
        atomicMax(&tmax[tile], t);
    }
}

__global__ void k_krange_from_t(uint32_t ntiles, const uint32_t *__restrict__ tmin,
                                const uint32_t *__restrict__ tmax, uint32_t kp, uint32_t *krange) {
    const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ntiles) return;
    uint32_t b = 0, e = 0;
    if (tmin[j] <= tmax[j] && tmin[j] != 0xffffffffu) {
        b = tmin[j] / 64 * 64;
        e = (tmax[j] + 1 + 63) / 64 * 64;
        if (e > kp) e = kp;
    }
    krange[2 * j] = b;
    krange[2 * j + 1] = e;
}

// Number of entries of p_list[0..cnt) strictly below x (p_list ascending).
__device__ __forceinline__ uint32_t count_below(const uint32_t *list, uint32_t cnt, uint32_t x,
                                                const uint32_t *map) {
    uint32_t lo = 0, hi = cnt;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        uint32_t v = map ? map[list[mid]] : list[mid];
        if (v < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

struct OutRow {
    bool top;          // a row of [Id X'] (else a row of R_D)
    uint32_t src;      // row index within X' or R_D
    uint32_t pos;      // output row position
    uint32_t pivot;    // original pivot column
};

// Output row j of the wave: j < npiv -> top row j, else R_D row j - npiv.
// col_perm[0..npiv) are the pivot columns of A ascending; col_perm[npiv + c]
// the non-pivot columns ascending; R_D's pivots col_perm[npiv + pivcol[t]]
// are ascending in t.
__device__ __forceinline__ OutRow out_row(uint32_t j, uint32_t npiv, uint32_t r,
                                          const uint32_t *col_perm, const uint32_t *pivcol) {
    OutRow o;
    if (j < npiv) {
        o.top = true; o.src = j; o.pivot = col_perm[j];
        o.pos = j + count_below(pivcol, r, o.pivot, col_perm + npiv);
    } else {
        o.top = false; o.src = j - npiv; o.pivot = col_perm[npiv + pivcol[o.src]];
        o.pos = o.src + count_below(col_perm, npiv, o.pivot, nullptr);
    }
    return o;
}

// Nonzero u16 entries among the four of v.
__device__ __forceinline__ uint32_t nz4(uint64_t v) {
    return ((v & 0xffffull) != 0) + ((v & 0xffff0000ull) != 0) + ((v & 0xffff00000000ull) != 0) +
           ((v >> 48) != 0);
}

// Rows are read as 8-byte chunks of four entries (rows start 8-byte aligned:
// ld is a multiple of 4); the nB % 4 entries past the last chunk one by one.
__global__ __launch_bounds__(256) void k_csr_count(uint32_t npiv, uint32_t nB,
                                                   const uint32_t *__restrict__ col_perm,
                                                   const uint16_t *__restrict__ Xp, uint64_t ldx,
                                                   const uint16_t *__restrict__ RD, uint64_t ldd,
                                                   const uint32_t *__restrict__ d_rank,
                                                   const uint32_t *__restrict__ pivcol,
                                                   uint64_t *cnt) {
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
    const uint32_t r = *d_rank;
    if (j >= npiv + r) return;
    OutRow o = out_row(j, npiv, r, col_perm, pivcol);
    const uint16_t *row = o.top ? Xp + (uint64_t)o.src * ldx : RD + (uint64_t)o.src * ldd;
    const gu64 *row8 = (const gu64 *)row;
    const uint32_t nq = nB / 4;
    uint32_t c = 0;
#pragma unroll 4
    for (uint32_t q = lane; q < nq; q += 64) c += nz4(row8[q]);
    for (uint32_t k = nq * 4 + lane; k < nB; k += 64) c += row[k] != 0 ? 1 : 0;
    for (int d = 32; d >= 1; d >>= 1) c += __shfl_xor(c, d, 64);
    if (lane == 0) cnt[o.pos] = c + (o.top ? 1 : 0);
}

// Orders one wave's LDS writes before its later LDS reads by other lanes.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One wave per output row: each lane takes a chunk of four entries, and the
// wave's exclusive prefix sum of the chunks' nonzero counts places them in an
// LDS staging run of up to 256 entries, which the wave then stores to the CSR
// arrays as contiguous, coalesced runs.
__global__ __launch_bounds__(256) void k_csr_emit(uint32_t npiv, uint32_t nB,
                                                  const uint32_t *__restrict__ col_perm,
                                                  const uint16_t *__restrict__ Xp, uint64_t ldx,
                                                  const uint16_t *__restrict__ RD, uint64_t ldd,
                                                  const uint32_t *__restrict__ d_rank,
                                                  const uint32_t *__restrict__ pivcol,
                                                  const uint64_t *__restrict__ row_ptr,
                                                  uint32_t *ocol, uint16_t *oval) {
    typedef __attribute__((address_space(1))) const uint64_t gu64;
    __shared__ uint32_t s_col[4][256];
    __shared__ uint16_t s_val[4][256];
    const uint32_t lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const uint32_t j = blockIdx.x * 4 + wv;
    const uint32_t r = *d_rank;
    if (j >= npiv + r) return;
    OutRow o = out_row(j, npiv, r, col_perm, pivcol);
    const uint16_t *row = o.top ? Xp + (uint64_t)o.src * ldx : RD + (uint64_t)o.src * ldd;
    const gu64 *row8 = (const gu64 *)row;
    const uint32_t *perm = col_perm + npiv;
    uint32_t *const sc = s_col[wv];
    uint16_t *const sv = s_val[wv];
    uint64_t out = row_ptr[o.pos];
    if (o.top) {
        if (lane == 0) { ocol[out] = o.pivot; oval[out] = 1; }
        out++;
    }
    const uint32_t nq = nB / 4;
    // software pipeline over chunks of 64 x 4 entries: the row chunk two
    // ahead and the original columns of the next chunk's nonzeros are in
    // flight while a chunk is compacted and stored
    uint64_t v1 = lane < nq ? row8[lane] : 0;
    uint64_t v2 = 64 + lane < nq ? row8[64 + lane] : 0;
    uint32_t pc[4];
#pragma unroll
    for (int e = 0; e < 4; e++) pc[e] = (v1 >> (16 * e)) & 0xffffu ? perm[4 * lane + e] : 0;
    for (uint32_t q0 = 0; q0 < nq; q0 += 64) {
        const uint32_t q = q0 + lane;
        const uint64_t v = v1;
        const uint32_t c4[4] = {pc[0], pc[1], pc[2], pc[3]};
        v1 = v2;  // (zero past the row: no column is fetched for it)
#pragma unroll
        for (int e = 0; e < 4; e++) pc[e] = (v1 >> (16 * e)) & 0xffffu ? perm[4 * (q + 64) + e] : 0;
        v2 = q + 128 < nq ? row8[q + 128] : 0;
        const uint32_t n = nz4(v);
        uint32_t incl = n;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = __shfl_up(incl, d, 64);
            if (lane >= (uint32_t)d) incl += t;
        }
        uint32_t at = incl - n;
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const uint32_t x = (uint32_t)(v >> (16 * e)) & 0xffffu;
            if (x) {
                sc[at] = c4[e];
                sv[at] = (uint16_t)x;
                at++;
            }
        }
        const uint32_t tot = __shfl(incl, 63, 64);
        wave_lds_sync();
        for (uint32_t i = lane; i < tot; i += 64) {
            ocol[out + i] = sc[i];
            oval[out + i] = sv[i];
        }
        wave_lds_sync();
        out += tot;
    }
    // the nB % 4 entries past the last chunk
    {
        const uint32_t k = nq * 4 + lane;
        const uint32_t x = k < nB ? row[k] : 0;
        const uint64_t mask = __ballot(x != 0);
        const uint64_t below = lane == 0 ? 0 : (mask & (~(uint64_t)0 >> (64 - lane)));
        if (x) {
            const uint64_t at = out + __popcll(below);
            ocol[at] = perm[k];
            oval[at] = (uint16_t)x;
        }
    }
}

struct CsrWs {
    uint64_t *cnt;
    uint64_t *scantmp;
    uint64_t *dinfo;
};

size_t csr_layout(uint32_t npiv, uint32_t maxr, void *ws, CsrWs *c) {
    WsCarve w(ws);
    CsrWs t;
    size_t n = (size_t)npiv + maxr + 1;
    t.cnt = w.take<uint64_t>(n);
    t.scantmp = w.take<uint64_t>(fl_scan_tmp_elems(n));
    t.dinfo = w.take<uint64_t>(4);
    if (c) *c = t;
    return w.off;
}

struct RrefWs {
    uint16_t *L;
    uint64_t ldl;
    int8_t *Lh, *Ll, *Rh, *Rl;
    uint32_t *tmin, *tmax, *krange;
    uint32_t *tfirst, *krange_m;  // per row of L / per 128-row tile of L
    uint64_t kp;
    uint32_t ntiles;
};

size_t rref_layout(const fl_split_info *info, fl_mode mode, void *ws, RrefWs *r) {
    WsCarve w(ws);
    RrefWs t = {};
    const uint32_t maxr = info->mD < info->nB ? info->mD : info->nB;
    if (mode == FL_MFMA_I8) {
        const uint64_t mp = ((uint64_t)info->npiv + 127) / 128 * 128;
        const uint64_t np = ((uint64_t)info->nB + 127) / 128 * 128;
        t.kp = ((uint64_t)maxr + 63) / 64 * 64;
        if (t.kp == 0) t.kp = 64;
        t.ntiles = (uint32_t)(np / 128);
        t.Lh = w.take<int8_t>(mp * t.kp);
        t.Ll = w.take<int8_t>(mp * t.kp);
        t.Rh = w.take<int8_t>(np * t.kp);
        t.Rl = w.take<int8_t>(np * t.kp);
        t.tmin = w.take<uint32_t>(t.ntiles ? t.ntiles : 1);
        t.tmax = w.take<uint32_t>(t.ntiles ? t.ntiles : 1);
        t.krange = w.take<uint32_t>(2 * (size_t)(t.ntiles ? t.ntiles : 1));
        t.tfirst = w.take<uint32_t>(mp ? mp : 1);
        t.krange_m = w.take<uint32_t>(2 * (mp / 128 ? mp / 128 : 1));
    } else {
        t.ldl = ((uint64_t)maxr + 7) & ~(uint64_t)7;
        t.L = w.take<uint16_t>((size_t)(info->npiv ? info->npiv : 1) * (t.ldl ? t.ldl : 1));
        const uint64_t np = ((uint64_t)info->nB + 127) / 128 * 128;
        t.ntiles = (uint32_t)(np / 128);
        t.tmin = w.take<uint32_t>(t.ntiles ? t.ntiles : 1);
        t.tmax = w.take<uint32_t>(t.ntiles ? t.ntiles : 1);
        t.krange = w.take<uint32_t>(2 * (size_t)(t.ntiles ? t.ntiles : 1));
        t.tfirst = w.take<uint32_t>(info->npiv ? info->npiv : 1);
    }
    if (r) *r = t;
    return w.off;
}

}  // namespace

extern "C" size_t fl_rref_workspace(const fl_split_info *info, fl_mode mode) {
    if (!info) return 0;
    return rref_layout(info, mode, nullptr, nullptr);
}

extern "C" fl_status fl_rref(const fl_split_info *info, const fl_split_out *s, uint16_t *X,
                             uint64_t ldx, const uint16_t *RD, uint64_t ldd,
                             const uint32_t *d_rank, const uint32_t *d_pivcol, fl_mode mode,
                             void *ws, size_t ws_bytes, hipStream_t stream) {
    fl_status st = fl_check_split(info, s);
    if (st != FL_OK) return st;
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_rref: bad mode");
    const uint32_t npiv = info->npiv, nB = info->nB;
    const uint32_t maxr = info->mD < nB ? info->mD : nB;
    if (npiv == 0 || nB == 0 || maxr == 0) return FL_OK;
    FL_ARG(X && RD && d_rank && d_pivcol, "fl_rref: NULL array");
    FL_ARG(ldx >= nB && ldx % 4 == 0 && ldd >= nB && ldd % 4 == 0,
           "fl_rref: ldx/ldd must be >= nB and multiples of 4");
    FL_ARG(((uintptr_t)X & 7) == 0 && ((uintptr_t)RD & 7) == 0, "fl_rref: X, RD must be 8-byte aligned");
    RrefWs r;
    size_t need = rref_layout(info, mode, ws, &r);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_rref: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    if (mode == FL_MFMA_I8) {
        // L = X[:, P_D] and R_D as limb planes; per 128-column tile of X the
        // range of R_D rows that are nonzero there
        dim3 g((unsigned)((r.kp / 4 + 255) / 256), npiv < 1024 ? npiv : 1024);
        const uint32_t mtiles = (npiv + 127) / 128;
        FL_HIP(fl_fill_u32(r.tfirst, 0xffffffffu, npiv, stream));
        FL_PROF("rref.limbs", stream, {
            hipLaunchKernelGGL(k_gather_pivcols_limbs, g, dim3(256), 0, stream, info->p, (const uint16_t *)X,
                               ldx, npiv, d_rank, d_pivcol, r.Lh, r.Ll, r.kp, r.tfirst);
            hipLaunchKernelGGL(k_tile_kbeg, dim3((mtiles + 255) / 256), dim3(256), 0, stream, npiv, mtiles,
                               (const uint32_t *)r.tfirst, (uint32_t)r.kp, r.krange_m);
            hipLaunchKernelGGL(fl_limbs_cols_kernel(), dim3(r.ntiles * 2, (unsigned)(r.kp / 64)), dim3(256), 0,
                               stream, info->p, RD, ldd, nB, maxr, d_rank, r.Rh, r.Rl, (uint32_t)r.kp,
                               (uint32_t *)nullptr);
        });
        FL_LAUNCH_CHECK("rref limbs");
        FL_HIP(fl_fill_u32(r.tmin, 0xffffffffu, r.ntiles, stream));
        FL_HIP(fl_fill_u32(r.tmax, 0, r.ntiles, stream));
        FL_PROF("rref.ranges", stream, {
            hipLaunchKernelGGL(k_rd_tile_ranges, dim3((maxr + 3) / 4), dim3(256), 0, stream, RD, ldd, nB,
                               d_rank, d_pivcol, r.tmin, r.tmax);
            hipLaunchKernelGGL(k_krange_from_t, dim3((r.ntiles + 255) / 256), dim3(256), 0, stream, r.ntiles,
                               (const uint32_t *)r.tmin, (const uint32_t *)r.tmax, (uint32_t)r.kp, r.krange);
        });
        FL_LAUNCH_CHECK("rref ranges");
        GemmPlanes gp = {r.Lh, r.Ll, r.Rh, r.Rl, r.kp, r.kp, 0, 0, 0, (uint32_t)r.kp, d_rank, r.krange_m,
                         r.krange, nullptr, X, ldx, npiv, nB};
        // groups of 4 row tiles per column tile on each XCD: the group shares
        // the column tile's R_D planes in L2 (measured: 4 beats grid order,
        // 16, and all row tiles per column)
        gp.group_m = 4;
        gp.max_wg = kGemmPerCu;  // (measured: a little faster than one workgroup per tile)
        FL_HIP(fl_mfma_gemm_planes(info->p, gp, stream, "rref.mfma"));
    } else {
        // the same zero-skipping as the MFMA form: per 128-column tile the R_D
        // rows nonzero there, per row of X its first nonzero pivot column
        FL_HIP(fl_fill_u32(r.tmin, 0xffffffffu, r.ntiles, stream));
        FL_HIP(fl_fill_u32(r.tmax, 0, r.ntiles, stream));
        FL_HIP(fl_fill_u32(r.tfirst, 0xffffffffu, npiv, stream));
        hipLaunchKernelGGL(k_rd_tile_ranges, dim3((maxr + 3) / 4), dim3(256), 0, stream, RD, ldd, nB, d_rank,
                           d_pivcol, r.tmin, r.tmax);
        hipLaunchKernelGGL(k_krange_from_t, dim3((r.ntiles + 255) / 256), dim3(256), 0, stream, r.ntiles,
                           (const uint32_t *)r.tmin, (const uint32_t *)r.tmax, (uint32_t)r.ldl, r.krange);
        dim3 g((maxr + 255) / 256, npiv < 1024 ? npiv : 1024);
        hipLaunchKernelGGL(k_gather_pivcols, g, dim3(256), 0, stream, (const uint16_t *)X, ldx, npiv,
                           d_rank, d_pivcol, r.L, r.ldl, r.tfirst);
        FL_LAUNCH_CHECK("k_gather_pivcols");
        FL_HIP(fl_gemm_sub_plain(info->p, npiv, nB, 0, d_rank, r.L, r.ldl, RD, ldd, X, ldx, stream,
                                 "rref.plain", r.krange, r.tfirst));
    }
    return FL_OK;
}

extern "C" size_t fl_rref_csr_workspace(const fl_split_info *info) {
    if (!info) return 0;
    const uint32_t maxr = info->mD < info->nB ? info->mD : info->nB;
    return csr_layout(info->npiv, maxr, nullptr, nullptr);
}

// Row counts of RREF(M) and their exclusive scan into row_ptr (device), no
// sync; c.dinfo[0] receives the total.
static fl_status csr_count_scan(const fl_split_info *info, const fl_split_out *s, const uint16_t *Xp,
                                uint64_t ldx, const uint16_t *RD, uint64_t ldd,
                                const uint32_t *d_rank, const uint32_t *d_pivcol, uint64_t *row_ptr,
                                void *ws, size_t ws_bytes, const char *who, CsrWs *cout,
                                hipStream_t stream) {
    fl_status st = fl_check_split(info, s);
    if (st != FL_OK) return st;
    FL_ARG(row_ptr && d_rank, "fl_rref_csr_size: NULL argument");
    const uint32_t npiv = info->npiv, nB = info->nB;
    const uint32_t maxr = info->mD < nB ? info->mD : nB;
    FL_ARG(npiv == 0 || nB == 0 || (Xp && ldx >= nB && ldx % 4 == 0 && ((uintptr_t)Xp & 7) == 0),
           "fl_rref_csr_size: bad X' (NULL, ldx < nB, ldx % 4, or not 8-byte aligned)");
    FL_ARG(maxr == 0 || (RD && d_pivcol && ldd >= nB && ldd % 4 == 0 && ((uintptr_t)RD & 7) == 0),
           "fl_rref_csr_size: bad R_D (NULL, ldd < nB, ldd % 4, or not 8-byte aligned)");
    CsrWs c;
    size_t need = csr_layout(npiv, maxr, ws, &c);
    if (!ws || ws_bytes < need) {
        fl_set_error((std::string(who) + ": workspace too small").c_str());
        return FL_ERR_WORKSPACE;
    }
    const size_t nrows_max = (size_t)npiv + maxr;
    FL_HIP(fl_fill_u64(c.cnt, 0, nrows_max + 1, stream));
    if (nrows_max) {
        hipLaunchKernelGGL(k_csr_count, dim3((unsigned)((nrows_max + 3) / 4)), dim3(256), 0, stream,
                           npiv, nB, (const uint32_t *)s->col_perm, Xp, ldx, RD, ldd, d_rank,
                           d_pivcol, c.cnt);
        FL_LAUNCH_CHECK("k_csr_count");
    }
    // rows beyond npiv + r have count 0, so the scan over the upper bound
    // yields row_ptr[rank] = nnz for every rank
    FL_HIP(fl_exclusive_scan_u64(c.cnt, row_ptr, nrows_max + 1, c.scantmp, c.dinfo, stream));
    *cout = c;
    return FL_OK;
}

extern "C" fl_status fl_rref_csr_size(const fl_split_info *info, const fl_split_out *s,
                                      const uint16_t *Xp, uint64_t ldx, const uint16_t *RD,
                                      uint64_t ldd, const uint32_t *d_rank,
                                      const uint32_t *d_pivcol, uint64_t *row_ptr,
                                      uint32_t *h_rank, uint64_t *h_nnz, void *ws, size_t ws_bytes,
                                      hipStream_t stream) {
    FL_ARG(h_rank && h_nnz, "fl_rref_csr_size: NULL argument");
    CsrWs c;
    fl_status st = csr_count_scan(info, s, Xp, ldx, RD, ldd, d_rank, d_pivcol, row_ptr, ws, ws_bytes,
                                  "fl_rref_csr_size", &c, stream);
    if (st != FL_OK) return st;
    const uint32_t maxr = info->mD < info->nB ? info->mD : info->nB;
    uint32_t r = 0;
    uint64_t tot = 0;
    if (maxr) FL_HIP(hipMemcpyAsync(&r, d_rank, sizeof(r), hipMemcpyDeviceToHost, stream));
    FL_HIP(hipMemcpyAsync(&tot, c.dinfo, sizeof(tot), hipMemcpyDeviceToHost, stream));
    FL_HIP(hipStreamSynchronize(stream));
    *h_rank = info->npiv + r;
    *h_nnz = tot;
    return FL_OK;
}

// ---- the read-off's size query without any allocation -------------------------
// The count/scan scratch lives in a file-scope device array (one copy per GPU,
// held until the process ends).  Host code never passes the array's name to a
// kernel: its device address is looked up once per device with
// hipGetSymbolAddress and kept here.
namespace {
constexpr size_t kCsrScratchBytes = (size_t)16 << 20;
__device__ __align__(256) unsigned char scratch[kCsrScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

fl_status csr_scratch(void **out) {
    int dev = 0;
    FL_HIP(hipGetDevice(&dev));
    FL_ARG(dev >= 0 && dev < kMaxDevices, "fl_rref_csr_size_noalloc: device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        FL_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        FL_ARG(ptr != nullptr, "fl_rref_csr_size_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FL_OK;
}
}  // namespace

extern "C" size_t fl_rref_csr_noalloc_scratch_bytes(void) { return kCsrScratchBytes; }

extern "C" fl_status fl_rref_csr_size_noalloc(const fl_split_info *info, const fl_split_out *s,
                                              const uint16_t *Xp, uint64_t ldx, const uint16_t *RD,
                                              uint64_t ldd, const uint32_t *d_rank,
                                              const uint32_t *d_pivcol, uint64_t *row_ptr,
                                              uint32_t *h_rank, uint64_t *h_nnz, hipStream_t stream) {
    fl_status st = fl_check_split(info, s);
    if (st != FL_OK) return st;
    const size_t need = fl_rref_csr_workspace(info);
    if (need > kCsrScratchBytes) {
        fl_set_error("fl_rref_csr_size_noalloc: npiv + min(mD, nB) rows need more than the 16 MiB "
                     "static scratch; use fl_rref_csr_size with a workspace");
        return FL_ERR_ARG;
    }
    void *ws = nullptr;
    st = csr_scratch(&ws);
    if (st != FL_OK) return st;
    return fl_rref_csr_size(info, s, Xp, ldx, RD, ldd, d_rank, d_pivcol, row_ptr, h_rank, h_nnz, ws,
                            kCsrScratchBytes, stream);
}

// Count, scan and emit without a host sync: col/val must hold the upper bound
// (npiv + min(mD, nB)) * (nB + 1) entries.
fl_status fl_rref_csr_enqueue(const fl_split_info *info, const fl_split_out *s, const uint16_t *Xp,
                              uint64_t ldx, const uint16_t *RD, uint64_t ldd,
                              const uint32_t *d_rank, const uint32_t *d_pivcol, uint64_t *row_ptr,
                              uint32_t *col, uint16_t *val, void *ws, size_t ws_bytes,
                              hipStream_t stream) {
    CsrWs c;
    fl_status st = csr_count_scan(info, s, Xp, ldx, RD, ldd, d_rank, d_pivcol, row_ptr, ws, ws_bytes,
                                  "fl_rref_csr_enqueue", &c, stream);
    if (st != FL_OK) return st;
    return fl_rref_to_csr(info, s, Xp, ldx, RD, ldd, d_rank, d_pivcol, row_ptr, col, val, ws, ws_bytes,
                          stream);
}

extern "C" fl_status fl_rref_to_csr(const fl_split_info *info, const fl_split_out *s,
                                    const uint16_t *Xp, uint64_t ldx, const uint16_t *RD,
                                    uint64_t ldd, const uint32_t *d_rank, const uint32_t *d_pivcol,
                                    const uint64_t *row_ptr, uint32_t *col, uint16_t *val,
                                    void *ws, size_t ws_bytes, hipStream_t stream) {
    (void)ws; (void)ws_bytes;
    fl_status st = fl_check_split(info, s);
    if (st != FL_OK) return st;
    FL_ARG(row_ptr && d_rank, "fl_rref_to_csr: NULL argument");
    const uint32_t npiv = info->npiv, nB = info->nB;
    const uint32_t maxr = info->mD < nB ? info->mD : nB;
    const size_t nrows_max = (size_t)npiv + maxr;
    if (nrows_max == 0) return FL_OK;
    FL_ARG(col && val, "fl_rref_to_csr: NULL col/val");
    FL_ARG(npiv == 0 || nB == 0 || (Xp && ldx >= nB && ldx % 4 == 0 && ((uintptr_t)Xp & 7) == 0),
           "fl_rref_to_csr: bad X' (NULL, ldx < nB, ldx % 4, or not 8-byte aligned)");
    FL_ARG(maxr == 0 || (RD && d_pivcol && ldd >= nB && ldd % 4 == 0 && ((uintptr_t)RD & 7) == 0),
           "fl_rref_to_csr: bad R_D (NULL, ldd < nB, ldd % 4, or not 8-byte aligned)");
    hipLaunchKernelGGL(k_csr_emit, dim3((unsigned)((nrows_max + 3) / 4)), dim3(256), 0, stream, npiv,
                       nB, (const uint32_t *)s->col_perm, Xp, ldx, RD, ldd, d_rank, d_pivcol,
                       row_ptr, col, val);
    FL_LAUNCH_CHECK("k_csr_emit");
    return FL_OK;
}
