// reduce.hip -- FL step 3 (paper Sec. 4.1 step 3): Dt = D - C X mod p, C
// reduced to zero by the identity block with the same operations applied to
// D; and the dense form of the contraction, fl_matmul_sub.
//
//   FL_PLAIN    Dt = dense(D), then every w-multiline group of C subtracts
//               its rows times X (one load of a row of X serves the w rows).
//   FL_MFMA_I8  C is expanded to a dense mD x npiv operand and the product
//               runs on the int8 matrix cores (limb form of gemm_mfma.hip);
//               the result is bit-identical.
#include "fl_internal.h"

hipError_t fl_ml_spmm(uint32_t w, uint32_t p, const uint64_t *gptr, const uint32_t *pos,
                      const uint16_t *val, uint32_t g0, uint32_t ngroups, uint32_t row_limit,
                      uint32_t pos_lo, const uint16_t *X, uint64_t ldx, uint16_t *out,
                      uint64_t ldo, uint32_t ncols, hipStream_t s, const char *site);
hipError_t fl_csr_to_dense(uint32_t rows, uint32_t cols, const uint64_t *rp, const uint32_t *ci,
                           const uint16_t *v, uint16_t *out, uint64_t ld, hipStream_t s);
fl_status fl_check_split(const fl_split_info *info, const fl_split_out *s);
hipError_t fl_gemm_sub_mfma(uint32_t p, uint32_t M, uint32_t N, uint32_t Kmax, const uint32_t *Kdev,
                            const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                            uint16_t *C, uint64_t ldc, void *ws, size_t ws_bytes, hipStream_t s,
                            const char *site);
size_t fl_gemm_sub_mfma_ws(uint32_t M, uint32_t N, uint32_t Kmax);

namespace {

typedef void (*fl_limbs_cols_fn)(uint32_t, const uint16_t *, uint64_t, uint32_t, uint32_t,
                                 const uint32_t *, int8_t *, int8_t *, uint32_t, uint32_t *);

// ---- MFMA form: C's multiline groups sorted by first column, so that each
// 128-row tile of the dense C operand is nonzero only on a short K range ----

constexpr uint32_t kBucketShift = 6;  // rows bucketed by first column / 64

// First and last column of every row of C (from its multiline group, one wave
// per group), its bucket (empty rows go to the last bucket) and the histogram.
__global__ __launch_bounds__(256) void k_row_extent(uint32_t w, uint32_t ngroups, uint32_t mD,
                                                    uint32_t nbuckets, const uint64_t *__restrict__ gptr,
                                                    const uint32_t *__restrict__ pos,
                                                    const uint16_t *__restrict__ val, uint32_t *first,
                                                    uint32_t *last, uint32_t *bucket, uint64_t *hist) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= ngroups) return;
    const uint64_t b = gptr[g], e = gptr[g + 1];
    for (uint32_t q = 0; q < w; q++) {
        const uint32_t row = g * w + q;
        if (row >= mD) break;
        uint32_t lo = 0xffffffffu, hi = 0;
        for (uint64_t k0 = b; k0 < e; k0 += 64) {
            const uint64_t k = k0 + lane;
            const bool nz = k < e && val[(uint64_t)w * k + q] != 0;
            const uint64_t m = __ballot(nz);
            if (m) {
                const uint32_t fpos = pos[k0 + __ffsll((long long)m) - 1];
                const uint32_t lpos = pos[k0 + 63 - __clzll(m)];
                lo = fpos < lo ? fpos : lo;
                hi = lpos + 1;
            }
        }
        if (lane == 0) {
            first[row] = lo;
            last[row] = hi;
            const uint32_t bk = lo != 0xffffffffu ? (lo >> kBucketShift) : nbuckets - 1;
            bucket[row] = bk;
            atomicAdd((unsigned long long *)&hist[bk], 1ull);
        }
    }
}

// order[off[bucket] + rank within bucket] = row; rank_of[row] = its position.
__global__ void k_row_scatter(uint32_t mD, const uint32_t *__restrict__ bucket,
                              const uint64_t *__restrict__ off, uint32_t *fill, uint32_t *order,
                              uint32_t *rank_of) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= mD) return;
    const uint32_t k = bucket[r];
    const uint32_t at = (uint32_t)off[k] + atomicAdd(&fill[k], 1u);
    order[at] = r;
    rank_of[r] = at;
}

// Per tile of 128 sorted rows: the K range spanned by its rows' columns, and
// the output row of every sorted row (~0u past the last row).
__global__ void k_tile_krange(uint32_t mD, uint32_t ntiles, const uint32_t *__restrict__ order,
                              const uint32_t *__restrict__ first, const uint32_t *__restrict__ last,
                              uint32_t kp, uint32_t *krange, uint32_t *row_map) {
    const uint32_t tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= ntiles) return;
    uint32_t lo = 0xffffffffu, hi = 0;
    for (uint32_t j = 0; j < 128; j++) {
        const uint32_t s = tile * 128 + j;
        const uint32_t r = s < mD ? order[s] : 0xffffffffu;
        row_map[s] = r;
        if (r == 0xffffffffu || first[r] == 0xffffffffu) continue;
        lo = first[r] < lo ? first[r] : lo;
        hi = last[r] > hi ? last[r] : hi;
    }
    uint32_t kb = 0, ke = 0;
    if (lo != 0xffffffffu) {
        kb = lo / 64 * 64;
        ke = (hi + 63) / 64 * 64;
        if (ke > kp) ke = kp;
    }
    krange[2 * tile] = kb;
    krange[2 * tile + 1] = ke;
}

// Zero the K range of every sorted row of tile blockIdx.x (row blockIdx.y).
__global__ __launch_bounds__(256) void k_tile_zero(const uint32_t *__restrict__ krange, int8_t *Ah,
                                                   int8_t *Al, uint64_t kp) {
    const uint32_t tile = blockIdx.x, row = tile * 128 + blockIdx.y;
    const uint32_t kb = krange[2 * tile], ke = krange[2 * tile + 1];
    const uint4 z = make_uint4(0, 0, 0, 0);
    for (uint32_t k = kb + threadIdx.x * 16; k < ke; k += blockDim.x * 16) {
        *(uint4 *)(Ah + (uint64_t)row * kp + k) = z;
        *(uint4 *)(Al + (uint64_t)row * kp + k) = z;
    }
}

// Nonzero entries of group g's rows -> their sorted rows of the limb planes.
__global__ __launch_bounds__(256) void k_tile_scatter(uint32_t w, uint32_t p, uint32_t ngroups,
                                                      uint32_t mD, const uint64_t *__restrict__ gptr,
                                                      const uint32_t *__restrict__ pos,
                                                      const uint16_t *__restrict__ val,
                                                      const uint32_t *__restrict__ rank_of, int8_t *Ah,
                                                      int8_t *Al, uint64_t kp) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= ngroups) return;
    for (uint32_t q = 0; q < w; q++) {
        const uint32_t row = g * w + q;
        if (row >= mD) break;
        const uint64_t srow = rank_of[row];
        for (uint64_t k = gptr[g] + lane; k < gptr[g + 1]; k += 64) {
            const uint32_t v = val[(uint64_t)w * k + q];
            if (!v) continue;
            int h, l;
            fl_split_limbs(v, p, h, l);
            Ah[srow * kp + pos[k]] = (int8_t)h;
            Al[srow * kp + pos[k]] = (int8_t)l;
        }
    }
}

struct ReduceWs {
    int8_t *Ah, *Al, *Xh, *Xl;
    uint32_t *first, *last, *bucket, *fill, *order, *rank_of, *krange, *row_map;
    uint32_t *xend;  // per 128-column tile of X: 1 + its last nonzero row (X given as u16 only)
    uint64_t *hist, *scantmp;
    uint64_t kp;
    uint32_t ntiles, nbuckets;
};

// x_planes: the workspace holds the limb planes of X (false when the caller
// passes them in).
size_t reduce_layout(const fl_split_info *info, fl_mode mode, bool x_planes, void *ws, ReduceWs *r) {
    WsCarve c(ws);
    ReduceWs t = {};
    if (mode == FL_MFMA_I8 && info->mD && info->nB && info->npiv) {
        t.ntiles = (info->mD + 127) / 128;
        t.nbuckets = (info->npiv >> kBucketShift) + 2;
        t.kp = ((uint64_t)info->npiv + 63) / 64 * 64;
        const uint64_t mp = (uint64_t)t.ntiles * 128;
        const uint64_t np = ((uint64_t)info->nB + 127) / 128 * 128;
        t.Ah = c.take<int8_t>(mp * t.kp);
        t.Al = c.take<int8_t>(mp * t.kp);
        if (x_planes) {
            t.Xh = c.take<int8_t>(np * t.kp);
            t.Xl = c.take<int8_t>(np * t.kp);
        }
        t.first = c.take<uint32_t>(info->mD);
        t.last = c.take<uint32_t>(info->mD);
        t.bucket = c.take<uint32_t>(info->mD);
        t.fill = c.take<uint32_t>(t.nbuckets);
        t.order = c.take<uint32_t>(info->mD);
        t.rank_of = c.take<uint32_t>(info->mD);
        t.krange = c.take<uint32_t>(2 * (size_t)t.ntiles);
        if (x_planes) t.xend = c.take<uint32_t>(np / 128);
        t.row_map = c.take<uint32_t>(mp);
        t.hist = c.take<uint64_t>(t.nbuckets);
        t.scantmp = c.take<uint64_t>(fl_scan_tmp_elems(t.nbuckets));
    }
    if (r) *r = t;
    return c.off;
}

}  // namespace

fl_limbs_cols_fn fl_limbs_cols_kernel();

namespace {
// The int8-MFMA form of the reduce: C's rows sorted by first column into
// 128-row tiles with their K ranges, C as limb planes, X's limb planes (Xh,
// Xl, row stride ldp) converted from X when X is given, then Dt -= C X.
fl_status reduce_mfma(const fl_split_info *info, const fl_split_out *s, const uint16_t *X, uint64_t ldx,
                      const int8_t *Xh, const int8_t *Xl, uint64_t ldp, const uint32_t *row_end, uint16_t *Dt,
                      uint64_t ldd, const ReduceWs &r, hipStream_t stream) {
    const uint32_t mD = info->mD, nB = info->nB, npiv = info->npiv, w = info->ml_width;
    const uint32_t ngroups = (mD + w - 1) / w;
    FL_HIP(fl_fill_u64(r.hist, 0, r.nbuckets, stream));
    FL_HIP(fl_fill_u32(r.fill, 0, r.nbuckets, stream));
    FL_PROF("reduce.sort", stream, {
        hipLaunchKernelGGL(k_row_extent, dim3((ngroups + 3) / 4), dim3(256), 0, stream, w, ngroups, mD,
                           r.nbuckets, (const uint64_t *)s->c_gptr, (const uint32_t *)s->c_pos,
                           (const uint16_t *)s->c_val, r.first, r.last, r.bucket, r.hist);
        (void)fl_exclusive_scan_u64(r.hist, r.hist, r.nbuckets, r.scantmp, nullptr, stream);
        hipLaunchKernelGGL(k_row_scatter, dim3((mD + 255) / 256), dim3(256), 0, stream, mD,
                           (const uint32_t *)r.bucket, (const uint64_t *)r.hist, r.fill, r.order, r.rank_of);
        hipLaunchKernelGGL(k_tile_krange, dim3((r.ntiles + 255) / 256), dim3(256), 0, stream, mD, r.ntiles,
                           (const uint32_t *)r.order, (const uint32_t *)r.first, (const uint32_t *)r.last,
                           (uint32_t)r.kp, r.krange, r.row_map);
    });
    FL_LAUNCH_CHECK("reduce sort");
    FL_PROF("reduce.limbs", stream, {
        hipLaunchKernelGGL(k_tile_zero, dim3(r.ntiles, 128), dim3(256), 0, stream, (const uint32_t *)r.krange,
                           r.Ah, r.Al, r.kp);
        hipLaunchKernelGGL(k_tile_scatter, dim3((ngroups + 3) / 4), dim3(256), 0, stream, w, info->p, ngroups,
                           mD, (const uint64_t *)s->c_gptr, (const uint32_t *)s->c_pos,
                           (const uint16_t *)s->c_val, (const uint32_t *)r.rank_of, r.Ah, r.Al, r.kp);
        if (X) {  // X's limb planes into the workspace, with the last nonzero row per column tile
            const uint32_t np = (nB + 127) / 128 * 128;
            (void)fl_fill_u32(r.xend, 0, np / 128, stream);
            hipLaunchKernelGGL(fl_limbs_cols_kernel(), dim3(np / 64, (unsigned)(r.kp / 64)), dim3(256), 0,
                               stream, info->p, X, ldx, nB, npiv, (const uint32_t *)nullptr, r.Xh, r.Xl,
                               (uint32_t)r.kp, r.xend);
        }
    });
    FL_LAUNCH_CHECK("reduce limbs");
    GemmPlanes gp = {r.Ah, r.Al, Xh, Xl, r.kp, ldp, 0, 0, 0, (uint32_t)r.kp, nullptr, r.krange,
                     nullptr, r.row_map, Dt, ldd, r.ntiles * 128, nB};
    // column tiles of X past whose last nonzero row C's K range starts: skipped
    gp.kcap_n = X ? r.xend : row_end;
    // groups of 4 row tiles per column tile on each XCD: the group shares the
    // column tile's X planes in L2 while C's limb planes are re-read from the
    // last-level cache (measured on the 60,000 x 80,000 workload: 4 beats
    // 8, 16, 32 and all row tiles per column tile by 4-15%)
    gp.group_m = 4;
    FL_HIP(fl_mfma_gemm_planes(info->p, gp, stream, "reduce.mfma"));
    return FL_OK;
}
}  // namespace

extern "C" size_t fl_reduce_cd_workspace(const fl_split_info *info, fl_mode mode) {
    if (!info) return 0;
    return reduce_layout(info, mode, true, nullptr, nullptr);
}

extern "C" size_t fl_reduce_cd_planes_workspace(const fl_split_info *info) {
    if (!info) return 0;
    return reduce_layout(info, FL_MFMA_I8, false, nullptr, nullptr);
}

extern "C" fl_status fl_reduce_cd(const fl_split_info *info, const fl_split_out *s,
                                  const uint16_t *X, uint64_t ldx, uint16_t *Dt, uint64_t ldd,
                                  fl_mode mode, void *ws, size_t ws_bytes, hipStream_t stream) {
    fl_status st = fl_check_split(info, s);
    if (st != FL_OK) return st;
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_reduce_cd: bad mode");
    const uint32_t mD = info->mD, nB = info->nB, npiv = info->npiv, w = info->ml_width;
    if (mD == 0 || nB == 0) return FL_OK;
    FL_ARG(Dt, "fl_reduce_cd: NULL Dt");
    FL_ARG(ldd >= nB && ldd % 4 == 0, "fl_reduce_cd: ldd must be >= nB and a multiple of 4");
    FL_ARG(((uintptr_t)Dt & 7) == 0, "fl_reduce_cd: Dt must be 8-byte aligned");
    FL_ARG(npiv == 0 || (X && ldx >= nB && ldx % 4 == 0 && ((uintptr_t)X & 7) == 0),
           "fl_reduce_cd: bad X (NULL, ldx < nB, ldx % 4, or misaligned)");
    ReduceWs r;
    size_t need = reduce_layout(info, mode, true, ws, &r);
    if (need && (!ws || ws_bytes < need)) {
        fl_set_error("fl_reduce_cd: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    FL_HIP(fl_csr_to_dense(mD, nB, s->d_ptr, s->d_col, s->d_val, Dt, ldd, stream));
    if (npiv == 0) return FL_OK;
    const uint32_t ngroups = (mD + w - 1) / w;
    if (mode == FL_PLAIN) {
        FL_HIP(fl_ml_spmm(w, info->p, s->c_gptr, s->c_pos, s->c_val, 0, ngroups, mD, 0, X, ldx, Dt,
                          ldd, nB, stream, "reduce.spmm"));
        return FL_OK;
    }
    return reduce_mfma(info, s, X, ldx, r.Xh, r.Xl, r.kp, nullptr, Dt, ldd, r, stream);
}

extern "C" fl_status fl_reduce_cd_planes(const fl_split_info *info, const fl_split_out *s, const int8_t *Xh,
                                         const int8_t *Xl, uint64_t ldp, const uint32_t *row_end, uint16_t *Dt,
                                         uint64_t ldd, void *ws, size_t ws_bytes, hipStream_t stream) {
    fl_status st = fl_check_split(info, s);
    if (st != FL_OK) return st;
    const uint32_t mD = info->mD, nB = info->nB, npiv = info->npiv;
    if (mD == 0 || nB == 0) return FL_OK;
    FL_ARG(Dt, "fl_reduce_cd_planes: NULL Dt");
    FL_ARG(ldd >= nB && ldd % 4 == 0, "fl_reduce_cd_planes: ldd must be >= nB and a multiple of 4");
    FL_ARG(((uintptr_t)Dt & 7) == 0, "fl_reduce_cd_planes: Dt must be 8-byte aligned");
    FL_ARG(npiv == 0 || (Xh && Xl && ldp >= ((uint64_t)npiv + 63) / 64 * 64 && ldp % 16 == 0 &&
                         ((uintptr_t)Xh & 15) == 0 && ((uintptr_t)Xl & 15) == 0),
           "fl_reduce_cd_planes: bad planes (NULL, ldp < npiv rounded up to 64, ldp % 16, or misaligned)");
    ReduceWs r;
    size_t need = reduce_layout(info, FL_MFMA_I8, false, ws, &r);
    if (need && (!ws || ws_bytes < need)) {
        fl_set_error("fl_reduce_cd_planes: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    FL_HIP(fl_csr_to_dense(mD, nB, s->d_ptr, s->d_col, s->d_val, Dt, ldd, stream));
    if (npiv == 0) return FL_OK;
    return reduce_mfma(info, s, nullptr, 0, Xh, Xl, ldp, row_end, Dt, ldd, r, stream);
}

extern "C" size_t fl_matmul_sub_workspace(uint32_t M, uint32_t N, uint32_t K, fl_mode mode) {
    return mode == FL_MFMA_I8 ? fl_gemm_sub_mfma_ws(M, N, K) : 0;
}

extern "C" fl_status fl_matmul_sub(uint32_t p, uint32_t M, uint32_t N, uint32_t K,
                                   const uint16_t *Cm, uint64_t ldc, const uint16_t *Xm,
                                   uint64_t ldx, uint16_t *Dm, uint64_t ldd, fl_mode mode,
                                   void *ws, size_t ws_bytes, hipStream_t stream) {
    FL_ARG(p >= 2 && p <= 65521, "fl_matmul_sub: p must be in [2, 65521]");
    FL_ARG(mode == FL_PLAIN || mode == FL_MFMA_I8, "fl_matmul_sub: bad mode");
    if (M == 0 || N == 0 || K == 0) return FL_OK;
    FL_ARG(Cm && Xm && Dm, "fl_matmul_sub: NULL array");
    FL_ARG(ldc >= K && ldx >= N && ldd >= N && ldx % 4 == 0 && ldd % 4 == 0,
           "fl_matmul_sub: leading dimensions too small or not multiples of 4");
    FL_ARG(((uintptr_t)Xm & 7) == 0 && ((uintptr_t)Dm & 7) == 0,
           "fl_matmul_sub: Xm, Dm must be 8-byte aligned");
    if (mode == FL_PLAIN) {
        FL_HIP(fl_gemm_sub_plain(p, M, N, K, nullptr, Cm, ldc, Xm, ldx, Dm, ldd, stream, "matmul.plain"));
        return FL_OK;
    }
    size_t need = fl_gemm_sub_mfma_ws(M, N, K);
    if (!ws || ws_bytes < need) {
        fl_set_error("fl_matmul_sub: workspace too small");
        return FL_ERR_WORKSPACE;
    }
    FL_HIP(fl_gemm_sub_mfma(p, M, N, K, nullptr, Cm, ldc, Xm, ldx, Dm, ldd, ws, ws_bytes, stream, "matmul"));
    return FL_OK;
}
