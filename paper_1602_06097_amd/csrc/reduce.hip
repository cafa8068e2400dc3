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
hipError_t fl_gemm_sub_plain(uint32_t p, uint32_t M, uint32_t N, uint32_t Kh, const uint32_t *Kdev,
                             const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                             uint16_t *C, uint64_t ldc, hipStream_t s, const char *site);
hipError_t fl_gemm_sub_mfma(uint32_t p, uint32_t M, uint32_t N, uint32_t Kmax, const uint32_t *Kdev,
                            const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                            uint16_t *C, uint64_t ldc, void *ws, size_t ws_bytes, hipStream_t s,
                            const char *site);
size_t fl_gemm_sub_mfma_ws(uint32_t M, uint32_t N, uint32_t Kmax);

namespace {

// Dense rows of C from its multiline groups: out[g*w+q][pos[k]] = val[w*k+q].
__global__ __launch_bounds__(256) void k_ml_to_dense(uint32_t w, uint32_t ngroups, uint32_t rows,
                                                     const uint64_t *__restrict__ gptr,
                                                     const uint32_t *__restrict__ pos,
                                                     const uint16_t *__restrict__ val,
                                                     uint16_t *out, uint64_t ld) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t g = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (g >= ngroups) return;
    for (uint64_t k = gptr[g] + lane; k < gptr[g + 1]; k += 64) {
        const uint32_t c = pos[k];
        for (uint32_t q = 0; q < w; q++) {
            const uint32_t row = g * w + q;
            if (row < rows) out[(uint64_t)row * ld + c] = val[(uint64_t)w * k + q];
        }
    }
}

struct ReduceWs {
    uint16_t *Cd;
    uint64_t ldc;
    void *gemm_ws;
    size_t gemm_ws_bytes;
};

size_t reduce_layout(const fl_split_info *info, fl_mode mode, void *ws, ReduceWs *r) {
    WsCarve c(ws);
    ReduceWs t = {};
    if (mode == FL_MFMA_I8) {
        t.ldc = ((uint64_t)info->npiv + 63) & ~(uint64_t)63;
        t.Cd = c.take<uint16_t>((size_t)(info->mD ? info->mD : 1) * (t.ldc ? t.ldc : 64));
        t.gemm_ws_bytes = fl_gemm_sub_mfma_ws(info->mD, info->nB, info->npiv);
        t.gemm_ws = c.take<char>(t.gemm_ws_bytes);
    }
    if (r) *r = t;
    return c.off;
}

}  // namespace

extern "C" size_t fl_reduce_cd_workspace(const fl_split_info *info, fl_mode mode) {
    if (!info) return 0;
    return reduce_layout(info, mode, nullptr, nullptr);
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
    size_t need = reduce_layout(info, mode, ws, &r);
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
    FL_HIP(fl_zero_rows_u16(r.Cd, r.ldc, mD, npiv, stream));
    hipLaunchKernelGGL(k_ml_to_dense, dim3((ngroups + 3) / 4), dim3(256), 0, stream, w, ngroups, mD,
                       (const uint64_t *)s->c_gptr, (const uint32_t *)s->c_pos,
                       (const uint16_t *)s->c_val, r.Cd, r.ldc);
    FL_LAUNCH_CHECK("k_ml_to_dense");
    FL_HIP(fl_gemm_sub_mfma(info->p, mD, nB, npiv, nullptr, r.Cd, r.ldc, X, ldx, Dt, ldd, r.gemm_ws,
                            r.gemm_ws_bytes, stream, "reduce"));
    return FL_OK;
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
