// gemm_plain.hip -- dense C = C - A B mod p on the vector ALUs (the tile is
// in valu_tile.h).
#include "fl_internal.h"
#include "valu_tile.h"

namespace {

using namespace fl_valu;

__global__ __launch_bounds__(256) void k_gemm_sub(fl::Mod md, uint32_t M, uint32_t N, uint32_t Kh,
                                                  const uint32_t *__restrict__ Kdev,
                                                  const uint16_t *__restrict__ A, uint64_t lda,
                                                  const uint16_t *__restrict__ B, uint64_t ldb,
                                                  uint16_t *C, uint64_t ldc, const uint32_t *__restrict__ krange_n,
                                                  const uint32_t *__restrict__ kfirst) {
    valu_gemm_tile(md, M, N, Kh, Kdev, A, lda, B, ldb, C, ldc, blockIdx.x, blockIdx.y, krange_n, kfirst);
}

}  // namespace

// C[M x N] -= A[M x K] B[K x N] (mod p).  K is taken from *Kdev when Kdev is
// non-NULL (a device-side size), else from Kh.  ldb, ldc multiples of 4, B and
// C 8-byte aligned; A needs no alignment.
// krange_n / kfirst: optional zero-skipping ranges (see valu_gemm_tile).
hipError_t fl_gemm_sub_plain(uint32_t p, uint32_t M, uint32_t N, uint32_t Kh, const uint32_t *Kdev,
                             const uint16_t *A, uint64_t lda, const uint16_t *B, uint64_t ldb,
                             uint16_t *C, uint64_t ldc, hipStream_t s, const char *site,
                             const uint32_t *krange_n, const uint32_t *kfirst) {
    if (M == 0 || N == 0) return hipSuccess;
    dim3 grid((N + kColsPerWave - 1) / kColsPerWave, (M + 4 * kRowsPerWave - 1) / (4 * kRowsPerWave));
    FL_PROF(site ? site : "gemm.plain", s,
            hipLaunchKernelGGL(k_gemm_sub, grid, dim3(256), 0, s, fl::make_mod(p), M, N, Kh, Kdev, A,
                               lda, B, ldb, C, ldc, krange_n, kfirst));
    return hipGetLastError();
}
