// Dense contractions for Gaussian embeddings (Algorithm 1 steps 3 and 6 with
// X and Y Gaussian): C = A B with FP64 accumulation, LDS-tiled.
#include "common.h"

namespace re {

namespace {

constexpr int BM = 64, BN = 64, BK = 16;

template <typename T>
__device__ __forceinline__ double ld(const T* p) {
  return (double)*p;
}

template <typename TA, typename TB, typename TC>
__global__ void __launch_bounds__(256) k_gemm_f64acc(int64_t M, int64_t N, int64_t K, const TA* __restrict__ A,
                                                     int64_t lda, const TB* __restrict__ B, int64_t ldb,
                                                     TC* __restrict__ C, int64_t ldc) {
  __shared__ double sa[BK][BM + 1];
  __shared__ double sb[BK][BN + 1];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t m0 = (int64_t)blockIdx.y * BM, n0 = (int64_t)blockIdx.x * BN;
  double acc[4][4] = {};
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    for (int e = threadIdx.x; e < BM * BK; e += 256) {
      const int r = e / BK, c = e % BK;
      const int64_t gm = m0 + r, gk = k0 + c;
      sa[c][r] = (gm < M && gk < K) ? ld(A + gm * lda + gk) : 0.0;
    }
    for (int e = threadIdx.x; e < BK * BN; e += 256) {
      const int r = e / BN, c = e % BN;
      const int64_t gk = k0 + r, gn = n0 + c;
      sb[r][c] = (gk < K && gn < N) ? ld(B + gk * ldb + gn) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < BK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sa[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sb[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t gm = m0 + ty + 16 * i, gn = n0 + tx + 16 * j;
      if (gm < M && gn < N) C[gm * ldc + gn] = (TC)acc[i][j];
    }
}

template <typename TA, typename TB, typename TC>
re_status go(hipStream_t s, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda, const void* B, int64_t ldb,
             void* C, int64_t ldc) {
  const dim3 grid((unsigned)cdiv(N, BN), (unsigned)cdiv(M, BM));
  if (grid.y > 65535) return RE_ERR_UNSUPPORTED;
  hipLaunchKernelGGL((k_gemm_f64acc<TA, TB, TC>), grid, dim3(256), 0, s, M, N, K, (const TA*)A, lda, (const TB*)B,
                     ldb, (TC*)C, ldc);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace

re_status launch_gemm_f64acc(hipStream_t s, int64_t M, int64_t N, int64_t K, const void* A, int ta, int64_t lda,
                             const void* B, int tb, int64_t ldb, void* C, int tc, int64_t ldc) {
  if (M <= 0 || N <= 0) return RE_OK;
  const int code = ta * 100 + tb * 10 + tc;
  switch (code) {
    case 0: return go<double, double, double>(s, M, N, K, A, lda, B, ldb, C, ldc);
    case 100: return go<float, double, double>(s, M, N, K, A, lda, B, ldb, C, ldc);
    case 110: return go<float, float, double>(s, M, N, K, A, lda, B, ldb, C, ldc);
    case 111: return go<float, float, float>(s, M, N, K, A, lda, B, ldb, C, ldc);
    case 10: return go<double, float, double>(s, M, N, K, A, lda, B, ldb, C, ldc);
    default: return RE_ERR_UNSUPPORTED;
  }
}

}  // namespace re
