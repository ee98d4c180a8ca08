// Subsampled randomized Hadamard embeddings (Eq. (Theta) with F = H/sqrt(N)),
// applied without their scale factors:
//   X side (Algorithm 1 step 3):  B[i][t] = (H_N (d .* [a_i, 0]))[S_t]
//   Y side (Algorithm 1 step 6):  C[s][t] = (H_M (d' .* [B[:,t], 0]))[S'_s]
// H is the unnormalised Sylvester-ordered Walsh-Hadamard matrix,
// H[p][q] = (-1)^popcount(p & q); N, M are n, m rounded up to powers of two.
#include "common.h"

namespace re {

namespace {

__device__ __forceinline__ bool sign_neg(const uint32_t* bits, int64_t i) { return (bits[i >> 5] >> (i & 31)) & 1u; }

template <typename T>
__device__ __forceinline__ T apply_sign(T v, bool neg) {
  return neg ? -v : v;
}

// ---------------------------------------------------------------------------
// X side, any power-of-two N that fits the LDS: one workgroup per row, the
// padded row staged in LDS, log2(N) butterfly stages separated by barriers.
// ---------------------------------------------------------------------------
template <typename TA, typename TC>
__global__ void __launch_bounds__(256) k_srht_rows_lds(const TA* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                       int logN, const uint32_t* __restrict__ bits,
                                                       const int32_t* __restrict__ sel, int64_t k,
                                                       TC* __restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  TC* s = reinterpret_cast<TC*>(smem_raw);
  const int N = 1 << logN;
  for (int64_t i = blockIdx.x; i < m; i += gridDim.x) {
    const TA* a = A + i * lda;
    for (int j = threadIdx.x; j < N; j += blockDim.x) s[j] = (j < n) ? apply_sign<TC>((TC)a[j], sign_neg(bits, j)) : TC(0);
    for (int lh = 0; lh < logN; ++lh) {
      __syncthreads();
      const int h = 1 << lh;
      for (int p = threadIdx.x; p < (N >> 1); p += blockDim.x) {
        const int j = ((p >> lh) << (lh + 1)) | (p & (h - 1));
        const TC x = s[j], y = s[j + h];
        s[j] = x + y;
        s[j + h] = x - y;
      }
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < k; t += blockDim.x) B[i * k + t] = s[sel[t]];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Y side.  H_M = H_{M/L} (x) H_L with the row index split (hi, lo):
//   lo pass: every block of L consecutive rows is signed and transformed over
//            its L rows, in place (rows past m read as zero);
//   hi pass: C[s][t] = sum_b (-1)^popcount(hi(S'_s) & b) Z[b L + lo(S'_s)][t].
// ---------------------------------------------------------------------------
constexpr int kColTile = 64;

template <typename T>
__global__ void __launch_bounds__(256) k_srht_cols_lo(T* __restrict__ B, int64_t m, int64_t k, int logL,
                                                      const uint32_t* __restrict__ bits) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = reinterpret_cast<T*>(smem_raw);  // [L][kColTile]
  const int L = 1 << logL;
  const int64_t row0 = (int64_t)blockIdx.x * L;
  const int64_t c0 = (int64_t)blockIdx.y * kColTile;
  const int tc = threadIdx.x % kColTile, tr = threadIdx.x / kColTile, rstep = blockDim.x / kColTile;
  const int64_t col = c0 + tc;
  for (int r = tr; r < L; r += rstep) {
    const int64_t row = row0 + r;
    T v = T(0);
    if (row < m && col < k) v = apply_sign<T>(B[row * k + col], sign_neg(bits, row));
    s[r * kColTile + tc] = v;
  }
  for (int lh = 0; lh < logL; ++lh) {
    __syncthreads();
    const int h = 1 << lh;
    for (int e = threadIdx.x; e < (L >> 1) * kColTile; e += blockDim.x) {
      const int c = e % kColTile, p = e / kColTile;
      const int j = ((p >> lh) << (lh + 1)) | (p & (h - 1));
      const T x = s[j * kColTile + c], y = s[(j + h) * kColTile + c];
      s[j * kColTile + c] = x + y;
      s[(j + h) * kColTile + c] = x - y;
    }
  }
  __syncthreads();
  if (col < k)
    for (int r = tr; r < L; r += rstep) B[(row0 + r) * k + col] = s[r * kColTile + tc];
}

template <typename T>
__global__ void __launch_bounds__(256) k_srht_cols_hi(const T* __restrict__ Z, int64_t nblk, int64_t k, int logL,
                                                      const int32_t* __restrict__ sel, int64_t l,
                                                      double* __restrict__ C) {
  const int64_t total = l * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / k, t = e - s * k;
    const int64_t idx = sel[s];
    const int64_t hi = idx >> logL, lo = idx & ((int64_t(1) << logL) - 1);
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) {
      const double z = (double)Z[((b << logL) + lo) * k + t];
      acc += (__popcll((unsigned long long)(hi & b)) & 1) ? -z : z;
    }
    C[e] = acc;
  }
}

int lds_limit() { return 160 * 1024; }

template <typename K>
re_status allow_lds(K kernel, size_t bytes) {
  if (bytes > (size_t)lds_limit()) return RE_ERR_UNSUPPORTED;
  if (bytes > 64 * 1024)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  return RE_OK;
}

}  // namespace

re_status launch_srht_rows(hipStream_t s, const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                           const uint32_t* bits, const int32_t* sel, int64_t k, void* B) {
  const int64_t N = next_pow2(n);
  const int logN = ilog2_exact(N);
  const int grid = (int)(m < 8192 ? m : 8192);
  if (m <= 0) return RE_OK;
  if (dtype == RE_F32) {
    const size_t lds = (size_t)N * sizeof(float);
    RE_TRY(allow_lds(k_srht_rows_lds<float, float>, lds));
    hipLaunchKernelGGL((k_srht_rows_lds<float, float>), dim3(grid), dim3(256), lds, s, (const float*)A, m, n, lda,
                       logN, bits, sel, k, (float*)B);
  } else {
    const size_t lds = (size_t)N * sizeof(double);
    RE_TRY(allow_lds(k_srht_rows_lds<double, double>, lds));
    hipLaunchKernelGGL((k_srht_rows_lds<double, double>), dim3(grid), dim3(256), lds, s, (const double*)A, m, n, lda,
                       logN, bits, sel, k, (double*)B);
  }
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

static int cols_logL(int64_t m) {
  const int logM = ilog2_exact(next_pow2(m));
  return logM < 8 ? logM : 8;
}

size_t srht_cols_rows_alloc(int64_t m) {
  const int64_t L = int64_t(1) << cols_logL(m);
  return (size_t)(cdiv(m, L) * L);
}

re_status launch_srht_cols(hipStream_t s, void* B, int bdtype, int64_t m, int64_t k, const uint32_t* bits,
                           const int32_t* sel, int64_t l, double* C) {
  if (m <= 0 || k <= 0 || l <= 0) return RE_OK;
  const int logL = cols_logL(m);
  const int64_t L = int64_t(1) << logL;
  const int64_t nblk = cdiv(m, L);
  const dim3 glo((unsigned)nblk, (unsigned)cdiv(k, kColTile));
  const int64_t total = l * k;
  const int ghi = (int)(cdiv(total, 256) < 65536 ? cdiv(total, 256) : 65536);
  if (bdtype == RE_F32) {
    const size_t lds = (size_t)L * kColTile * sizeof(float);
    RE_TRY(allow_lds(k_srht_cols_lo<float>, lds));
    hipLaunchKernelGGL(k_srht_cols_lo<float>, glo, dim3(256), lds, s, (float*)B, m, k, logL, bits);
    hipLaunchKernelGGL(k_srht_cols_hi<float>, dim3(ghi), dim3(256), 0, s, (const float*)B, nblk, k, logL, sel, l, C);
  } else {
    const size_t lds = (size_t)L * kColTile * sizeof(double);
    RE_TRY(allow_lds(k_srht_cols_lo<double>, lds));
    hipLaunchKernelGGL(k_srht_cols_lo<double>, glo, dim3(256), lds, s, (double*)B, m, k, logL, bits);
    hipLaunchKernelGGL(k_srht_cols_hi<double>, dim3(ghi), dim3(256), 0, s, (const double*)B, nblk, k, logL, sel, l,
                       C);
  }
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
