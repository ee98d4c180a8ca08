// Hashed randomized DCT of the rows of A (the HRTT embedding X, Sec. 3.3; the
// paper's experimental X): B[i][b] = sqrt(k) sum_{j : h(j) = b} s(j) (F D a_i)_j
// with D the signs of the SRHT's X (stream 3), F the orthonormal DCT-II of
// length N (n zero-padded to a power of two, at least 2) and a CountSketch
// (bucket h(j) = floor(w0 k / 2^64), sign s(j) from the lowest bit of w1, both
// from Philox4x64-10 at counter (j, 0, 7, 0)).  The factor sqrt(k) lets every
// X kind share the estimates' 1/sqrt(k l) scale.
//
// The DCT of a row is Makhoul's: v = (a_0, a_2, ..., a_3, a_1) (even entries
// forward, odd ones backward), V = FFT_N(v), (F a)_q = c_q Re(e^{-i pi q / (2N)}
// V_q).  One workgroup per row keeps the N complex values in LDS and runs an
// in-place radix-2 decimation-in-time FFT over the bit-reversed sequence; each
// bucket's sum then runs over a fixed list of its coordinates (one thread per
// bucket), so every run gives the same bits.
#include <limits.h>

#include "common.h"
#include "hrtt.h"

namespace re {

namespace {

constexpr uint64_t kXHashStream = 7;
constexpr int kHrttThreads = 1024;

// code[j] = bucket of coordinate j, bit 31 set for a negative sign.
__global__ void k_hash_code(int64_t N, int64_t k, uint64_t seed, int32_t* __restrict__ code) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= N) return;
  const u64x4 w = philox((uint64_t)j, 0, kXHashStream, 0, seed);
  const uint64_t b = __umul64hi(w.x, (uint64_t)k);
  code[j] = (int32_t)((uint32_t)b | ((w.y & 1u) ? 0x80000000u : 0u));
}

// cnt[b] = coordinates hashed to bucket b (one thread per bucket, all N in order).
__global__ void k_hash_count(const int32_t* __restrict__ code, int64_t N, int64_t k, int32_t* __restrict__ cnt) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= k) return;
  int32_t c = 0;
  for (int64_t j = 0; j < N; ++j) c += (code[j] & 0x7fffffff) == b;
  cnt[b] = c;
}

// ptr[0..k] = exclusive prefix sums of cnt (in place: cnt has k + 1 slots).
__global__ void k_hash_scan(int32_t* __restrict__ ptr, int64_t k) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int32_t s = 0;
  for (int64_t b = 0; b < k; ++b) {
    const int32_t c = ptr[b];
    ptr[b] = s;
    s += c;
  }
  ptr[k] = s;
}

// list[ptr[b] ..] = the coordinates of bucket b in increasing order, sign bit kept.
__global__ void k_hash_fill(const int32_t* __restrict__ code, int64_t N, int64_t k, const int32_t* __restrict__ ptr,
                            int32_t* __restrict__ list) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= k) return;
  int32_t p = ptr[b];
  for (int64_t j = 0; j < N; ++j) {
    const int32_t c = code[j];
    if ((c & 0x7fffffff) == b) list[p++] = (int32_t)((uint32_t)j | ((uint32_t)c & 0x80000000u));
  }
}

// FFT twiddles W[t] = e^{-2 pi i t / N} (t < N/2) and the DCT's post-twiddles
// E[q] = e^{-i pi q / (2N)} (q < N), from FP64 sincospi rounded to FP32.
__global__ void k_dct_twiddles(int64_t N, float2* __restrict__ W, float2* __restrict__ E) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= N) return;
  double sv, cv;
  if (t < N / 2) {
    sincospi(2.0 * (double)t / (double)N, &sv, &cv);
    W[t] = make_float2((float)cv, (float)-sv);
  }
  sincospi((double)t / (2.0 * (double)N), &sv, &cv);
  E[t] = make_float2((float)cv, (float)-sv);
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

__global__ void __launch_bounds__(kHrttThreads) k_hrtt_rows(const float* __restrict__ A, int64_t m, int64_t n,
                                                            int64_t lda, int lgN, const uint32_t* __restrict__ bits,
                                                            const float2* __restrict__ W,
                                                            const float2* __restrict__ E,
                                                            const int32_t* __restrict__ ptr,
                                                            const int32_t* __restrict__ list, int64_t k, float sk,
                                                            float* __restrict__ B, int64_t ldb) {
  extern __shared__ float2 X[];  // N complex values
  const int N = 1 << lgN, half_n = N >> 1;
  const int tid = threadIdx.x, nth = blockDim.x;
  const float nrm = sqrtf(2.0f / (float)N), nrm0 = sqrtf(1.0f / (float)N);
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    const float* __restrict__ a = A + row * lda;
    // signs, Makhoul's reordering, bit-reversed placement
    for (int p = tid; p < N; p += nth) {
      const int j = p < half_n ? 2 * p : 2 * (N - 1 - p) + 1;
      float v = j < n ? a[j] : 0.0f;
      if ((bits[j >> 5] >> (j & 31)) & 1u) v = -v;
      X[__brev((unsigned)p) >> (32 - lgN)] = make_float2(v, 0.0f);
    }
    __syncthreads();
    // radix-2 decimation in time: stage s joins pairs half = 2^s apart
    for (int s = 0; s < lgN; ++s) {
      const int half = 1 << s;
      for (int u = tid; u < half_n; u += nth) {
        const int pos = u & (half - 1);
        const int i0 = ((u >> s) << (s + 1)) + pos, i1 = i0 + half;
        const float2 w = W[pos << (lgN - 1 - s)];
        const float2 x0 = X[i0], x1 = cmul(X[i1], w);
        X[i0] = make_float2(x0.x + x1.x, x0.y + x1.y);
        X[i1] = make_float2(x0.x - x1.x, x0.y - x1.y);
      }
      __syncthreads();
    }
    // DCT-II value q, kept in the real slot of X[q]
    for (int q = tid; q < N; q += nth) {
      const float2 c = X[q], e = E[q];
      X[q].x = (c.x * e.x - c.y * e.y) * (q ? nrm : nrm0);
    }
    __syncthreads();
    // CountSketch: one thread per bucket over its fixed coordinate list
    for (int64_t b = tid; b < k; b += nth) {
      float acc = 0.0f;
      const int32_t p1 = ptr[b + 1];
      for (int32_t t = ptr[b]; t < p1; ++t) {
        const int32_t c = list[t];
        const float v = X[c & 0x7fffffff].x;
        acc += c < 0 ? -v : v;
      }
      B[row * ldb + b] = acc * sk;
    }
    __syncthreads();
  }
}

}  // namespace

int64_t hrtt_npad(int64_t n) {
  const int64_t p = next_pow2(n);
  return p < 2 ? 2 : p;
}

size_t hrtt_scratch_bytes(int64_t n, int64_t k) {
  const int64_t N = hrtt_npad(n);
  return (size_t)N * 4 + (size_t)(k + 1) * 4 + (size_t)N * 4 + (size_t)N * 12 + 4 * 256;
}

re_status launch_hrtt_rows(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, int64_t k, uint64_t seed,
                           const uint32_t* sign_bits, void* scratch, float* B, int64_t ldb) {
  const int64_t N = hrtt_npad(n);
  if (N > kHrttMaxN || k < 1 || k > N) return RE_ERR_UNSUPPORTED;
  char* base = (char*)scratch;
  int32_t* code = (int32_t*)base;
  int32_t* ptr = (int32_t*)(base + ((N * 4 + 255) / 256) * 256);
  int32_t* list = (int32_t*)((char*)ptr + (((k + 1) * 4 + 255) / 256) * 256);
  float2* W = (float2*)((char*)list + ((N * 4 + 255) / 256) * 256);
  float2* E = W + N / 2;
  const unsigned gN = (unsigned)cdiv(N, 256), gk = (unsigned)cdiv(k, 256);
  hipLaunchKernelGGL(k_hash_code, dim3(gN), dim3(256), 0, s, N, k, seed, code);
  hipLaunchKernelGGL(k_hash_count, dim3(gk), dim3(256), 0, s, (const int32_t*)code, N, k, ptr);
  hipLaunchKernelGGL(k_hash_scan, dim3(1), dim3(64), 0, s, ptr, k);
  hipLaunchKernelGGL(k_hash_fill, dim3(gk), dim3(256), 0, s, (const int32_t*)code, N, k, (const int32_t*)ptr, list);
  hipLaunchKernelGGL(k_dct_twiddles, dim3(gN), dim3(256), 0, s, N, W, E);
  RE_TRY_HIP(hipGetLastError());
  int lgN = 0;
  while ((int64_t(1) << lgN) < N) ++lgN;
  const size_t lds = (size_t)N * sizeof(float2);
  if (lds > 65536)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_hrtt_rows, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = (int)((160 * 1024) / (lds + 1024));
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 2) per_cu = 2;  // 1024 threads per workgroup: two fill a CU
  int64_t grid = 256 * (int64_t)per_cu;
  if (grid > m) grid = m;
  hipLaunchKernelGGL(k_hrtt_rows, dim3((unsigned)grid), dim3(kHrttThreads), lds, s, A, m, n, lda, lgN, sign_bits,
                     (const float2*)W, (const float2*)E, (const int32_t*)ptr, (const int32_t*)list, k,
                     sqrtf((float)k), B, ldb);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
