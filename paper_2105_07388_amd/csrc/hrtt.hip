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

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Twiddles come from sincospif (FP32, within 2 ulp; the arguments t / N are
// exact), so the FFT needs no table reads; the next row's entries are loaded
// into registers while the current row is transformed.
__global__ void __launch_bounds__(kHrttThreads) k_hrtt_rows(const float* __restrict__ A, int64_t m, int64_t n,
                                                            int64_t lda, int lgN, const uint32_t* __restrict__ bits,
                                                            const int32_t* __restrict__ ptr,
                                                            const int32_t* __restrict__ list, int64_t k, float sk,
                                                            float* __restrict__ B, int64_t ldb) {
  extern __shared__ float2 X[];  // N complex values
  constexpr int kPer = kHrttMaxN / kHrttThreads;  // entries of a row per thread at most
  const int N = 1 << lgN, half_n = N >> 1;
  const int tid = threadIdx.x, nth = blockDim.x;
  const float nrm = sqrtf(2.0f / (float)N), nrm0 = sqrtf(1.0f / (float)N);
  const float inv_n = 1.0f / (float)N;
  // signed entries of one row in Makhoul's order: thread tid holds positions tid + q nth
  float v[kPer];
  auto load_row = [&](int64_t row) {
    const float* __restrict__ a = A + row * lda;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int p = tid + q * nth;
      float x = 0.0f;
      if (p < N) {
        const int j = p < half_n ? 2 * p : 2 * (N - 1 - p) + 1;
        if (j < n) x = a[j];
        if ((bits[j >> 5] >> (j & 31)) & 1u) x = -x;
      }
      v[q] = x;
    }
  };
  int64_t row = blockIdx.x;
  if (row < m) load_row(row);
  for (; row < m; row += gridDim.x) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int p = tid + q * nth;
      if (p < N) X[__brev((unsigned)p) >> (32 - lgN)] = make_float2(v[q], 0.0f);
    }
    __syncthreads();
    if (row + gridDim.x < m) load_row(row + gridDim.x);  // in flight during the transform
    // radix-2 decimation in time: stage s joins pairs half = 2^s apart with
    // twiddle e^{-2 pi i pos / 2^(s+1)}
    for (int s = 0; s < lgN; ++s) {
      const int half = 1 << s;
      const float tw = 1.0f / (float)half;  // twiddle angle step in units of pi
      for (int u = tid; u < half_n; u += nth) {
        const int pos = u & (half - 1);
        const int i0 = ((u >> s) << (s + 1)) + pos, i1 = i0 + half;
        float sw, cw;
        sincospif((float)pos * tw, &sw, &cw);
        const float2 w = make_float2(cw, -sw);
        const float2 x0 = X[i0], x1 = cmul(X[i1], w);
        X[i0] = make_float2(x0.x + x1.x, x0.y + x1.y);
        X[i1] = make_float2(x0.x - x1.x, x0.y - x1.y);
      }
      __syncthreads();
    }
    // DCT-II value q = c_q Re(e^{-i pi q / (2N)} V_q), kept in the real slot of X[q]
    for (int q = tid; q < N; q += nth) {
      float se, ce;
      sincospif(0.5f * (float)q * inv_n, &se, &ce);
      const float2 c = X[q];
      X[q].x = (c.x * ce + c.y * se) * (q ? nrm : nrm0);
    }
    __syncthreads();
    // CountSketch: one thread per bucket over its fixed coordinate list
    for (int64_t b = tid; b < k; b += nth) {
      float acc = 0.0f;
      const int32_t p1 = ptr[b + 1];
      int32_t t = ptr[b];
      for (; t + 3 < p1; t += 4) {  // four list entries in flight, same summation order
        int32_t c[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] = list[t + q];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float x = X[c[q] & 0x7fffffff].x;
          acc += c[q] < 0 ? -x : x;
        }
      }
      for (; t < p1; ++t) {
        const int32_t c = list[t];
        const float x = X[c & 0x7fffffff].x;
        acc += c < 0 ? -x : x;
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
  return (size_t)N * 4 + (size_t)(k + 1) * 4 + (size_t)N * 4 + 3 * 256;
}

re_status launch_hrtt_rows(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, int64_t k, uint64_t seed,
                           const uint32_t* sign_bits, void* scratch, float* B, int64_t ldb) {
  const int64_t N = hrtt_npad(n);
  if (N > kHrttMaxN || k < 1 || k > N) return RE_ERR_UNSUPPORTED;
  char* base = (char*)scratch;
  int32_t* code = (int32_t*)base;
  int32_t* ptr = (int32_t*)(base + ((N * 4 + 255) / 256) * 256);
  int32_t* list = (int32_t*)((char*)ptr + (((k + 1) * 4 + 255) / 256) * 256);
  const unsigned gN = (unsigned)cdiv(N, 256), gk = (unsigned)cdiv(k, 256);
  hipLaunchKernelGGL(k_hash_code, dim3(gN), dim3(256), 0, s, N, k, seed, code);
  hipLaunchKernelGGL(k_hash_count, dim3(gk), dim3(256), 0, s, (const int32_t*)code, N, k, ptr);
  hipLaunchKernelGGL(k_hash_scan, dim3(1), dim3(64), 0, s, ptr, k);
  hipLaunchKernelGGL(k_hash_fill, dim3(gk), dim3(256), 0, s, (const int32_t*)code, N, k, (const int32_t*)ptr, list);
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
                     (const int32_t*)ptr, (const int32_t*)list, k, sqrtf((float)k), B, ldb);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
