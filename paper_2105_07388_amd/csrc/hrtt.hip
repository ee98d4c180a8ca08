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
// V_q).  One workgroup per row keeps the N complex values in LDS and runs a
// Stockham FFT of radix-16 passes (the 16-point DFTs in registers), so a row
// of 16384 takes four passes over LDS; each bucket's sum then runs over a
// fixed list of its coordinates (one thread per bucket), so every run gives
// the same bits.
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

constexpr int brev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r = (r << 1) | ((i >> b) & 1);
  return r;
}

constexpr int log2_c(int r) { return r <= 1 ? 0 : 1 + log2_c(r >> 1); }

// R-point DFT (R <= 16) in registers, in place: radix-2 decimation in time
// over values already in bit-reversed order (t[brev(r)] = input r), twiddles
// e^{-2 pi i t / 16} written out (cos and sin of multiples of pi / 8); the
// output is in natural order.
template <int R>
__device__ __forceinline__ void dft_reg(float2 (&t)[R]) {
  constexpr float c1 = 0.923879532511286756f, s1 = 0.382683432365089772f, c2 = 0.707106781186547524f;
  const float2 w16[8] = {make_float2(1.0f, 0.0f), make_float2(c1, -s1), make_float2(c2, -c2), make_float2(s1, -c1),
                         make_float2(0.0f, -1.0f), make_float2(-s1, -c1), make_float2(-c2, -c2), make_float2(-c1, -s1)};
#pragma unroll
  for (int half = 1; half < R; half *= 2)
#pragma unroll
    for (int g = 0; g < R; g += 2 * half)
#pragma unroll
      for (int pos = 0; pos < half; ++pos) {
        const float2 a = t[g + pos], b = cmul(t[g + pos + half], w16[pos * (16 / (2 * half))]);
        t[g + pos] = make_float2(a.x + b.x, a.y + b.y);
        t[g + pos + half] = make_float2(a.x - b.x, a.y - b.y);
      }
}

// One Stockham pass of radix R over the N values in LDS (natural order in,
// natural order out after the last pass): task j reads X[j + r N/R], turns it
// by e^{-2 pi i (j mod Ns) r / (Ns R)}, takes the R-point DFT and writes it to
// X[(j / Ns) Ns R + (j mod Ns) + r Ns].  All reads finish before any write.
template <int R>
__device__ __forceinline__ void stockham_pass(float2* X, int N, int Ns, int tid, int nth) {
  constexpr int TASKS = R == 16 ? 1 : R == 8 ? 2 : 4;  // tasks per thread (N <= 16384, 1024 threads)
  const int T = N / R;
  float2 v[TASKS][R];
#pragma unroll
  for (int q = 0; q < TASKS; ++q) {
    const int j = tid + q * nth;
    if (j < T) {
      const int kk = j & (Ns - 1);
      constexpr int L = log2_c(R);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][brev_c(r, L)] = X[j + r * T];  // bit-reversed for dft_reg
      if (Ns > 1) {
        const float step = 2.0f * (float)kk / (float)(Ns * R);  // exact: powers of two
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float sw, cw;
          sincospif(step * (float)r, &sw, &cw);
          v[q][brev_c(r, L)] = cmul(v[q][brev_c(r, L)], make_float2(cw, -sw));
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TASKS; ++q) {
    const int j = tid + q * nth;
    if (j < T) {
      dft_reg<R>(v[q]);
      const int kk = j & (Ns - 1);
      const int base = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) X[base + r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// Twiddles come from sincospif (FP32, within 2 ulp; the arguments are exact),
// so the FFT reads no tables.
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
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    // signed entries in Makhoul's order, natural positions (four loads in flight)
    const float* __restrict__ a = A + row * lda;
#pragma unroll
    for (int q0 = 0; q0 < kPer; q0 += 4) {
      float x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = tid + (q0 + q) * nth;
        x[q] = 0.0f;
        if (p < N) {
          const int j = p < half_n ? 2 * p : 2 * (N - 1 - p) + 1;
          if (j < n) x[q] = a[j];
          if ((bits[j >> 5] >> (j & 31)) & 1u) x[q] = -x[q];
        }
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int p = tid + (q0 + q) * nth;
        if (p < N) X[p] = make_float2(x[q], 0.0f);
      }
    }
    __syncthreads();
    // FFT_N by Stockham passes of radix 16 while 16 divides what is left, then 8, 4 or 2
    int Ns = 1, rem = N;
    while (rem > 1) {
      if (rem >= 16) {
        stockham_pass<16>(X, N, Ns, tid, nth);
        Ns *= 16;
        rem >>= 4;
      } else if (rem == 8) {
        stockham_pass<8>(X, N, Ns, tid, nth);
        Ns *= 8;
        rem = 1;
      } else if (rem == 4) {
        stockham_pass<4>(X, N, Ns, tid, nth);
        Ns *= 4;
        rem = 1;
      } else {
        stockham_pass<2>(X, N, Ns, tid, nth);
        Ns *= 2;
        rem = 1;
      }
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
