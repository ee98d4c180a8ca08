// Subsampled randomized Hadamard embeddings (Eq. (Theta) with F = H/sqrt(N)),
// applied without their scale factors:
//   X side (Algorithm 1 step 3):  B[i][t] = (H_N (d .* [a_i, 0]))[S_t]
//   Y side (Algorithm 1 step 6):  C[s][t] = (H_M (d' .* [B[:,t], 0]))[S'_s]
// H is the unnormalised Sylvester-ordered Walsh-Hadamard matrix,
// H[p][q] = (-1)^popcount(p & q); N, M are n, m rounded up to powers of two.
#include <stdlib.h>
#include <string.h>

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

// Rows longer than the LDS holds, N' = 2^(logN + logH): one work item per
// (row, c < 2^logH) builds v_c[j] = sum_h (-1)^popcount(c & h) (d .* a)[h N + j]
// (the Kronecker split H_N' = H_{2^logH} (x) H_N), transforms it in LDS and
// writes the sampled outputs at positions c N + p.  Item u is (row, c) with
// row = 8 (u / 2^(logH+3)) + u mod 8 and c = (u / 8) mod 2^logH: the items of a
// row are 8 apart, so under a grid that is a multiple of 8 (workgroup b runs on
// XCD b mod 8) they run side by side on one XCD and share its L2.
__device__ __forceinline__ bool sub_item(int64_t u, int64_t m, int logH, int64_t& row, int& c) {
  const int64_t slot = u >> 3;
  c = (int)(slot & ((1 << logH) - 1));
  row = ((slot >> logH) << 3) | (u & 7);
  return row < m;
}

template <typename T>
__global__ void __launch_bounds__(256) k_srht_rows_lds_sub(const T* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                           int logN, int logH, const uint32_t* __restrict__ bits,
                                                           const int32_t* __restrict__ sel, int64_t k,
                                                           T* __restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* s = reinterpret_cast<T*>(smem_raw);
  const int N = 1 << logN;
  const int64_t items = (((m + 7) >> 3) << 3) << logH;
  for (int64_t u = blockIdx.x; u < items; u += gridDim.x) {
    int64_t i;
    int c;
    if (!sub_item(u, m, logH, i, c)) continue;  // uniform over the workgroup
    const T* a = A + i * lda;
    for (int j = threadIdx.x; j < N; j += blockDim.x) {
      T acc = T(0);
      for (int h = 0; h < (1 << logH); ++h) {
        const int64_t q = ((int64_t)h << logN) + j;
        if (q >= n) break;
        const T v = apply_sign<T>(a[q], sign_neg(bits, q));
        acc += (__popc(c & h) & 1) ? -v : v;
      }
      s[j] = acc;
    }
    for (int lh = 0; lh < logN; ++lh) {
      __syncthreads();
      const int h = 1 << lh;
      for (int p = threadIdx.x; p < (N >> 1); p += blockDim.x) {
        const int j = ((p >> lh) << (lh + 1)) | (p & (h - 1));
        const T x = s[j], y = s[j + h];
        s[j] = x + y;
        s[j + h] = x - y;
      }
    }
    __syncthreads();
    for (int64_t t = threadIdx.x; t < k; t += blockDim.x) {
      const int p = sel[t];
      if ((p >> logN) == c) B[i * k + t] = s[p & (N - 1)];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// X side, N = 2^14 FP32 rows (the streaming pass that dominates the method):
// 256 threads, 64 values per thread, no padding (n = N).
//   load     thread t reads float4 chunks t + 256 j (j < 16): it holds the
//            positions q = 1024 j + 4 t + c, so its register bits are q's bits
//            {0, 1, 10..13}; signs are XOR masks prepared once per thread;
//   phase 1  the six butterfly stages over those bits, in registers;
//   LDS      the row is written to LDS at f(q) = q ^ (((q >> 8) & 15) << 2),
//            a bijection that keeps both access patterns below free of bank
//            conflicts for 32- and 64-bank LDS;
//   phase 2  thread t re-reads the 64 positions whose bits {2..7} vary
//            (the others fixed by t) and applies those six stages in place;
//   output   only the k sampled outputs are completed: each needs the four
//            values that differ in bits {8, 9} (the last two stages).
// ---------------------------------------------------------------------------
constexpr int kN14 = 1 << 14;

__device__ __forceinline__ int lds_swz14(int q) { return q ^ (((q >> 8) & 15) << 2); }

typedef float fx4 __attribute__((ext_vector_type(4)));

// 16-byte load of data read exactly once (non-temporal hint).
__device__ __forceinline__ fx4 ld_stream(const float* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const fx4*>(p));
}

__device__ __forceinline__ void fwht64(float* x) {
#pragma unroll
  for (int h = 1; h < 64; h <<= 1) {
#pragma unroll
    for (int e = 0; e < 64; ++e) {
      if (!(e & h)) {
        const float a = x[e], b = x[e | h];
        x[e] = a + b;
        x[e | h] = a - b;
      }
    }
  }
}

__global__ void __launch_bounds__(256, 2) k_srht_rows_n14(const float* __restrict__ A, int64_t m, int64_t lda,
                                                          const uint32_t* __restrict__ bits,
                                                          const int32_t* __restrict__ sel, int k,
                                                          float* __restrict__ B) {
  __shared__ __align__(16) float lds[kN14];
  const int t = threadIdx.x, w = t >> 6;
  uint32_t msk[64];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint32_t wb = bits[32 * j + (t >> 3)] >> (4 * (t & 7));
#pragma unroll
    for (int c = 0; c < 4; ++c) msk[4 * j + c] = ((wb >> c) & 1u) << 31;
  }
  int wa[4];  // phase-1 store address of chunk j is wa[j & 3] + 1024 j
#pragma unroll
  for (int r = 0; r < 4; ++r) wa[r] = (4 * t) ^ ((4 * r + w) << 2);
  const int base = (t & 3) + 256 * ((t >> 2) & 3) + 1024 * (t >> 4);
  const int sw = ((t >> 2) & 3) | (((t >> 4) & 3) << 2);
  int ra[16];  // phase-2 address of value u = 16 h + i is ra[i] + 64 h
#pragma unroll
  for (int i = 0; i < 16; ++i) ra[i] = base + 4 * (i ^ sw);

  // software pipeline: the loads of the next row are issued as soon as the
  // current row has left the registers for LDS, so they overlap phase 2,
  // the output step and the barriers
  float x[64];
  int64_t row = blockIdx.x;
  if (row < m) {
    const float* src = A + row * lda + 4 * t;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const fx4 v = ld_stream(src + 1024 * j);
      x[4 * j + 0] = v.x;
      x[4 * j + 1] = v.y;
      x[4 * j + 2] = v.z;
      x[4 * j + 3] = v.w;
    }
  }
  for (; row < m; row += gridDim.x) {
#pragma unroll
    for (int e = 0; e < 64; ++e) x[e] = __uint_as_float(__float_as_uint(x[e]) ^ msk[e]);
    fwht64(x);
#pragma unroll
    for (int j = 0; j < 16; ++j)
      *reinterpret_cast<float4*>(&lds[wa[j & 3] + 1024 * j]) = make_float4(x[4 * j], x[4 * j + 1], x[4 * j + 2], x[4 * j + 3]);
    const int64_t next = row + gridDim.x;
    if (next < m) {
      const float* src = A + next * lda + 4 * t;
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const fx4 v = ld_stream(src + 1024 * j);
        x[4 * j + 0] = v.x;
        x[4 * j + 1] = v.y;
        x[4 * j + 2] = v.z;
        x[4 * j + 3] = v.w;
      }
    }
    __syncthreads();
    float y[64];
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) y[16 * h + i] = lds[ra[i] + 64 * h];
    fwht64(y);
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[ra[i] + 64 * h] = y[16 * h + i];
    __syncthreads();
    for (int s = t; s < k; s += 256) {
      const int p = sel[s];
      const int ph = (p >> 8) & 3, pl = p & ~0x300;
      const float v0 = lds[lds_swz14(pl)], v1 = lds[lds_swz14(pl | 0x100)];
      const float v2 = lds[lds_swz14(pl | 0x200)], v3 = lds[lds_swz14(pl | 0x300)];
      // (H_4 [v0 v1 v2 v3])[ph] with the Sylvester signs (-1)^popcount(ph & b)
      const float a01 = (ph & 1) ? v0 - v1 : v0 + v1;
      const float a23 = (ph & 1) ? v2 - v3 : v2 + v3;
      B[row * k + s] = (ph & 2) ? a01 - a23 : a01 + a23;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// X side, N = 2^14 FP32 rows, 512 threads with 32 values each (twice the
// wavefronts per CU of the kernel above, at most 128 VGPRs):
//   load     thread t holds q = 2048 j + 4 t + c (j < 8): register bits {0, 1, 11, 12, 13};
//   phase 1  those five butterfly stages in registers;
//   LDS      f(q) = q ^ (((q >> 7) & 15) << 2), conflict-free for both patterns;
//   phase 2  thread t holds the 32 positions whose bits {2..6} vary: five stages;
//   output   bits {7..10} are finished only for the k sampled outputs: each sums
//            its 16 partial values with the Sylvester signs of its bits 7..10.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void fwht32(float* x) {
#pragma unroll
  for (int h = 1; h < 32; h <<= 1) {
#pragma unroll
    for (int e = 0; e < 32; ++e) {
      if (!(e & h)) {
        const float a = x[e], b = x[e | h];
        x[e] = a + b;
        x[e | h] = a - b;
      }
    }
  }
}

__global__ void __launch_bounds__(512, 2) __attribute__((amdgpu_waves_per_eu(4))) k_srht_rows_n14w(const float* __restrict__ A, int64_t m, int64_t lda,
                                                           const uint32_t* __restrict__ bits,
                                                           const int32_t* __restrict__ sel, int k,
                                                           float* __restrict__ B) {
  __shared__ __align__(16) float lds[kN14];
  const int t = threadIdx.x;
  uint32_t msk = 0;  // bit 4 j + c: sign of position 2048 j + 4 t + c
#pragma unroll
  for (int j = 0; j < 8; ++j) msk |= ((bits[64 * j + (t >> 3)] >> (4 * (t & 7))) & 15u) << (4 * j);
  const int wa = (4 * t) ^ (((t >> 5) & 15) << 2);  // phase-1 store of chunk j at wa + 2048 j
  const int base = (t & 3) + 128 * ((t >> 2) & 15) + 2048 * (t >> 6);
  const int sw = (t >> 2) & 15;
  int ra[16];  // phase-2 value u = 16 h + i lives at ra[i] + 64 h
#pragma unroll
  for (int i = 0; i < 16; ++i) ra[i] = base + 4 * (i ^ sw);
  // this thread's sampled output (k <= 512): its 16 partial values and their signs
  const bool has = t < k;
  int pa[16];
  uint32_t sgn = 0;
  {
    const int p = has ? sel[t] : 0;
    const int pl = p & ~(15 << 7), ph = (p >> 7) & 15;
#pragma unroll
    for (int b = 0; b < 16; ++b) {
      pa[b] = (pl ^ (b << 2)) + 128 * b;
      sgn |= (uint32_t)(__popc(ph & b) & 1) << b;
    }
  }
  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    const float* src = A + row * lda + 4 * t;
    float x[32];
    // keep the 32 shifted sign masks from being hoisted into 32 live registers
    asm volatile("" : "+v"(msk));
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const fx4 v = ld_stream(src + 2048 * j);
      x[4 * j + 0] = v.x;
      x[4 * j + 1] = v.y;
      x[4 * j + 2] = v.z;
      x[4 * j + 3] = v.w;
    }
#pragma unroll
    for (int e = 0; e < 32; ++e) x[e] = __uint_as_float(__float_as_uint(x[e]) ^ ((msk << (31 - e)) & 0x80000000u));
    fwht32(x);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      *reinterpret_cast<float4*>(&lds[wa + 2048 * j]) = make_float4(x[4 * j], x[4 * j + 1], x[4 * j + 2], x[4 * j + 3]);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) x[16 * h + i] = lds[ra[i] + 64 * h];
    fwht32(x);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[ra[i] + 64 * h] = x[16 * h + i];
    __syncthreads();
    if (has) {
      float v[16];
#pragma unroll
      for (int b = 0; b < 16; ++b) v[b] = __uint_as_float(__float_as_uint(lds[pa[b]]) ^ (((sgn >> b) & 1u) << 31));
#pragma unroll
      for (int w = 8; w > 0; w >>= 1)
#pragma unroll
        for (int b = 0; b < w; ++b) v[b] += v[b + w];
      B[row * k + t] = v[0];
    }
    for (int s = t + 512; s < k; s += 512) {  // samples beyond the first 512
      const int p = sel[s];
      const int pl = p & ~(15 << 7), ph = (p >> 7) & 15;
      float acc = 0.0f;
      for (int b = 0; b < 16; ++b) {
        const float val = lds[(pl ^ (b << 2)) + 128 * b];
        acc += (__popc(ph & b) & 1) ? -val : val;
      }
      B[row * k + s] = acc;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// X side, FP32 rows of any N = 2^P with 11 <= P <= 15 (zero-padded when
// n < N): the scheme above with NT = N / 32 threads of 32 values each.
//   load     thread t reads float4 chunks at 4 t + (N / 8) j (j < 8): its
//            register bits are q's bits {0, 1, P-3, P-2, P-1};
//   phase 1  those five stages in registers;
//   LDS      f(q) = q ^ (((q >> 7) & SWM) << 2) with SWM covering
//            min(P - 10, 4) bits: the bits 7.. that phase 2 takes from t;
//   phase 2  thread t holds the 32 positions whose bits {2..6} vary (its
//            other bits: {0, 1} from t bits 0-1, {7 .. P-4} from t bits
//            2 .. P-9, {P-3 .. P-1} from the top three bits of t): five stages;
//   output   bits {7 .. P-4} are finished only for the k sampled outputs,
//            each a signed sum of its 2^(P-10) partial values.
//
// Longer rows (SUB, N' = 2^(P + logH) > 2^15): H_N' = H_{2^logH} (x) H_N, so
// the sampled output at position c N + p (c < 2^logH, p < N) is entry p of
// H_N v_c, v_c[j] = sum_h (-1)^popcount(c & h) (d .* a)[h N + j].  Each work
// item is one (row, c): it accumulates v_c chunk by chunk (reading the whole
// row), transforms it as above and keeps the samples that fall in chunk c.
// The 2^logH items of a row are numbered 8 apart, so with a grid that is a
// multiple of 8 they run side by side on one XCD and all but the first read
// of the row are served from that XCD's L2.
// ---------------------------------------------------------------------------
template <int P, bool PADDED, bool SUB>
__global__ void __launch_bounds__(1 << (P - 5)) k_srht_rows_reg(const float* __restrict__ A, int64_t m, int64_t n,
                                                               int64_t lda, const uint32_t* __restrict__ bits,
                                                               const int32_t* __restrict__ sel, int k,
                                                               float* __restrict__ B, int logH) {
  constexpr int N = 1 << P, NT = N >> 5, CS = N >> 3;
  constexpr int NB = P - 10;                      // unresolved bits 7 .. P-4
  constexpr int SWB = NB < 4 ? NB : 4, SWM = (1 << SWB) - 1;
  __shared__ __align__(16) float lds[N];
  const int t = threadIdx.x;
  uint32_t msk = 0;  // bit 4 j + c: sign of position CS j + 4 t + c
  if constexpr (!SUB) {
#pragma unroll
    for (int j = 0; j < 8; ++j) msk |= ((bits[(CS >> 5) * j + (t >> 3)] >> (4 * (t & 7))) & 15u) << (4 * j);
  }
  const int wa = (4 * t) ^ (((t >> 5) & SWM) << 2);  // phase-1 store of chunk j at wa + CS j
  const int base = (t & 3) + 128 * ((t >> 2) & ((1 << NB) - 1)) + CS * (t >> (P - 8));
  const int sw = (t >> 2) & SWM;
  int ra[16];  // phase-2 value u = 16 h + i lives at ra[i] + 64 h
#pragma unroll
  for (int i = 0; i < 16; ++i) ra[i] = base + 4 * (i ^ sw);
  const int64_t items = SUB ? (((m + 7) >> 3) << 3) << logH : m;
  for (int64_t u = blockIdx.x; u < items; u += gridDim.x) {
    int64_t row = u;
    int cc = 0;  // SUB: which chunk of the long row's outputs this item produces
    if constexpr (SUB) {
      if (!sub_item(u, m, logH, row, cc)) continue;  // uniform over the workgroup
    }
    float x[32];
    if constexpr (!SUB) {
      const float* src = A + row * lda + 4 * t;
      asm volatile("" : "+v"(msk));
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        fx4 v;
        if constexpr (PADDED) {
          const int64_t q0 = 4 * t + (int64_t)CS * j;
          if (q0 + 3 < n) {
            v = *reinterpret_cast<const fx4*>(src + CS * j);
          } else {
            v = fx4{0.f, 0.f, 0.f, 0.f};
            for (int c = 0; c < 4; ++c)
              if (q0 + c < n) v[c] = src[CS * j + c];
          }
        } else {
          v = ld_stream(src + CS * j);
        }
        x[4 * j + 0] = v.x;
        x[4 * j + 1] = v.y;
        x[4 * j + 2] = v.z;
        x[4 * j + 3] = v.w;
      }
#pragma unroll
      for (int e = 0; e < 32; ++e) x[e] = __uint_as_float(__float_as_uint(x[e]) ^ ((msk << (31 - e)) & 0x80000000u));
    } else {
#pragma unroll
      for (int e = 0; e < 32; ++e) x[e] = 0.0f;
      for (int h = 0; h < (1 << logH); ++h) {
        const int64_t qh = (int64_t)h << P;  // chunk h of the long row
        if (qh >= n) break;                  // the rest is padding
        const float* src = A + row * lda + qh + 4 * t;
        uint32_t mh = 0;
#pragma unroll
        for (int j = 0; j < 8; ++j)
          mh |= ((bits[(qh >> 5) + (CS >> 5) * j + (t >> 3)] >> (4 * (t & 7))) & 15u) << (4 * j);
        if (__popc(cc & h) & 1) mh = ~mh;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          fx4 v;
          const int64_t q0 = qh + 4 * t + (int64_t)CS * j;
          if (!PADDED || q0 + 3 < n) {
            v = *reinterpret_cast<const fx4*>(src + CS * j);
          } else {
            v = fx4{0.f, 0.f, 0.f, 0.f};
            for (int c = 0; c < 4; ++c)
              if (q0 + c < n) v[c] = src[CS * j + c];
          }
#pragma unroll
          for (int c = 0; c < 4; ++c)
            x[4 * j + c] += __uint_as_float(__float_as_uint(v[c]) ^ ((mh << (31 - (4 * j + c))) & 0x80000000u));
        }
      }
    }
    fwht32(x);
#pragma unroll
    for (int j = 0; j < 8; ++j)
      *reinterpret_cast<float4*>(&lds[wa + CS * j]) = make_float4(x[4 * j], x[4 * j + 1], x[4 * j + 2], x[4 * j + 3]);
    __syncthreads();
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) x[16 * h + i] = lds[ra[i] + 64 * h];
    fwht32(x);
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int i = 0; i < 16; ++i) lds[ra[i] + 64 * h] = x[16 * h + i];
    __syncthreads();
    for (int s = t; s < k; s += NT) {
      int p = sel[s];
      if constexpr (SUB) {
        if ((p >> P) != cc) continue;
        p &= N - 1;
      }
      const int pl = p & ~(((1 << NB) - 1) << 7), ph = (p >> 7) & ((1 << NB) - 1);
      float v[1 << NB];
#pragma unroll
      for (int b = 0; b < (1 << NB); ++b) {
        const float val = lds[(pl ^ ((b & SWM) << 2)) + 128 * b];
        v[b] = __uint_as_float(__float_as_uint(val) ^ ((uint32_t)(__popc(ph & b) & 1) << 31));
      }
#pragma unroll
      for (int w = (1 << NB) >> 1; w > 0; w >>= 1)
#pragma unroll
        for (int b = 0; b < w; ++b) v[b] += v[b + w];
      B[row * k + s] = v[0];
    }
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
__global__ void __launch_bounds__(256) k_srht_cols_lo(T* __restrict__ B, int64_t m, int64_t k, int64_t ldb,
                                                      int logL, const uint32_t* __restrict__ bits) {
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
    if (row < m && col < k) v = apply_sign<T>(B[row * ldb + col], sign_neg(bits, row));
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
    for (int r = tr; r < L; r += rstep) B[(row0 + r) * ldb + col] = s[r * kColTile + tc];
}

template <typename T>
__global__ void __launch_bounds__(256) k_srht_cols_hi(const T* __restrict__ Z, int64_t nblk, int64_t k, int64_t ldz,
                                                      int logL, const int32_t* __restrict__ sel, int64_t l,
                                                      double* __restrict__ C) {
  const int64_t total = l * k;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / k, t = e - s * k;
    const int64_t idx = sel[s];
    const int64_t hi = idx >> logL, lo = idx & ((int64_t(1) << logL) - 1);
    double acc = 0.0;
    for (int64_t b = 0; b < nblk; ++b) {
      const double z = (double)Z[((b << logL) + lo) * ldz + t];
      acc += (__popcll((unsigned long long)(hi & b)) & 1) ? -z : z;
    }
    C[e] = acc;
  }
}

// ---------------------------------------------------------------------------
// Y side, FP32 with L = 256 and four-column vectors: the same butterflies and
// the same block sums as the two kernels above, in the same order (identical
// results), arranged so that every thread issues all of its loads at once.
//   lo: a workgroup owns 256 rows x 64 columns.  Thread (q = tid & 15,
//       g = tid >> 4) first holds rows 16 g + i (i < 16) of columns 4q..4q+3
//       and runs the stages over row bits 0..3 in registers; the tile passes
//       through LDS once, after which the thread holds rows g + 16 i and runs
//       the stages over bits 4..7.
//   hi: a workgroup owns one low index v and 64 columns: it stages the rows
//       b L + v of every block b in LDS, then each sample s with lo(S'_s) = v
//       adds its signed terms over ascending b in FP64.
// ---------------------------------------------------------------------------
constexpr int kMaxBlkV = 512;  // blocks the hi kernel stages (m <= 131072)

__device__ __forceinline__ void bfly4(fx4& x, fx4& y) {
  const fx4 a = x, b = y;
  x = a + b;
  y = a - b;
}

__device__ __forceinline__ void bfly16(fx4 (&v)[16]) {
#pragma unroll
  for (int h = 1; h < 16; h <<= 1)
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (!(i & h)) bfly4(v[i], v[i + h]);
}

__global__ void __launch_bounds__(256) k_srht_cols_lo_v(float* __restrict__ B, int64_t m, int64_t k, int64_t ldb,
                                                        const uint32_t* __restrict__ bits) {
  __shared__ __align__(16) float s[256 * kColTile];
  const int64_t row0 = (int64_t)blockIdx.x * 256;
  const int tid = threadIdx.x, q = tid & 15, g = tid >> 4;
  const int64_t col = (int64_t)blockIdx.y * kColTile + 4 * q;
  const bool has = col < k;  // k % 4 == 0: all four columns or none
  const fx4 zero = {0.f, 0.f, 0.f, 0.f};
  fx4 v[16];
  // sign bits of rows 16 g .. 16 g + 15 (row0 is a multiple of 256)
  const uint32_t word = row0 + 16 * g < m ? bits[(row0 + 16 * g) >> 5] >> ((16 * g) & 16) : 0u;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t row = row0 + 16 * g + i;
    v[i] = (has && row < m) ? *reinterpret_cast<const fx4*>(B + row * ldb + col) : zero;
  }
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int64_t row = row0 + 16 * g + i;
    if (row < m && ((word >> i) & 1u)) v[i] = -v[i];
  }
  bfly16(v);  // stages over row bits 0..3
#pragma unroll
  for (int i = 0; i < 16; ++i) *reinterpret_cast<fx4*>(s + (16 * g + i) * kColTile + 4 * q) = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = *reinterpret_cast<const fx4*>(s + (g + 16 * i) * kColTile + 4 * q);
  bfly16(v);  // stages over row bits 4..7
  if (has)
#pragma unroll
    for (int i = 0; i < 16; ++i) *reinterpret_cast<fx4*>(B + (row0 + g + 16 * i) * ldb + col) = v[i];
}

__global__ void __launch_bounds__(256) k_srht_cols_hi_v(const float* __restrict__ Z, int nblk, int64_t k,
                                                        int64_t ldz, const int32_t* __restrict__ sel, int64_t l,
                                                        double* __restrict__ C) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  float* s = reinterpret_cast<float*>(smem_raw);  // [nblk][kColTile]
  __shared__ int list[kMaxBlkV];
  __shared__ int wcnt[4];
  const int v = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t c0 = (int64_t)blockIdx.y * kColTile;
  const int q = tid & 15, g = tid >> 4;
  const bool has = c0 + 4 * q < k;
  const fx4 zero = {0.f, 0.f, 0.f, 0.f};
  // the first 256 blocks' rows are requested before the sample scan so that
  // the scan runs under their latency
  fx4 r[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int b = g + 16 * i;
    r[i] = (has && b < nblk) ? *reinterpret_cast<const fx4*>(Z + ((int64_t)b * 256 + v) * ldz + c0 + 4 * q) : zero;
  }
  // the samples with low index v, in ascending order (distinct rows, so at
  // most one per block: nblk <= kMaxBlkV)
  int tot = 0;
  for (int64_t w0 = 0; w0 < l; w0 += 256) {
    const int64_t e = w0 + tid;
    const bool hit = e < l && (sel[e] & 255) == v;
    const uint64_t mask = __ballot(hit);
    if (lane == 0) wcnt[wave] = __popcll(mask);
    __syncthreads();
    int pos = tot + __popcll(mask & ((1ull << lane) - 1));
    for (int w = 0; w < wave; ++w) pos += wcnt[w];
    if (hit && pos < kMaxBlkV) list[pos] = (int)e;
    tot += (wcnt[0] + wcnt[1]) + (wcnt[2] + wcnt[3]);
    __syncthreads();
  }
  if (tot == 0) return;  // uniform: no sample has this low index
  if (tot > kMaxBlkV) tot = kMaxBlkV;
  for (int b0 = 0; b0 < nblk; b0 += 256) {
    if (b0 > 0)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int b = b0 + g + 16 * i;
        r[i] = (has && b < nblk) ? *reinterpret_cast<const fx4*>(Z + ((int64_t)b * 256 + v) * ldz + c0 + 4 * q) : zero;
      }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int b = b0 + g + 16 * i;
      if (b < nblk) *reinterpret_cast<fx4*>(s + b * kColTile + 4 * q) = r[i];
    }
  }
  __syncthreads();
  // wavefront w takes the samples w, w + 4, ...: its 64 lanes are the 64
  // columns of one sample, so the sample's high index and the sign of each
  // block are uniform (scalar unit); the sign goes onto the FP32 value before
  // it is widened, which gives the same FP64 terms as negating after
  for (int o0 = wave * kColTile; o0 < tot * kColTile; o0 += 256) {
    const int64_t srow = list[o0 / kColTile];
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane(sel[srow] >> 8);
    if (c0 + lane >= k) continue;
    double acc = 0.0;
#pragma unroll 16
    for (int b = 0; b < nblk; ++b) {
      const uint32_t neg = (uint32_t)(__builtin_popcount(hi & (uint32_t)b) & 1) << 31;
      acc += (double)__uint_as_float(__float_as_uint(s[b * kColTile + lane]) ^ neg);
    }
    C[srow * k + c0 + lane] = acc;
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

static int num_cus() {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

// RANKEST_SRHT_ROWS=lds sends every FP32 row transform to the one-row-per-
// workgroup LDS kernel (a reference for the register-tiled ones).
static bool srht_rows_lds_forced() {
  static const bool forced = [] {
    const char* v = getenv("RANKEST_SRHT_ROWS");
    return v && strcmp(v, "lds") == 0;
  }();
  return forced;
}

re_status launch_srht_rows(hipStream_t s, const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                           const uint32_t* bits, const int32_t* sel, int64_t k, void* B) {
  const int64_t N = next_pow2(n);
  const int logN = ilog2_exact(N);
  const int grid = (int)(m < 8192 ? m : 8192);
  if (m <= 0) return RE_OK;
  if (dtype == RE_F32 && n == kN14 && lda % 4 == 0 && ((uintptr_t)A % 16) == 0 && k <= INT32_MAX) {
    // 32 workgroups per CU's worth (8192 on 256 CUs), each striding over the
    // rows (8 rows apiece at m = 65536): against two per CU, each holding its
    // CU for the whole pass, the pass itself is about 1 % faster and the
    // kernels of estimates in flight on other streams find CUs as workgroups
    // retire (joint rate 678 against 631 estimates/s at four in flight).
    // RANKEST_N14W_GRID sets another workgroup count (tuning).
    static const int64_t grid_env = getenv("RANKEST_N14W_GRID") ? atoll(getenv("RANKEST_N14W_GRID")) : 0;
    const int64_t g = grid_env > 0 ? grid_env : 32 * (int64_t)num_cus();
    static const int variant = getenv("RANKEST_FWHT14") ? atoi(getenv("RANKEST_FWHT14")) : 1;
    if (variant == 1)
      hipLaunchKernelGGL(k_srht_rows_n14w, dim3((unsigned)(m < g ? m : g)), dim3(512), 0, s, (const float*)A, m, lda,
                         bits, sel, (int)k, (float*)B);
    else
      hipLaunchKernelGGL(k_srht_rows_n14, dim3((unsigned)(m < g ? m : g)), dim3(256), 0, s, (const float*)A, m, lda,
                         bits, sel, (int)k, (float*)B);
    RE_TRY_HIP(hipGetLastError());
    return RE_OK;
  }
  if (logN > 30) return RE_ERR_UNSUPPORTED;  // sampled positions are 32-bit
  // 16-byte aligned FP32 rows of N >= 2^11: the register-tiled transform,
  // over sub-rows of 2^15 with their chunk sums when N is longer.
  if (dtype == RE_F32 && logN >= 11 && lda % 4 == 0 && ((uintptr_t)A % 16) == 0 && k <= INT32_MAX &&
      !srht_rows_lds_forced()) {
    const bool pad = n != N;
    const int P = logN < 15 ? logN : 15;
    const int logH = logN - P;
    const void* fn = nullptr;
    switch (P) {
      case 11: fn = pad ? (const void*)k_srht_rows_reg<11, true, false> : (const void*)k_srht_rows_reg<11, false, false>; break;
      case 12: fn = pad ? (const void*)k_srht_rows_reg<12, true, false> : (const void*)k_srht_rows_reg<12, false, false>; break;
      case 13: fn = pad ? (const void*)k_srht_rows_reg<13, true, false> : (const void*)k_srht_rows_reg<13, false, false>; break;
      case 14: fn = pad ? (const void*)k_srht_rows_reg<14, true, false> : (const void*)k_srht_rows_reg<14, false, false>; break;
      default:
        if (logH == 0)
          fn = pad ? (const void*)k_srht_rows_reg<15, true, false> : (const void*)k_srht_rows_reg<15, false, false>;
        else
          fn = pad ? (const void*)k_srht_rows_reg<15, true, true> : (const void*)k_srht_rows_reg<15, false, true>;
        break;
    }
    const int nt = 1 << (P - 5);
    int per = 0;
    RE_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, nt, 0));
    const int64_t items = logH ? ((m + 7) / 8 * 8) << logH : m;
    int64_t g = (int64_t)(per > 0 ? per : 1) * num_cus();
    if (logH) g = g < 8 ? 8 : g / 8 * 8;  // a multiple of 8 keeps a row's items on one XCD
    if (items < g) g = items;
    const int kk = (int)k;
    void* args[] = {(void*)&A, (void*)&m, (void*)&n, (void*)&lda, (void*)&bits, (void*)&sel, (void*)&kk, (void*)&B,
                    (void*)&logH};
    RE_TRY_HIP(hipLaunchKernel(fn, dim3((unsigned)g), dim3(nt), args, 0, s));
    return RE_OK;
  }
  // Everything else: one row (or, past the LDS, one (row, chunk) item) per
  // workgroup with the row staged in LDS: up to 2^15 FP32 or 2^14 FP64 values.
  const int maxLog = dtype == RE_F32 ? 15 : 14;
  if (logN > maxLog) {
    const int logH = logN - maxLog;
    const size_t lds = (size_t)(1 << maxLog) * (dtype == RE_F32 ? sizeof(float) : sizeof(double));
    const int64_t items = ((m + 7) / 8 * 8) << logH;
    int64_t g = 8192;
    if (items < g) g = items;
    if (dtype == RE_F32) {
      RE_TRY(allow_lds(k_srht_rows_lds_sub<float>, lds));
      hipLaunchKernelGGL(k_srht_rows_lds_sub<float>, dim3((unsigned)g), dim3(256), lds, s, (const float*)A, m, n, lda,
                         maxLog, logH, bits, sel, k, (float*)B);
    } else {
      RE_TRY(allow_lds(k_srht_rows_lds_sub<double>, lds));
      hipLaunchKernelGGL(k_srht_rows_lds_sub<double>, dim3((unsigned)g), dim3(256), lds, s, (const double*)A, m, n,
                         lda, maxLog, logH, bits, sel, k, (double*)B);
    }
    RE_TRY_HIP(hipGetLastError());
    return RE_OK;
  }
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

re_status launch_srht_cols_lo(hipStream_t s, void* B, int bdtype, int64_t m, int64_t k, int64_t ldb,
                              const uint32_t* bits) {
  if (m <= 0 || k <= 0) return RE_OK;
  const int logL = cols_logL(m);
  const int64_t L = int64_t(1) << logL;
  const dim3 glo((unsigned)cdiv(m, L), (unsigned)cdiv(k, kColTile));
  if (bdtype == RE_F32 && logL == 8 && k % 4 == 0 && ldb % 4 == 0 && ((uintptr_t)B & 15) == 0) {
    hipLaunchKernelGGL(k_srht_cols_lo_v, glo, dim3(256), 0, s, (float*)B, m, k, ldb, bits);
  } else if (bdtype == RE_F32) {
    const size_t lds = (size_t)L * kColTile * sizeof(float);
    RE_TRY(allow_lds(k_srht_cols_lo<float>, lds));
    hipLaunchKernelGGL(k_srht_cols_lo<float>, glo, dim3(256), lds, s, (float*)B, m, k, ldb, logL, bits);
  } else {
    const size_t lds = (size_t)L * kColTile * sizeof(double);
    RE_TRY(allow_lds(k_srht_cols_lo<double>, lds));
    hipLaunchKernelGGL(k_srht_cols_lo<double>, glo, dim3(256), lds, s, (double*)B, m, k, ldb, logL, bits);
  }
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_srht_cols_hi(hipStream_t s, const void* B, int bdtype, int64_t m, int64_t k, int64_t ldb,
                              const int32_t* sel, int64_t l, double* C) {
  if (m <= 0 || k <= 0 || l <= 0) return RE_OK;
  const int logL = cols_logL(m);
  const int64_t nblk = cdiv(m, int64_t(1) << logL);
  const int64_t total = l * k;
  const int ghi = (int)(cdiv(total, 256) < 65536 ? cdiv(total, 256) : 65536);
  if (bdtype == RE_F32 && logL == 8 && nblk <= kMaxBlkV && k % 4 == 0 && ldb % 4 == 0 && ((uintptr_t)B & 15) == 0) {
    const size_t lds = (size_t)nblk * kColTile * sizeof(float);
    RE_TRY(allow_lds(k_srht_cols_hi_v, lds));
    hipLaunchKernelGGL(k_srht_cols_hi_v, dim3(256, (unsigned)cdiv(k, kColTile)), dim3(256), lds, s, (const float*)B,
                       (int)nblk, k, ldb, sel, l, C);
  } else if (bdtype == RE_F32)
    hipLaunchKernelGGL(k_srht_cols_hi<float>, dim3(ghi), dim3(256), 0, s, (const float*)B, nblk, k, ldb, logL, sel, l,
                       C);
  else
    hipLaunchKernelGGL(k_srht_cols_hi<double>, dim3(ghi), dim3(256), 0, s, (const double*)B, nblk, k, ldb, logL, sel,
                       l, C);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_srht_cols(hipStream_t s, void* B, int bdtype, int64_t m, int64_t k, const uint32_t* bits,
                           const int32_t* sel, int64_t l, double* C) {
  if (m <= 0 || k <= 0 || l <= 0) return RE_OK;
  RE_TRY(launch_srht_cols_lo(s, B, bdtype, m, k, k, bits));
  return launch_srht_cols_hi(s, B, bdtype, m, k, k, sel, l, C);
}

}  // namespace re
