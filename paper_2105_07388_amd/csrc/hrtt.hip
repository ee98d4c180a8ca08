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
// V_q).  v is real, so V comes from one complex FFT of half the length:
// z_p = v_{2p} + i v_{2p+1}, Z = FFT_M(z) with M = N / 2, then
// V_q = E_q + e^{-2 pi i q / N} O_q and V_{q+M} = E_q - e^{-2 pi i q / N} O_q,
// where E_q = (Z_q + conj Z_{M-q}) / 2 and O_q = (Z_q - conj Z_{M-q}) / (2i) are
// the transforms of the even and odd samples; V_{N-q} = conj V_q gives
// (F a)_{N-q} from the same product.  A row's M complex values (64 KiB at
// N = 16384) sit in LDS, so two rows run on each CU, one per workgroup; the
// FFT is a Stockham one (a pass of radix 2, 4 or 8 first when lg M is not a
// multiple of 4, fused into the loads for radix 2, then radix-16 passes with
// the 16-point DFTs in registers and twiddles from a quarter-wave cosine
// table).  Each thread owns a fixed chunk of the bucket-sorted coordinate
// list, kept in registers for the whole launch: it sums its chunk's runs, and
// each bucket then adds the run sums that fall in it, always in the same
// order, so every run gives the same bits.
#include <limits.h>

#include "common.h"
#include "hrtt.h"

namespace re {

namespace {

constexpr uint64_t kXHashStream = 7;
constexpr int kRowThreads = 512;
// a thread's chunk of the list (N / 512 entries) fits the 32-bit run-end mask
static_assert(kHrttMaxN / kRowThreads <= 32, "list chunk larger than the run-end mask");
constexpr int kBuildThreads = 1024;
static_assert(kHrttMaxN <= 16 * kBuildThreads, "the hash sort holds at most 16 keys per thread");

// Hash lists and their run structure, one workgroup.  Each coordinate j gets
// the key (bucket << 15) | (j << 1) | sign; a stable radix sort of the N keys
// on their bucket bits, in LDS, puts them in (bucket, j) order.  ptr[0..k] = first list position of each
// bucket (ptr[k] = N); list[ptr[b] ..] = the coordinates of bucket b in
// increasing order, the sign in bit 31; code16[p] = the same entry in 16 bits
// (coordinate, sign in bit 15).  The list is cut into chunks of C =
// max(N / 512, 1) positions; a run is a maximal piece of a chunk inside one
// bucket, numbered in list order.  ends[t] = bit i set where position tC + i
// ends a run; rbase[t] = number of the first run of chunk t; runs rlo[b] ..
// rhi[b] make up bucket b (rlo > rhi for an empty bucket).
// Longer transforms are cut into chunks of N coordinates: workgroup c builds
// the lists of coordinates c N .. c N + N - 1 (local indices in list and
// code16) into the arrays at byte offset c * chunk_bytes.
__global__ void __launch_bounds__(kBuildThreads) k_hash_build(int N, int k, uint64_t seed, int32_t* __restrict__ ptr,
                                                              int32_t* __restrict__ list, uint16_t* __restrict__ code16,
                                                              uint32_t* __restrict__ ends,
                                                              int32_t* __restrict__ rbase, int32_t* __restrict__ rlo,
                                                              int32_t* __restrict__ rhi, size_t chunk_bytes) {
  extern __shared__ uint32_t key[];  // N keys, then N + 1 words: the sort's buffer, later the k + 1 bucket starts
  uint32_t* tmp = key + N;
  int32_t* sptr = (int32_t*)(key + N);  // written only after the sorted keys are back in key
  __shared__ uint32_t smask[kRowThreads];
  __shared__ int32_t sbase[kRowThreads];
  __shared__ int wsum[kBuildThreads / 64];
  const int tid = threadIdx.x, nth = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const uint64_t j0 = (uint64_t)blockIdx.x * (uint64_t)N;
  {
    const size_t off = (size_t)blockIdx.x * chunk_bytes;
    ptr = (int32_t*)((char*)ptr + off);
    list = (int32_t*)((char*)list + off);
    code16 = (uint16_t*)((char*)code16 + off);
    ends = (uint32_t*)((char*)ends + off);
    rbase = (int32_t*)((char*)rbase + off);
    rlo = (int32_t*)((char*)rlo + off);
    rhi = (int32_t*)((char*)rhi + off);
  }
  for (int j = tid; j < N; j += nth) {
    const u64x4 w = philox(j0 + (uint64_t)j, 0, kXHashStream, 0, seed);
    const uint32_t b = (uint32_t)__umul64hi(w.x, (uint64_t)k);
    key[j] = (b << 15) | ((uint32_t)j << 1) | (uint32_t)(w.y & 1u);
  }
  __syncthreads();
  // Sort by (bucket, index): a stable least-significant-digit radix sort on
  // the bucket bits, one bit per pass, of keys that start in index order.
  // Thread t owns the E consecutive positions from t E; a pass counts its
  // zeros, finds the zeros before it by a workgroup prefix sum and writes
  // zeros then ones, each in their order, to the other buffer.
  {
    const int E = (N + nth - 1) / nth;
    const int p0 = tid * E < N ? tid * E : N, p1 = p0 + E < N ? p0 + E : N;
    int nbits = 0;
    while ((1 << nbits) < k) ++nbits;
    uint32_t* src = key;
    uint32_t* dst = tmp;
    const int cnt = p1 - p0;  // 0 or E (N and nth are powers of two, E <= 16)
    for (int bit = 0; bit < nbits; ++bit) {
      const int sh = 15 + bit;
      // the thread's keys into registers, as 16-byte reads when E = 16
      uint32_t v[16];
      if (E == 16 && cnt == 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const uint4 x = *reinterpret_cast<const uint4*>(src + p0 + 4 * q);
          v[4 * q] = x.x;
          v[4 * q + 1] = x.y;
          v[4 * q + 2] = x.z;
          v[4 * q + 3] = x.w;
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) v[e] = e < cnt ? src[p0 + e] : 0u;
      }
      int z = 0;
#pragma unroll
      for (int e = 0; e < 16; ++e) z += (e < cnt) & !((v[e] >> sh) & 1u);
      int incl = z;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(incl, off, 64);
        if (lane >= off) incl += y;
      }
      if (lane == 63) wsum[wave] = incl;
      __syncthreads();
      int before = 0, total = 0;
      for (int w = 0; w < nth / 64; ++w) {
        before += w < wave ? wsum[w] : 0;
        total += wsum[w];
      }
      int zi = before + incl - z, oi = total + (p0 - (before + incl - z));
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        if (e >= cnt) break;
        if ((v[e] >> sh) & 1u) dst[oi++] = v[e];
        else dst[zi++] = v[e];
      }
      __syncthreads();  // dst complete; wsum free for the next pass
      uint32_t* t = src;
      src = dst;
      dst = t;
    }
    if (src != key) {
      for (int p = tid; p < N; p += nth) key[p] = src[p];
      __syncthreads();
    }
  }
  // list, bucket starts (every bucket from the previous key's up to this one starts here)
  for (int p = tid; p < N; p += nth) {
    const uint32_t kp = key[p];
    const int b = (int)(kp >> 15), j = (int)((kp >> 1) & 0x3fffu), neg = (int)(kp & 1u);
    list[p] = (int32_t)((uint32_t)j | (neg ? 0x80000000u : 0u));
    code16[p] = (uint16_t)(j | (neg ? 0x8000 : 0));
    const int bprev = p ? (int)(key[p - 1] >> 15) : -1;
    for (int bb = bprev + 1; bb <= b; ++bb) sptr[bb] = p;
    if (p == N - 1)
      for (int bb = b + 1; bb <= k; ++bb) sptr[bb] = N;
  }
  __syncthreads();
  for (int b = tid; b <= k; b += nth) ptr[b] = sptr[b];
  // runs: per chunk the run-end mask, then prefix sums of the run counts (chunks <= 512)
  const int C = N >= kRowThreads ? N / kRowThreads : 1, nch = N / C;
  if (tid < nch) {
    uint32_t msk = 0;
    for (int i = 0; i < C; ++i) {
      const int p = tid * C + i;
      if (i == C - 1 || (key[p + 1] >> 15) != (key[p] >> 15)) msk |= 1u << i;
    }
    smask[tid] = msk;
    ends[tid] = msk;
    sbase[tid] = __popc(msk);
  }
  __syncthreads();
  if (tid < 64) {
    const int ch = (nch + 63) / 64;
    const int lo = min(nch, tid * ch), hi = min(nch, lo + ch);
    int sum = 0;
    for (int t = lo; t < hi; ++t) sum += sbase[t];
    int incl = sum;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int y = __shfl_up(incl, off, 64);
      if (tid >= off) incl += y;
    }
    int run = incl - sum;
    for (int t = lo; t < hi; ++t) {
      const int c = sbase[t];
      sbase[t] = run;
      run += c;
    }
  }
  __syncthreads();
  if (tid < nch) rbase[tid] = sbase[tid];
  // a bucket's runs: from the first run end at or after its start to its last position
  for (int b = tid; b < k; b += nth) {
    const int s0 = sptr[b], e = sptr[b + 1];
    if (e > s0) {
      const int first = min(s0 - s0 % C + C - 1, e - 1);
      const int t0 = first / C, t1 = (e - 1) / C;
      rlo[b] = sbase[t0] + __popc(smask[t0] & ((1u << (first % C)) - 1u));
      rhi[b] = sbase[t1] + __popc(smask[t1] & ((1u << ((e - 1) % C)) - 1u));
    } else {
      rlo[b] = 1;
      rhi[b] = 0;
    }
  }
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// LDS slots with one pad per 16 complex values, so that strided Stockham
// writes spread over the banks: complex value i at pz(i), real value q (the
// float view of the same storage) at px(q).
__device__ __forceinline__ int pz(int i) { return i + (i >> 4); }
__device__ __forceinline__ int px(int q) { return q + ((q >> 5) << 1); }

constexpr int brev_c(int i, int bits) {
  int r = 0;
  for (int b = 0; b < bits; ++b) r = (r << 1) | ((i >> b) & 1);
  return r;
}

constexpr int log2_c(int r) { return r <= 1 ? 0 : 1 + log2_c(r >> 1); }

// e^{-2 pi i t / M} for 0 <= t < M as the product of two table entries:
// tw[u] = e^{-2 pi i u / M} for u < 64 and tw[64 + v] = e^{-2 pi i 64 v / M}
// for v < M / 64.
__device__ __forceinline__ float2 twiddle(const float2* tw, int t) {
  const float2 f = tw[t & 63];
  return (t >> 6) ? cmul(f, tw[64 + (t >> 6)]) : f;
}

// a e^{-2 pi i t / 16}; t is a constant once the DFT's loops are unrolled, so
// the products by 1 and -i cost nothing and those by e^{-i pi / 4} and
// e^{-3 i pi / 4} two multiplies.
__device__ __forceinline__ float2 mul_w16(float2 a, int t) {
  constexpr float c1 = 0.923879532511286756f, s1 = 0.382683432365089772f, c2 = 0.707106781186547524f;
  switch (t) {
    case 0: return a;
    case 1: return cmul(a, make_float2(c1, -s1));
    case 2: return make_float2(c2 * (a.x + a.y), c2 * (a.y - a.x));
    case 3: return cmul(a, make_float2(s1, -c1));
    case 4: return make_float2(a.y, -a.x);
    case 5: return cmul(a, make_float2(-s1, -c1));
    case 6: return make_float2(c2 * (a.y - a.x), -c2 * (a.x + a.y));
    default: return cmul(a, make_float2(-c1, -s1));
  }
}

// R-point DFT (R <= 16) in registers, in place: radix-2 decimation in time
// over values already in bit-reversed order (t[brev(r)] = input r); the
// output is in natural order.
template <int R>
__device__ __forceinline__ void dft_reg(float2 (&t)[R]) {
#pragma unroll
  for (int half = 1; half < R; half *= 2)
#pragma unroll
    for (int g = 0; g < R; g += 2 * half)
#pragma unroll
      for (int pos = 0; pos < half; ++pos) {
        const float2 a = t[g + pos], b = mul_w16(t[g + pos + half], pos * (16 / (2 * half)));
        t[g + pos] = cadd(a, b);
        t[g + pos + half] = csub(a, b);
      }
}

// One Stockham pass of radix R over the M = 2^LGM values in LDS (natural
// order in, natural order out after the last pass), Ns = 2^LGNS: task j reads
// Z[j + r M/R], turns it by e^{-2 pi i (j mod Ns) r / (Ns R)}, takes the
// R-point DFT and writes it to Z[(j / Ns) Ns R + (j mod Ns) + r Ns].  All reads
// finish before any write.
template <int R, int LGM, int LGNS>
__device__ __forceinline__ void fft_pass(float2* Z, const float2* tw, int tid) {
  constexpr int L = log2_c(R), M = 1 << LGM, T = M / R, Ns = 1 << LGNS;
  constexpr int TASKS = T > kRowThreads ? T / kRowThreads : 1;
  float2 v[TASKS][R];
#pragma unroll
  for (int q = 0; q < TASKS; ++q) {
    const int j = tid + q * kRowThreads;
    if (T >= kRowThreads || j < T) {
      const int kk = j & (Ns - 1);
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][brev_c(r, L)] = Z[pz(j + r * T)];
      if constexpr (Ns > 1) {
        // w^r for w = e^{-2 pi i t1 / M}: the powers w^(2^b) from the table, the
        // rest as products of at most L of them
        const int t1 = kk << (LGM - LGNS - L);
        float2 wp[L], w[R];
#pragma unroll
        for (int b = 0; b < L; ++b) wp[b] = twiddle(tw, t1 << b);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const int hb = log2_c(r);
          w[r] = r == (1 << hb) ? wp[hb] : cmul(w[r - (1 << hb)], wp[hb]);
          v[q][brev_c(r, L)] = cmul(v[q][brev_c(r, L)], w[r]);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < TASKS; ++q) {
    const int j = tid + q * kRowThreads;
    if (T >= kRowThreads || j < T) {
      dft_reg<R>(v[q]);
      const int kk = j & (Ns - 1);
      const int base = (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) Z[pz(base + r * Ns)] = v[q][r];
    }
  }
  __syncthreads();
}

// The radix-16 passes from Ns = 2^LGNS up to M.
template <int LGM, int LGNS>
__device__ __forceinline__ void fft_rest(float2* Z, const float2* tw, int tid) {
  if constexpr (LGNS < LGM) {
    fft_pass<16, LGM, LGNS>(Z, tw, tid);
    fft_rest<LGM, LGNS + 4>(Z, tw, tid);
  }
}

// e^{-2 pi i t / (4N)} for 0 <= t < N from ts[u] = e^{-2 pi i u / (4N)}, u < 256,
// and ts[256 + v] = e^{-2 pi i 256 v / (4N)}; 64 more entries after those hold
// e^{-2 pi i u / N}, u < 64, the fine part of e^{-2 pi i q / N}.
__device__ __forceinline__ float2 split_twiddle(const float2* ts, int t) {
  const float2 f = ts[t & 255];
  return (t >> 8) ? cmul(f, ts[256 + (t >> 8)]) : f;
}

// x times the signs in the low four bits of sg (bit set: negative), by the sign bit.
__device__ __forceinline__ float4 signed4(float4 x, uint32_t sg) {
  x.x = __uint_as_float(__float_as_uint(x.x) ^ ((sg & 1u) << 31));
  x.y = __uint_as_float(__float_as_uint(x.y) ^ (((sg >> 1) & 1u) << 31));
  x.z = __uint_as_float(__float_as_uint(x.z) ^ (((sg >> 2) & 1u) << 31));
  x.w = __uint_as_float(__float_as_uint(x.w) ^ (((sg >> 3) & 1u) << 31));
  return x;
}

// Entries 4p .. 4p+3 of a row, zero past n (unsigned).  FULL: n covers every
// quad, so the load has no branch and the loads of a thread stay in flight together.
template <bool FULL>
__device__ __forceinline__ float4 load_quad(const float* __restrict__ a, int p, int64_t n) {
  const int64_t j = 4 * (int64_t)p;
  if (FULL) return *(const float4*)(a + j);
  float4 x;
  if (j + 3 < n) {
    x = *(const float4*)(a + j);
  } else {
    x.x = j < n ? a[j] : 0.0f;
    x.y = j + 1 < n ? a[j + 1] : 0.0f;
    x.z = j + 2 < n ? a[j + 2] : 0.0f;
    x.w = 0.0f;
  }
  return x;
}

// N = 2^LGN: one workgroup per row at a time (two per CU); VEC: rows are
// 16-byte aligned and the loads are float4.  LDS: M + M/16 complex slots, the
// FFT twiddles (64 + max(M / 64, 1) complex values), the split twiddles
// (256 + max(N / 256, 1) + 64), then one float per run.
// HASH: the CountSketch of the hashed DCT (list and runs from k_hash_build);
// otherwise the subsampled DCT: B[i][b] = sk (F D a_i)_{sel[b]}, no run floats.
template <bool VEC, int LGN, bool HASH>
__global__ void __launch_bounds__(kRowThreads) __attribute__((amdgpu_waves_per_eu(4)))
k_hrtt_rows(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const uint32_t* __restrict__ bits,
            const uint16_t* __restrict__ code16, const uint32_t* __restrict__ ends_g, const int32_t* __restrict__ rbase_g,
            const int32_t* __restrict__ rlo_g, const int32_t* __restrict__ rhi_g, const int32_t* __restrict__ sel,
            int k, float sk, float* __restrict__ B, int64_t ldb) {
  constexpr int N = 1 << LGN, LGM = LGN - 1, M = N >> 1;
  constexpr int C = N >= kRowThreads ? N / kRowThreads : 1;                 // list entries per thread
  constexpr int QUADS = (N / 4 + kRowThreads - 1) / kRowThreads;           // float4 loads per thread
  constexpr bool FUSED = VEC && (LGM & 3) == 1 && M >= 4;                  // radix-2 pass in the loads
  constexpr int FPAIRS = (M / 4 + kRowThreads - 1) / kRowThreads;          // fused load pairs per thread
  constexpr int SPAIRS = M >= 2 ? (M / 2 + kRowThreads - 1) / kRowThreads : 1;  // split pairs per thread
  constexpr bool QFULL = N / 4 > 0 && (N / 4) % kRowThreads == 0;  // every float4 slot in range
  constexpr bool PFULL = M / 4 > 0 && (M / 4) % kRowThreads == 0;  // every fused pair slot in range
  constexpr int TWN = 64 + (M / 64 > 1 ? M / 64 : 1);
  constexpr int TSN = 256 + (N / 256 > 1 ? N / 256 : 1) + 64;
  extern __shared__ float2 Z[];
  float* Xf = (float*)Z;
  float2* tw = Z + (M + (M >> 4));
  float2* ts = tw + TWN;
  float* P = (float*)(ts + TSN);
  const int tid0 = threadIdx.x;
  const int tid = tid0;

  // set-up: twiddle table, this thread's chunk of the list and its runs, the signs of the loads
  for (int u = tid; u < TWN; u += kRowThreads) {
    const int t = u < 64 ? u : 64 * (u - 64);
    double sv, cv;
    sincospi(2.0 * (double)t / (double)M, &sv, &cv);
    tw[u] = make_float2((float)cv, (float)-sv);
  }
  for (int u = tid; u < TSN; u += kRowThreads) {  // e^{-2 pi i t / (4N)}: 256 fine, N / 256 coarse, 64 at step 4
    const int t = u < 256 ? u : u < TSN - 64 ? 256 * (u - 256) : 4 * (u - (TSN - 64));
    double sv, cv;
    sincospi((double)t / (double)(2 * N), &sv, &cv);
    ts[u] = make_float2((float)cv, (float)-sv);
  }
  const bool lister = HASH && tid * C < N;
  uint32_t ends = 0;
  int32_t rb = 0;
  if (lister) {
    ends = ends_g[tid];
    rb = rbase_g[tid];
  }
  uint32_t sgn = 0;
  if constexpr (FUSED) {
#pragma unroll
    for (int i = 0; i < FPAIRS; ++i) {
      const int p = tid + i * kRowThreads;
      if (PFULL || p < M / 4) {
        const int p2 = M / 2 - 1 - p;
        sgn |= ((bits[p >> 3] >> ((p & 7) * 4)) & 15u) << (8 * i);
        sgn |= ((bits[p2 >> 3] >> ((p2 & 7) * 4)) & 15u) << (8 * i + 4);
      }
    }
  } else if constexpr (VEC && N >= 4) {
#pragma unroll
    for (int i = 0; i < QUADS; ++i) {
      const int p = tid + i * kRowThreads;
      if (QFULL || p < N / 4) sgn |= ((bits[p >> 3] >> ((p & 7) * 4)) & 15u) << (4 * i);
    }
  }
  const bool one_bucket = k <= kRowThreads;
  int32_t lo0 = 1, hi0 = 0;
  if (one_bucket && tid < k) {
    if constexpr (HASH) {
      lo0 = rlo_g[tid];
      hi0 = rhi_g[tid];
    } else {
      lo0 = sel[tid];
    }
  }
  const float c = sqrtf(2.0f / (float)N), c0 = sqrtf(1.0f / (float)N);
  __syncthreads();

  const bool full_rows = n == N;  // every quad in range: branch-free loads
  float4 x[FUSED ? 2 * FPAIRS : 1];
  auto fetch = [&](const float* __restrict__ a, int t) {
    if (full_rows) {
#pragma unroll
      for (int i = 0; i < FPAIRS; ++i) {
        const int p = t + i * kRowThreads;
        if (PFULL || p < M / 4) {
          x[2 * i] = load_quad<true>(a, p, n);
          x[2 * i + 1] = load_quad<true>(a, M / 2 - 1 - p, n);
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < FPAIRS; ++i) {
        const int p = t + i * kRowThreads;
        if (PFULL || p < M / 4) {
          x[2 * i] = load_quad<false>(a, p, n);
          x[2 * i + 1] = load_quad<false>(a, M / 2 - 1 - p, n);
        }
      }
    }
  };

  for (int64_t row = blockIdx.x; row < m; row += gridDim.x) {
    // the thread index and the sign word, opaque to the optimiser here, so that
    // the row's LDS addresses and sign masks are recomputed per row instead of
    // held (and spilled) across rows
    int tid = tid0;
    uint32_t sg = sgn;
    asm volatile("" : "+v"(tid), "+v"(sg));
    const float* __restrict__ a = A + row * lda;
    // 1. z (or its first radix-2 pass) into LDS
    if constexpr (FUSED) {
      fetch(a, tid);
#pragma unroll
      for (int i = 0; i < FPAIRS; ++i) {
        const int p = tid + i * kRowThreads;
        if (PFULL || p < M / 4) {
          const int p2 = M / 2 - 1 - p;
          const float4 u = signed4(x[2 * i], sg >> (8 * i)), w = signed4(x[2 * i + 1], sg >> (8 * i + 4));
          const float2 zp = make_float2(u.x, u.z), zp_hi = make_float2(w.w, w.y);   // z_p, z_{p + M/2}
          const float2 zq = make_float2(w.x, w.z), zq_hi = make_float2(u.w, u.y);   // z_{p2}, z_{p2 + M/2}
          Z[pz(2 * p)] = cadd(zp, zp_hi);
          Z[pz(2 * p + 1)] = csub(zp, zp_hi);
          Z[pz(2 * p2)] = cadd(zq, zq_hi);
          Z[pz(2 * p2 + 1)] = csub(zq, zq_hi);
        }
      }
    } else if constexpr (VEC && N >= 4) {
      float4 x[QUADS];
      if (full_rows) {
#pragma unroll
        for (int i = 0; i < QUADS; ++i) {
          const int p = tid + i * kRowThreads;
          if (QFULL || p < N / 4) x[i] = load_quad<true>(a, p, n);
        }
      } else {
#pragma unroll
        for (int i = 0; i < QUADS; ++i) {
          const int p = tid + i * kRowThreads;
          if (QFULL || p < N / 4) x[i] = load_quad<false>(a, p, n);
        }
      }
#pragma unroll
      for (int i = 0; i < QUADS; ++i) {
        const int p = tid + i * kRowThreads;
        if (QFULL || p < N / 4) {
          const float4 y = signed4(x[i], sg >> (4 * i));
          Z[pz(p)] = make_float2(y.x, y.z);
          Z[pz(M - 1 - p)] = make_float2(y.w, y.y);
        }
      }
    } else {
      for (int t = tid; t < N; t += kRowThreads) {
        const int64_t j = t < M ? 2 * (int64_t)t : 2 * (int64_t)(N - 1 - t) + 1;
        float x = j < n ? a[j] : 0.0f;
        if ((bits[j >> 5] >> (j & 31)) & 1u) x = -x;
        Xf[px(t)] = x;
      }
    }
    __syncthreads();
    // 2. Z = FFT_M(z)
    if constexpr (FUSED) {
      fft_rest<LGM, 1>(Z, tw, tid);
    } else if constexpr ((LGM & 3) == 1) {
      fft_pass<2, LGM, 0>(Z, tw, tid);
      fft_rest<LGM, 1>(Z, tw, tid);
    } else if constexpr ((LGM & 3) == 2) {
      fft_pass<4, LGM, 0>(Z, tw, tid);
      fft_rest<LGM, 2>(Z, tw, tid);
    } else if constexpr ((LGM & 3) == 3) {
      fft_pass<8, LGM, 0>(Z, tw, tid);
      fft_rest<LGM, 3>(Z, tw, tid);
    } else {
      fft_rest<LGM, 0>(Z, tw, tid);
    }

    // 3. DCT-II values from Z: pairs (q, M - q) give (F a) at q, N - q, M + q and
    //    M - q; q = 0 gives them at 0, M, M/2 and 3M/2
    constexpr bool SFULL = M / 2 > 0 && (M / 2) % kRowThreads == 0;  // every pair slot in range
    float out[SPAIRS][4];
#pragma unroll
    for (int i = 0; i < SPAIRS; ++i) {
      const int q = tid + i * kRowThreads;
      if (i == 0 && q == 0) {
        const float2 z0 = Z[pz(0)];
        out[0][0] = c0 * (z0.x + z0.y);                          // 0
        out[0][1] = c * 0.707106781186547524f * (z0.x - z0.y);   // M
        if constexpr (M >= 2) {
          const float2 zh = Z[pz(M / 2)];
          const float2 Uh = cmul(split_twiddle(ts, M / 2), make_float2(zh.x, -zh.y));  // e^{-i pi / 8}
          out[0][2] = c * Uh.x;    // M / 2
          out[0][3] = -c * Uh.y;   // 3M / 2
        }
      } else if (SFULL || q < M / 2) {
        const float2 zq = Z[pz(q)], zr = Z[pz(M - q)];
        const float2 E = make_float2(zq.x + zr.x, zq.y - zr.y);   // 2 E_q
        const float2 O = make_float2(zq.y + zr.y, zr.x - zq.x);   // 2 O_q
        const float2 t1 = split_twiddle(ts, q);            // e^{-i pi q / (2N)}
        const float2 wq = ts[TSN - 64 + (q & 63)];            // e^{-2 pi i q / N}: fine part
        const float2 P = cmul((q >> 6) ? cmul(wq, ts[256 + (q >> 6)]) : wq, O);
        const float2 U = cmul(t1, cadd(E, P));
        // e^{-i pi / 4} t1 for the upper half
        const float h = 0.707106781186547524f;
        const float2 t2 = make_float2(h * (t1.x + t1.y), h * (t1.y - t1.x));
        const float2 U2 = cmul(t2, csub(E, P));
        const float hc = 0.5f * c;
        out[i][0] = hc * U.x;     // q
        out[i][1] = -hc * U.y;    // N - q
        out[i][2] = hc * U2.x;    // M + q
        out[i][3] = -hc * U2.y;   // M - q
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SPAIRS; ++i) {
      const int q = tid + i * kRowThreads;
      if (i == 0 && q == 0) {
        Xf[px(0)] = out[0][0];
        Xf[px(M)] = out[0][1];
        if constexpr (M >= 2) {
          Xf[px(M / 2)] = out[0][2];
          Xf[px(3 * M / 2)] = out[0][3];
        }
      } else if (SFULL || q < M / 2) {
        Xf[px(q)] = out[i][0];
        Xf[px(N - q)] = out[i][1];
        Xf[px(M + q)] = out[i][2];
        Xf[px(M - q)] = out[i][3];
      }
    }
    __syncthreads();
    if constexpr (!HASH) {
      // 4'. the sampled coordinates (the next row's loads overwrite X)
      for (int b = tid; b < k; b += kRowThreads) B[row * ldb + b] = Xf[px(one_bucket ? lo0 : sel[b])] * sk;
      __syncthreads();
      continue;
    }
    // 4. CountSketch: the sums of this thread's runs, each stored by its number
    if (lister) {
      uint32_t cw[(C + 1) / 2];  // the chunk's 16-bit list entries, two a word
      if constexpr (C % 8 == 0) {
#pragma unroll
        for (int i = 0; i < C / 8; ++i) {
          const uint4 w = *(const uint4*)(code16 + tid * C + 8 * i);
          cw[4 * i] = w.x;
          cw[4 * i + 1] = w.y;
          cw[4 * i + 2] = w.z;
          cw[4 * i + 3] = w.w;
        }
      } else {
#pragma unroll
        for (int i = 0; i < C; ++i) {
          const uint32_t e = code16[tid * C + i];
          cw[i >> 1] = (i & 1) ? (cw[i >> 1] | (e << 16)) : e;
        }
      }
      float acc = 0.0f;
      int r = rb;
#pragma unroll
      for (int i = 0; i < C; ++i) {
        const uint32_t e = (cw[i >> 1] >> ((i & 1) * 16)) & 0xffffu;
        const float x = Xf[px((int)(e & 0x3fffu))];
        acc += (e & 0x8000u) ? -x : x;
        if ((ends >> i) & 1u) {
          P[r++] = acc;
          acc = 0.0f;
        }
      }
    }
    __syncthreads();
    // 5. each bucket adds its runs in order (the next row writes Z and X, not the run sums)
    for (int b = tid; b < k; b += kRowThreads) {
      const int32_t lo = one_bucket ? lo0 : rlo_g[b], hi = one_bucket ? hi0 : rhi_g[b];
      float sum = 0.0f;
      for (int r = lo; r <= hi; ++r) sum += P[r];
      B[row * ldb + b] = sum * sk;
    }
  }
}

// ---------------------------------------------------------------------------
// Rows longer than one workgroup's LDS (N > 16384): Makhoul's DCT through a
// four-step split of the M = N / 2 point complex FFT, M = M1 M2 with
// M2 = 8192.  With p = p2 + M2 p1 and q = q1 + M1 q2,
//   Z_q = sum_p2 e^{-2 pi i p2 q2 / M2} [ e^{-2 pi i p2 q1 / M}
//         sum_p1 e^{-2 pi i p1 q1 / M1} z_{p2 + M2 p1} ],
// so one work item per (row, q1) reads the whole row, forms the bracket for
// its q1 (an M1-term sum and a twiddle per p2), runs the 8192-point FFT in
// LDS and writes Z_{q1 + M1 q2} for every q2 to W (natural order, M complex
// values per row).  The items of a row are numbered 8 apart, so under a grid
// that is a multiple of 8 they share one XCD's L2 while they read the row.
// Then the DCT values come from the pairs (Z_q, Z_{M-q}) as in the one-row
// kernel: sampled (SRCT) straight into B, or (HRTT) all N into T, whose
// chunked bucket lists give the CountSketch sums.
// ---------------------------------------------------------------------------
constexpr int kLongLgM2 = 13, kLongM2 = 1 << kLongLgM2;
constexpr int kLongPairs = kLongM2 / 2 / kRowThreads;  // (p2, M2 - 1 - p2) pairs per thread

// Entries 4p .. 4p+3 of a row of n >= 1 entries, zero past n, without branches:
// every load reads an entry in range (the index clamped to n - 1).
__device__ __forceinline__ float4 clamped_quad(const float* __restrict__ a, int p, int n) {
  const int j = 4 * p;
  float v[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float x = a[j + c < n ? j + c : n - 1];
    v[c] = j + c < n ? x : 0.0f;
  }
  return make_float4(v[0], v[1], v[2], v[3]);
}

// LDS: M2 + M2/16 complex slots, the FFT twiddles (64 + M2/64), then
// e^{-2 pi i t / M} as 256 fine and M/256 coarse factors.
template <bool VEC>
__global__ void __launch_bounds__(kRowThreads) k_dct_long_fft(const float* __restrict__ A, int64_t rows, int64_t n,
                                                              int64_t lda, int lgM, const uint32_t* __restrict__ bits,
                                                              float2* __restrict__ W) {
  constexpr int M2 = kLongM2, LGM2 = kLongLgM2, TWN = 64 + M2 / 64;
  const int M = 1 << lgM, lgM1 = lgM - LGM2, M1 = 1 << lgM1;
  extern __shared__ float2 Z[];
  float2* tw = Z + (M2 + (M2 >> 4));
  float2* tf = tw + TWN;
  float2* tc = tf + 256;
  const int tid0 = threadIdx.x;
  for (int u = tid0; u < TWN; u += kRowThreads) {
    const int t = u < 64 ? u : 64 * (u - 64);
    double sv, cv;
    sincospi(2.0 * (double)t / (double)M2, &sv, &cv);
    tw[u] = make_float2((float)cv, (float)-sv);
  }
  for (int u = tid0; u < 256 + (M >> 8); u += kRowThreads) {
    const int t = u < 256 ? u : 256 * (u - 256);
    double sv, cv;
    sincospi(2.0 * (double)t / (double)M, &sv, &cv);
    tf[u] = make_float2((float)cv, (float)-sv);  // tc = tf + 256 continues the same array
  }
  __syncthreads();
  auto cis = [&](int t) {  // e^{-2 pi i t / M}
    t &= M - 1;
    const float2 f = tf[t & 255];
    return (t >> 8) ? cmul(f, tc[t >> 8]) : f;
  };
  const int64_t items = (((rows + 7) >> 3) << 3) << lgM1;
  for (int64_t u = blockIdx.x; u < items; u += gridDim.x) {
    const int64_t slot = u >> 3;
    const int q1 = (int)(slot & (M1 - 1));
    const int64_t row = ((slot >> lgM1) << 3) | (u & 7);
    if (row >= rows) continue;  // uniform over the workgroup
    // the thread index, opaque to the optimiser here, so that the item's LDS
    // addresses are recomputed per item instead of held (and spilled) across items
    int tid = tid0;
    asm volatile("" : "+v"(tid));
    const float* __restrict__ a = A + row * lda;
    // thread t owns p2 = t + 512 i and M2 - 1 - p2; quad p gives z_p = (x0, x2) and
    // z_{M-1-p} = (x3, x1), and M - 1 - (p2 + M2 p1) = (M2 - 1 - p2) + M2 (M1 - 1 - p1)
    constexpr int G = 4;  // pairs per group: eight loads in flight
#pragma unroll
    for (int g0 = 0; g0 < kLongPairs; g0 += G) {
      float2 lo[G], hi[G];  // brackets at p2 and at M2 - 1 - p2
#pragma unroll
      for (int e = 0; e < G; ++e) lo[e] = hi[e] = make_float2(0.0f, 0.0f);
#pragma unroll 1
      for (int p1 = 0; p1 < (M1 >> 1); ++p1) {
        const float2 wf = cis(p1 * q1 * M2), wb = cis((M1 - 1 - p1) * q1 * M2);  // e^{-2 pi i p1' q1 / M1}
        const float* __restrict__ ap = a + 4 * (int64_t)M2 * p1;
        const int64_t np = n - 4 * (int64_t)M2 * p1;  // the entries left from this chunk on
        const uint32_t* __restrict__ bp = bits + (M2 >> 3) * p1;
        if (VEC && np >= 4 * (int64_t)M2) {  // the whole chunk in range: unchecked float4 loads
          float4 xa[G], xb[G];
#pragma unroll
          for (int e = 0; e < G; ++e) {
            const int p2 = tid + (g0 + e) * kRowThreads, p2b = M2 - 1 - p2;
            xa[e] = signed4(*(const float4*)(ap + 4 * p2), bp[p2 >> 3] >> ((p2 & 7) * 4));
            xb[e] = signed4(*(const float4*)(ap + 4 * p2b), bp[p2b >> 3] >> ((p2b & 7) * 4));
          }
#pragma unroll
          for (int e = 0; e < G; ++e) {
            lo[e] = cadd(lo[e], cadd(cmul(wf, make_float2(xa[e].x, xa[e].z)), cmul(wb, make_float2(xb[e].w, xb[e].y))));
            hi[e] = cadd(hi[e], cadd(cmul(wf, make_float2(xb[e].x, xb[e].z)), cmul(wb, make_float2(xa[e].w, xa[e].y))));
          }
        } else if (np > 0) {  // the chunk holding the end of the row (or unaligned rows): one quad at a time
          const int nl = (int)(np < 4 * (int64_t)M2 ? np : 4 * (int64_t)M2);
#pragma unroll
          for (int e = 0; e < G; ++e) {
            const int p2 = tid + (g0 + e) * kRowThreads, p2b = M2 - 1 - p2;
            const float4 xa = signed4(clamped_quad(ap, p2, nl), bp[p2 >> 3] >> ((p2 & 7) * 4));
            const float4 xb = signed4(clamped_quad(ap, p2b, nl), bp[p2b >> 3] >> ((p2b & 7) * 4));
            lo[e] = cadd(lo[e], cadd(cmul(wf, make_float2(xa.x, xa.z)), cmul(wb, make_float2(xb.w, xb.y))));
            hi[e] = cadd(hi[e], cadd(cmul(wf, make_float2(xb.x, xb.z)), cmul(wb, make_float2(xa.w, xa.y))));
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }
#pragma unroll
      for (int e = 0; e < G; ++e) {
        const int p2 = tid + (g0 + e) * kRowThreads;
        Z[pz(p2)] = cmul(cis(p2 * q1), lo[e]);
        Z[pz(M2 - 1 - p2)] = cmul(cis((M2 - 1 - p2) * q1), hi[e]);
      }
    }
    __syncthreads();
    fft_pass<2, LGM2, 0>(Z, tw, tid);
    fft_rest<LGM2, 1>(Z, tw, tid);
    float2* __restrict__ w = W + row * (int64_t)M;
    for (int q2 = tid; q2 < M2; q2 += kRowThreads) w[q1 + (q2 << lgM1)] = Z[pz(q2)];
    __syncthreads();
  }
}

// DCT-II value j of a row from Z (Makhoul): with q = j mod M and r = (M - q) mod M,
// E = (Z_q + conj Z_r) / 2, O = (Z_q - conj Z_r) / (2i), V_j = E +- e^{-2 pi i q / N} O
// (+ for j < M), (F a)_j = c_j Re(e^{-i pi j / (2N)} V_j).  The two unit factors
// depend on j only: t1 = e^{-i pi j / (2N)}, t2 = +- t1 e^{-2 pi i q / N}.
struct DctTw {
  float2 t1, t2;
  int q, r;
  float c;
};

__device__ __forceinline__ DctTw dct_tw(int64_t j, int lgN) {
  const int64_t N = int64_t(1) << lgN, M = N >> 1;
  DctTw d;
  d.q = (int)(j & (M - 1));
  d.r = (int)((M - d.q) & (M - 1));
  double s1, c1, s2, c2;
  sincospi((double)j / (double)(2 * N), &s1, &c1);
  sincospi((double)j / (double)(2 * N) + 2.0 * (double)d.q / (double)N, &s2, &c2);
  const double sg = j < M ? 1.0 : -1.0;
  d.t1 = make_float2((float)c1, (float)-s1);
  d.t2 = make_float2((float)(sg * c2), (float)(-sg * s2));
  d.c = j == 0 ? (float)sqrt(1.0 / (double)N) : (float)sqrt(2.0 / (double)N);
  return d;
}

__device__ __forceinline__ float dct_value(const float2* __restrict__ z, const DctTw& d) {
  const float2 zq = z[d.q], zr = z[d.r];
  const float2 E = make_float2(0.5f * (zq.x + zr.x), 0.5f * (zq.y - zr.y));
  const float2 O = make_float2(0.5f * (zq.y + zr.y), 0.5f * (zr.x - zq.x));
  // Re(t1 E + t2 O)
  return d.c * ((d.t1.x * E.x - d.t1.y * E.y) + (d.t2.x * O.x - d.t2.y * O.y));
}

// SRCT: B[i][b] = sk (F D a_i)_{sel[b]} for the rows of W; thread (b, row group).
__global__ void __launch_bounds__(256) k_dct_long_sample(const float2* __restrict__ W, int64_t rows, int lgN,
                                                        const int32_t* __restrict__ sel, int64_t k, float sk,
                                                        float* __restrict__ B, int64_t ldb) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= k) return;
  const DctTw d = dct_tw(sel[b], lgN);
  const int64_t M = int64_t(1) << (lgN - 1);
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) B[i * ldb + b] = sk * dct_value(W + i * M, d);
}

// HRTT, first part: T[i][j] = (F D a_i)_j for every j (coalesced in j).
__global__ void __launch_bounds__(256) k_dct_long_values(const float2* __restrict__ W, int64_t rows, int lgN,
                                                        float* __restrict__ T) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t N = int64_t(1) << lgN, M = N >> 1;
  if (j >= N) return;
  const DctTw d = dct_tw(j, lgN);
  for (int64_t i = blockIdx.y; i < rows; i += gridDim.y) T[i * N + j] = dct_value(W + i * M, d);
}

// HRTT, second part, one workgroup per row: each chunk of the row's values
// (NC = 16384 coordinates, 64 KiB) is staged in LDS, every bucket sums its
// list entries of that chunk (increasing coordinate, with their signs) and
// adds the chunk's sum to its total in LDS, chunks in order; then
// B[i][b] = sk * total.
constexpr int kBucketThreads = 512;

__global__ void __launch_bounds__(kBucketThreads) k_dct_long_buckets(const float* __restrict__ T, int64_t rows,
                                                                    int64_t N, int chunks,
                                                                    const int32_t* __restrict__ ptr,
                                                                    const uint16_t* __restrict__ code16,
                                                                    size_t chunk_bytes, int k, float sk,
                                                                    float* __restrict__ B, int64_t ldb) {
  constexpr int NC = (int)kHrttMaxN;
  __shared__ __align__(16) float tl[NC];
  __shared__ float acc[NC];  // k <= NC bucket totals
  const int tid = threadIdx.x;
  for (int64_t i = blockIdx.x; i < rows; i += gridDim.x) {
    for (int b = tid; b < k; b += kBucketThreads) acc[b] = 0.0f;
    for (int c = 0; c < chunks; ++c) {
      const float4* src = reinterpret_cast<const float4*>(T + i * N + (int64_t)c * NC);
      for (int q = tid; q < NC / 4; q += kBucketThreads) reinterpret_cast<float4*>(tl)[q] = src[q];
      __syncthreads();
      const int32_t* pc = (const int32_t*)((const char*)ptr + (size_t)c * chunk_bytes);
      const uint16_t* cc = (const uint16_t*)((const char*)code16 + (size_t)c * chunk_bytes);
      for (int b = tid; b < k; b += kBucketThreads) {
        float part = 0.0f;
        for (int p = pc[b]; p < pc[b + 1]; ++p) {
          const uint32_t e = cc[p];
          const float x = tl[e & 0x3fffu];
          part += (e & 0x8000u) ? -x : x;
        }
        acc[b] += part;
      }
      __syncthreads();
    }
    for (int b = tid; b < k; b += kBucketThreads) B[i * ldb + b] = sk * acc[b];
    __syncthreads();
  }
}

}  // namespace

int64_t hrtt_npad(int64_t n) {
  const int64_t p = next_pow2(n);
  return p < 2 ? 2 : p;
}

// Scratch of one call, each piece on a 256-byte boundary: ptr (k + 1), list (N),
// code16 (N, 16-bit), ends and rbase (512 each), rlo and rhi (k each).
namespace {
struct HashScratch {
  int32_t *ptr, *list, *rbase, *rlo, *rhi;
  uint16_t* code16;
  uint32_t* ends;
  size_t bytes;
};
HashScratch carve_hash(void* base, int64_t N, int64_t k) {
  HashScratch h{};
  size_t off = 0;
  // with base == nullptr only the size is wanted: no pointer is formed
  auto take = [&](int64_t count) {
    char* p = base ? (char*)base + off : nullptr;
    off += (size_t)((count * 4 + 255) / 256) * 256;
    return p;
  };
  h.ptr = (int32_t*)take(k + 1);
  h.list = (int32_t*)take(N);
  h.code16 = (uint16_t*)take((N + 1) / 2);
  h.ends = (uint32_t*)take(kRowThreads);
  h.rbase = (int32_t*)take(kRowThreads);
  h.rlo = (int32_t*)take(k);
  h.rhi = (int32_t*)take(k);
  h.bytes = off;
  return h;
}
}  // namespace

// Coordinates per hash chunk and the chunk count of a transform of length N.
static int64_t hash_chunk(int64_t N) { return N < kHrttMaxN ? N : kHrttMaxN; }
static int64_t hash_chunks(int64_t N) { return N / hash_chunk(N); }

size_t hrtt_scratch_bytes(int64_t n, int64_t k) {
  const int64_t N = hrtt_npad(n);
  return (size_t)hash_chunks(N) * carve_hash(nullptr, hash_chunk(N), k).bytes;
}

// Rows of one pass of the long-row path and its workspace: W (rows x N / 2
// complex) and, for the hashed DCT, T (rows x N).
static int64_t long_rows(int64_t m, int64_t N, bool hash) {
  const int64_t per = N * 4 * (hash ? 2 : 1);
  int64_t r = (kDctLongWsBytes / per) / 8 * 8;
  if (r < 8) r = 8;
  const int64_t m8 = (m + 7) / 8 * 8;
  return r < m8 ? r : m8;
}

size_t dct_long_ws_bytes(int64_t m, int64_t n, bool hash) {
  const int64_t N = hrtt_npad(n);
  if (N <= kHrttMaxN) return 0;
  return (size_t)long_rows(m, N, hash) * (size_t)N * 4 * (hash ? 2 : 1);
}

template <bool VEC, bool HASH>
static const void* rows_kernel(int lgN) {
  switch (lgN) {
    case 1: return (const void*)k_hrtt_rows<VEC, 1, HASH>;
    case 2: return (const void*)k_hrtt_rows<VEC, 2, HASH>;
    case 3: return (const void*)k_hrtt_rows<VEC, 3, HASH>;
    case 4: return (const void*)k_hrtt_rows<VEC, 4, HASH>;
    case 5: return (const void*)k_hrtt_rows<VEC, 5, HASH>;
    case 6: return (const void*)k_hrtt_rows<VEC, 6, HASH>;
    case 7: return (const void*)k_hrtt_rows<VEC, 7, HASH>;
    case 8: return (const void*)k_hrtt_rows<VEC, 8, HASH>;
    case 9: return (const void*)k_hrtt_rows<VEC, 9, HASH>;
    case 10: return (const void*)k_hrtt_rows<VEC, 10, HASH>;
    case 11: return (const void*)k_hrtt_rows<VEC, 11, HASH>;
    case 12: return (const void*)k_hrtt_rows<VEC, 12, HASH>;
    case 13: return (const void*)k_hrtt_rows<VEC, 13, HASH>;
    case 14: return (const void*)k_hrtt_rows<VEC, 14, HASH>;
    default: return nullptr;
  }
}

// One launch of the rows kernel (either variant) on all CUs, two workgroups
// per CU when the LDS allows.
static re_status launch_rows(hipStream_t s, bool hash, const float* A, int64_t m, int64_t n, int64_t lda, int64_t k,
                             const uint32_t* sign_bits, const HashScratch* h, const int32_t* sel, float sk, float* B,
                             int64_t ldb) {
  const int64_t N = hrtt_npad(n);
  int lgN = 0;
  while ((int64_t(1) << lgN) < N) ++lgN;
  const int64_t M = N / 2, twn = 64 + (M / 64 > 1 ? M / 64 : 1), tsn = 256 + (N / 256 > 1 ? N / 256 : 1) + 64;
  const size_t lds = (size_t)(M + (M >> 4) + twn + tsn) * sizeof(float2) +
                     (hash ? (size_t)(k + kRowThreads) * sizeof(float) : 0);
  const bool vec = ((uintptr_t)A & 15) == 0 && (lda & 3) == 0;
  const void* fn = hash ? (vec ? rows_kernel<true, true>(lgN) : rows_kernel<false, true>(lgN))
                        : (vec ? rows_kernel<true, false>(lgN) : rows_kernel<false, false>(lgN));
  if (fn == nullptr) return RE_ERR_UNSUPPORTED;
  if (lds > 65536) RE_TRY_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per_cu = (int)((160 * 1024) / lds);
  if (per_cu < 1) per_cu = 1;
  if (per_cu > 2) per_cu = 2;  // 512 threads of at most 128 VGPRs: two workgroups per CU
  int64_t grid = 256 * (int64_t)per_cu;
  if (grid > m) grid = m;
  const uint16_t* ccode = hash ? h->code16 : nullptr;
  const uint32_t* cends = hash ? h->ends : nullptr;
  const int32_t* crbase = hash ? h->rbase : nullptr;
  const int32_t* crlo = hash ? h->rlo : nullptr;
  const int32_t* crhi = hash ? h->rhi : nullptr;
  int ki = (int)k;
  void* args[] = {(void*)&A,     (void*)&m,     (void*)&n,      (void*)&lda,  (void*)&sign_bits,
                  (void*)&ccode, (void*)&cends, (void*)&crbase, (void*)&crlo, (void*)&crhi,
                  (void*)&sel,   (void*)&ki,    (void*)&sk,     (void*)&B,    (void*)&ldb};
  RE_TRY_HIP(hipLaunchKernel(fn, dim3((unsigned)grid), dim3(kRowThreads), args, lds, s));
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

bool dct_x_supported(int64_t n, int64_t k, bool hash) {
  const int64_t N = hrtt_npad(n);
  if (N > kDctMaxN || k < 1 || k > N) return false;
  return !(hash && N > kHrttMaxN && k > kHrttMaxN);  // a chunk's bucket starts live in its build's LDS
}

re_status launch_hrtt_hash(hipStream_t s, int64_t n, int64_t k, uint64_t seed, void* scratch) {
  const int64_t N = hrtt_npad(n);
  if (!dct_x_supported(n, k, true)) return RE_ERR_UNSUPPORTED;
  const int64_t NC = hash_chunk(N);
  const HashScratch h = carve_hash(scratch, NC, k);
  const size_t lds_build = (size_t)(2 * NC + 1) * 4;  // keys, then the sort buffer that later holds the k + 1 <= NC + 1 bucket starts
  if (lds_build > 65536)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_hash_build, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds_build));
  hipLaunchKernelGGL(k_hash_build, dim3((unsigned)hash_chunks(N)), dim3(kBuildThreads), lds_build, s, (int)NC, (int)k,
                     seed, h.ptr, h.list, h.code16, h.ends, h.rbase, h.rlo, h.rhi, h.bytes);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

// Rows past 16384 coordinates: for each block of rows, the four-step FFT
// items into W, then the sampled values (SRCT) or all values into T and the
// bucket sums (HRTT).
static re_status launch_long(hipStream_t s, bool hash, const float* A, int64_t m, int64_t n, int64_t lda, int64_t k,
                             const uint32_t* sign_bits, const HashScratch* h, const int32_t* sel, float sk, float* B,
                             int64_t ldb, void* ws) {
  const int64_t N = hrtt_npad(n), M = N / 2;
  int lgN = 0;
  while ((int64_t(1) << lgN) < N) ++lgN;
  const int lgM = lgN - 1, lgM1 = lgM - kLongLgM2;
  if (ws == nullptr) return RE_ERR_INVALID_ARG;
  const int64_t R = long_rows(m, N, hash);
  float2* W = (float2*)ws;
  float* T = (float*)((char*)ws + (size_t)R * (size_t)M * sizeof(float2));
  const bool vec = ((uintptr_t)A & 15) == 0 && (lda & 3) == 0;
  const void* fn = vec ? (const void*)k_dct_long_fft<true> : (const void*)k_dct_long_fft<false>;
  const size_t lds = (size_t)(kLongM2 + kLongM2 / 16 + 64 + kLongM2 / 64 + 256 + (M >> 8)) * sizeof(float2);
  if (lds > 65536) RE_TRY_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  int per = 0;
  RE_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kRowThreads, lds));
  int cus = 0, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess || cus <= 0)
    cus = 256;
  int64_t g = (int64_t)(per > 0 ? per : 1) * cus;
  g = g < 8 ? 8 : g / 8 * 8;  // a multiple of 8 keeps a row's items on one XCD
  const int chunks = (int)hash_chunks(N);
  for (int64_t r0 = 0; r0 < m; r0 += R) {
    int64_t rows = m - r0 < R ? m - r0 : R;
    int lgMv = lgM;
    const float* Ar = A + r0 * lda;
    const int64_t items = ((rows + 7) / 8 * 8) << lgM1;
    const unsigned grid = (unsigned)(items < g ? items : g);
    void* args[] = {(void*)&Ar, (void*)&rows, (void*)&n, (void*)&lda, (void*)&lgMv, (void*)&sign_bits, (void*)&W};
    RE_TRY_HIP(hipLaunchKernel(fn, dim3(grid), dim3(kRowThreads), args, lds, s));
    const unsigned gy = (unsigned)((rows + 15) / 16);
    if (!hash) {
      hipLaunchKernelGGL(k_dct_long_sample, dim3((unsigned)cdiv(k, 256), gy), dim3(256), 0, s, (const float2*)W, rows,
                         lgN, sel, k, sk, B + r0 * ldb, ldb);
    } else {
      hipLaunchKernelGGL(k_dct_long_values, dim3((unsigned)(N / 256), gy), dim3(256), 0, s, (const float2*)W, rows,
                         lgN, T);
      const unsigned gb = (unsigned)(rows < 2 * (int64_t)cus ? rows : 2 * (int64_t)cus);
      hipLaunchKernelGGL(k_dct_long_buckets, dim3(gb), dim3(kBucketThreads), 0, s, (const float*)T, rows, N, chunks,
                         (const int32_t*)h->ptr, (const uint16_t*)h->code16, h->bytes, (int)k, sk, B + r0 * ldb,
                         ldb);
    }
    RE_TRY_HIP(hipGetLastError());
  }
  return RE_OK;
}

re_status launch_hrtt_rows(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, int64_t k,
                           const uint32_t* sign_bits, const void* scratch, float* B, int64_t ldb, void* ws) {
  const int64_t N = hrtt_npad(n);
  if (!dct_x_supported(n, k, true)) return RE_ERR_UNSUPPORTED;
  const HashScratch h = carve_hash((void*)scratch, hash_chunk(N), k);
  if (N > kHrttMaxN) return launch_long(s, true, A, m, n, lda, k, sign_bits, &h, nullptr, sqrtf((float)k), B, ldb, ws);
  return launch_rows(s, true, A, m, n, lda, k, sign_bits, &h, nullptr, sqrtf((float)k), B, ldb);
}

re_status launch_srct_rows(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, int64_t k,
                           const uint32_t* sign_bits, const int32_t* sel, float* B, int64_t ldb, void* ws) {
  const int64_t N = hrtt_npad(n);
  if (!dct_x_supported(n, k, false)) return RE_ERR_UNSUPPORTED;
  if (N > kHrttMaxN) return launch_long(s, false, A, m, n, lda, k, sign_bits, nullptr, sel, sqrtf((float)N), B, ldb, ws);
  return launch_rows(s, false, A, m, n, lda, k, sign_bits, nullptr, sel, sqrtf((float)N), B, ldb);
}

}  // namespace re
