// Low-precision Gaussian contraction B = A X (Algorithm 1 step 3) on the
// MFMA units: A is read once in FP32 and rounded to BF16 or FP16 as it is
// staged (FP16 after an exact power-of-two scale 2^s that keeps its entries
// inside the FP16 range), X holds Gaussian entries already rounded to the same
// format, products accumulate in FP32 and B = 2^-s (A_f X) is written in FP32.
//
// Tiling: a workgroup owns 128 rows of A and 512 columns of B (all of them
// when k <= 512, so A is fetched from HBM once); its eight wavefronts, two per
// SIMD, each own a 64 x 128 block made of 32x32 MFMA tiles
// (v_mfma_f32_32x32x16_{bf16,f16}).  K advances 32 at a time.
//
// X is stored step-major: tile st holds, for every column c < kx (k rounded
// up to 512), the 32 values X[32 st .. 32 st + 31][c] (zero past n and past
// k), so the 32 KB a workgroup needs for one step are contiguous.  They are
// copied global -> LDS by buffer loads that write LDS directly (no registers),
// four stages deep, issued three steps ahead.  A goes through registers (four
// steps ahead), is rounded there and written to one of three LDS buffers two
// steps before it is used; with three buffers the first MFMA operands of the
// next step are read before the barrier that ends the current one.
#include "common.h"

#include <type_traits>

namespace re {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float fx4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

constexpr int kBM = 128;     // rows of A per workgroup
constexpr int kBN = 512;     // columns of B per workgroup
constexpr int kKS = 32;      // K per step
constexpr int kRowPad = 40;  // A's LDS row stride in 16-bit elements (80 bytes)
constexpr int kXStages = 4;  // X tiles in LDS
constexpr int kABufs = 3;    // A tiles in LDS

template <typename T>
struct LpTraits;
template <>
struct LpTraits<__bf16> {
  typedef bf16x8 vec8;
  static __device__ __forceinline__ uint16_t cvt(float v) {
    const __bf16 h = (__bf16)v;
    return __builtin_bit_cast(uint16_t, h);
  }
  static __device__ __forceinline__ f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct LpTraits<_Float16> {
  typedef f16x8 vec8;
  static __device__ __forceinline__ uint16_t cvt(float v) {
    const _Float16 h = (_Float16)v;
    return __builtin_bit_cast(uint16_t, h);
  }
  static __device__ __forceinline__ f32x16 mfma(vec8 a, vec8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// Workgroup -> (row block, column block): the column blocks of one row block
// get consecutive slots on the same XCD (workgroups are dealt to the eight
// XCDs round-robin), so A's rows are fetched from HBM once and re-read from
// that XCD's L2.
__device__ __forceinline__ void tile_of(int nrb, int ncb, int& rb, int& cb) {
  const int b = blockIdx.x;
  const int nfull = (nrb / 8) * 8;
  if (b < nfull * ncb) {
    const int xcd = b & 7, slot = b >> 3;
    const int group = slot / ncb;
    cb = slot - group * ncb;
    rb = group * 8 + xcd;
  } else {  // row blocks past the last multiple of eight: plain order
    const int idx = b - nfull * ncb;
    rb = nfull + idx / ncb;
    cb = idx - (idx / ncb) * ncb;
  }
}

// s_waitcnt immediate that waits until at most N vector-memory loads of this
// wavefront are outstanding (expcnt and lgkmcnt left alone)
constexpr int vm_wait(int N) { return 0x0F70 | (N & 15) | ((N >> 4) << 14); }

// This wavefront's LDS writes done, then the workgroup barrier; the memory
// clobber keeps the compiler from moving LDS accesses across it.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// X tile in LDS: 512 columns x 32 values (64 bytes a column), the four
// 16-byte chunks of column c stored in the order j ^ ((c >> 1) & 3), which
// keeps the 16-byte operand reads of eight consecutive columns on distinct banks.
__device__ __forceinline__ int xoff(int c, int j) { return c * 32 + 8 * (j ^ ((c >> 1) & 3)); }

__device__ __forceinline__ uint64_t uniform64(uint64_t v) {
  return ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)(v >> 32)) << 32) |
         (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((uint32_t)v);
}

// SCALED: FP16, A multiplied by 2^s before rounding.  VEC_A: rows of A are
// 16-byte aligned (A and lda), so a thread's four values come in one load.
template <typename T, bool SCALED, bool VEC_A>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
k_gemm_lp(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda, const T* __restrict__ Xtiles, int64_t kx,
          int64_t k, float scale, float unscale, float* __restrict__ B, int nrb, int ncb) {
  typedef LpTraits<T> Tr;
  typedef typename Tr::vec8 vec8;
  constexpr int WN = 128, NT = 4, MT = 2;
  __shared__ __align__(16) uint16_t sA[kABufs][kBM * kRowPad];
  __shared__ __align__(1024) uint16_t sX0[kBN * kKS];
  __shared__ __align__(1024) uint16_t sX1[kBN * kKS];
  __shared__ __align__(1024) uint16_t sX2[kBN * kKS];
  __shared__ __align__(1024) uint16_t sX3[kBN * kKS];
  uint16_t* const sX[kXStages] = {sX0, sX1, sX2, sX3};
  int rb, cb;
  tile_of(nrb, ncb, rb, cb);
  if (rb >= nrb) return;
  const int64_t row0 = (int64_t)rb * kBM, col0 = (int64_t)cb * kBN;
  const int tid = threadIdx.x, lane = tid & 63, w8 = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wn = w8 & 3, wm = w8 >> 2;  // this wavefront's 128 columns and 64 rows
  const int64_t nst = (n + kKS - 1) / kKS, nfull = n / kKS;

  // A: thread t stages rows t / 8 and t / 8 + 64, values 4 (t % 8) .. + 3 of
  // the step (rows past m read row m - 1; their products are not stored)
  const float* arow[2];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    int64_t gr = row0 + (tid >> 3) + 64 * i;
    gr = gr < m ? gr : m - 1;
    arow[i] = A + gr * lda + 4 * (tid & 7);
  }
  auto load_a = [&](int64_t st, fx4 (&ra)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const float* p = arow[i] + st * kKS;
      if constexpr (VEC_A) {
        ra[i] = __builtin_nontemporal_load(reinterpret_cast<const fx4*>(p));
      } else {
        ra[i] = fx4{p[0], p[1], p[2], p[3]};
      }
    }
  };
  auto load_a_masked = [&](int64_t st, fx4 (&ra)[2]) {  // the partial last step: zeros past n
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      fx4 v = {0.f, 0.f, 0.f, 0.f};
      const int64_t gk = st * kKS + 4 * (tid & 7);
      for (int q = 0; q < 4; ++q)
        if (gk + q < n) v[q] = arow[i][st * kKS + q];
      ra[i] = v;
    }
  };
  auto store_a = [&](int buf, const fx4 (&ra)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = (tid >> 3) + 64 * i, kk = 4 * (tid & 7);
      fx4 v = ra[i];
      if constexpr (SCALED) v = v * scale;
      u16x4 h;
      h.x = Tr::cvt(v.x);
      h.y = Tr::cvt(v.y);
      h.z = Tr::cvt(v.z);
      h.w = Tr::cvt(v.w);
      *reinterpret_cast<u16x4*>(&sA[buf][r * kRowPad + kk]) = h;
    }
  };

  // X: copy i of wavefront w fills the 1 KB block 8 i + w of a stage (columns
  // 16 (8 i + w) .. + 15); lane t takes column 16 (8 i + w) + t / 4 and the
  // chunk that belongs at slot t % 4.  The buffer resource is rebased on
  // every step (scalar arithmetic), so offsets stay below 32 KB.
  uint32_t xoffs;
  {
    const int c = 16 * w8 + (lane >> 2);
    const int j = (lane & 3) ^ ((c >> 1) & 3);  // the same for column c + 128 i
    xoffs = (uint32_t)((c * kKS + 8 * j) * 2);
  }
  const uint64_t xbase = uniform64((uint64_t)(Xtiles + col0 * kKS));
  const uint64_t xstep = (uint64_t)kx * kKS * 2;
  auto dma_x = [&](int64_t st, uint16_t* sx) {
    const __amdgpu_buffer_rsrc_t xr =
        __builtin_amdgcn_make_buffer_rsrc((void*)(xbase + (uint64_t)st * xstep), (short)0, kBN * kKS * 2, 0x00020000);
#pragma unroll
    for (int i = 0; i < 4; ++i)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(xr, (lds_void*)(sx + (8 * i + w8) * 512), 16, xoffs + i * 128 * 64, 0,
                                               0, 0);
  };

  f32x16 acc[MT][NT];
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[mi][ni][q] = 0.f;
  // MFMA operands of one 16-deep half step: lane l takes row / column l % 32
  // of a 32 x 32 tile and the 8 values at 8 (2 ks + l / 32)
  struct Frag {
    vec8 a[MT], b[NT];
  };
  auto read_frag = [&](int buf, const uint16_t* sx, int ks, Frag& f) {
    const int j = 2 * ks + (lane >> 5);
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
      f.a[mi] = *reinterpret_cast<const vec8*>(&sA[buf][(64 * wm + 32 * mi + (lane & 31)) * kRowPad + 8 * j]);
#pragma unroll
    for (int ni = 0; ni < NT; ++ni)
      f.b[ni] = *reinterpret_cast<const vec8*>(&sx[xoff(WN * wn + 32 * ni + (lane & 31), j)]);
  };
  auto mma = [&](const Frag& f) {
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
      for (int ni = 0; ni < NT; ++ni) acc[mi][ni] = Tr::mfma(f.a[mi], f.b[ni], acc[mi][ni]);
  };

  // the vector-memory counter completes loads in issue order; the waits below
  // count on X's copies of a step being issued before its A loads
  auto issue_order = [] {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
  };
  Frag f0, f1;
  if (nst >= 16) {
    // A of step t is loaded into register set t % 3 at step t - 4 and written
    // to LDS buffer t % 3 at step t - 2; X of step t is copied into stage t % 4
    // at step t - 3.  Prologue: X of 0 .. 2 issued, A of 0 and 1 written, A of
    // 2 and 3 issued; wait for all but the last two A loads; first operands.
    fx4 ra[3][2];
    dma_x(0, sX0);
    dma_x(1, sX1);
    dma_x(2, sX2);
    issue_order();
    load_a(0, ra[0]);
    load_a(1, ra[1]);
    store_a(0, ra[0]);
    store_a(1, ra[1]);
    load_a(2, ra[2]);
    load_a(3, ra[0]);
    __builtin_amdgcn_s_waitcnt(vm_wait(4));
    lds_barrier();
    read_frag(0, sX0, 0, f0);
    // step st = J mod 12: issue X of st + 3 and A of st + 4; the second half
    // step's operands, both halves' MFMAs; A of st + 2 rounded into LDS; X of
    // st + 2 awaited (issued one step earlier: at most that step's two A loads
    // and this step's six loads still outstanding); barrier; the first
    // operands of st + 1 (published one barrier earlier)
    auto steady = [&](int64_t st, auto Jc) {
      constexpr int J = decltype(Jc)::value;
      dma_x(st + 3, sX[(J + 3) % kXStages]);
      issue_order();
      load_a(st + 4, ra[(J + 1) % 3]);
      __builtin_amdgcn_sched_barrier(0);
      read_frag(J % kABufs, sX[J % kXStages], 1, f1);
      mma(f0);
      mma(f1);
      __builtin_amdgcn_sched_barrier(0);
      store_a((J + 2) % kABufs, ra[(J + 2) % 3]);
      __builtin_amdgcn_s_waitcnt(vm_wait(8));
      lds_barrier();
      read_frag((J + 1) % kABufs, sX[(J + 1) % kXStages], 0, f0);
      __builtin_amdgcn_sched_barrier(0);
    };
    // the same step near the end, where loads past the last step are skipped
    // and everything issued is awaited
    auto last = [&](int64_t st, auto Jc) {
      constexpr int J = decltype(Jc)::value;
      if (st >= nst) return;
      if (st + 3 < nst) dma_x(st + 3, sX[(J + 3) % kXStages]);
      if (st + 4 < nst) {
        if (st + 4 < nfull) load_a(st + 4, ra[(J + 1) % 3]);
        else load_a_masked(st + 4, ra[(J + 1) % 3]);
      }
      read_frag(J % kABufs, sX[J % kXStages], 1, f1);
      mma(f0);
      mma(f1);
      if (st + 2 < nst) store_a((J + 2) % kABufs, ra[(J + 2) % 3]);
      __builtin_amdgcn_s_waitcnt(vm_wait(0));
      lds_barrier();
      if (st + 1 < nst) read_frag((J + 1) % kABufs, sX[(J + 1) % kXStages], 0, f0);
    };
    int64_t st = 0;
    // twelve steps (the period of the 3 buffers and 4 stages) while every
    // load they issue is a full step: st + 11 + 4 < nfull
    for (; st + 15 < nfull; st += 12) {
      steady(st, std::integral_constant<int, 0>());
      steady(st + 1, std::integral_constant<int, 1>());
      steady(st + 2, std::integral_constant<int, 2>());
      steady(st + 3, std::integral_constant<int, 3>());
      steady(st + 4, std::integral_constant<int, 4>());
      steady(st + 5, std::integral_constant<int, 5>());
      steady(st + 6, std::integral_constant<int, 6>());
      steady(st + 7, std::integral_constant<int, 7>());
      steady(st + 8, std::integral_constant<int, 8>());
      steady(st + 9, std::integral_constant<int, 9>());
      steady(st + 10, std::integral_constant<int, 10>());
      steady(st + 11, std::integral_constant<int, 11>());
    }
    // at most 16 steps remain (nst <= nfull + 1 <= st + 16)
    last(st, std::integral_constant<int, 0>());
    last(st + 1, std::integral_constant<int, 1>());
    last(st + 2, std::integral_constant<int, 2>());
    last(st + 3, std::integral_constant<int, 3>());
    last(st + 4, std::integral_constant<int, 4>());
    last(st + 5, std::integral_constant<int, 5>());
    last(st + 6, std::integral_constant<int, 6>());
    last(st + 7, std::integral_constant<int, 7>());
    last(st + 8, std::integral_constant<int, 8>());
    last(st + 9, std::integral_constant<int, 9>());
    last(st + 10, std::integral_constant<int, 10>());
    last(st + 11, std::integral_constant<int, 11>());
    last(st + 12, std::integral_constant<int, 0>());
    last(st + 13, std::integral_constant<int, 1>());
    last(st + 14, std::integral_constant<int, 2>());
    last(st + 15, std::integral_constant<int, 3>());
  } else {  // short K: one step at a time
    for (int64_t st = 0; st < nst; ++st) {
      fx4 ra[2];
      if (st < nfull) load_a(st, ra);
      else load_a_masked(st, ra);
      if (st > 0) lds_barrier();
      dma_x(st, sX0);
      store_a(0, ra);
      __builtin_amdgcn_s_waitcnt(vm_wait(0));
      lds_barrier();
      read_frag(0, sX0, 0, f0);
      read_frag(0, sX0, 1, f1);
      mma(f0);
      mma(f1);
    }
  }
  // accumulator layout of a 32x32 tile: value q of lane l is at
  // row 8 (q / 4) + 4 (l / 32) + (q % 4), column l % 32
#pragma unroll
  for (int mi = 0; mi < MT; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t r = row0 + 64 * wm + 32 * mi + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int64_t c = col0 + WN * wn + 32 * ni + (lane & 31);
        if (r < m && c < k) B[r * k + c] = acc[mi][ni][q] * unscale;
      }
}

int64_t x_cols(int64_t k) { return cdiv(k, kBN) * kBN; }

// Gaussian X in the step-major tiles: element (st, c, q) is
// X[32 st + q][c] = round_fmt(N(32 st + q, c)), zero past n or k.  The value
// is rounded once from FP64; the conversion to T is then exact.
template <typename T>
__global__ void k_gauss_tiles(int fmt, int64_t n, int64_t k, int64_t kx, uint64_t seed, T* __restrict__ out) {
  const int64_t total = (n + kKS - 1) / kKS * kx * kKS;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t st = e / (kx * kKS), rem = e - st * kx * kKS, c = rem / kKS, i = st * kKS + (rem - c * kKS);
    double v = 0.0;
    if (i < n && c < k) v = round_fmt(gauss01((uint64_t)i, (uint64_t)c, kXGauss, seed), fmt);
    out[e] = (T)(float)v;
  }
}

template <typename T, bool SCALED>
re_status launch_t(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, const void* Xtiles, int64_t k,
                   int scale_exp, float* B) {
  const float scale = ldexpf(1.0f, scale_exp), unscale = ldexpf(1.0f, -scale_exp);
  const bool vec_a = (lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
  const int nrb = (int)cdiv(m, kBM), ncb = (int)cdiv(k, kBN);
  const dim3 grid((unsigned)(nrb * ncb)), block(512);
  if (vec_a)
    hipLaunchKernelGGL((k_gemm_lp<T, SCALED, true>), grid, block, 0, s, A, m, n, lda, (const T*)Xtiles, x_cols(k), k,
                       scale, unscale, B, nrb, ncb);
  else
    hipLaunchKernelGGL((k_gemm_lp<T, SCALED, false>), grid, block, 0, s, A, m, n, lda, (const T*)Xtiles, x_cols(k), k,
                       scale, unscale, B, nrb, ncb);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

// Sampled statistics of A for the precision choice: sum of squares and the
// largest magnitude over a strided sample of rows and columns.
// Sampled sum of squares and largest magnitude of A on a grid of rows and
// columns.  Workgroup g takes sampled rows g, g + G, ... and writes one
// partial pair; k_sample_finish adds the G pairs in order.
constexpr int kStatsGroups = 256;
__global__ void __launch_bounds__(256) k_sample_stats(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                      int64_t rstep, int64_t cstep, double* __restrict__ part) {
  __shared__ double s_sum[256];
  __shared__ float s_max[256];
  double sum = 0.0;
  float mx = 0.0f;
  const int64_t nr = (m + rstep - 1) / rstep, nc = (n + cstep - 1) / cstep;
  for (int64_t r = blockIdx.x; r < nr; r += gridDim.x) {
    const float* row = A + r * rstep * lda;
    for (int64_t c = threadIdx.x; c < nc; c += blockDim.x) {
      const float v = row[c * cstep];
      sum += (double)v * (double)v;
      mx = fmaxf(mx, fabsf(v));
    }
  }
  s_sum[threadIdx.x] = sum;
  s_max[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_sum[threadIdx.x] += s_sum[threadIdx.x + w];
      s_max[threadIdx.x] = fmaxf(s_max[threadIdx.x], s_max[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s_sum[0];
    part[2 * blockIdx.x + 1] = (double)s_max[0];
  }
}

__global__ void k_sample_finish(const double* __restrict__ part, int groups, int64_t count, double* __restrict__ out) {
  if (threadIdx.x != 0) return;
  double sum = 0.0, mx = 0.0;
  for (int g = 0; g < groups; ++g) {
    sum += part[2 * g];
    mx = fmax(mx, part[2 * g + 1]);
  }
  out[0] = sum;
  out[1] = mx;
  out[2] = (double)count;
}

}  // namespace

size_t gemm_lp_x_bytes(int64_t n, int64_t k) { return (size_t)cdiv(n, kKS) * (size_t)x_cols(k) * kKS * 2; }

re_status launch_gemm_lp_x(hipStream_t s, int fmt, int64_t n, int64_t k, uint64_t seed, void* Xtiles) {
  if (n <= 0 || k <= 0) return RE_OK;
  const int64_t total = cdiv(n, kKS) * x_cols(k) * kKS;
  const unsigned g = (unsigned)(cdiv(total, 256) < 65536 ? cdiv(total, 256) : 65536);
  if (fmt == kBF16)
    hipLaunchKernelGGL(k_gauss_tiles<__bf16>, dim3(g), dim3(256), 0, s, fmt, n, k, x_cols(k), seed, (__bf16*)Xtiles);
  else if (fmt == kF16)
    hipLaunchKernelGGL(k_gauss_tiles<_Float16>, dim3(g), dim3(256), 0, s, fmt, n, k, x_cols(k), seed,
                       (_Float16*)Xtiles);
  else
    return RE_ERR_INVALID_ARG;
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_gemm_lp(hipStream_t s, int fmt, const float* A, int64_t m, int64_t n, int64_t lda, const void* Xtiles,
                         int64_t k, int scale_exp, float* B) {
  if (m <= 0 || k <= 0) return RE_OK;
  if (fmt == kBF16) return launch_t<__bf16, false>(s, A, m, n, lda, Xtiles, k, 0, B);
  if (fmt == kF16) return launch_t<_Float16, true>(s, A, m, n, lda, Xtiles, k, scale_exp, B);
  return RE_ERR_INVALID_ARG;
}

// out3 must provide 4 + 2 * 256 doubles: the three results, then the
// per-workgroup partials.
re_status launch_sample_stats(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, double* out3) {
  // about 2^17 entries on a coprime-ish grid of rows and columns
  int64_t rstep = m > 512 ? m / 512 : 1, cstep = n > 256 ? n / 256 : 1;
  if (rstep > 1 && rstep % 2 == 0) --rstep;
  if (cstep > 1 && cstep % 2 == 0) --cstep;
  const int64_t nr = (m + rstep - 1) / rstep, nc = (n + cstep - 1) / cstep;
  const int groups = (int)(nr < kStatsGroups ? nr : kStatsGroups);
  double* part = out3 + 4;
  hipLaunchKernelGGL(k_sample_stats, dim3(groups), dim3(256), 0, s, A, m, n, lda, rstep, cstep, part);
  hipLaunchKernelGGL(k_sample_finish, dim3(1), dim3(64), 0, s, part, groups, nr * nc, out3);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
