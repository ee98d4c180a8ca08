// Low-precision Gaussian contraction B = A X (Algorithm 1 step 3) on the
// MFMA units: A is read once in FP32 and rounded to BF16 or FP16 as it is
// loaded (FP16 after an exact power-of-two scale 2^s that keeps its entries
// inside the FP16 range), X holds Gaussian entries already rounded to the same
// format, products accumulate in FP32 and B = 2^-s (A_f X) is written in FP32.
//
// Tiling: a workgroup owns 64 WM rows of A and BN = 4 * WN columns of B; each
// of its 4 WM wavefronts owns a 64 x WN block made of 32x32 MFMA tiles
// (v_mfma_f32_32x32x16_{bf16,f16}).  K advances 32 at a time through
// double-buffered LDS tiles whose rows are padded to 80 bytes, which keeps the
// 16-byte operand reads free of bank conflicts.
#include "common.h"

namespace re {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float fx4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64;      // rows of A per workgroup
constexpr int kBK = 32;      // K per step
constexpr int kRowPad = 40;  // LDS row stride in 16-bit elements (80 bytes)

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

// WM wavefront rows: a workgroup of 256 WM threads owns BM = 64 WM rows, so
// each X tile staged in LDS serves WM times as many rows of A.
template <typename T, int WN, int WM>
__global__ void __launch_bounds__(256 * WM) k_gemm_lp(const float* __restrict__ A, int64_t m, int64_t n, int64_t lda,
                                                      const T* __restrict__ Xt, int64_t k, float scale, float unscale,
                                                      float* __restrict__ B, int nrb, int ncb, int vec_a, int vec_x) {
  typedef LpTraits<T> Tr;
  typedef typename Tr::vec8 vec8;
  constexpr int BN = 4 * WN, BM = kBM * WM, NTH = 256 * WM;
  constexpr int NT = WN / 32;  // 32-wide MFMA tiles per wavefront along N
  __shared__ __align__(16) uint16_t sA[2][BM * kRowPad];
  __shared__ __align__(16) uint16_t sX[2][BN * kRowPad];
  int rb, cb;
  tile_of(nrb, ncb, rb, cb);
  if (rb >= nrb) return;
  const int64_t row0 = (int64_t)rb * BM, col0 = (int64_t)cb * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = (tid >> 6) & 3, wm = tid >> 8;

  // global -> register staging: A DA K steps ahead (it streams from HBM; three
  // steps where the registers allow it: four measured slower), X one step ahead (every workgroup
  // walks the same K range, so X stays in L2)
  constexpr int DA = WM == 2 ? 3 : 1;
  fx4 ra0[2], ra1[2], ra2[2];
  u32x4 rx[BN * 4 / NTH];
  auto load_a = [&](int64_t k0, fx4 (&ra)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = (tid >> 3) + (NTH / 8) * i, kk = 4 * (tid & 7);
      const int64_t gr = row0 + r, gk = k0 + kk;
      fx4 v = {0.f, 0.f, 0.f, 0.f};
      if (gr < m) {
        if (vec_a && gk + 3 < n) {
          v = __builtin_nontemporal_load(reinterpret_cast<const fx4*>(A + gr * lda + gk));
        } else {
          for (int q = 0; q < 4; ++q)
            if (gk + q < n) v[q] = A[gr * lda + gk + q];
        }
      }
      ra[i] = v;
    }
  };
  auto load_x = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < BN * 4 / NTH; ++i) {
      const int c = (tid >> 2) + (NTH / 4) * i, kk = 8 * (tid & 3);
      const int64_t gc = col0 + c, gk = k0 + kk;
      u32x4 v = {0u, 0u, 0u, 0u};
      if (gc < k) {
        if (vec_x && gk + 7 < n) {
          v = *reinterpret_cast<const u32x4*>(Xt + gc * n + gk);
        } else {
          uint16_t h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
          for (int q = 0; q < 8; ++q)
            if (gk + q < n) h[q] = __builtin_bit_cast(uint16_t, Xt[gc * n + gk + q]);
          v = u32x4{h[0] | (uint32_t)h[1] << 16, h[2] | (uint32_t)h[3] << 16, h[4] | (uint32_t)h[5] << 16,
                    h[6] | (uint32_t)h[7] << 16};
        }
      }
      rx[i] = v;
    }
  };
  auto store_tile = [&](int buf, const fx4 (&ra)[2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int r = (tid >> 3) + (NTH / 8) * i, kk = 4 * (tid & 7);
      u16x4 h;
      h.x = Tr::cvt(ra[i].x * scale);
      h.y = Tr::cvt(ra[i].y * scale);
      h.z = Tr::cvt(ra[i].z * scale);
      h.w = Tr::cvt(ra[i].w * scale);
      *reinterpret_cast<u16x4*>(&sA[buf][r * kRowPad + kk]) = h;
    }
#pragma unroll
    for (int i = 0; i < BN * 4 / NTH; ++i) {
      const int c = (tid >> 2) + (NTH / 4) * i, kk = 8 * (tid & 3);
      *reinterpret_cast<u32x4*>(&sX[buf][c * kRowPad + kk]) = rx[i];
    }
  };

  f32x16 acc[2][NT];
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni)
#pragma unroll
      for (int q = 0; q < 16; ++q) acc[mi][ni][q] = 0.f;

  const int64_t nsteps = (n + kBK - 1) / kBK;
  auto compute = [&](int buf) {
#pragma unroll
    for (int ks = 0; ks < 2; ++ks) {
      // operand fragments: lane l takes row/column l % 32 and K values 8 (l / 32) .. + 7
      const int kk = 16 * ks + 8 * (lane >> 5);
      vec8 af[2], bf[NT];
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
        af[mi] = *reinterpret_cast<const vec8*>(&sA[buf][(64 * wm + 32 * mi + (lane & 31)) * kRowPad + kk]);
#pragma unroll
      for (int ni = 0; ni < NT; ++ni)
        bf[ni] = *reinterpret_cast<const vec8*>(&sX[buf][(WN * wave + 32 * ni + (lane & 31)) * kRowPad + kk]);
#pragma unroll
      for (int mi = 0; mi < 2; ++mi)
#pragma unroll
        for (int ni = 0; ni < NT; ++ni) acc[mi][ni] = Tr::mfma(af[mi], bf[ni], acc[mi][ni]);
    }
  };
  // step st computes from LDS buffer st & 1; A of steps st + 1 .. st + DA is in
  // flight (DA = 3: set j holds the steps = j mod 3; DA = 1: one set)
  load_a(0, ra0);
  load_x(0);
  if constexpr (DA == 3) {
    if (nsteps > 1) load_a(kBK, ra1);
    if (nsteps > 2) load_a(2 * kBK, ra2);
  }
  store_tile(0, ra0);
  __syncthreads();
  auto step = [&](int64_t st, fx4 (&ra_next)[2], fx4 (&ra_free)[2]) {
    // ra_next holds A of step st + 1; ra_free (step st, already in LDS) takes st + DA
    if (st + 1 < nsteps) load_x((st + 1) * kBK);
    if (st + DA < nsteps) load_a((st + DA) * kBK, ra_free);
    compute(st & 1);
    if (st + 1 < nsteps) {
      store_tile((st & 1) ^ 1, ra_next);
      __syncthreads();
    }
  };
  if constexpr (DA == 3) {
    for (int64_t st = 0; st < nsteps; st += 3) {
      step(st, ra1, ra0);
      if (st + 1 < nsteps) step(st + 1, ra2, ra1);
      if (st + 2 < nsteps) step(st + 2, ra0, ra2);
    }
  } else {
    for (int64_t st = 0; st < nsteps; ++st) step(st, ra0, ra0);
  }
  // accumulator layout of a 32x32 tile: value q of lane l is at
  // row 8 (q / 4) + 4 (l / 32) + (q % 4), column l % 32
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < NT; ++ni)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int64_t r = row0 + 64 * wm + 32 * mi + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
        const int64_t c = col0 + WN * wave + 32 * ni + (lane & 31);
        if (r < m && c < k) B[r * k + c] = acc[mi][ni][q] * unscale;
      }
}

template <typename T>
re_status launch_t(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, const void* Xt, int64_t k,
                   int scale_exp, float* B) {
  const float scale = ldexpf(1.0f, scale_exp), unscale = ldexpf(1.0f, -scale_exp);
  const int vec_a = (lda % 4 == 0) && ((uintptr_t)A % 16 == 0);
  const int vec_x = (n % 8 == 0) && ((uintptr_t)Xt % 16 == 0);
  // two wavefront rows (128 rows of A per X tile) while that still gives at
  // least one workgroup per CU
  const int wm = cdiv(m, 128) * cdiv(k, k > 256 ? 512 : 256) >= 256 ? 2 : 1;
  const int nrb = (int)cdiv(m, kBM * wm);
  if (k > 256) {
    const int ncb = (int)cdiv(k, 512);
    if (wm == 2)
      hipLaunchKernelGGL((k_gemm_lp<T, 128, 2>), dim3((unsigned)(nrb * ncb)), dim3(512), 0, s, A, m, n, lda,
                         (const T*)Xt, k, scale, unscale, B, nrb, ncb, vec_a, vec_x);
    else
      hipLaunchKernelGGL((k_gemm_lp<T, 128, 1>), dim3((unsigned)(nrb * ncb)), dim3(256), 0, s, A, m, n, lda,
                         (const T*)Xt, k, scale, unscale, B, nrb, ncb, vec_a, vec_x);
  } else {
    const int ncb = (int)cdiv(k, 256);
    if (wm == 2)
      hipLaunchKernelGGL((k_gemm_lp<T, 64, 2>), dim3((unsigned)(nrb * ncb)), dim3(512), 0, s, A, m, n, lda,
                         (const T*)Xt, k, scale, unscale, B, nrb, ncb, vec_a, vec_x);
    else
      hipLaunchKernelGGL((k_gemm_lp<T, 64, 1>), dim3((unsigned)(nrb * ncb)), dim3(256), 0, s, A, m, n, lda,
                         (const T*)Xt, k, scale, unscale, B, nrb, ncb, vec_a, vec_x);
  }
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

re_status launch_gemm_lp(hipStream_t s, int fmt, const float* A, int64_t m, int64_t n, int64_t lda, const void* Xt,
                         int64_t k, int scale_exp, float* B) {
  if (m <= 0 || k <= 0) return RE_OK;
  if (fmt == kBF16) return launch_t<__bf16>(s, A, m, n, lda, Xt, k, scale_exp, B);
  if (fmt == kF16) return launch_t<_Float16>(s, A, m, n, lda, Xt, k, scale_exp, B);
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
