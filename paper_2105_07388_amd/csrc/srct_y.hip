// The subsampled randomized DCT as Y (Sec. 4 with F a DCT; Sec. 6 takes it for
// Theta = Y): C[s][t] = sqrt(M) (F D b_t)_{q_s} for the k columns b_t of B
// (m x k, zero-padded to M = a power of two), F the orthonormal DCT-II, D the
// SRHT's Y signs, q the sampled outputs.
//
// The DCT of a column goes through a DFT of the same length (Makhoul's
// reordering v[j] = x[2j], v[M-1-j] = x[2j+1] for j < M/2):
//   sum_i x_i cos(pi q (2i+1) / (2M)) = Re(e^{-i pi q / (2M)} V[q]),  V = DFT_M(v),
// and the DFT splits as M = M1 M2 with j = j1 + M1 j2 (four-step):
//   V[q] = sum_{j1 < M1} e^{-2 pi i q j1 / M} U[j1][q mod M2],
//   U[j1][q2] = sum_{j2 < M2} v[j1 + M1 j2] e^{-2 pi i q2 j2 / M2}.
// Level 1 (k_srct_y_lo) forms U, M2-point DFTs of strided pieces of every
// column, in registers, and keeps it: it is the stored first level through
// which the sketch grows (new columns of B get level 1 once; more sampled rows
// only need level 2 again).  Level 2 (k_srct_y_hi) forms the l sampled rows:
//   C[s][t] = sqrt(2) c_q sum_{j1} (cos phi U_re + sin phi U_im),
//   phi = pi q (4 j1 + 1) / (2M),  c_0 = 1/sqrt(2), c_q = 1 otherwise,
// a real weighted sum over M1 terms; the samples are grouped by q mod M2 so
// that each workgroup reads one slice U[.][q2][tile] for all its rows.
#include <math.h>

#include "common.h"
#include "srct_y.h"

namespace re {

namespace {

constexpr int kSrctM2 = 32;       // DFT length of level 1 (M2 = min(M, 32))
constexpr int kSrctRows = 8;      // sampled rows per level-2 workgroup
constexpr int kSrctCols = 2;      // columns per lane in level 2 (a workgroup covers 128)
constexpr int kSrctChunk = 64;    // j1 values whose weights share one LDS load

__device__ __forceinline__ bool neg_bit(const uint32_t* bits, int64_t i) { return (bits[i >> 5] >> (i & 31)) & 1u; }

template <typename T>
struct Cx {
  T re, im;
};

// In-register DFT of length L (power of two <= 32) of real input x: radix-2
// decimation in time over the bit-reversed order, twiddles e^{-2 pi i k / L}.
template <typename T, int L>
__device__ __forceinline__ void dft_reg(const T (&x)[L], Cx<T> (&X)[L]) {
  constexpr int LG = L == 1 ? 0 : L == 2 ? 1 : L == 4 ? 2 : L == 8 ? 3 : L == 16 ? 4 : 5;
#pragma unroll
  for (int i = 0; i < L; ++i) {
    int r = 0;
#pragma unroll
    for (int b = 0; b < LG; ++b) r |= ((i >> b) & 1) << (LG - 1 - b);
    X[r].re = x[i];
    X[r].im = T(0);
  }
#pragma unroll
  for (int h = 1; h < L; h <<= 1) {  // butterflies of span h, twiddle step L / (2h)
#pragma unroll
    for (int base = 0; base < L; base += 2 * h) {
#pragma unroll
      for (int j = 0; j < h; ++j) {
        // w = e^{-2 pi i j / (2h)} = e^{-i pi j / h}
        const double ang = -3.14159265358979323846 * (double)j / (double)h;
        const T wr = (T)__builtin_cos(ang), wi = (T)__builtin_sin(ang);
        const Cx<T> a = X[base + j], b = X[base + j + h];
        const T tr = b.re * wr - b.im * wi, ti = b.re * wi + b.im * wr;
        X[base + j] = Cx<T>{a.re + tr, a.im + ti};
        X[base + j + h] = Cx<T>{a.re - tr, a.im - ti};
      }
    }
  }
}

// Level 1: for j1 < M1 and the columns t < k of B (leading dimension ldb),
// U[(j1 M2 + q2) ldu + t] = sum_{j2 < M2} v[j1 + M1 j2][t] e^{-2 pi i q2 j2 / M2}.
// Thread (j1, t): the 64 lanes of a wavefront take consecutive columns, so each
// load of a row of B and each store of U is one contiguous segment.
template <typename T, int L>
__global__ void __launch_bounds__(256) k_srct_y_lo(const T* __restrict__ B, int64_t m, int64_t k, int64_t ldb,
                                                   int64_t M, const uint32_t* __restrict__ bits, T* __restrict__ Ure,
                                                   T* __restrict__ Uim, int64_t ldu) {
  const int64_t M1 = M / L;
  const int64_t j1 = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t t = (int64_t)blockIdx.y * 64 + (threadIdx.x & 63);
  if (j1 >= M1 || t >= k) return;
  T x[L];
#pragma unroll
  for (int j2 = 0; j2 < L; ++j2) {
    const int64_t j = j1 + M1 * j2;
    const int64_t i = j < M / 2 ? 2 * j : 2 * M - 1 - 2 * j;  // Makhoul's reordering
    T v = T(0);
    if (i < m) {
      v = B[i * ldb + t];
      if (neg_bit(bits, i)) v = -v;
    }
    x[j2] = v;
  }
  Cx<T> X[L];
  dft_reg<T, L>(x, X);
#pragma unroll
  for (int q2 = 0; q2 < L; ++q2) {
    const int64_t o = (j1 * L + q2) * ldu + t;
    Ure[o] = X[q2].re;
    Uim[o] = X[q2].im;
  }
}

// The sampled rows grouped by class q mod M2: order[] lists the rows s of class
// 0, then class 1, ... (ascending s within a class); start[c] is the first
// position of class c, start[M2] = l.  One workgroup: the rows go in chunks of
// 64 (one wavefront each); a chunk's class histogram and each row's rank among
// the earlier rows of its chunk and class come from one ballot per class, the
// chunks' histograms are summed up per class.  LDS: (nchunk + 2) M2 ints.
constexpr int kClsThreads = 256;
__global__ void __launch_bounds__(kClsThreads) k_srct_y_classes(const int32_t* __restrict__ sel, int64_t l, int M2,
                                                                int32_t* __restrict__ order,
                                                                int32_t* __restrict__ start) {
  extern __shared__ int32_t sh[];
  const int nchunk = (int)((l + 63) / 64);
  int32_t* base = sh;                  // [nchunk][M2]: rows of the class in the chunk, then in earlier chunks
  int32_t* size = base + nchunk * M2;  // [M2]
  int32_t* cstart = size + M2;         // [M2]
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t lt = lane ? ((uint64_t)-1 >> (64 - lane)) : 0;  // lanes below this one
  for (int z = wave; z < nchunk; z += kClsThreads / 64) {
    const int64_t s = (int64_t)z * 64 + lane;
    const int c = s < l ? (sel[s] & (M2 - 1)) : -1;
    for (int cc = 0; cc < M2; ++cc) {
      const uint64_t msk = __ballot(c == cc);
      if (lane == 0) base[z * M2 + cc] = __popcll(msk);
    }
  }
  __syncthreads();
  if (threadIdx.x < M2) {  // per class: exclusive prefix over the chunks
    const int c = threadIdx.x;
    int acc = 0;
    for (int z = 0; z < nchunk; ++z) {
      const int v = base[z * M2 + c];
      base[z * M2 + c] = acc;
      acc += v;
    }
    size[c] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int c = 0; c < M2; ++c) {
      cstart[c] = acc;
      start[c] = acc;
      acc += size[c];
    }
    start[M2] = acc;
  }
  __syncthreads();
  for (int z = wave; z < nchunk; z += kClsThreads / 64) {
    const int64_t s = (int64_t)z * 64 + lane;
    const int c = s < l ? (sel[s] & (M2 - 1)) : -1;
    int rank = 0;
    for (int cc = 0; cc < M2; ++cc) {
      const uint64_t msk = __ballot(c == cc);
      if (c == cc) rank = __popcll(msk & lt);
    }
    if (c >= 0) order[cstart[c] + base[z * M2 + c] + rank] = (int32_t)s;
  }
}

// Level 2: workgroup (class c, row group g, column tile) forms the rows
// order[start[c] + 8 g + r], r < 8, of C for 128 columns (two per lane).  The
// four wavefronts split each chunk of 64 j1 values (16 each) and add their
// sums at the end in a fixed order; the weights (cos phi, sin phi) of a chunk
// are computed once per workgroup into LDS, in FP64 from the angle reduced
// exactly modulo 2 pi (M is a power of two).
template <typename T>
__global__ void __launch_bounds__(256) k_srct_y_hi(const T* __restrict__ Ure, const T* __restrict__ Uim, int64_t ldu,
                                                   int64_t M, int M2, int64_t k, const int32_t* __restrict__ sel,
                                                   const int32_t* __restrict__ order,
                                                   const int32_t* __restrict__ start, double* __restrict__ C,
                                                   int64_t ldc) {
  __shared__ double2 w[kSrctRows][kSrctChunk];
  __shared__ double part[4][kSrctRows][64 * kSrctCols];
  __shared__ int64_t qs[kSrctRows];
  const int c = blockIdx.x % M2;
  const int g = blockIdx.x / M2;
  const int r0 = start[c] + g * kSrctRows, r1 = start[c + 1];
  if (r0 >= r1) return;  // uniform over the workgroup
  const int nr = r1 - r0 < kSrctRows ? r1 - r0 : kSrctRows;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t tb = (int64_t)blockIdx.y * 64 * kSrctCols + lane;
  const int64_t M1 = M / M2, mask = 4 * M - 1;
  if (threadIdx.x < kSrctRows) qs[threadIdx.x] = threadIdx.x < nr ? (int64_t)sel[order[r0 + threadIdx.x]] : 0;
  double acc[kSrctCols][kSrctRows];
#pragma unroll
  for (int u = 0; u < kSrctCols; ++u)
#pragma unroll
    for (int r = 0; r < kSrctRows; ++r) acc[u][r] = 0.0;
  // this wavefront's 16 j1 values of a chunk, both columns, real and imaginary.
  // The loads of a chunk are issued together, from clamped in-range addresses
  // (values out of range are zeroed afterwards), and a chunk's loads are issued
  // before the previous chunk is used: two register sets alternate, so the
  // compiler can wait for the older set alone.
  constexpr int JW = kSrctChunk / 4;
  T ar[JW][kSrctCols], ai[JW][kSrctCols], br[JW][kSrctCols], bi[JW][kSrctCols];
  const int64_t kc = k - 1;
  auto fetch = [&](int64_t j0, T (&vr)[JW][kSrctCols], T (&vi)[JW][kSrctCols]) {
#pragma unroll
    for (int i = 0; i < JW; ++i) {
      const int64_t j1 = j0 + wave * JW + i;
      const int64_t o = ((j1 < M1 ? j1 : M1 - 1) * M2 + c) * ldu;
#pragma unroll
      for (int u = 0; u < kSrctCols; ++u) {
        const int64_t t = tb + 64 * u;
        vr[i][u] = Ure[o + (t < k ? t : kc)];
        vi[i][u] = Uim[o + (t < k ? t : kc)];
      }
    }
  };
  auto weights = [&](int64_t j0) {
    for (int e = threadIdx.x; e < kSrctRows * kSrctChunk; e += 256) {
      const int r = e / kSrctChunk, jj = e % kSrctChunk;
      double cv = 0.0, sv = 0.0;
      if (r < nr && j0 + jj < M1) {
        // phi / pi = q (4 j1 + 1) / (2M), reduced modulo 2 exactly
        const int64_t p = (qs[r] * (4 * (j0 + jj) + 1)) & mask;
        sincospi((double)p / (double)(2 * M), &sv, &cv);
      }
      w[r][jj] = make_double2(cv, sv);
    }
  };
  // weights of j1 >= M1 are zero, so the clamped values there add nothing; a
  // column past k is never stored
  auto use = [&](const T (&vr)[JW][kSrctCols], const T (&vi)[JW][kSrctCols]) {
#pragma unroll
    for (int i = 0; i < JW; ++i) {
      const int jj = wave * JW + i;
#pragma unroll
      for (int r = 0; r < kSrctRows; ++r) {
        const double2 wv = w[r][jj];
#pragma unroll
        for (int u = 0; u < kSrctCols; ++u)
          acc[u][r] = fma(wv.x, (double)vr[i][u], fma(wv.y, (double)vi[i][u], acc[u][r]));
      }
    }
  };
  fetch(0, ar, ai);
  for (int64_t j0 = 0; j0 < M1; j0 += 2 * kSrctChunk) {
    __syncthreads();  // the previous chunk's weights are no longer read
    weights(j0);
    __syncthreads();
    if (j0 + kSrctChunk < M1) fetch(j0 + kSrctChunk, br, bi);
    use(ar, ai);
    if (j0 + kSrctChunk >= M1) break;
    __syncthreads();
    weights(j0 + kSrctChunk);
    __syncthreads();
    if (j0 + 2 * kSrctChunk < M1) fetch(j0 + 2 * kSrctChunk, ar, ai);
    use(br, bi);
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kSrctCols; ++u)
#pragma unroll
    for (int r = 0; r < kSrctRows; ++r) part[wave][r][lane + 64 * u] = acc[u][r];
  __syncthreads();
  if (wave != 0) return;
  for (int r = 0; r < nr; ++r) {
    const int s = order[r0 + r];
    const double cq = qs[r] == 0 ? 1.0 : 1.4142135623730951;  // sqrt(2) c_q
#pragma unroll
    for (int u = 0; u < kSrctCols; ++u) {
      const int64_t t = tb + 64 * u;
      const int x = lane + 64 * u;
      if (t < k) C[(int64_t)s * ldc + t] = cq * (((part[0][r][x] + part[1][r][x]) + part[2][r][x]) + part[3][r][x]);
    }
  }
}

template <typename T, int L>
re_status lo_case(hipStream_t s, const T* B, int64_t m, int64_t k, int64_t ldb, int64_t M, const uint32_t* bits,
                  T* Ure, T* Uim, int64_t ldu) {
  const dim3 grid((unsigned)cdiv(M / L, 4), (unsigned)cdiv(k, 64));
  hipLaunchKernelGGL((k_srct_y_lo<T, L>), grid, dim3(256), 0, s, B, m, k, ldb, M, bits, Ure, Uim, ldu);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

template <typename T>
re_status lo_any(hipStream_t s, const T* B, int64_t m, int64_t k, int64_t ldb, int64_t M, const uint32_t* bits,
                 T* Ure, T* Uim, int64_t ldu) {
  switch (srct_y_m2(M)) {
    case 2: return lo_case<T, 2>(s, B, m, k, ldb, M, bits, Ure, Uim, ldu);
    case 4: return lo_case<T, 4>(s, B, m, k, ldb, M, bits, Ure, Uim, ldu);
    case 8: return lo_case<T, 8>(s, B, m, k, ldb, M, bits, Ure, Uim, ldu);
    case 16: return lo_case<T, 16>(s, B, m, k, ldb, M, bits, Ure, Uim, ldu);
    case 32: return lo_case<T, 32>(s, B, m, k, ldb, M, bits, Ure, Uim, ldu);
    default: return RE_ERR_INVALID_ARG;
  }
}

}  // namespace

int64_t srct_y_npad(int64_t m) { return m < 2 ? 2 : next_pow2(m); }

int srct_y_m2(int64_t M) { return M < kSrctM2 ? (int)M : kSrctM2; }

size_t srct_y_u_bytes(int64_t m, int64_t k, int dtype) {
  return (size_t)2 * srct_y_npad(m) * k * (dtype == RE_F64 ? 8 : 4);
}

size_t srct_y_order_bytes(int64_t l) { return (size_t)(l + kSrctM2 + 1) * 4; }

re_status launch_srct_y_lo(hipStream_t s, const void* B, int bdtype, int64_t m, int64_t k, int64_t ldb,
                           const uint32_t* bits, void* U, int64_t ldu) {
  if (m <= 0 || k <= 0) return RE_OK;
  const int64_t M = srct_y_npad(m);
  const size_t half = (size_t)M * ldu;
  if (bdtype == RE_F64)
    return lo_any<double>(s, (const double*)B, m, k, ldb, M, bits, (double*)U, (double*)U + half, ldu);
  return lo_any<float>(s, (const float*)B, m, k, ldb, M, bits, (float*)U, (float*)U + half, ldu);
}

re_status launch_srct_y_hi(hipStream_t s, const void* U, int bdtype, int64_t m, int64_t k, int64_t ldu,
                           const int32_t* sel, int64_t l, int32_t* order_scratch, double* C) {
  if (m <= 0 || k <= 0 || l <= 0) return RE_OK;
  const int64_t M = srct_y_npad(m);
  const int M2 = srct_y_m2(M);
  int32_t* order = order_scratch;
  int32_t* start = order_scratch + l;
  const size_t cls_lds = (size_t)((cdiv(l, 64) + 2) * M2) * 4;
  if (cls_lds > 160 * 1024) return RE_ERR_UNSUPPORTED;
  if (cls_lds > 64 * 1024)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_srct_y_classes, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)cls_lds));
  hipLaunchKernelGGL(k_srct_y_classes, dim3(1), dim3(kClsThreads), cls_lds, s, sel, l, M2, order, start);
  RE_TRY_HIP(hipGetLastError());
  // row groups per class: at most ceil(l / 8) for one class; empty groups exit
  const int64_t groups = cdiv(l, kSrctRows);
  const int64_t gx = groups * M2;
  if (gx > INT32_MAX) return RE_ERR_UNSUPPORTED;
  const dim3 grid((unsigned)gx, (unsigned)cdiv(k, 64 * kSrctCols));
  const size_t half = (size_t)M * ldu;
  if (bdtype == RE_F64)
    hipLaunchKernelGGL(k_srct_y_hi<double>, grid, dim3(256), 0, s, (const double*)U, (const double*)U + half, ldu, M,
                       M2, k, sel, order, start, C, k);
  else
    hipLaunchKernelGGL(k_srct_y_hi<float>, grid, dim3(256), 0, s, (const float*)U, (const float*)U + half, ldu, M, M2,
                       k, sel, order, start, C, k);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
