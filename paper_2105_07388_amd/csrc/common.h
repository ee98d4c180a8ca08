// Internal definitions shared by the HIP translation units of librankest.
// Nothing here is part of the public C ABI (include/rankest.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rankest.h"

#define RE_HIDDEN __attribute__((visibility("hidden")))

namespace re {

// ---------------------------------------------------------------------------
// Sketch specification: Philox4x64-10 (Salmon et al., SC'11), key = (seed, 0),
// counter = (a, b, stream, block).  Streams name the random objects of
// Algorithm 1: the column embedding X and the row embedding Y (Theta).
// ---------------------------------------------------------------------------
enum Stream : uint64_t {
  kXGauss = 1,  // X[i][j], counter (i, j)
  kYGauss = 2,  // Y[i][j], counter (j, i)
  kXSign = 3,   // D of the column SRHT, counter (i, 0)
  kYSign = 4,   // D of the row SRHT, counter (i, 0)
  kXSel = 5,    // sampling keys of the column SRHT, counter (i, 0)
  kYSel = 6,    // sampling keys of the row SRHT, counter (i, 0)
};

struct u64x4 {
  uint64_t x, y, z, w;
};

// Philox4x64-10: ten rounds of the 4x64 S-box with multipliers M0, M1; the
// key is bumped by the Weyl increments W0, W1 before every round but the first.
__device__ __forceinline__ u64x4 philox(uint64_t a, uint64_t b, uint64_t c, uint64_t d, uint64_t seed) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  uint64_t k0 = seed, k1 = 0;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * a, hi0 = __umul64hi(M0, a);
    const uint64_t lo1 = M1 * c, hi1 = __umul64hi(M1, c);
    const uint64_t na = hi1 ^ b ^ k0, nc = hi0 ^ d ^ k1;
    a = na;
    b = lo1;
    c = nc;
    d = lo0;
    k0 += W0;
    k1 += W1;
  }
  return {a, b, c, d};
}

// Standard normal from two Philox words by the Box-Muller transform:
// u1 = (top 53 bits + 1) 2^-53 in (0, 1], u2 = top 53 bits 2^-53 in [0, 1).
__device__ __forceinline__ double gauss01(uint64_t a, uint64_t b, uint64_t stream, uint64_t seed) {
  const u64x4 w = philox(a, b, stream, 0, seed);
  const double u1 = (double)((w.x >> 11) + 1) * 0x1.0p-53;
  const double u2 = (double)(w.y >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// Value formats of the sketch entries used by a contraction.
enum Fmt : int { kF64 = 0, kF32 = 1, kBF16 = 2, kF16 = 3 };

// Round an FP64 value to nearest-even in a binary format with `p` significand
// bits whose lowest normal binade starts at 2^(emin-1); returns it as FP64.
__device__ __forceinline__ double rne_to(double v, int p, int emin) {
  if (v == 0.0) return v;
  int e = ilogb(v) + 1;
  if (e < emin) e = emin;
  const double q = ldexp(1.0, e - p);
  return rint(v / q) * q;
}

__device__ __forceinline__ double round_fmt(double v, int fmt) {
  switch (fmt) {
    case kF32: return (double)(float)v;
    case kBF16: return rne_to(v, 8, -125);
    case kF16: return rne_to(v, 11, -13);
    default: return v;
  }
}

// ---------------------------------------------------------------------------
// Host-side helpers.
// ---------------------------------------------------------------------------
// On failure the runtime's per-thread last error is read (and so cleared),
// so that a later call's hipGetLastError() check does not see it again.
#define RE_TRY_HIP(expr)                          \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) {                       \
      (void)hipGetLastError();                    \
      return RE_ERR_HIP;                          \
    }                                             \
  } while (0)

#define RE_TRY(expr)                              \
  do {                                            \
    re_status _s = (expr);                        \
    if (_s != RE_OK) return _s;                   \
  } while (0)

static inline int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

static inline int ilog2_exact(int64_t p) {
  int l = 0;
  while ((int64_t(1) << l) < p) ++l;
  return l;
}

static inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------------------
// Launchers implemented in the .hip translation units.
// ---------------------------------------------------------------------------
RE_HIDDEN re_status launch_philox(hipStream_t s, const uint64_t* ctr, uint64_t seed, int64_t count, uint64_t* out);
RE_HIDDEN re_status launch_gauss_fill(hipStream_t s, int fmt, int64_t rows, int64_t cols, uint64_t seed,
                                      int stream_id, int swap_ab, void* out);
RE_HIDDEN re_status launch_sign_bits(hipStream_t s, int64_t npad, uint64_t seed, int stream_id, uint32_t* bits);
// Scratch for selection: keys (8*npad bytes) + candidates (16*kSelCap) + 2 counters.
RE_HIDDEN size_t select_scratch_bytes(int64_t npad);
RE_HIDDEN re_status launch_select(hipStream_t s, int64_t npad, int64_t k, uint64_t seed, int stream_id, void* scratch,
                                  int32_t* idx);

// SRHT along rows (X side): B[i][t] = (H_npad (d .* [A_i, 0]))[S_t].
RE_HIDDEN re_status launch_srht_rows(hipStream_t s, const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                                     const uint32_t* sign_bits, const int32_t* sel, int64_t k, void* B);
// SRHT along columns (Y side): C[s][t] = (H_mpad (d .* [B_:t, 0]))[S_s]; B is
// m x k (FP32 or FP64, row-major) and is overwritten; C is l x k FP64.
RE_HIDDEN size_t srht_cols_rows_alloc(int64_t m);  // rows B must provide
RE_HIDDEN re_status launch_srht_cols(hipStream_t s, void* B, int bdtype, int64_t m, int64_t k,
                                     const uint32_t* sign_bits, const int32_t* sel, int64_t l, double* C);
// Its two levels separately, on k columns of a matrix with leading dimension
// ldb: the first transforms blocks of rows in place (signs applied), the
// second forms the l sampled rows from those blocks.
RE_HIDDEN re_status launch_srht_cols_lo(hipStream_t s, void* B, int bdtype, int64_t m, int64_t k, int64_t ldb,
                                        const uint32_t* sign_bits);
RE_HIDDEN re_status launch_srht_cols_hi(hipStream_t s, const void* B, int bdtype, int64_t m, int64_t k, int64_t ldb,
                                        const int32_t* sel, int64_t l, double* C);

// Dense products for Gaussian sketches.
// C[M x N] (ldc) = A[M x K] (lda, type ta) * B[K x N] (ldb, type tb), FP64 accumulate, output type tc.
RE_HIDDEN re_status launch_gemm_f64acc(hipStream_t s, int64_t M, int64_t N, int64_t K, const void* A, int ta,
                                       int64_t lda, const void* B, int tb, int64_t ldb, void* C, int tc, int64_t ldc);

// Low-precision contraction B = 2^-s round_fmt(2^s A) X, fmt BF16 or F16,
// FP32 accumulation and output.  X is held in step-major tiles written by
// launch_gemm_lp_x (gemm_lp_x_bytes(n, k) bytes): Gaussian entries of stream
// kXGauss rounded to fmt.
RE_HIDDEN size_t gemm_lp_x_bytes(int64_t n, int64_t k);
RE_HIDDEN re_status launch_gemm_lp_x(hipStream_t s, int fmt, int64_t n, int64_t k, uint64_t seed, void* Xtiles);
RE_HIDDEN re_status launch_gemm_lp(hipStream_t s, int fmt, const float* A, int64_t m, int64_t n, int64_t lda,
                                   const void* Xtiles, int64_t k, int scale_exp, float* B);
// Sampled sum of squares, largest magnitude and sample count of A (3 doubles).
RE_HIDDEN re_status launch_sample_stats(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, double* out3);

// Small dense SVD of an l x k FP64 row-major matrix: singular values, descending.
RE_HIDDEN size_t svd_scratch_bytes(int64_t l, int64_t k);
// spin_limit: polls of a grid barrier before it reports RE_ERR_NO_CONVERGENCE
// (0: the default; negative: give up at the first poll).  xcd: the XCD (of
// eight) that holds the workgroups of the multi-workgroup bidiagonalisation,
// so that sketches of different streams need not share one.  allow_plain:
// the bidiagonalisation pinned to one XCD may take a plain launch (the
// cooperative form runs one kernel at a time device-wide), 1 with a short
// barrier poll limit, 2 with the default one; *used_plain (if given) tells
// whether it did, so that a caller can redo a give-up (C is left untouched).
// A sketch small enough for one workgroup takes the batched form's per-lane
// bisection (the same bits as a block of a batch), or with multisect_small
// the 64-way multisection (shorter on one small sketch; for inputs the
// batched form never takes).
RE_HIDDEN re_status launch_svd(hipStream_t s, const double* C, int64_t l, int64_t k, double scale, void* scratch,
                               double* sigma, int32_t* info, long spin_limit = 0, int xcd = 0,
                               int allow_plain = 0, bool* used_plain = nullptr, bool multisect_small = false);
RE_HIDDEN re_status launch_rank_count(hipStream_t s, const double* sigma, int64_t k, int32_t r1, double eps,
                                      const int32_t* info, int32_t* out3);
// Gap statistics of descending estimates (search without a tolerance).
struct GapOut {
  int32_t g, a, reached, status;
  double ratio_g, ratio_a, s1;
};
RE_HIDDEN re_status launch_gap(hipStream_t s, const double* sigma, int64_t k, int32_t r1, double gamma,
                               double floor_rel, const int32_t* info, GapOut* out);
RE_HIDDEN re_status launch_nonfinite_scan(hipStream_t s, const void* A, int dtype, int64_t m, int64_t n, int64_t lda,
                                          int32_t* count);

}  // namespace re
