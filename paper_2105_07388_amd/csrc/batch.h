// Descriptor tables of the batched form (device memory, filled by the host).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rankest.h"

namespace re {

// Largest leading dimension of the persistent contraction (it indexes a
// 256-row tile with 32-bit offsets).
constexpr int64_t kMaxBatchLda = int64_t(1) << 23;

// One block of the FP32 contraction B = A X[:n]: its work items are
// item0 .. item0 + (row tiles x column chunks) - 1.
struct GemmDesc {
  const float* A;
  float* B;
  int64_t m, n, lda, ldb;
  int64_t item0;
  int64_t ncc;  // column chunks
};

// One block of C = Y[:, :m] B.
struct YDesc {
  const float* B;
  double* C;
  int64_t m, ldb;
};

// One small bidiagonal problem and its count.
struct SvDesc {
  const double* d;
  const double* e;
  double* sigma;
  const int32_t* info;
  int32_t* out3;  // r, flags, status
  int32_t k, r1;
  double scale, eps;
};

// Per-call header of a batched launch (device memory, written before the graph runs).
struct BatchHeader {
  uint64_t seed;
};

// B = A X for one FP32 matrix with the persistent kernel (B leading
// dimension ldb); dscratch receives its descriptor.
__attribute__((visibility("hidden"))) re_status launch_gemm_f32_single(hipStream_t s, const float* A, int64_t m,
                                                                      int64_t n, int64_t lda, const float* X, int64_t k,
                                                                      float* B, int64_t ldb, GemmDesc* dscratch,
                                                                      unsigned* queue);
// Rows r0.. and columns c0.. of a Gaussian sketch, FP32, leading dimension ld.
__attribute__((visibility("hidden"))) re_status launch_gauss_sub(hipStream_t s, int64_t rows, int64_t cols, int64_t r0,
                                                                int64_t c0, uint64_t seed, int stream_id, int swap_ab,
                                                                int64_t ld, float* out);
__attribute__((visibility("hidden"))) re_status launch_gauss_sub64(hipStream_t s, int64_t rows, int64_t cols,
                                                                  int64_t r0, int64_t c0, uint64_t seed, int stream_id,
                                                                  int swap_ab, int64_t ld, double* out);
// C = Y[:, :m] B (l x k FP64) for one block with the batched kernel's
// arithmetic; with m above one group of rows it splits m over workgroups,
// which needs ygemm_split_bytes(l, k, m) of `parts` (nullptr: no split).
__attribute__((visibility("hidden"))) re_status launch_ygemm_single(hipStream_t s, const float* B, int64_t m, int64_t k,
                                                                   int64_t ldb, const float* Y, int64_t ldy, int64_t l,
                                                                   double* C, YDesc* dscratch, double* parts);
__attribute__((visibility("hidden"))) size_t ygemm_split_bytes(int64_t l, int64_t k, int64_t m);
__attribute__((visibility("hidden"))) re_status launch_gauss_master(hipStream_t s, const BatchHeader* hdr, int64_t nmax,
                                                                   int64_t k, int64_t l, int64_t mmax, float* X,
                                                                   float* Y);
__attribute__((visibility("hidden"))) re_status launch_gemm_f32_persistent(hipStream_t s, const GemmDesc* desc, int nblk,
                                                                          const float* X, int64_t k, int64_t total,
                                                                          unsigned* queue, int waves, int grid, int bk,
                                                                          int mt);
__attribute__((visibility("hidden"))) int64_t gemm_items(int64_t m, int64_t k, int rows_per_item);
__attribute__((visibility("hidden"))) int gemm_col_chunks(int64_t k);
__attribute__((visibility("hidden"))) re_status launch_ygemm_batched(hipStream_t s, const YDesc* desc, int nblk,
                                                                    const float* Y, int64_t ldy, int64_t l, int64_t k);
__attribute__((visibility("hidden"))) re_status launch_ygemm_grid(hipStream_t s, const YDesc* desc, int nblk,
                                                                 const float* Y, int64_t ldy, int64_t l, int64_t k,
                                                                 unsigned groups, double* parts);
// Batched small SVDs: C[b] (l[b] x k[b], each fitting one workgroup's LDS) ->
// d[b], e[b]; then singular values and counts per SvDesc.
__attribute__((visibility("hidden"))) size_t batched_svd_lds_bytes(int64_t lmax, int64_t kmax);
__attribute__((visibility("hidden"))) re_status launch_bidiag_batched(hipStream_t s, const double* const* C,
                                                                     double* const* d, double* const* e,
                                                                     const int32_t* l, const int32_t* k, int32_t* info,
                                                                     int nblk, int64_t lmax, int64_t kmax);
__attribute__((visibility("hidden"))) re_status launch_sv_count_batched(hipStream_t s, const SvDesc* desc, int nblk,
                                                                       int64_t kmax);

}  // namespace re
