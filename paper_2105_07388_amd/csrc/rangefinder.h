// Launchers of the rangefinder stage (Algorithm 3, Sec. 5.1): the width rule,
// the thin QR of the kept sketch columns and B = Q^T A.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rankest.h"

#define RE_RF_HIDDEN __attribute__((visibility("hidden")))

namespace re {

// Width rule over the descending estimates sigma[0..k): out4 = {r, w, status,
// flags}; r = -1 when no r with r + p <= k qualifies, 0 for a zero sketch.
// norm_a <= 0 uses sigma[0] for ||A||.  info: status of the small SVD;
// tail: scratch of r1 + 1 doubles.
RE_RF_HIDDEN re_status launch_rf_width(hipStream_t s, const double* sigma, int64_t k, int32_t r1, int64_t n,
                                       double eps, int32_t p, double norm_a, const int32_t* info, double* tail,
                                       int32_t* out4);

// Split of the m rows of a Gram product or of Q^T A into chunks (a multiple
// of 16 rows each): the number of chunks and their length.
RE_RF_HIDDEN void rf_row_split(int64_t m, int64_t tiles, int64_t* splits, int64_t* rows_per_split);

// parts[s] (w x w, row-major, upper 64 x 64 tiles only) = V[rows of chunk s]^T
// V[rows of chunk s], FP64 products; V is m x w (FP32 if v32, else FP64), ldv.
RE_RF_HIDDEN re_status launch_rf_gram(hipStream_t s, const void* V, bool v32, int64_t m, int64_t w, int64_t ldv,
                                      int64_t splits, int64_t rows_per_split, double* parts);
// out[a][c] (ld ldo) = sum over s in order of parts[s][a][c] (rows x cols per
// part); upper: only a <= c.
RE_RF_HIDDEN re_status launch_rf_sum_parts(hipStream_t s, const double* parts, int64_t splits, int64_t rows,
                                           int64_t cols, bool upper, double* out, int64_t ldo);
// Cholesky factor of G (+ shift for the first pass) and the inverse of the
// factor (w x w, upper, row-major, zero rows / columns for dropped columns);
// keep[c] = new index of column c or -1; cnt2 = {kept columns, status};
// rdiag (w doubles, or NULL) receives the factor's diagonal.
RE_RF_HIDDEN size_t rf_chol_lds_bytes(int64_t w);
RE_RF_HIDDEN re_status launch_rf_chol(hipStream_t s, double* G, int64_t w, bool shift, int64_t m, double* Rinv,
                                      int32_t* keep, int32_t* cnt2, double* rdiag);
// sigma (k, descending) = |R3_jj R2_jj R1_jj| scale from the three passes'
// diagonals (rdiag3: 3 x k doubles, pass-major).
RE_RF_HIDDEN re_status launch_qr_sigma(hipStream_t s, const double* rdiag3, int64_t k, double scale, double* sigma);
// Q (ldq) = V Rinv for the w columns; column c goes to keep[c] (skipped when
// negative) if keep is given, else to c.  V as in launch_rf_gram.
RE_RF_HIDDEN re_status launch_rf_apply(hipStream_t s, const void* V, bool v32, int64_t m, int64_t w, int64_t ldv,
                                       const double* Rinv, const int32_t* keep, double* Q, int64_t ldq);
// C = Y B (l x k, FP64, leading dimension k) for a Gaussian Y (l x m FP32,
// ldy) and B (m x k FP32, ldb): 64 x 64 tiles on the FP64 matrix cores, the m
// rows split into chunks when the tiles alone cannot fill the chip, chunk
// partials (yb_parts_bytes of scratch) summed in a fixed order.
RE_RF_HIDDEN size_t yb_parts_bytes(int64_t l, int64_t k, int64_t m);
RE_RF_HIDDEN re_status launch_yb_tiled(hipStream_t s, const float* B, int64_t m, int64_t k, int64_t ldb, const float* Y,
                                       int64_t ldy, int64_t l, double* C, double* parts);
// parts[s] (w x n) = Q[rows of chunk s]^T A[rows of chunk s], FP32
// matrix-core products of FP32 A with Q rounded to FP32 (q32: m x w floats of
// scratch), FP64 accumulation across every 256 rows.
// FP64 C = A B on the matrix cores, K split over slices when M is short and K
// long (parts: gemm64_parts_bytes; nullptr when that is 0).
RE_RF_HIDDEN size_t gemm64_parts_bytes(int64_t M, int64_t N, int64_t K);
RE_RF_HIDDEN re_status launch_gemm64(hipStream_t s, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                                     const double* B, int64_t ldb, double* C, int64_t ldc, double* parts);
RE_RF_HIDDEN int64_t rf_qta_col_tiles(int64_t n);
RE_RF_HIDDEN re_status launch_rf_qta(hipStream_t s, const double* Q, int64_t ldq, int64_t w, const float* A,
                                     int64_t m, int64_t n, int64_t lda, int64_t splits, int64_t rows_per_split,
                                     float* q32, double* parts);

}  // namespace re
