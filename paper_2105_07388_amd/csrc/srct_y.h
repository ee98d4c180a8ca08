// Launchers of the subsampled randomized DCT as Y (Sec. 4 with F a DCT),
// applied along the columns of B in two levels (a stored first level of
// 32-point DFTs, then the sampled rows).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rankest.h"

namespace re {

// M: the transform length for m rows (next power of two, at least 2).
__attribute__((visibility("hidden"))) int64_t srct_y_npad(int64_t m);
// Level-1 DFT length for transform length M: min(M, 32).
__attribute__((visibility("hidden"))) int srct_y_m2(int64_t M);
// Bytes of the stored first level U (real and imaginary planes, M x k each, in
// B's type) and of the class-ordering scratch of level 2.
__attribute__((visibility("hidden"))) size_t srct_y_u_bytes(int64_t m, int64_t k, int dtype);
__attribute__((visibility("hidden"))) size_t srct_y_order_bytes(int64_t l);
// Level 1 on k columns of B (m x k, leading dimension ldb, FP32 or FP64): the
// signed, reordered, zero-padded columns cut into M / M2 strided pieces and
// their M2-point DFTs, into U (two planes of M rows, leading dimension ldu:
// column t of B goes to column t of U, so appended columns of B go to the
// same columns of U).
__attribute__((visibility("hidden"))) re_status launch_srct_y_lo(hipStream_t s, const void* B, int bdtype, int64_t m,
                                                                int64_t k, int64_t ldb, const uint32_t* sign_bits,
                                                                void* U, int64_t ldu);
// Level 2: C (l x k FP64, leading dimension k) = the l sampled rows sel (< M)
// of sqrt(M) F D B from U (k columns, leading dimension ldu).
__attribute__((visibility("hidden"))) re_status launch_srct_y_hi(hipStream_t s, const void* U, int bdtype, int64_t m,
                                                                int64_t k, int64_t ldu, const int32_t* sel, int64_t l,
                                                                int32_t* order_scratch, double* C);

}  // namespace re
