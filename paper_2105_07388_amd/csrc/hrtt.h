// Launchers of the hashed and the subsampled randomized DCT embeddings (HRTT and
// SRCT X, Sec. 3.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rankest.h"

namespace re {

// Rows of the DCT held in one workgroup's LDS: N complex FP32 values.
constexpr int64_t kHrttMaxN = 16384;

// N = the transform length for n columns (next power of two, at least 2).
__attribute__((visibility("hidden"))) int64_t hrtt_npad(int64_t n);
// Scratch of one call: bucket codes, bucket pointers, coordinate lists.
__attribute__((visibility("hidden"))) size_t hrtt_scratch_bytes(int64_t n, int64_t k);
// Draw the HRTT X of width k for n columns: its bucket lists and their run
// structure into `scratch` (hrtt_scratch_bytes).  RE_ERR_UNSUPPORTED when
// N > kHrttMaxN or k > N.
__attribute__((visibility("hidden"))) re_status launch_hrtt_hash(hipStream_t s, int64_t n, int64_t k, uint64_t seed,
                                                                void* scratch);
// B (m x k FP32, ldb) = A X for the HRTT X drawn into `scratch`; sign_bits: the
// SRHT X signs for N coordinates.
__attribute__((visibility("hidden"))) re_status launch_hrtt_rows(hipStream_t s, const float* A, int64_t m, int64_t n,
                                                                int64_t lda, int64_t k, const uint32_t* sign_bits,
                                                                const void* scratch, float* B, int64_t ldb);
// B (m x k FP32, ldb) = A X for the subsampled randomized DCT X:
// B[i][b] = sqrt(N) (F D a_i)_{sel[b]}, sel the k sampled coordinates (< N).
__attribute__((visibility("hidden"))) re_status launch_srct_rows(hipStream_t s, const float* A, int64_t m, int64_t n,
                                                                int64_t lda, int64_t k, const uint32_t* sign_bits,
                                                                const int32_t* sel, float* B, int64_t ldb);

}  // namespace re
