// Launchers of the hashed and the subsampled randomized DCT embeddings (HRTT and
// SRCT X, Sec. 3.3).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rankest.h"

namespace re {

// Rows of the DCT held in one workgroup's LDS: N complex FP32 values.  Longer
// rows (up to kDctMaxN) go through a four-step split of the FFT with a
// workspace in HBM (dct_long_ws_bytes), and the hashed DCT's lists are built
// per chunk of kHrttMaxN coordinates (so k <= kHrttMaxN there).
constexpr int64_t kHrttMaxN = 16384;
constexpr int64_t kDctMaxN = int64_t(1) << 20;
constexpr int64_t kDctLongWsBytes = int64_t(256) << 20;  // rows per pass: as many as fit this

// Whether the DCT X of width k (hashed or subsampled) takes n columns.
__attribute__((visibility("hidden"))) bool dct_x_supported(int64_t n, int64_t k, bool hash);
// Workspace of the long-row path for an m-row A (0 when N <= kHrttMaxN).
__attribute__((visibility("hidden"))) size_t dct_long_ws_bytes(int64_t m, int64_t n, bool hash);

// N = the transform length for n columns (next power of two, at least 2).
__attribute__((visibility("hidden"))) int64_t hrtt_npad(int64_t n);
// Scratch of one call: bucket codes, bucket pointers, coordinate lists.
__attribute__((visibility("hidden"))) size_t hrtt_scratch_bytes(int64_t n, int64_t k);
// Draw the HRTT X of width k for n columns: its bucket lists and their run
// structure into `scratch` (hrtt_scratch_bytes).  RE_ERR_UNSUPPORTED unless
// dct_x_supported(n, k, true).
__attribute__((visibility("hidden"))) re_status launch_hrtt_hash(hipStream_t s, int64_t n, int64_t k, uint64_t seed,
                                                                void* scratch);
// B (m x k FP32, ldb) = A X for the HRTT X drawn into `scratch`; sign_bits: the
// SRHT X signs for N coordinates; ws: dct_long_ws_bytes(m, n, true) bytes.
__attribute__((visibility("hidden"))) re_status launch_hrtt_rows(hipStream_t s, const float* A, int64_t m, int64_t n,
                                                                int64_t lda, int64_t k, const uint32_t* sign_bits,
                                                                const void* scratch, float* B, int64_t ldb, void* ws);
// B (m x k FP32, ldb) = A X for the subsampled randomized DCT X:
// B[i][b] = sqrt(N) (F D a_i)_{sel[b]}, sel the k sampled coordinates (< N);
// ws: dct_long_ws_bytes(m, n, false) bytes.
__attribute__((visibility("hidden"))) re_status launch_srct_rows(hipStream_t s, const float* A, int64_t m, int64_t n,
                                                                int64_t lda, int64_t k, const uint32_t* sign_bits,
                                                                const int32_t* sel, float* B, int64_t ldb, void* ws);

}  // namespace re
