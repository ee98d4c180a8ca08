// Driver for the library built with AddressSanitizer and UndefinedBehavior-
// Sanitizer on its host code (GPU code is built as usual).  It calls the C ABI
// the way a C caller would: argument errors on every entry point first (no GPU
// needed), then, when a GPU is present, the estimate in each form on small
// synthetic matrices, the forced error paths (workspace cap, barrier that
// gives up, NaN input) and the handle's teardown.  Exit status 0 and the line
// "host sanitizer driver ok" mean no check failed and no sanitizer report
// stopped the run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "rankest.h"

static int g_fails = 0;
// a call's status against the expected one, both printed on a mismatch
#define EXPECT_ST(call, want)                                                                          \
  do {                                                                                                 \
    const re_status st_ = (call);                                                                      \
    if (st_ != (want)) {                                                                               \
      fprintf(stderr, "check failed at line %d: %s returned %d (%s), expected %d\n", __LINE__, #call, \
              (int)st_, re_status_string(st_), (int)(want));                                          \
      ++g_fails;                                                                                       \
    }                                                                                                  \
  } while (0)
#define EXPECT(cond)                                                     \
  do {                                                                   \
    if (!(cond)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fails;                                                         \
    }                                                                    \
  } while (0)

// A = U diag(s) V^T with U, V built from cosines (exactly orthogonal up to
// rounding: columns of a DCT-II basis), s_i = 10^-i for i < r, zero after.
static std::vector<double> low_rank(int64_t m, int64_t n, int r) {
  std::vector<double> A((size_t)m * n, 0.0);
  for (int t = 0; t < r; ++t) {
    const double s = std::pow(10.0, -t);
    const double cu = std::sqrt(2.0 / m), cv = std::sqrt(2.0 / n);
    for (int64_t i = 0; i < m; ++i) {
      const double u = cu * std::cos(M_PI * (i + 0.5) * (t + 1) / m);
      for (int64_t j = 0; j < n; ++j) A[i * n + j] += s * u * cv * std::cos(M_PI * (j + 0.5) * (t + 1) / n);
    }
  }
  return A;
}

static void host_paths() {
  for (int s = 1; s >= -8; --s) EXPECT(re_status_string((re_status)s) != nullptr);
  EXPECT(re_r1_from_k(1) == 1);
  EXPECT(re_r1_from_k(11) == 10);
  EXPECT(re_r1_from_k(384) == 349);
  EXPECT(re_singular_values_noalloc_fits(576, 384) == 1);
  EXPECT(re_singular_values_noalloc_fits(100000, 5000) == 0);
  EXPECT(re_sketch_y_rows(1000) >= 1000);
  const double sig[5] = {1.0, 0.5, 1e-6, 5e-7, 0.0};
  int32_t r = -1;
  double q = 0.0;
  EXPECT(re_gap_rank(sig, 5, 4, &r, &q) == RE_OK && r == 2 && q == 0.5 / 1e-6);
  EXPECT_ST(re_gap_rank(nullptr, 5, 4, &r, &q), RE_ERR_INVALID_ARG);
  EXPECT_ST(re_create(nullptr, nullptr), RE_ERR_INVALID_ARG);
  EXPECT_ST(re_destroy(nullptr), RE_OK);
  EXPECT_ST(re_set_limits(nullptr, 0, 0), RE_ERR_INVALID_ARG);
  EXPECT_ST(re_set_profiling(nullptr, 1), RE_ERR_INVALID_ARG);
  size_t bytes = 0;
  EXPECT_ST(re_workspace_bytes(nullptr, &bytes), RE_ERR_INVALID_ARG);
  re_sketch sk = {RE_GAUSSIAN, RE_GAUSSIAN, 8, 12, RE_PREC_NATIVE};
  int32_t r1 = 0;
  uint32_t fl = 0;
  double sigma[8];
  EXPECT(re_rank_estimate(nullptr, (const void*)16, RE_F32, 100, 50, 50, 1e-3, &sk, 0, &r, sigma, &r1, &fl) ==
         RE_ERR_INVALID_ARG);
  EXPECT_ST(re_singular_values(nullptr, nullptr, 10, 5, 1.0, nullptr), RE_ERR_INVALID_ARG);
}

static void gpu_paths() {
  re_handle h = nullptr;
  EXPECT_ST(re_create(&h, nullptr), RE_OK);
  if (!h) return;
  const int64_t m = 1500, n = 700;
  const std::vector<double> Ad = low_rank(m, n, 5);
  std::vector<float> Af(Ad.begin(), Ad.end());
  float* A32 = nullptr;
  double* A64 = nullptr;
  EXPECT(hipMalloc(&A32, Af.size() * 4) == hipSuccess);
  EXPECT(hipMalloc(&A64, Ad.size() * 8) == hipSuccess);
  EXPECT(hipMemcpy(A32, Af.data(), Af.size() * 4, hipMemcpyHostToDevice) == hipSuccess);
  EXPECT(hipMemcpy(A64, Ad.data(), Ad.size() * 8, hipMemcpyHostToDevice) == hipSuccess);
  std::vector<double> sigma(1024);
  int32_t r = -1, r1 = 0;
  uint32_t fl = 0;
  // every sketch kind and format the single estimate takes (values 1, 0.1,
  // 0.01, 1e-3, 1e-4: three above eps = 3e-3)
  const int kinds[][3] = {{RE_GAUSSIAN, RE_GAUSSIAN, RE_PREC_NATIVE}, {RE_SRHT, RE_SRHT, RE_PREC_NATIVE},
                          {RE_GAUSSIAN, RE_SRHT, RE_PREC_BF16},       {RE_GAUSSIAN, RE_GAUSSIAN, RE_PREC_AUTO},
                          {RE_HRTT, RE_SRHT, RE_PREC_NATIVE},         {RE_SRCT, RE_SRCT, RE_PREC_NATIVE}};
  for (const auto& kd : kinds) {
    re_sketch sk = {kd[0], kd[1], 40, 60, kd[2]};
    const re_status st = re_rank_estimate(h, A32, RE_F32, m, n, n, 3e-3, &sk, 7, &r, sigma.data(), &r1, &fl);
    EXPECT(st == RE_OK);
    if (st == RE_OK) EXPECT(r == 3);
  }
  {
    re_sketch sk = {RE_GAUSSIAN, RE_GAUSSIAN, 40, 60, RE_PREC_NATIVE};
    EXPECT(re_rank_estimate(h, A64, RE_F64, m, n, n, 3e-3, &sk, 7, &r, sigma.data(), &r1, &fl) == RE_OK && r == 3);
    // argument errors on a live handle leave it usable
    re_sketch bad = {RE_GAUSSIAN, RE_GAUSSIAN, 800, 900, RE_PREC_NATIVE};
    EXPECT_ST(re_rank_estimate(h, A32, RE_F32, m, n, n, 1e-3, &bad, 7, &r, sigma.data(), &r1, &fl), RE_ERR_INVALID_ARG);
    EXPECT(re_rank_estimate(h, A32, RE_F32, m, n, n - 1, 3e-3, &sk, 7, &r, sigma.data(), &r1, &fl) ==
           RE_ERR_INVALID_ARG);
    EXPECT_ST(re_rank_estimate(h, A32, RE_F32, m, n, n, 0.0, &sk, 7, &r, sigma.data(), &r1, &fl), RE_ERR_INVALID_ARG);
    // profiling and stage times
    double ms[RE_NUM_STAGES];
    EXPECT_ST(re_set_profiling(h, 1), RE_OK);
    EXPECT_ST(re_rank_estimate(h, A32, RE_F32, m, n, n, 3e-3, &sk, 7, &r, sigma.data(), &r1, &fl), RE_OK);
    EXPECT(re_last_stage_ms(h, ms) == RE_OK && ms[RE_STAGE_AX] >= 0.0);
    EXPECT_ST(re_set_profiling(h, 0), RE_OK);
    size_t bytes = 0;
    EXPECT(re_workspace_bytes(h, &bytes) == RE_OK && bytes > 0);
    // workspace cap: NO_MEMORY from a fresh handle, then recovery
    re_handle h2 = nullptr;
    EXPECT_ST(re_create(&h2, nullptr), RE_OK);
    EXPECT_ST(re_set_limits(h2, 4096, 0), RE_OK);
    EXPECT_ST(re_rank_estimate(h2, A32, RE_F32, m, n, n, 3e-3, &sk, 7, &r, sigma.data(), &r1, &fl), RE_ERR_NO_MEMORY);
    EXPECT_ST(re_set_limits(h2, 0, 0), RE_OK);
    EXPECT(re_rank_estimate(h2, A32, RE_F32, m, n, n, 3e-3, &sk, 7, &r, sigma.data(), &r1, &fl) == RE_OK && r == 3);
    EXPECT_ST(re_destroy(h2), RE_OK);
  }
  // the multi-workgroup small SVD: forced give-up, then the values
  {
    const int64_t l = 576, k = 384;
    std::vector<double> C((size_t)l * k);
    for (int64_t i = 0; i < l; ++i)
      for (int64_t j = 0; j < k; ++j) C[i * k + j] = std::sin(0.37 * i + 1.3 * j) + (i == j ? 2.0 : 0.0);
    double *Cd = nullptr, *sd = nullptr;
    EXPECT(hipMalloc(&Cd, C.size() * 8) == hipSuccess);
    EXPECT(hipMalloc(&sd, k * 8) == hipSuccess);
    EXPECT(hipMemcpy(Cd, C.data(), C.size() * 8, hipMemcpyHostToDevice) == hipSuccess);
    EXPECT_ST(re_set_limits(h, 0, -1), RE_OK);
    EXPECT_ST(re_singular_values(h, Cd, l, k, 1.0, sd), RE_ERR_NO_CONVERGENCE);
    EXPECT_ST(re_set_limits(h, 0, 0), RE_OK);
    EXPECT_ST(re_singular_values(h, Cd, l, k, 1.0, sd), RE_OK);
    std::vector<double> s(k);
    EXPECT(hipMemcpy(s.data(), sd, k * 8, hipMemcpyDeviceToHost) == hipSuccess);
    for (int64_t i = 1; i < k; ++i) EXPECT(s[i] <= s[i - 1] && s[i] >= 0.0);
    // NaN in the sketch
    C[5] = NAN;
    EXPECT(hipMemcpy(Cd, C.data(), C.size() * 8, hipMemcpyHostToDevice) == hipSuccess);
    EXPECT_ST(re_singular_values(h, Cd, l, k, 1.0, sd), RE_ERR_NONFINITE);
    (void)hipFree(Cd);
    (void)hipFree(sd);
  }
  // batched form on three views of A
  {
    re_block blocks[3] = {{A32, 1500, 700, 700}, {A32, 900, 400, 700}, {A32, 1200, 650, 700}};
    re_sketch sk = {RE_GAUSSIAN, RE_GAUSSIAN, 24, 36, RE_PREC_NATIVE};
    int32_t rb[3];
    std::vector<double> sb(3 * 24);
    uint32_t fb[3];
    EXPECT_ST(re_rank_estimate_batched(h, blocks, 3, RE_F32, 3e-3, &sk, 3, rb, sb.data(), fb), RE_OK);
  }
  // adaptive width and the gap search
  {
    re_adaptive ad = {8, 256, 1.5, nullptr, 0.0};
    int32_t k_out = 0, l_out = 0, rounds = 0, kp = 0;
    EXPECT_ST(re_rank_adaptive(h, A32, RE_F32, m, n, n, 3e-3, &ad, 5, &r, sigma.data(), &k_out, &l_out, &rounds, &kp,
                            &fl), RE_OK);
    re_gap_search gs = {16, 16, 128, RE_GAUSSIAN, 1.5, 100.0, 1e-5};
    int32_t am = 0, kk = 0, ll = 0, rr = 0;
    double ratio = 0.0, aratio = 0.0;
    std::vector<double> spectra(8 * 128);
    EXPECT_ST(re_rank_gap(h, A32, RE_F32, m, n, n, &gs, 5, &r, &ratio, &am, &aratio, sigma.data(), &kk, &ll, &rr,
                       spectra.data(), 8, &fl), RE_OK);
  }
  // NaN in A
  {
    Af[123] = NAN;
    EXPECT(hipMemcpy(A32, Af.data(), Af.size() * 4, hipMemcpyHostToDevice) == hipSuccess);
    re_sketch sk = {RE_GAUSSIAN, RE_GAUSSIAN, 40, 60, RE_PREC_NATIVE};
    EXPECT_ST(re_rank_estimate(h, A32, RE_F32, m, n, n, 3e-3, &sk, 7, &r, sigma.data(), &r1, &fl), RE_ERR_NONFINITE);
  }
  (void)hipFree(A32);
  (void)hipFree(A64);
  EXPECT_ST(re_destroy(h), RE_OK);
}

int main() {
  host_paths();
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0) {
    gpu_paths();
    printf("GPU paths run on device 0\n");
  } else {
    (void)hipGetLastError();
    printf("no GPU: host paths only\n");
  }
  if (g_fails) {
    printf("host sanitizer driver: %d checks failed\n", g_fails);
    return 1;
  }
  printf("host sanitizer driver ok\n");
  return 0;
}
