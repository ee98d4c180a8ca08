// Internal declarations of the learned sketch-size policy (MLP kernels).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rankest.h"

namespace re {

// 35 inputs -> 64 ReLU -> 64 ReLU -> 1; parameter vector W1 (64 x 35),
// b1, W2 (64 x 64), b2, w3, b3.
constexpr int kMlpIn = RE_MLP_INPUTS, kMlpH = 64, kMlpParams = RE_MLP_PARAMS;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kMlpH * kMlpIn, kOffW2 = kOffB1 + kMlpH, kOffB2 = kOffW2 + kMlpH * kMlpH,
              kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpH;
static_assert(kOffB3 + 1 == kMlpParams, "parameter layout");

// Floats of activation scratch for a batch (z1, z2, dz1, dz2: 64 each; dy).
inline size_t mlp_scratch_floats(int64_t batch) { return (size_t)batch * (4 * kMlpH + 1); }

__attribute__((visibility("hidden"))) re_status launch_mlp_forward(hipStream_t s, const float* P, const float* X,
                                                                  int64_t batch, float* y, float* z1, float* z2);
__attribute__((visibility("hidden"))) re_status launch_mlp_loss_grad(hipStream_t s, const float* P, const float* X,
                                                                    const float* T, int64_t batch, float* scratch,
                                                                    float* grad, float* loss);
__attribute__((visibility("hidden"))) re_status launch_mlp_adam(hipStream_t s, float* P, const float* G, float* M,
                                                               float* V, int64_t n, float lr, float beta1, float beta2,
                                                               float eps, float c1, float c2);

}  // namespace re
