// The sketch-size network of the learned policy: forward, mean-squared-error
// gradient and Adam, FP32.  Small and launch-bound by design: the whole
// parameter vector (26 KB) sits in LDS, one thread carries one sample through
// the forward pass, and every gradient entry is summed over the batch by one
// thread in sample order, so training is deterministic.
#include "common.h"
#include "learned.h"

namespace re {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ void load_params(const float* __restrict__ P, float* sp) {
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) sp[i] = P[i];
  __syncthreads();
}

// y_s = w3 . relu(W2 relu(W1 x_s + b1) + b2) + b3; keeps z1, z2 when asked.
__global__ void __launch_bounds__(kThreads) k_mlp_forward(const float* __restrict__ P, const float* __restrict__ X,
                                                          int64_t batch, float* __restrict__ y, float* __restrict__ z1,
                                                          float* __restrict__ z2) {
  __shared__ float sp[kMlpParams];
  load_params(P, sp);
  const int64_t smp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (smp >= batch) return;
  float x[kMlpIn];
#pragma unroll
  for (int f = 0; f < kMlpIn; ++f) x[f] = X[smp * kMlpIn + f];
  float h1[kMlpH];
#pragma unroll
  for (int i = 0; i < kMlpH; ++i) {
    float z = sp[kOffB1 + i];
#pragma unroll
    for (int f = 0; f < kMlpIn; ++f) z = fmaf(sp[kOffW1 + i * kMlpIn + f], x[f], z);
    if (z1) z1[smp * kMlpH + i] = z;
    h1[i] = z > 0.0f ? z : 0.0f;
  }
  float out = sp[kOffB3];
  for (int j = 0; j < kMlpH; ++j) {
    float z = sp[kOffB2 + j];
#pragma unroll
    for (int i = 0; i < kMlpH; ++i) z = fmaf(sp[kOffW2 + j * kMlpH + i], h1[i], z);
    if (z2) z2[smp * kMlpH + j] = z;
    out = fmaf(sp[kOffW3 + j], z > 0.0f ? z : 0.0f, out);
  }
  y[smp] = out;
}

// Per-sample output and hidden-layer error terms of L = (1/B) sum (y - t)^2:
// dy = 2 (y - t) / B, dz2 = dy w3 [z2 > 0], dz1 = (W2^T dz2) [z1 > 0].
__global__ void __launch_bounds__(kThreads) k_mlp_backprop(const float* __restrict__ P, const float* __restrict__ T,
                                                           int64_t batch, const float* __restrict__ y,
                                                           const float* __restrict__ z1, const float* __restrict__ z2,
                                                           float* __restrict__ dz1, float* __restrict__ dz2,
                                                           float* __restrict__ dy) {
  __shared__ float sp[kMlpParams];
  load_params(P, sp);
  const int64_t smp = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (smp >= batch) return;
  const float d = 2.0f * (y[smp] - T[smp]) / (float)batch;
  dy[smp] = d;
  float e2[kMlpH];
#pragma unroll
  for (int j = 0; j < kMlpH; ++j) {
    e2[j] = z2[smp * kMlpH + j] > 0.0f ? d * sp[kOffW3 + j] : 0.0f;
    dz2[smp * kMlpH + j] = e2[j];
  }
  for (int i = 0; i < kMlpH; ++i) {
    float g = 0.0f;
#pragma unroll
    for (int j = 0; j < kMlpH; ++j) g = fmaf(sp[kOffW2 + j * kMlpH + i], e2[j], g);
    dz1[smp * kMlpH + i] = z1[smp * kMlpH + i] > 0.0f ? g : 0.0f;
  }
}

// One thread per parameter, summed over the batch in sample order.
__global__ void __launch_bounds__(kThreads) k_mlp_wgrad(const float* __restrict__ X, int64_t batch,
                                                        const float* __restrict__ z1, const float* __restrict__ z2,
                                                        const float* __restrict__ dz1, const float* __restrict__ dz2,
                                                        const float* __restrict__ dy, float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  float g = 0.0f;
  if (p < kOffB1) {
    const int i = p / kMlpIn, f = p % kMlpIn;
    for (int64_t s = 0; s < batch; ++s) g = fmaf(dz1[s * kMlpH + i], X[s * kMlpIn + f], g);
  } else if (p < kOffW2) {
    const int i = p - kOffB1;
    for (int64_t s = 0; s < batch; ++s) g += dz1[s * kMlpH + i];
  } else if (p < kOffB2) {
    const int j = (p - kOffW2) / kMlpH, i = (p - kOffW2) % kMlpH;
    for (int64_t s = 0; s < batch; ++s) {
      const float h = z1[s * kMlpH + i];
      g = fmaf(dz2[s * kMlpH + j], h > 0.0f ? h : 0.0f, g);
    }
  } else if (p < kOffW3) {
    const int j = p - kOffB2;
    for (int64_t s = 0; s < batch; ++s) g += dz2[s * kMlpH + j];
  } else if (p < kOffB3) {
    const int j = p - kOffW3;
    for (int64_t s = 0; s < batch; ++s) {
      const float h = z2[s * kMlpH + j];
      g = fmaf(dy[s], h > 0.0f ? h : 0.0f, g);
    }
  } else {
    for (int64_t s = 0; s < batch; ++s) g += dy[s];
  }
  G[p] = g;
}

// Mean squared error, one workgroup: strided partial sums, then a fixed tree.
__global__ void __launch_bounds__(kThreads) k_mlp_loss(const float* __restrict__ y, const float* __restrict__ T,
                                                       int64_t batch, float* __restrict__ loss) {
  __shared__ float part[kThreads];
  float a = 0.0f;
  for (int64_t s = threadIdx.x; s < batch; s += kThreads) {
    const float d = y[s] - T[s];
    a = fmaf(d, d, a);
  }
  part[threadIdx.x] = a;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = part[0] / (float)batch;
}

// Adam (Kingma & Ba): c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t).
__global__ void k_mlp_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ M,
                           float* __restrict__ V, int64_t n, float lr, float beta1, float beta2, float eps, float c1,
                           float c2) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = beta1 * M[i] + (1.0f - beta1) * g;
  const float v = beta2 * V[i] + (1.0f - beta2) * g * g;
  M[i] = m;
  V[i] = v;
  P[i] -= lr * (m * c1) / (sqrtf(v * c2) + eps);
}

}  // namespace

re_status launch_mlp_forward(hipStream_t s, const float* P, const float* X, int64_t batch, float* y, float* z1,
                             float* z2) {
  if (batch <= 0) return RE_OK;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)cdiv(batch, kThreads)), dim3(kThreads), 0, s, P, X, batch, y, z1,
                     z2);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_mlp_loss_grad(hipStream_t s, const float* P, const float* X, const float* T, int64_t batch,
                               float* scratch, float* grad, float* loss) {
  if (batch <= 0) return RE_ERR_INVALID_ARG;
  float* z1 = scratch;
  float* z2 = z1 + batch * kMlpH;
  float* dz1 = z2 + batch * kMlpH;
  float* dz2 = dz1 + batch * kMlpH;
  float* dy = dz2 + batch * kMlpH;
  float* y = dy + batch;  // the caller provides mlp_scratch_floats(batch) + batch floats
  const unsigned g = (unsigned)cdiv(batch, kThreads);
  hipLaunchKernelGGL(k_mlp_forward, dim3(g), dim3(kThreads), 0, s, P, X, batch, y, z1, z2);
  hipLaunchKernelGGL(k_mlp_backprop, dim3(g), dim3(kThreads), 0, s, P, T, batch, y, z1, z2, dz1, dz2, dy);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3((unsigned)cdiv(kMlpParams, kThreads)), dim3(kThreads), 0, s, X, batch, z1, z2,
                     dz1, dz2, dy, grad);
  if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(kThreads), 0, s, y, T, batch, loss);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_mlp_adam(hipStream_t s, float* P, const float* G, float* M, float* V, int64_t n, float lr,
                          float beta1, float beta2, float eps, float c1, float c2) {
  if (n <= 0) return RE_OK;
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)cdiv(n, 256)), dim3(256), 0, s, P, G, M, V, n, lr, beta1, beta2, eps,
                     c1, c2);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
