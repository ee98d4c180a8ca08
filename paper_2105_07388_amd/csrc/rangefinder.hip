// Rangefinder stage of rank estimation combined with the randomized
// rangefinder (Algorithm 3, Sec. 5.1): the width rule over the extended
// estimates (Eq. errRFfro), the thin QR of the first w = r + p columns of the
// sketch A X, and B = Q^T A.
//
// The paper leaves the thin QR method open.  Here it is shifted CholeskyQR3
// (Fukaya, Kannan, Nakatsukasa, Zhang and Yamamoto, SIAM J. Sci. Comput. 2020):
// three passes of  G = V^T V,  G + s I = R^T R,  V <- V R^-1, the first with
// the shift s = 11 (m w + w (w + 1)) u ||V||_F^2, the other two unshifted.
// Every pass is two tall contractions over the m rows on the FP64 matrix
// cores and one w x w factorisation; no pass reads A.  A column whose pivot
// falls below 16 u times the largest diagonal is numerically dependent on the
// earlier ones (the shifted pass never gets there: its pivots are at least s);
// it is left out of Q (its span adds nothing at FP64 precision), so Q has
// orthonormal columns even for an exactly rank-deficient sketch.
#include <limits.h>

#include "common.h"
#include "rangefinder.h"

namespace re {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr double kU64 = 0x1.0p-53;  // FP64 unit roundoff

// ---------------------------------------------------------------------------
// Width rule (Algorithm 3 steps 4-5): tail[r] = sum_{j=r}^{r1-1} s_j^2 (0-based,
// accumulated from the end), the extension s_j = s_{r1-1} for j >= r1, and the
// smallest r >= 1 with (1 + r/(p-1))^(1/2) (tail + extension)^(1/2) <= eps ||A||.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rf_width(const double* __restrict__ sigma, int k, int r1, int64_t n,
                                                  double eps, int p, double norm_a, const int32_t* __restrict__ info,
                                                  double* __restrict__ tail, int32_t* __restrict__ out) {
  __shared__ int s_best, s_bad;
  const int tid = threadIdx.x;
  if (tid == 0) {
    s_best = INT_MAX;
    s_bad = 0;
  }
  __syncthreads();
  int bad = 0;
  for (int i = tid; i < k; i += blockDim.x) bad |= !isfinite(sigma[i]);
  if (bad) atomicOr(&s_bad, 1);
  if (tid == 0) {
    double t = 0.0;
    tail[r1] = 0.0;
    for (int j = r1 - 1; j >= 0; --j) {
      t += sigma[j] * sigma[j];
      tail[j] = t;
    }
  }
  __syncthreads();
  const double s1 = sigma[0];
  const double target = eps * (norm_a > 0.0 ? norm_a : s1);
  const double ext = sigma[r1 - 1] * sigma[r1 - 1];
  for (int r = 1 + tid; r + p <= k; r += blockDim.x) {
    const double head = r < r1 ? tail[r] : 0.0;
    const double extra = (double)(n - (r > r1 ? r : r1)) * ext;
    const double b = sqrt(1.0 + (double)r / (double)(p - 1)) * sqrt(head + extra);
    if (b <= target) atomicMin(&s_best, r);
  }
  __syncthreads();
  if (tid != 0) return;
  int32_t st = info ? info[0] : 0;
  if (st == 0 && s_bad) st = RE_ERR_NONFINITE;
  int32_t r = 0, w = 0;
  uint32_t flags = 0;
  if (st == 0) {
    if (!(s1 > 0.0)) {
      flags |= RE_FLAG_ZERO;
    } else if (s_best == INT_MAX) {
      r = -1;
      flags |= RE_FLAG_NOT_CONVERGED;
    } else {
      r = s_best;
      w = r + p;
    }
  }
  out[0] = r;
  out[1] = w;
  out[2] = st;
  out[3] = (int32_t)flags;
}

// ---------------------------------------------------------------------------
// Gram partials: parts[s][a][c] = sum over the rows i of chunk s of V[i][a] V[i][c]
// for the 64 x 64 tiles with tile row <= tile column.  Four wavefronts, each a
// 32 x 32 quarter as 2 x 2 v_mfma_f64_16x16x4f64 tiles (operand lane q: row or
// column q % 16, K index q / 16; accumulator r of lane q: row q / 16 + 4 r,
// column q % 16).  K steps of 16 rows through double-buffered LDS.
// ---------------------------------------------------------------------------
constexpr int kGBK = 16, kGP = 80;  // rows per K step; LDS pitch in doubles

template <typename TI>
__global__ void __launch_bounds__(256) k_rf_gram(const TI* __restrict__ V, int64_t m, int64_t w, int64_t ldv,
                                                 int64_t rps, double* __restrict__ parts) {
  const int tj = blockIdx.x, ti = blockIdx.y;
  if (ti > tj) return;
  __shared__ double sU[2][kGBK * kGP], sV[2][kGBK * kGP];
  const int64_t ib = (int64_t)blockIdx.z * rps;
  const int64_t ie = ib + rps < m ? ib + rps : m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q16 = lane & 15, kq = lane >> 4, wy = wave >> 1, wx = wave & 1;
  const int64_t a0 = (int64_t)ti * 64, b0 = (int64_t)tj * 64;
  const int lr = tid >> 4, lc = (tid & 15) * 4;  // loader: row, first of 4 columns
  double ru[4], rv[4];
  auto load = [&](int64_t i0) {
    const int64_t i = i0 + lr;
    const bool ok = i < ie;
    const TI* __restrict__ row = V + (ok ? i : 0) * ldv;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t a = a0 + lc + q, b = b0 + lc + q;
      ru[q] = (ok && a < w) ? (double)row[a] : 0.0;
      rv[q] = (ok && b < w) ? (double)row[b] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sU[buf][lr * kGP + lc + q] = ru[q];
      sV[buf][lr * kGP + lc + q] = rv[q];
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t nsteps = (ie - ib + kGBK - 1) / kGBK;
  load(ib);
  store(0);
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    if (st + 1 < nsteps) load(ib + (st + 1) * kGBK);
#pragma unroll
    for (int kk = 0; kk < kGBK; kk += 4) {
      const double* u = &sU[buf][(kk + kq) * kGP + wy * 32 + q16];
      const double* v = &sV[buf][(kk + kq) * kGP + wx * 32 + q16];
      const double u0 = u[0], u1 = u[16], v0 = v[0], v1 = v[16];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0, v0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0, v1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1, v0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1, v1, acc[1][1], 0, 0, 0);
    }
    if (st + 1 < nsteps) store(buf ^ 1);
    __syncthreads();
  }
  double* __restrict__ part = parts + (int64_t)blockIdx.z * w * w;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t a = a0 + wy * 32 + x * 16 + kq + 4 * r, c = b0 + wx * 32 + y * 16 + q16;
        if (a < w && c < w) part[a * w + c] = acc[x][y][r];
      }
}

// out[a][c] = sum_s parts[s][a][c], s in increasing order (deterministic).
__global__ void k_rf_sum_parts(const double* __restrict__ parts, int64_t splits, int64_t rows, int64_t cols, int upper,
                               double* __restrict__ out, int64_t ldo) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t a = e / cols, c = e - a * cols;
    if (upper && a > c) continue;
    double t = 0.0;
    for (int64_t s = 0; s < splits; ++s) t += parts[s * total + e];
    out[a * ldo + c] = t;
  }
}

// ---------------------------------------------------------------------------
// Cholesky factor and its inverse, one workgroup.  G (w x w, upper triangle
// used) is factored in place (in LDS when it fits, else in global memory):
// right-looking, one pivot per step, G + s I = R^T R.  Then R^-1 by rows from
// the bottom: Rinv[t][c] = (delta_tc - sum_{t<j<=c} R[t][j] Rinv[j][c]) / R[t][t].
// ---------------------------------------------------------------------------
constexpr int kCholThreads = 1024;
constexpr int64_t kCholLdsMaxW = 136;  // w^2 doubles within 148 KiB

__device__ double block_sum(double v, double* red) {
  // fixed-shape tree: the same order for every call with the same blockDim
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ double block_max(double v, double* red) {
  const int tid = threadIdx.x;
  red[tid] = v;
  __syncthreads();
  for (int h = blockDim.x >> 1; h > 0; h >>= 1) {
    if (tid < h) red[tid] = fmax(red[tid], red[tid + h]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kCholThreads) k_rf_chol(double* __restrict__ G, int w, int shift, int64_t m,
                                                         int use_lds, double* __restrict__ Rinv,
                                                         int32_t* __restrict__ keep, int32_t* __restrict__ cnt2,
                                                         double* __restrict__ rdiag) {
  extern __shared__ double lds[];
  __shared__ double red[kCholThreads];
  __shared__ int s_bad;
  const int tid = threadIdx.x, nth = blockDim.x;
  double* R = use_lds ? lds : G;
  if (tid == 0) s_bad = 0;
  if (use_lds)
    for (int64_t e = tid; e < (int64_t)w * w; e += nth) lds[e] = G[e];
  __syncthreads();
  double tr = 0.0, mx = 0.0;
  int bad = 0;
  for (int j = tid; j < w; j += nth) {
    const double d = R[(int64_t)j * w + j];
    bad |= !isfinite(d);
    tr += d;
    mx = fmax(mx, d);
  }
  if (bad) atomicOr(&s_bad, 1);
  tr = block_sum(tr, red);
  mx = block_max(mx, red);
  const double s = shift ? 11.0 * ((double)m * w + (double)w * (w + 1)) * kU64 * tr : 0.0;
  const double thr = 16.0 * kU64 * (mx + s);
  for (int j = tid; j < w; j += nth) R[(int64_t)j * w + j] += s;
  __syncthreads();
  for (int j = 0; j < w; ++j) {
    double* Rj = R + (int64_t)j * w;
    const double d = Rj[j];
    const bool kj = isfinite(d) && d > thr;
    const double rjj = kj ? sqrt(d) : 0.0, inv = kj ? 1.0 / rjj : 0.0;
    for (int c = j + 1 + tid; c < w; c += nth) Rj[c] *= inv;
    __syncthreads();
    if (tid == 0) {
      Rj[j] = rjj;
      if (!isfinite(d)) s_bad = 1;
    }
    const int L = w - j - 1;
    for (int e = tid; e < L * L; e += nth) {
      const int a = j + 1 + e / L, b = j + 1 + e % L;
      if (a <= b) R[(int64_t)a * w + b] -= Rj[a] * Rj[b];
    }
    __syncthreads();
  }
  if (rdiag)
    for (int j = tid; j < w; j += nth) rdiag[j] = R[(int64_t)j * w + j];
  if (tid == 0) {
    int cnt = 0;
    for (int j = 0; j < w; ++j) keep[j] = R[(int64_t)j * w + j] > 0.0 ? cnt++ : -1;
    cnt2[0] = cnt;
    cnt2[1] = s_bad ? (int32_t)RE_ERR_NONFINITE : 0;
  }
  for (int t = w - 1; t >= 0; --t) {
    const double* Rt = R + (int64_t)t * w;
    const double rtt = Rt[t];
    for (int c = tid; c < w; c += nth) {
      double x = 0.0;
      if (c >= t && rtt > 0.0 && R[(int64_t)c * w + c] > 0.0) {
        double acc = c == t ? 1.0 : 0.0;
        for (int j = t + 1; j <= c; ++j) acc -= Rt[j] * Rinv[(int64_t)j * w + c];
        x = acc / rtt;
      }
      Rinv[(int64_t)t * w + c] = x;
    }
    __syncthreads();
  }
}

// Blocked form of the same factorisation and inverse for 136 < w <= 2200, in
// blocks of CB = 16 rows (8 rows above w = 1100, where 16 rows of w doubles
// would overflow LDS): the diagonal block is factored in LDS, the block
// row of R solved column by column (one thread per column) and kept in LDS,
// and the trailing matrix in global memory takes one rank-16 update per
// element (16 products per read-modify-write instead of one).  The inverse
// runs over block rows from the bottom: the diagonal block's inverse D^-1 by
// back substitution, then for every column c to the right
// Rinv[I][c] = -D^-1 sum_t R[I][t] Rinv[t][c] with 16 accumulators per thread.
// The pivot rule (shift, dependence threshold) is the unblocked one.
constexpr int kCholBlkThreads = 1024;
constexpr int64_t kCholBlkMaxW = 1100;   // 16-row blocks: 16 rows of w doubles within 138 KiB of LDS
constexpr int64_t kCholBlk8MaxW = 2200;  // 8-row blocks beyond that

template <int CB>
__global__ void __launch_bounds__(kCholBlkThreads) k_rf_chol_blk(double* __restrict__ R, int w, int shift, int64_t m,
                                                             double* __restrict__ Rinv, int32_t* __restrict__ keep,
                                                             int32_t* __restrict__ cnt2, double* __restrict__ rdiag) {
  extern __shared__ double P[];  // CB x w: the current block row (row stride w)
  __shared__ double D[CB * CB], Di[CB * CB];
  __shared__ double red[kCholThreads];
  __shared__ int s_bad;
  const int tid = threadIdx.x, nth = blockDim.x;
  if (tid == 0) s_bad = 0;
  double tr = 0.0, mx = 0.0;
  int bad = 0;
  for (int j = tid; j < w; j += nth) {
    const double d = R[(int64_t)j * w + j];
    bad |= !isfinite(d);
    tr += d;
    mx = fmax(mx, d);
  }
  __syncthreads();
  if (bad) atomicOr(&s_bad, 1);
  tr = block_sum(tr, red);
  mx = block_max(mx, red);
  const double s = shift ? 11.0 * ((double)m * w + (double)w * (w + 1)) * kU64 * tr : 0.0;
  const double thr = 16.0 * kU64 * (mx + s);
  for (int j = tid; j < w; j += nth) R[(int64_t)j * w + j] += s;
  __syncthreads();
  for (int J = 0; J < w; J += CB) {
    const int jb = w - J < CB ? w - J : CB;
    // diagonal block (upper triangle) into LDS, factored in place
    if (tid < jb * jb) {
      const int i = tid / jb, j = tid % jb;
      D[i * CB + j] = i <= j ? R[(int64_t)(J + i) * w + J + j] : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < jb; ++j) {
      const double d = D[j * CB + j];
      const bool kj = isfinite(d) && d > thr;
      const double rjj = kj ? sqrt(d) : 0.0, inv = kj ? 1.0 / rjj : 0.0;
      __syncthreads();
      if (tid < jb) {
        if (tid > j) D[j * CB + tid] *= inv;
        if (tid == j) {
          D[j * CB + j] = rjj;
          if (!isfinite(d)) s_bad = 1;
        }
      }
      __syncthreads();
      if (tid < jb * jb) {
        const int a = tid / jb, b = tid % jb;
        if (a > j && b >= a) D[a * CB + b] -= D[j * CB + a] * D[j * CB + b];
      }
      __syncthreads();
    }
    // block row of R: forward substitution with D^T, one thread per column,
    // kept in LDS (rows past jb zero, so the update below needs no guard)
    for (int c = J + jb + tid; c < w; c += nth) {
#pragma unroll
      for (int i = 0; i < CB; ++i) P[i * w + c] = i < jb ? R[(int64_t)(J + i) * w + c] : 0.0;  // loads in flight together
      for (int i = 0; i < jb; ++i) {
        double v = P[i * w + c];
        for (int t = 0; t < i; ++t) v -= D[t * CB + i] * P[t * w + c];
        const double dii = D[i * CB + i];
        const double x = dii > 0.0 ? v / dii : 0.0;
        R[(int64_t)(J + i) * w + c] = x;
        P[i * w + c] = x;
      }
    }
    if (tid < jb * jb) {
      const int i = tid / jb, j = tid % jb;
      if (i <= j) R[(int64_t)(J + i) * w + J + j] = D[i * CB + j];
    }
    __syncthreads();
    // trailing matrix: rank-jb update of the upper triangle
    const int c0 = J + jb, L = w - c0;
    for (int e = tid; e < L * L; e += nth) {
      const int a = c0 + e / L, b = c0 + e % L;
      if (a > b) continue;
      double acc = 0.0;
#pragma unroll
      for (int i = 0; i < CB; ++i) acc += P[i * w + a] * P[i * w + b];
      R[(int64_t)a * w + b] -= acc;
    }
    __syncthreads();
  }
  if (rdiag)
    for (int j = tid; j < w; j += nth) rdiag[j] = R[(int64_t)j * w + j];
  if (tid == 0) {
    int cnt = 0;
    for (int j = 0; j < w; ++j) keep[j] = R[(int64_t)j * w + j] > 0.0 ? cnt++ : -1;
    cnt2[0] = cnt;
    cnt2[1] = s_bad ? (int32_t)RE_ERR_NONFINITE : 0;
  }
  for (int I = ((w - 1) / CB) * CB; I >= 0; I -= CB) {
    const int ib = w - I < CB ? w - I : CB, W2 = w - I;
    // block row of R (rows past ib zero) and the diagonal block's inverse Di
    for (int e = tid; e < CB * W2; e += nth) {
      const int i = e / W2, c = I + e % W2;
      P[i * w + c] = i < ib ? R[(int64_t)(I + i) * w + c] : 0.0;
    }
    __syncthreads();
    if (tid < CB) {  // column tid of Di by back substitution
      const int cc = tid;
      const bool ckept = cc < ib && P[cc * w + I + cc] > 0.0;
      for (int i = CB - 1; i >= 0; --i) {
        double v = 0.0;
        if (i <= cc && ckept) {
          const double rii = P[i * w + I + i];
          if (rii > 0.0) {
            v = i == cc ? 1.0 : 0.0;
            for (int t = i + 1; t <= cc; ++t) v -= P[i * w + I + t] * Di[t * CB + cc];
            v /= rii;
          }
        }
        Di[i * CB + cc] = v;
        if (i < ib && cc < ib) Rinv[(int64_t)(I + i) * w + I + cc] = v;
      }
    }
    __syncthreads();
    for (int c = I + ib + tid; c < w; c += nth) {
      double y[CB];
#pragma unroll
      for (int i = 0; i < CB; ++i) y[i] = 0.0;
      constexpr int U = CB == 16 ? 1 : 4;  // loads in flight together; the summation order is unchanged
      int t = I + ib;
      for (; t + U - 1 <= c; t += U) {
        double rv[U];
#pragma unroll
        for (int q = 0; q < U; ++q) rv[q] = Rinv[(int64_t)(t + q) * w + c];
#pragma unroll
        for (int q = 0; q < U; ++q)
#pragma unroll
          for (int i = 0; i < CB; ++i) y[i] += P[i * w + t + q] * rv[q];
      }
      for (; t <= c; ++t) {
        const double rv = Rinv[(int64_t)t * w + c];
#pragma unroll
        for (int i = 0; i < CB; ++i) y[i] += P[i * w + t] * rv;
      }
      for (int i = 0; i < ib; ++i) {
        double o = 0.0;
        for (int j = i; j < CB; ++j) o -= Di[i * CB + j] * y[j];
        Rinv[(int64_t)(I + i) * w + c] = o;
      }
    }
    for (int e = tid; e < ib * I; e += nth) {
      const int i = e / I, c = e % I;
      Rinv[(int64_t)(I + i) * w + c] = 0.0;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// C = A Bm over one chunk of K: 64 x 64 output tiles of the M x N product of a
// row-major A (M x K, lda) and a row-major Bm (K x N, ldb), FP64 products of
// the stored values (FP32 or FP64).  Chunk z = blockIdx.z covers K indices
// [z kps, (z+1) kps) and writes its tile to out + z sstride; with `tri` the K
// range also stops at the tile's last column (Bm upper triangular).  Column c
// is written to column map[c] (skipped when negative) if map is given.  Same
// wavefront layout and MFMA as the Gram kernel; the A tile is stored row by
// row (pitch 17 doubles).
// ---------------------------------------------------------------------------
constexpr int kABK = 16, kAPV = kABK + 1, kAPR = 80;

template <typename TA, typename TB>
__global__ void __launch_bounds__(256) k_nn64(const TA* __restrict__ A, int64_t M, int64_t lda,
                                              const TB* __restrict__ Bm, int64_t ldb, int64_t N, int64_t K,
                                              int64_t kps, int tri, const int32_t* __restrict__ map,
                                              double* __restrict__ out, int64_t ldo, int64_t sstride) {
  __shared__ double sV[2][64 * kAPV], sR[2][kABK * kAPR];
  const int64_t c0 = (int64_t)blockIdx.x * 64, i0 = (int64_t)blockIdx.y * 64;
  const int64_t kb = (int64_t)blockIdx.z * kps;
  int64_t ke = kb + kps < K ? kb + kps : K;
  if (tri && c0 + 64 < ke) ke = c0 + 64;
  double* __restrict__ o = out + (int64_t)blockIdx.z * sstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q16 = lane & 15, kq = lane >> 4, wy = wave >> 1, wx = wave & 1;
  const int vr = tid >> 2, vk = (tid & 3) * 4;   // A loader: row, first of 4 K values
  const int rr = tid >> 4, rc = (tid & 15) * 4;  // Bm loader: K row, first of 4 columns
  double xv[4], xr[4];
  const bool vrow_ok = i0 + vr < M;
  const TA* __restrict__ vrow = A + (vrow_ok ? i0 + vr : 0) * lda;
  auto load = [&](int64_t t0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t t = t0 + vk + q;
      xv[q] = (vrow_ok && t < ke) ? (double)vrow[t] : 0.0;
      const int64_t tr = t0 + rr, c = c0 + rc + q;
      xr[q] = (tr < ke && c < N) ? (double)Bm[tr * ldb + c] : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sV[buf][vr * kAPV + vk + q] = xv[q];
      sR[buf][rr * kAPR + rc + q] = xr[q];
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int64_t nsteps = ke > kb ? (ke - kb + kABK - 1) / kABK : 0;
  load(kb);
  store(0);
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    if (st + 1 < nsteps) load(kb + (st + 1) * kABK);
#pragma unroll
    for (int kk = 0; kk < kABK; kk += 4) {
      const double u0 = sV[buf][(wy * 32 + q16) * kAPV + kk + kq];
      const double u1 = sV[buf][(wy * 32 + 16 + q16) * kAPV + kk + kq];
      const double* rp = &sR[buf][(kk + kq) * kAPR + wx * 32 + q16];
      const double v0 = rp[0], v1 = rp[16];
      acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0, v0, acc[0][0], 0, 0, 0);
      acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u0, v1, acc[0][1], 0, 0, 0);
      acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1, v0, acc[1][0], 0, 0, 0);
      acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(u1, v1, acc[1][1], 0, 0, 0);
    }
    if (st + 1 < nsteps) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      const int64_t c = c0 + wx * 32 + y * 16 + q16;
      if (c >= N) continue;
      const int64_t oc = map ? (int64_t)map[c] : c;
      if (oc < 0) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wy * 32 + x * 16 + kq + 4 * r;
        if (i < M) o[i * ldo + oc] = acc[x][y][r];
      }
    }
}

// ---------------------------------------------------------------------------
// parts[s] (w x n) = Q[rows of chunk s]^T A[rows of chunk s] for FP32 copies
// of Q (m x w, leading dimension w) and A.  A workgroup owns 32 MC rows of the
// output (columns of Q) by 128 columns (of A): four wavefronts, each 32
// columns and MC v_mfma_f32_32x32x2f32 tiles (operand lane l: row or column
// l % 32, K index l / 32; accumulator q of lane l: row 8 (q/4) + 4 (l/32) +
// q%4, column l % 32).  K steps of 32 rows through double-buffered LDS; the
// FP32 accumulators are added into FP64 ones every 256 rows.  Workgroups are
// spread so that the MC-row tiles sharing one column panel of A sit on the
// same XCD (consecutive workgroup ids go round-robin over the 8 XCDs) and
// read that panel through the same L2.
// ---------------------------------------------------------------------------
constexpr int kQBK = 32, kQBJ = 128, kQFlush = 256 / kQBK;

__global__ void k_to_f32(const double* __restrict__ Q, int64_t ldq, int64_t m, int64_t w, float* __restrict__ out) {
  const int64_t total = m * w;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / w, c = e - i * w;
    out[e] = (float)Q[i * ldq + c];
  }
}

template <int MC>
__global__ void __launch_bounds__(256) k_rf_qta(const float* __restrict__ Q, int64_t w, const float* __restrict__ A,
                                               int64_t m, int64_t n, int64_t lda, int64_t rps, int64_t ctiles,
                                               int64_t ntiles, double* __restrict__ parts) {
  constexpr int BC = 32 * MC, QPER = kQBK * BC / 256, APER = kQBK * kQBJ / 256;
  __shared__ float sQ[2][kQBK * BC], sA[2][kQBK * kQBJ];
  const int64_t per_xcd = gridDim.x / 8;
  const int64_t tile = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (tile >= ntiles) return;
  const int64_t c0 = (tile % ctiles) * BC, j0 = (tile / ctiles) * kQBJ;
  const int64_t ib = (int64_t)blockIdx.y * rps;
  const int64_t ie = ib + rps < m ? ib + rps : m;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  float xq[QPER], xa[APER];
  auto load = [&](int64_t i0) {
#pragma unroll
    for (int q = 0; q < QPER; ++q) {
      const int e = tid + 256 * q, r = e / BC, c = e % BC;
      const int64_t i = i0 + r;
      xq[q] = (i < ie && c0 + c < w) ? Q[i * w + c0 + c] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < APER; ++q) {
      const int e = tid + 256 * q, r = e / kQBJ, c = e % kQBJ;
      const int64_t i = i0 + r;
      xa[q] = (i < ie && j0 + c < n) ? A[i * lda + j0 + c] : 0.0f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < QPER; ++q) sQ[buf][tid + 256 * q] = xq[q];
#pragma unroll
    for (int q = 0; q < APER; ++q) sA[buf][tid + 256 * q] = xa[q];
  };
  f32x16 acc[MC];
  double acc64[MC][16];
#pragma unroll
  for (int mi = 0; mi < MC; ++mi)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      acc[mi][q] = 0.0f;
      acc64[mi][q] = 0.0;
    }
  auto flush = [&]() {
#pragma unroll
    for (int mi = 0; mi < MC; ++mi)
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        acc64[mi][q] += (double)acc[mi][q];
        acc[mi][q] = 0.0f;
      }
  };
  const int64_t nsteps = (ie - ib + kQBK - 1) / kQBK;
  load(ib);
  store(0);
  __syncthreads();
  for (int64_t st = 0; st < nsteps; ++st) {
    const int buf = st & 1;
    if (st + 1 < nsteps) load(ib + (st + 1) * kQBK);
#pragma unroll
    for (int kk = 0; kk < kQBK; kk += 2) {
      const float b = sA[buf][(kk + (lane >> 5)) * kQBJ + wave * 32 + (lane & 31)];
#pragma unroll
      for (int mi = 0; mi < MC; ++mi) {
        const float a = sQ[buf][(kk + (lane >> 5)) * BC + mi * 32 + (lane & 31)];
        acc[mi] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[mi], 0, 0, 0);
      }
    }
    if (st + 1 < nsteps) store(buf ^ 1);
    if ((st + 1) % kQFlush == 0) flush();
    __syncthreads();
  }
  flush();
  double* __restrict__ part = parts + (int64_t)blockIdx.y * w * n;
  const int64_t j = j0 + wave * 32 + (lane & 31);
  if (j >= n) return;
#pragma unroll
  for (int mi = 0; mi < MC; ++mi)
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int64_t c = c0 + mi * 32 + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
      if (c < w) part[c * n + j] = acc64[mi][q];
    }
}

// ---------------------------------------------------------------------------
// Estimates from the diagonal of R (the alternative step 7 of Sec. 5): the
// sketch's R = R3 R2 R1 is the product of the three passes' triangular factors,
// so |R_jj| = |R3_jj R2_jj R1_jj|; scaled by 1/sqrt(k l) and placed in
// descending order by counting, for each value, the values above it (ties by
// index), which gives the same order on every run.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_qr_sigma(const double* __restrict__ rd, int64_t k, double scale,
                                                 double* __restrict__ sigma) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double vj = fabs(rd[j] * rd[k + j] * rd[2 * k + j]) * scale;
  int64_t rank = 0;
  for (int64_t i = 0; i < k; ++i) {
    const double vi = fabs(rd[i] * rd[k + i] * rd[2 * k + i]) * scale;
    rank += (vi > vj) || (vi == vj && i < j);
  }
  sigma[rank] = vj;
}

}  // namespace

re_status launch_rf_width(hipStream_t s, const double* sigma, int64_t k, int32_t r1, int64_t n, double eps, int32_t p,
                          double norm_a, const int32_t* info, double* tail, int32_t* out4) {
  if (k < 1 || r1 < 1 || r1 > k || p < 2) return RE_ERR_INVALID_ARG;
  hipLaunchKernelGGL(k_rf_width, dim3(1), dim3(256), 0, s, sigma, (int)k, (int)r1, n, eps, (int)p, norm_a, info, tail,
                     out4);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

void rf_row_split(int64_t m, int64_t tiles, int64_t* splits, int64_t* rows_per_split) {
  const int64_t target = 2048;  // workgroups per launch: 8 per CU
  int64_t sp = target / (tiles > 0 ? tiles : 1);
  const int64_t most = cdiv(m, 256);
  if (sp > most) sp = most;
  if (sp < 1) sp = 1;
  const int64_t rps = cdiv(cdiv(m, sp), 256) * 256;
  *rows_per_split = rps;
  *splits = cdiv(m, rps);
}

re_status launch_rf_gram(hipStream_t s, const void* V, bool v32, int64_t m, int64_t w, int64_t ldv, int64_t splits,
                         int64_t rows_per_split, double* parts) {
  const int64_t T = cdiv(w, 64);
  const dim3 grid((unsigned)T, (unsigned)T, (unsigned)splits);
  if (v32)
    hipLaunchKernelGGL(k_rf_gram<float>, grid, dim3(256), 0, s, (const float*)V, m, w, ldv, rows_per_split, parts);
  else
    hipLaunchKernelGGL(k_rf_gram<double>, grid, dim3(256), 0, s, (const double*)V, m, w, ldv, rows_per_split, parts);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_rf_sum_parts(hipStream_t s, const double* parts, int64_t splits, int64_t rows, int64_t cols,
                              bool upper, double* out, int64_t ldo) {
  const int64_t total = rows * cols;
  int64_t blocks = cdiv(total, 256);
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_rf_sum_parts, dim3((unsigned)blocks), dim3(256), 0, s, parts, splits, rows, cols, upper ? 1 : 0,
                     out, ldo);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

size_t rf_chol_lds_bytes(int64_t w) { return w <= kCholLdsMaxW ? (size_t)(w * w * 8) : 0; }

re_status launch_rf_chol(hipStream_t s, double* G, int64_t w, bool shift, int64_t m, double* Rinv, int32_t* keep,
                         int32_t* cnt2, double* rdiag) {
  if (w < 1 || w > 46340) return RE_ERR_INVALID_ARG;  // w^2 within int range of the trailing loop
  if (w > kCholLdsMaxW && w <= kCholBlk8MaxW) {
    const bool b16 = w <= kCholBlkMaxW;
    const size_t pb = (size_t)(b16 ? 16 : 8) * w * 8;
    const void* fn = b16 ? (const void*)k_rf_chol_blk<16> : (const void*)k_rf_chol_blk<8>;
    if (pb > 65536) RE_TRY_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)pb));
    if (b16)
      hipLaunchKernelGGL(k_rf_chol_blk<16>, dim3(1), dim3(kCholBlkThreads), pb, s, G, (int)w, shift ? 1 : 0, m, Rinv,
                         keep, cnt2, rdiag);
    else
      hipLaunchKernelGGL(k_rf_chol_blk<8>, dim3(1), dim3(kCholBlkThreads), pb, s, G, (int)w, shift ? 1 : 0, m, Rinv,
                         keep, cnt2, rdiag);
    RE_TRY_HIP(hipGetLastError());
    return RE_OK;
  }
  const size_t lds = rf_chol_lds_bytes(w);
  if (lds > 65536)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_rf_chol, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  hipLaunchKernelGGL(k_rf_chol, dim3(1), dim3(kCholThreads), lds, s, G, (int)w, shift ? 1 : 0, m, lds ? 1 : 0, Rinv,
                     keep, cnt2, rdiag);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_rf_apply(hipStream_t s, const void* V, bool v32, int64_t m, int64_t w, int64_t ldv, const double* Rinv,
                          const int32_t* keep, double* Q, int64_t ldq) {
  const dim3 grid((unsigned)cdiv(w, 64), (unsigned)cdiv(m, 64), 1);
  if (v32)
    hipLaunchKernelGGL((k_nn64<float, double>), grid, dim3(256), 0, s, (const float*)V, m, ldv, Rinv, w, w, w, w, 1,
                       keep, Q, ldq, (int64_t)0);
  else
    hipLaunchKernelGGL((k_nn64<double, double>), grid, dim3(256), 0, s, (const double*)V, m, ldv, Rinv, w, w, w, w, 1,
                       keep, Q, ldq, (int64_t)0);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

void yb_split(int64_t l, int64_t k, int64_t m, int64_t* splits, int64_t* rows_per_split) {
  rf_row_split(m, cdiv(l, 64) * cdiv(k, 64), splits, rows_per_split);
}

size_t yb_parts_bytes(int64_t l, int64_t k, int64_t m) {
  int64_t sp = 0, rps = 0;
  yb_split(l, k, m, &sp, &rps);
  return sp > 1 ? (size_t)sp * l * k * 8 : 0;
}

re_status launch_yb_tiled(hipStream_t s, const float* B, int64_t m, int64_t k, int64_t ldb, const float* Y, int64_t ldy,
                          int64_t l, double* C, double* parts) {
  int64_t sp = 0, rps = 0;
  yb_split(l, k, m, &sp, &rps);
  if (sp > 1 && !parts) return RE_ERR_INVALID_ARG;
  const dim3 grid((unsigned)cdiv(k, 64), (unsigned)cdiv(l, 64), (unsigned)sp);
  double* out = sp > 1 ? parts : C;
  hipLaunchKernelGGL((k_nn64<float, float>), grid, dim3(256), 0, s, Y, l, ldy, B, ldb, k, m, rps, 0,
                     (const int32_t*)nullptr, out, k, sp > 1 ? l * k : (int64_t)0);
  RE_TRY_HIP(hipGetLastError());
  if (sp > 1) return launch_rf_sum_parts(s, parts, sp, l, k, false, C, k);
  return RE_OK;
}

// FP64 C (M x N, ldc) = A (M x K) B (K x N) on the FP64 matrix cores (the
// 64 x 64 tiles of k_nn64).  K is split into S slices only when M is short
// (fewer than 64 row tiles) and K long, so that a short, wide product still
// fills the chip: slices of 4096 rows (at most 32) past K = 4096, of 256 rows
// from K = 513 to 4096 (a 60 x 40 product over 2000 rows is otherwise one
// workgroup's sequential sweep); the slices' partial products are then summed
// in slice order.  S depends on M and K alone, so every column of C gets the
// same arithmetic whatever N is (a product over the appended columns of B
// gives the bits of the same columns in a wider product).
void gemm64_split(int64_t M, int64_t K, int64_t* splits, int64_t* rows_per_split) {
  int64_t sp = 1;
  if (cdiv(M, 64) < 64 && K > 4096) sp = cdiv(K, 4096) < 32 ? cdiv(K, 4096) : 32;
  else if (cdiv(M, 64) < 64 && K > 512) sp = cdiv(K, 256);
  const int64_t rps = cdiv(cdiv(K, sp), kABK) * kABK;
  *rows_per_split = rps;
  *splits = cdiv(K, rps);
}

size_t gemm64_parts_bytes(int64_t M, int64_t N, int64_t K) {
  int64_t sp = 0, rps = 0;
  gemm64_split(M, K, &sp, &rps);
  return sp > 1 ? (size_t)sp * M * N * 8 : 0;
}

re_status launch_gemm64(hipStream_t s, int64_t M, int64_t N, int64_t K, const double* A, int64_t lda, const double* B,
                        int64_t ldb, double* C, int64_t ldc, double* parts) {
  if (M <= 0 || N <= 0) return RE_OK;
  int64_t sp = 0, rps = 0;
  gemm64_split(M, K, &sp, &rps);
  if (sp > 1 && !parts) return RE_ERR_INVALID_ARG;
  if (cdiv(M, 64) > 65535 || sp > 65535) return RE_ERR_UNSUPPORTED;
  const dim3 grid((unsigned)cdiv(N, 64), (unsigned)cdiv(M, 64), (unsigned)sp);
  double* out = sp > 1 ? parts : C;
  hipLaunchKernelGGL((k_nn64<double, double>), grid, dim3(256), 0, s, A, M, lda, B, ldb, N, K, rps, 0,
                     (const int32_t*)nullptr, out, sp > 1 ? N : ldc, sp > 1 ? M * N : (int64_t)0);
  RE_TRY_HIP(hipGetLastError());
  if (sp > 1) return launch_rf_sum_parts(s, parts, sp, M, N, false, C, ldc);
  return RE_OK;
}

int64_t rf_qta_col_tiles(int64_t n) { return cdiv(n, kQBJ); }

re_status launch_qr_sigma(hipStream_t s, const double* rdiag3, int64_t k, double scale, double* sigma) {
  hipLaunchKernelGGL(k_qr_sigma, dim3((unsigned)cdiv(k, 256)), dim3(256), 0, s, rdiag3, k, scale, sigma);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_rf_qta(hipStream_t s, const double* Q, int64_t ldq, int64_t w, const float* A, int64_t m, int64_t n,
                        int64_t lda, int64_t splits, int64_t rows_per_split, float* q32, double* parts) {
  int64_t blocks = cdiv(m * w, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(k_to_f32, dim3((unsigned)blocks), dim3(256), 0, s, Q, ldq, m, w, q32);
  const int mc = w >= 128 ? 4 : (int)cdiv(w, 32);
  const int64_t ctiles = cdiv(w, 32 * mc), ntiles = ctiles * rf_qta_col_tiles(n);
  const int64_t grid = cdiv(ntiles, 8) * 8;
  const dim3 g((unsigned)grid, (unsigned)splits);
#define RE_QTA_CASE(MC)                                                                                              \
  if (mc == MC) {                                                                                                    \
    hipLaunchKernelGGL(k_rf_qta<MC>, g, dim3(256), 0, s, (const float*)q32, w, A, m, n, lda, rows_per_split, ctiles, \
                       ntiles, parts);                                                                               \
    RE_TRY_HIP(hipGetLastError());                                                                                   \
    return RE_OK;                                                                                                    \
  }
  RE_QTA_CASE(1)
  RE_QTA_CASE(2)
  RE_QTA_CASE(3)
  RE_QTA_CASE(4)
#undef RE_QTA_CASE
  return RE_ERR_INVALID_ARG;
}

}  // namespace re
