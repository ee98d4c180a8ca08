// Algorithm 1 steps 7-8: singular values of the small l x k sketch C = Y A X
// in FP64, then the count of estimates above eps * sigma_1.
//
// Singular values are computed by
//   (1) Householder bidiagonalisation C = Q B P^T (Golub-Kahan), run by P
//       co-resident workgroups that each own the rows r = w (mod P) of a
//       working copy; every column step needs one reduction over all rows,
//       so the workgroups meet at one grid barrier per column;
//   (2) the singular values of the upper bidiagonal B, which are the positive
//       eigenvalues of the 2k x 2k Golub-Kahan tridiagonal with zero diagonal
//       and off-diagonal (d1, e1, d2, e2, ..., dk); each value is found by
//       multisection on Sturm counts, one wavefront per singular value.
// Both steps are backward stable, so each sigma_i is within a small multiple
// of u ||C|| of its exact value.
#include <stdlib.h>

#include <string.h>

#include "common.h"
#include "batch.h"

namespace re {

namespace {

constexpr int kBidiagThreads = 256;
constexpr int kWaves = kBidiagThreads / 64;

struct BidiagArgs {
  const double* C;   // l x k input, row-major
  double* W;         // l x k working copy
  double* part;      // [2][P][k + 1] partial reductions
  double* rowbuf;    // [2][k + 1] the pivot row
  double* red;       // [2][k + 1] reduced partials (k_bidiag_g2)
  double* d;         // k diagonal of B
  double* e;         // k - 1 superdiagonal of B
  unsigned* bar;     // grid barrier counter
  int32_t* info;     // status (0 ok, RE_ERR_*)
  int64_t l, k;
  int P;
  long spin_limit;   // polls of a grid barrier before it gives up (< 0: at once)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Cross-lane moves of a double by a DPP pattern (two 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const uint64_t u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Sum over each row of 16 lanes, result in every lane of the row:
// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror.
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x140>(v);
  return v;
}

// Sum over the wavefront, result in every lane.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = row16_sum(v);
  const uint64_t u = __double_as_longlong(v);
  double t = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, 16 * r);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), 16 * r);
    t += __longlong_as_double(((uint64_t)hi << 32) | lo);
  }
  return t;
}

// Grid barrier over the P workgroups of the bidiagonalisation.  The counter
// grows monotonically; a bounded wait (at most `limit` polls; a negative limit
// fails at once, a test hook) turns a missing workgroup into an error instead
// of a hang.
__device__ __forceinline__ bool barrier_gives_up(long& spins, long limit) { return limit < 0 || ++spins > limit; }

__device__ bool grid_barrier(unsigned* bar, unsigned target, int32_t* info, long limit) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (barrier_gives_up(spins, limit)) {
        ok = 0;
        __hip_atomic_store(info, (int32_t)RE_ERR_NO_CONVERGENCE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return ok != 0;
}

// Column step partials of column c over this workgroup's rows r >= c:
//   part[0] = sum W[r][c]^2,  part[1 + (j - c - 1)] = sum W[r][c] W[r][j]  (j > c)
// and, from the owner of row c, rowbuf = W[c][c..k).  Columns are taken in
// chunks of kPartChunk so that the per-wavefront accumulators fit in LDS for
// any k; every sum runs over the rows in the same order.
constexpr int kPartChunk = 1024;
__device__ void column_partials(const BidiagArgs& a, int64_t c, int w, double* gacc /* [kWaves][kPartChunk] LDS */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t k = a.k, len = k - c;  // len = 1 + (k - c - 1)
  double* g = gacc + (int64_t)wave * kPartChunk;
  const int64_t par = c & 1;
  double* out = a.part + (par * a.P + w) * (k + 1);
  for (int64_t j0 = 0; j0 < len; j0 += kPartChunk) {
    const int64_t jn = len - j0 < kPartChunk ? len - j0 : kPartChunk;
    for (int64_t j = lane; j < jn; j += 64) g[j] = 0.0;
    for (int64_t r = w + (int64_t)wave * a.P; r < a.l; r += (int64_t)kWaves * a.P) {
      if (r < c) continue;
      const double* row = a.W + r * k + c + j0;
      const double x = a.W[r * k + c];
      for (int64_t j = lane; j < jn; j += 64) g[j] += x * row[j];
      if (r == c)
        for (int64_t j = lane; j < jn; j += 64) a.rowbuf[par * (k + 1) + j0 + j] = row[j];
    }
    __syncthreads();
    for (int64_t j = threadIdx.x; j < jn; j += blockDim.x) {
      double s = 0.0;
      for (int v = 0; v < kWaves; ++v) s += gacc[(int64_t)v * kPartChunk + j];
      out[j0 + j] = s;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(kBidiagThreads) k_bidiag(BidiagArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t k = a.k, l = a.l;
  double* wv = reinterpret_cast<double*>(smem_raw);  // [k+1] column-step coefficients w_j
  double* vv = wv + (k + 1);                           // [k+1] row reflector v
  double* gacc = vv + (k + 1);                         // [kWaves][k+1]
  __shared__ double s_scalars[4];
  const int w = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  unsigned epoch = 0;

  // private copy of this workgroup's rows; non-finite input is reported
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  for (int64_t r = w + (int64_t)wave * a.P; r < l; r += (int64_t)kWaves * a.P)
    for (int64_t j = lane; j < k; j += 64) {
      const double x = a.C[r * k + j];
      if (!isfinite(x)) s_bad = 1;
      a.W[r * k + j] = x;
    }
  __syncthreads();
  if (s_bad) __hip_atomic_store(a.info, (int32_t)RE_ERR_NONFINITE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  column_partials(a, 0, w, gacc);
  if (!grid_barrier(a.bar, (unsigned)a.P * ++epoch, a.info, a.spin_limit)) return;

  for (int64_t c = 0; c < k; ++c) {
    const int64_t par = c & 1, len = k - c;
    // ---- reduce the partials of column c (every workgroup, same order) ----
    for (int64_t j = threadIdx.x; j < len; j += blockDim.x) {
      double s = 0.0;
      for (int p = 0; p < a.P; ++p) s += a.part[(par * a.P + p) * (k + 1) + j];
      wv[j] = s;  // wv[0] = ||x||^2, wv[j] = x . W[:, c + j]
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double s0 = wv[0], x0 = a.rowbuf[par * (k + 1)];
      const double nx = sqrt(s0);
      double alpha = 0.0, tau = 0.0;
      if (nx > 0.0) {
        alpha = -copysign(nx, x0);
        tau = 1.0 / (s0 - alpha * x0);
      }
      s_scalars[0] = alpha;
      s_scalars[1] = tau;
      s_scalars[2] = x0 - alpha;  // first entry of the column reflector u
      if (w == 0) a.d[c] = alpha;
    }
    __syncthreads();
    const double alpha = s_scalars[0], tau = s_scalars[1], u0 = s_scalars[2];
    // w_j = tau (x . W[:, j] - alpha W[c][j]); updated pivot row y_j = W[c][j] - u0 w_j
    for (int64_t j = 1 + threadIdx.x; j < len; j += blockDim.x) {
      const double row = a.rowbuf[par * (k + 1) + j];
      const double wj = tau * (wv[j] - alpha * row);
      wv[j] = wj;
      vv[j] = row - u0 * wj;
    }
    __syncthreads();
    // ---- row reflector of the updated pivot row (entries c+1 .. k-1) ----
    if (len > 1) {
      double p = 0.0;
      for (int64_t j = 1 + threadIdx.x; j < len; j += blockDim.x) p += vv[j] * vv[j];
      p = wave_sum(p);
      if (lane == 0) gacc[wave] = p;
      __syncthreads();
      if (threadIdx.x == 0) {
        double ny2 = 0.0;
        for (int v = 0; v < kWaves; ++v) ny2 += gacc[v];
        const double y0 = vv[1], ny = sqrt(ny2);
        double beta = 0.0, tau2 = 0.0;
        if (ny > 0.0) {
          beta = -copysign(ny, y0);
          tau2 = 1.0 / (ny2 - beta * y0);
        }
        s_scalars[3] = tau2;
        vv[1] = y0 - beta;
        if (w == 0) a.e[c] = beta;
      }
      __syncthreads();
    }
    const double tau2 = (len > 1) ? s_scalars[3] : 0.0;
    // ---- apply both reflectors to this workgroup's rows r > c ----
    for (int64_t r = w + (int64_t)wave * a.P; r < l; r += (int64_t)kWaves * a.P) {
      if (r <= c) continue;
      double* row = a.W + r * k;
      const double ur = row[c];
      double z = 0.0;
      for (int64_t j = 1 + lane; j < len; j += 64) {
        const double v = row[c + j] - ur * wv[j];
        row[c + j] = v;
        z += v * vv[j];
      }
      z = wave_sum(z) * tau2;
      for (int64_t j = 1 + lane; j < len; j += 64) row[c + j] -= z * vv[j];
    }
    __syncthreads();
    if (c + 1 < k) {
      column_partials(a, c + 1, w, gacc);
      if (!grid_barrier(a.bar, (unsigned)a.P * ++epoch, a.info, a.spin_limit)) return;
    }
  }
}

// ---- bidiagonalisation with the rows resident in LDS ----------------------
// Same reduction as k_bidiag, organised for latency: 1024 threads, each
// workgroup keeps its rows (r = w mod P) in LDS, the scalars of each step
// are recomputed by every thread instead of broadcast, and the values
// exchanged between workgroups (partials, pivot row) travel through
// agent-coherent stores and loads, so a grid barrier needs only the
// completion of those stores and one counter.
constexpr int kB2Threads = 1024;
constexpr int kB2Waves = kB2Threads / 64;

struct Bidiag2Args {
  const double* C;
  double* part;    // [2][P][k + 1]
  double* rowbuf;  // [2][k + 1]
  double* d;
  double* e;
  unsigned* bar;
  int32_t* info;
  int64_t l, k, kp;  // kp: LDS row stride in doubles (kp = 16 mod 32)
  int P, nr_max;
  int xstride;       // launched workgroups per participant (participants: blockIdx.x % xstride == xoff)
  int xoff;
  long spin_limit;   // polls of a grid barrier before it gives up (< 0: at once)
};

__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The exchange between participants goes only through agent-scope atomic
// stores and loads (st_coh / ld_coh), which bypass the non-coherent caches;
// a wave's vmcnt(0) waits for its stores' acknowledgements, so they are
// visible device-wide before the workgroup barrier and the counter increment
// that follows it, and the loads after the spin are issued only once the
// counter has reached the target.  Release / acquire orders on the counter
// would add an L2 writeback and invalidate per barrier: measured at 576 x 384,
// 2.68 ms against 2.05 ms for the bidiagonalisation, and the rate of four
// estimates in flight fell from 682 to 543 per second.
__device__ bool grid_sync_coh(unsigned* bar, unsigned target, int32_t* info, long limit) {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wave's coherent stores are complete
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    long spins = 0;
    ok = 1;
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (barrier_gives_up(spins, limit)) {
        ok = 0;
        __hip_atomic_store(info, (int32_t)RE_ERR_NO_CONVERGENCE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// ---- global-memory bidiagonalisation, rows held in registers --------------
//
// The same column steps as k_bidiag for sketches too wide for LDS, organised
// for memory-level parallelism: one wavefront owns a row at a time and holds
// its trailing part W[r][c .. k) in registers (lane j mod 64, up to 64 T
// columns), so a column step reads and writes each row once: it applies both
// reflectors and accumulates the next column's partial products x_r W[r][j]
// from the same registers.  The P partial vectors are reduced in two levels
// (each workgroup sums a slice of the columns over all P, then every
// workgroup reads the reduced vector), so each column step moves 2 P (k - c)
// partials instead of P^2 (k - c); it costs two grid barriers.  W is private
// to the wavefront that owns each row, so only the exchanged vectors (partials,
// reduced column, pivot row) travel by coherent stores and loads, and the
// barriers need no cache writeback or invalidation.
constexpr int kG2MaxP = 256;
template <int T>
__global__ void __launch_bounds__(kBidiagThreads) k_bidiag_g2(BidiagArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t k = a.k, l = a.l;
  const int P = a.P, w = blockIdx.x;
  double* wv = reinterpret_cast<double*>(smem_raw);  // [k+1] column-step coefficients w_j
  double* vv = wv + (k + 1);                           // [k+1] row reflector v
  double* gl = vv + (k + 1);                           // [kWaves][64 T] per-wavefront partials
  __shared__ double s_red[kBidiagThreads];
  __shared__ double s_scalars[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int gw = w * kWaves + wave, nw = P * kWaves;  // rows r = gw (mod nw)
  unsigned epoch = 0;
  double rv[T], g[T];

  // this wavefront's partials g (index j - 1 relative to the row segment) into
  // LDS, then the workgroup's sum into part[par][w][0 .. n)
  auto flush_partials = [&](int64_t par, int64_t n) {
#pragma unroll
    for (int t = 0; t < T; ++t) gl[(int64_t)wave * 64 * T + lane + 64 * t] = g[t];
    __syncthreads();
    double* out = a.part + (par * P + w) * (k + 1);
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
      st_coh(&out[j], (gl[j] + gl[64 * T + j]) + (gl[2 * 64 * T + j] + gl[3 * 64 * T + j]));
    __syncthreads();
  };

  // copy of this workgroup's rows (non-finite input is reported) and the
  // partials of column 0: part[j] = sum_r W[r][0] W[r][j]
  __shared__ int s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
#pragma unroll
  for (int t = 0; t < T; ++t) g[t] = 0.0;
  for (int64_t r = gw; r < l; r += nw) {
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t j = lane + 64 * t;
      rv[t] = j < k ? a.C[r * k + j] : 0.0;
    }
    bool bad = false;
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t j = lane + 64 * t;
      if (j < k) {
        bad |= !isfinite(rv[t]);
        a.W[r * k + j] = rv[t];
        if (r == 0) st_coh(&a.rowbuf[j], rv[t]);
      }
    }
    if (bad) s_bad = 1;
    const double x = __shfl(rv[0], 0, 64);
#pragma unroll
    for (int t = 0; t < T; ++t) g[t] += x * rv[t];
  }
  flush_partials(0, k);
  if (s_bad) __hip_atomic_store(a.info, (int32_t)RE_ERR_NONFINITE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (!grid_sync_coh(a.bar, (unsigned)P * ++epoch, a.info, a.spin_limit)) return;

  for (int64_t c = 0; c < k; ++c) {
    const int64_t par = c & 1, len = k - c;
    // ---- level 1: this workgroup's slice of the columns summed over all P partials ----
    {
      const int64_t S = (len + P - 1) / P, j0 = (int64_t)w * S;
      const int64_t ns = j0 >= len ? 0 : (len - j0 < S ? len - j0 : S);
      if (ns > kBidiagThreads) {
        for (int64_t jj = threadIdx.x; jj < ns; jj += blockDim.x) {
          double s = 0.0;
          for (int p = 0; p < P; ++p) s += ld_coh(&a.part[(par * P + p) * (k + 1) + j0 + jj]);
          st_coh(&a.red[par * (k + 1) + j0 + jj], s);
        }
      } else if (ns > 0) {
        const int G = kBidiagThreads / (int)ns;  // threads per column
        const int jj = threadIdx.x % (int)ns, gg = threadIdx.x / (int)ns;
        double s = 0.0;
        if (gg < G)
          for (int p = gg; p < P; p += G) s += ld_coh(&a.part[(par * P + p) * (k + 1) + j0 + jj]);
        s_red[threadIdx.x] = s;
        __syncthreads();
        if (threadIdx.x < ns) {
          double tot = 0.0;
          for (int q = 0; q < G; ++q) {
            const int idx = q * (int)ns + (int)threadIdx.x;
            if (idx < kBidiagThreads) tot += s_red[idx];
          }
          st_coh(&a.red[par * (k + 1) + j0 + threadIdx.x], tot);
        }
      }
    }
    if (!grid_sync_coh(a.bar, (unsigned)P * ++epoch, a.info, a.spin_limit)) return;
    // ---- level 2: the reduced column, both reflectors (every workgroup, same arithmetic) ----
    for (int64_t j = threadIdx.x; j < len; j += blockDim.x) wv[j] = ld_coh(&a.red[par * (k + 1) + j]);
    for (int64_t j = threadIdx.x; j < len; j += blockDim.x) vv[j] = ld_coh(&a.rowbuf[par * (k + 1) + j]);
    __syncthreads();
    if (threadIdx.x == 0) {
      const double s0 = wv[0], x0 = vv[0];
      const double nx = sqrt(s0);
      double alpha = 0.0, tau = 0.0;
      if (nx > 0.0) {
        alpha = -copysign(nx, x0);
        tau = 1.0 / (s0 - alpha * x0);
      }
      s_scalars[0] = alpha;
      s_scalars[1] = tau;
      s_scalars[2] = x0 - alpha;
      if (w == 0) a.d[c] = alpha;
    }
    __syncthreads();
    const double alpha = s_scalars[0], tau = s_scalars[1], u0 = s_scalars[2];
    for (int64_t j = 1 + threadIdx.x; j < len; j += blockDim.x) {
      const double row = vv[j];  // the pivot row, replaced by the updated row in place
      const double wj = tau * (wv[j] - alpha * row);
      wv[j] = wj;
      vv[j] = row - u0 * wj;
    }
    __syncthreads();
    if (len > 1) {
      double p = 0.0;
      for (int64_t j = 1 + threadIdx.x; j < len; j += blockDim.x) p += vv[j] * vv[j];
      p = wave_sum(p);
      if (lane == 0) s_red[wave] = p;
      __syncthreads();
      if (threadIdx.x == 0) {
        double ny2 = 0.0;
        for (int v = 0; v < kWaves; ++v) ny2 += s_red[v];
        const double y0 = vv[1], ny = sqrt(ny2);
        double beta = 0.0, tau2 = 0.0;
        if (ny > 0.0) {
          beta = -copysign(ny, y0);
          tau2 = 1.0 / (ny2 - beta * y0);
        }
        s_scalars[3] = tau2;
        vv[1] = y0 - beta;
        if (w == 0) a.e[c] = beta;
      }
      __syncthreads();
    }
    const double tau2 = (len > 1) ? s_scalars[3] : 0.0;
    if (len == 1) break;
    // ---- this wavefront's rows r > c: both reflectors, then the partials of column c + 1 ----
#pragma unroll
    for (int t = 0; t < T; ++t) g[t] = 0.0;
    const int64_t par1 = par ^ 1;
    for (int64_t r = gw; r < l; r += nw) {
      if (r <= c) continue;
      double* row = a.W + r * k + c;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int64_t j = lane + 64 * t;
        rv[t] = j < len ? row[j] : 0.0;
      }
      const double ur = __shfl(rv[0], 0, 64);  // W[r][c]
      double z = 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int64_t j = lane + 64 * t;
        if (j >= 1 && j < len) {
          const double v = rv[t] - ur * wv[j];
          rv[t] = v;
          z += v * vv[j];
        }
      }
      z = wave_sum(z) * tau2;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int64_t j = lane + 64 * t;
        if (j >= 1 && j < len) {
          rv[t] -= z * vv[j];
          row[j] = rv[t];
          if (r == c + 1) st_coh(&a.rowbuf[par1 * (k + 1) + j - 1], rv[t]);
        }
      }
      const double x = __shfl(rv[0], 1, 64);  // W[r][c + 1]
      // g[t] at lane holds the partial for j - 1 = lane + 64 t - 1: shift by one lane
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int64_t j = lane + 64 * t;
        if (j >= 1 && j < len) g[t] += x * rv[t];
      }
    }
    // g[t] belongs to index j - 1 (j = lane + 64 t): store it there
#pragma unroll
    for (int t = 0; t < T; ++t) {
      const int64_t j = lane + 64 * t;
      if (j >= 1 && j < len) gl[(int64_t)wave * 64 * T + j - 1] = g[t];
    }
    __syncthreads();
    {
      double* out = a.part + (par1 * P + w) * (k + 1);
      for (int64_t j = threadIdx.x; j < len - 1; j += blockDim.x)
        st_coh(&out[j], (gl[j] + gl[64 * T + j]) + (gl[2 * 64 * T + j] + gl[3 * 64 * T + j]));
    }
    __syncthreads();
    if (!grid_sync_coh(a.bar, (unsigned)P * ++epoch, a.info, a.spin_limit)) return;
  }
}

// Partials of column c from this workgroup's rows r >= c (thread per column):
// part[j] = sum_r W[r][c] W[r][c + j]; the owner of row c also sends W[c][c..k).
__device__ void partials_lds(const Bidiag2Args& a, const double* Wl, int nr, int64_t c, int w) {
  const int64_t k = a.k, len = k - c;
  const int P = a.P;
  const int64_t par = c & 1;
  const int i0 = c > w ? (int)((c - w + P - 1) / P) : 0;
  const bool owner = (c % P) == w;
  const int iown = (int)(c / P);
  const int64_t kp = a.kp;
  for (int64_t j = threadIdx.x; j < len; j += blockDim.x) {
    double g[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int i = i0;
    for (; i + 7 < nr; i += 8) {
      const double* r0 = Wl + (int64_t)i * kp + c;
#pragma unroll
      for (int q = 0; q < 8; ++q) g[q] += r0[q * kp] * r0[q * kp + j];
    }
    for (; i < nr; ++i) {
      const double* r0 = Wl + (int64_t)i * kp + c;
      g[0] += r0[0] * r0[j];
    }
    st_coh(&a.part[(par * P + w) * (k + 1) + j], ((g[0] + g[1]) + (g[2] + g[3])) + ((g[4] + g[5]) + (g[6] + g[7])));
    if (owner) st_coh(&a.rowbuf[par * (k + 1) + j], Wl[(int64_t)iown * kp + c + j]);
  }
}

__global__ void __launch_bounds__(kB2Threads) k_bidiag_lds(Bidiag2Args a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int64_t k = a.k, l = a.l, kp = a.kp;
  const int P = a.P, w = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nr = (int)((l - w + P - 1) / P);
  double* Wl = reinterpret_cast<double*>(smem_raw);  // [nr_max][kp]
  double* wv = Wl + (int64_t)a.nr_max * kp;           // [k + 1]
  double* vv = wv + (k + 1);                           // [k + 1]
  double* red = vv + (k + 1);                          // [kB2Waves]
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)nr * k; e += kB2Threads) {
    const int64_t i = e / k, j = e - i * k;
    const double x = a.C[(w + P * i) * k + j];
    if (!isfinite(x)) s_bad = 1;
    Wl[i * kp + j] = x;
  }
  __syncthreads();
  if (s_bad) __hip_atomic_store(a.info, (int32_t)RE_ERR_NONFINITE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned epoch = 0;
  partials_lds(a, Wl, nr, 0, w);
  if (!grid_sync_coh(a.bar, (unsigned)P * ++epoch, a.info, a.spin_limit)) return;

  for (int64_t c = 0; c < k; ++c) {
    const int64_t par = c & 1, len = k - c;
    // reduce the partials of column c; vv holds the pivot row W[c][c..k)
    for (int64_t j = tid; j < len; j += kB2Threads) {
      // issue the coherent loads in batches of 16, then add them in order
      const double* src = a.part + par * P * (k + 1) + j;
      const double rb = ld_coh(&a.rowbuf[par * (k + 1) + j]);
      double s = 0.0;
      for (int p0 = 0; p0 < P; p0 += 16) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (p0 + q < P) ? ld_coh(src + (int64_t)(p0 + q) * (k + 1)) : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += v[q];
      }
      wv[j] = s;
      vv[j] = rb;
    }
    __syncthreads();
    // column reflector (every thread): H x = alpha e1, u = x - alpha e1, tau = 2 / u.u
    const double s0 = wv[0], x0 = vv[0];
    const double nx = sqrt(s0);
    const double alpha = nx > 0.0 ? -copysign(nx, x0) : 0.0;
    const double tau = nx > 0.0 ? 1.0 / (s0 - alpha * x0) : 0.0;
    const double u0 = x0 - alpha;
    if (w == 0 && tid == 0) a.d[c] = alpha;
    // w_j = tau (x . W[:, c+j] - alpha W[c][c+j]); updated pivot row y_j = W[c][c+j] - u0 w_j
    double pp = 0.0;
    for (int64_t j = 1 + tid; j < len; j += kB2Threads) {
      const double row = vv[j];
      const double wj = tau * (wv[j] - alpha * row);
      const double y = row - u0 * wj;
      wv[j] = wj;
      vv[j] = y;
      pp += y * y;
    }
    pp = wave_sum_dpp(pp);
    if (lane == 0) red[wave] = pp;
    __syncthreads();
    double ny2 = 0.0;
#pragma unroll
    for (int v = 0; v < kB2Waves; ++v) ny2 += red[v];
    const double y0 = len > 1 ? vv[1] : 0.0;
    const double ny = sqrt(ny2);
    const double beta = ny > 0.0 ? -copysign(ny, y0) : 0.0;
    const double tau2 = ny > 0.0 ? 1.0 / (ny2 - beta * y0) : 0.0;
    const double v1 = y0 - beta;  // first entry of the row reflector; vv[j] for j >= 2
    if (w == 0 && tid == 0 && len > 1) a.e[c] = beta;
    // apply both reflectors to the rows r > c: 16 lanes per row, 4 rows per
    // wavefront; the second pass recomputes the column-step values from LDS
    const int l16 = lane & 15;
    for (int i = 4 * wave + (lane >> 4); i - (lane >> 4) < nr; i += 4 * kB2Waves) {
      const int64_t r = w + (int64_t)P * i;
      const bool live = i < nr && r > c;  // every lane takes part in the row sums
      double* row = Wl + (int64_t)(live ? i : 0) * kp + c;
      const double ur = live ? row[0] : 0.0;
      const int64_t jend = live ? len : 0;
      double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
      for (int64_t j = 1 + l16; j < jend; j += 64) {
        const int64_t j1 = j + 16, j2 = j + 32, j3 = j + 48;
        z0 += (row[j] - ur * wv[j]) * (j == 1 ? v1 : vv[j]);
        if (j1 < jend) z1 += (row[j1] - ur * wv[j1]) * vv[j1];
        if (j2 < jend) z2 += (row[j2] - ur * wv[j2]) * vv[j2];
        if (j3 < jend) z3 += (row[j3] - ur * wv[j3]) * vv[j3];
      }
      const double z = row16_sum((z0 + z1) + (z2 + z3)) * tau2;
      for (int64_t j = 1 + l16; j < jend; j += 64) {
        const int64_t j1 = j + 16, j2 = j + 32, j3 = j + 48;
        const double a0 = row[j], b0 = wv[j], c0 = j == 1 ? v1 : vv[j];
        const double a1 = j1 < jend ? row[j1] : 0.0, b1 = j1 < jend ? wv[j1] : 0.0, c1 = j1 < jend ? vv[j1] : 0.0;
        const double a2 = j2 < jend ? row[j2] : 0.0, b2 = j2 < jend ? wv[j2] : 0.0, c2 = j2 < jend ? vv[j2] : 0.0;
        const double a3 = j3 < jend ? row[j3] : 0.0, b3 = j3 < jend ? wv[j3] : 0.0, c3 = j3 < jend ? vv[j3] : 0.0;
        row[j] = (a0 - ur * b0) - z * c0;
        if (j1 < jend) row[j1] = (a1 - ur * b1) - z * c1;
        if (j2 < jend) row[j2] = (a2 - ur * b2) - z * c2;
        if (j3 < jend) row[j3] = (a3 - ur * b3) - z * c3;
      }
    }
    __syncthreads();
    if (c + 1 < k) {
      partials_lds(a, Wl, nr, c + 1, w);
      if (!grid_sync_coh(a.bar, (unsigned)P * ++epoch, a.info, a.spin_limit)) return;
    }
  }
}

// ---- bidiagonalisation with register-cached reflectors --------------------
// The LDS-resident scheme above, reorganised to move less data through LDS:
// one wavefront updates one row at a time with its 64 lanes (lane q owns the
// columns c + 1 + q + 64 t, t < KPL), the reflector coefficients of those
// columns stay in registers for all of the wavefront's rows, the updated
// entries stay in registers between the row dot product and the write-back,
// and the partial sums of the next column step are accumulated while the
// rows are written (each wavefront adds its rows in order, the wavefronts
// meet in at most 8 LDS slots), so no separate pass over the rows is needed.
__device__ __forceinline__ double bcast_lane0(double v) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

template <int KPL, int NT>
__global__ void __launch_bounds__(NT) k_bidiag_reg(Bidiag2Args a_in) {
  constexpr int NW = NT / 64;
  constexpr int SLOTS = NW < 8 ? NW : 8;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // Every xstride-th workgroup (from xoff) takes part; with xstride = 8 and the dispatch of
  // consecutive workgroups to the 8 XCDs in turn these all sit on one XCD.
  // The others leave at once.
  if ((int)(blockIdx.x % a_in.xstride) != a_in.xoff) return;
  Bidiag2Args a = a_in;
  const int64_t k = a.k, l = a.l, kp = a.kp;
  const int P = a.P, w = blockIdx.x / a.xstride;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nr = (int)((l - w + P - 1) / P);
  double* Wl = reinterpret_cast<double*>(smem_raw);  // [nr_max][kp]
  double* wv = Wl + (int64_t)a.nr_max * kp;           // [k + 1]
  double* vv = wv + (k + 1);                           // [k + 1]
  double* red = vv + (k + 1);                          // [NW]
  double* pw = red + NW;                               // [SLOTS][k + 1]
  double* sink = pw + SLOTS * (k + 1);                 // [NT]: target of masked-off stores
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int64_t e = tid; e < (int64_t)nr * k; e += NT) {
    const int64_t i = e / k, j = e - i * k;
    const double x = a.C[(w + P * i) * k + j];
    if (!isfinite(x)) s_bad = 1;
    Wl[i * kp + j] = x;
  }
  __syncthreads();
  if (s_bad) __hip_atomic_store(a.info, (int32_t)RE_ERR_NONFINITE, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  unsigned epoch = 0;
  partials_lds(a, Wl, nr, 0, w);
  if (!grid_sync_coh(a.bar, (unsigned)P * ++epoch, a.info, a.spin_limit)) return;

  for (int64_t c = 0; c < k; ++c) {
    const int64_t par = c & 1, len = k - c;
    for (int64_t j = tid; j < len; j += NT) {
      const double* src = a.part + par * P * (k + 1) + j;
      const double rb = ld_coh(&a.rowbuf[par * (k + 1) + j]);
      double s = 0.0;
      for (int p0 = 0; p0 < P; p0 += 16) {
        double v[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (p0 + q < P) ? ld_coh(src + (int64_t)(p0 + q) * (k + 1)) : 0.0;
#pragma unroll
        for (int q = 0; q < 16; ++q) s += v[q];
      }
      wv[j] = s;
      vv[j] = rb;
    }
    __syncthreads();
    const double s0 = wv[0], x0 = vv[0];
    const double nx = sqrt(s0);
    const double alpha = nx > 0.0 ? -copysign(nx, x0) : 0.0;
    const double tau = nx > 0.0 ? 1.0 / (s0 - alpha * x0) : 0.0;
    const double u0 = x0 - alpha;
    if (w == 0 && tid == 0) a.d[c] = alpha;
    double pp = 0.0;
    for (int64_t j = 1 + tid; j < len; j += NT) {
      const double row = vv[j];
      const double wj = tau * (wv[j] - alpha * row);
      const double y = row - u0 * wj;
      wv[j] = wj;
      vv[j] = y;
      pp += y * y;
    }
    pp = wave_sum_dpp(pp);
    if (lane == 0) red[wave] = pp;
    __syncthreads();
    double ny2 = 0.0;
#pragma unroll
    for (int v = 0; v < NW; ++v) ny2 += red[v];
    const double y0 = len > 1 ? vv[1] : 0.0;
    const double ny = sqrt(ny2);
    const double beta = ny > 0.0 ? -copysign(ny, y0) : 0.0;
    const double tau2 = ny > 0.0 ? 1.0 / (ny2 - beta * y0) : 0.0;
    const double v1 = y0 - beta;
    if (w == 0 && tid == 0 && len > 1) a.e[c] = beta;
    // this lane's reflector coefficients, columns c + j with j = 1 + lane + 64 t
    // (loads are issued unconditionally from a clamped in-range index and
    // masked afterwards, so each batch of LDS reads costs one wait)
    double cw[KPL], cv[KPL], pa[KPL];
#pragma unroll
    for (int t = 0; t < KPL; ++t) {
      const int64_t j = 1 + lane + 64 * t, jc = j < len ? j : len - 1;
      const double a = wv[jc], b = vv[jc];
      cw[t] = j < len ? a : 0.0;
      cv[t] = j < len ? (j == 1 ? v1 : b) : 0.0;
      pa[t] = 0.0;
    }
    for (int i = wave; i < nr; i += NW) {
      if (w + (int64_t)P * i <= c) continue;  // rows above the pivot are final
      double* row = Wl + (int64_t)i * kp + c;
      double raw[KPL];
#pragma unroll
      for (int t = 0; t < KPL; ++t) {
        const int64_t j = 1 + lane + 64 * t, jc = j < len ? j : len - 1;
        raw[t] = row[jc];
      }
      const double ur = row[0];
      double tv[KPL];
      double zp = 0.0;
#pragma unroll
      for (int t = 0; t < KPL; ++t) {
        const int64_t j = 1 + lane + 64 * t;
        tv[t] = j < len ? raw[t] - ur * cw[t] : 0.0;
        zp += tv[t] * cv[t];
      }
      const double z = wave_sum_dpp(zp) * tau2;
      const double x1 = bcast_lane0(tv[0] - z * cv[0]);  // the row's new entry in column c + 1
      // masked-off lanes (j >= len) have tv = cv = 0, so nv = 0 adds nothing
      // to pa; their store goes to this thread's sink slot
#pragma unroll
      for (int t = 0; t < KPL; ++t) {
        const int64_t j = 1 + lane + 64 * t;
        const double nv = tv[t] - z * cv[t];
        *(j < len ? row + j : sink + tid) = nv;
        pa[t] += x1 * nv;
      }
    }
    if (c + 1 < k) {
      // partials of column c + 1: part[j - 1] = sum over rows of W[r][c+1] W[r][c+j]
      if constexpr (NW > SLOTS) {  // wavefronts past the slots hand their sums over first
        if (wave >= SLOTS) {
          double* dst = pw + (int64_t)(wave - SLOTS) * (k + 1);
#pragma unroll
          for (int t = 0; t < KPL; ++t) {
            const int64_t j = 1 + lane + 64 * t;
            if (j < len) dst[j - 1] = pa[t];
          }
        }
        __syncthreads();
      }
      if (wave < SLOTS) {
        double* dst = pw + (int64_t)wave * (k + 1);
#pragma unroll
        for (int t = 0; t < KPL; ++t) {
          const int64_t j = 1 + lane + 64 * t;
          if (j < len) dst[j - 1] = (wave + SLOTS < NW ? dst[j - 1] : 0.0) + pa[t];
        }
      }
      __syncthreads();
      const int64_t par1 = (c + 1) & 1, len1 = len - 1;
      const bool owner = ((c + 1) % P) == w;
      const int iown = (int)((c + 1) / P);
      for (int64_t j = tid; j < len1; j += NT) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) s += pw[(int64_t)q * (k + 1) + j];
        st_coh(&a.part[(par1 * P + w) * (k + 1) + j], s);
        if (owner) st_coh(&a.rowbuf[par1 * (k + 1) + j], Wl[(int64_t)iown * kp + c + 1 + j]);
      }
      if (!grid_sync_coh(a.bar, (unsigned)P * ++epoch, a.info, a.spin_limit)) return;
    }
  }
}

// ---- bidiagonalisation of a sketch held by one workgroup ----------------
// When the whole l x k sketch fits in LDS one workgroup reduces it alone:
// the column partials go straight to LDS and workgroup barriers replace the
// grid barrier.  Launched with one workgroup per problem, so it also runs
// many independent sketches at once (problem b = blockIdx.x).
struct SmallBatch {
  const double* const* C;  // per problem: l x k row-major input (NULL: single problem below)
  double* const* d;        // per problem: k diagonal entries
  double* const* e;        // per problem: k - 1 superdiagonal entries
  const int32_t* l;        // per problem rows
  const int32_t* k;        // per problem columns
  int32_t* info;           // per problem status
  int kp;                  // LDS row stride in doubles (kp = 16 mod 32, kp >= max k)
  const double* C1;        // the single problem when C is NULL
  double* d1;
  double* e1;
  int32_t l1, k1;
};

__global__ void __launch_bounds__(kB2Threads) k_bidiag_1wg(SmallBatch sb) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const bool one = sb.C == nullptr;
  const int64_t l = one ? sb.l1 : sb.l[b], k = one ? sb.k1 : sb.k[b], kp = sb.kp;
  const double* C = one ? sb.C1 : sb.C[b];
  double* dd = one ? sb.d1 : sb.d[b];
  double* ee = one ? sb.e1 : sb.e[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* Wl = reinterpret_cast<double*>(smem_raw);  // [l][kp]
  double* wv = Wl + l * kp;                           // [k + 1]
  double* vv = wv + (k + 1);                          // [k + 1]
  double* red = vv + (k + 1);                         // [kB2Waves]
  double* part = red + kB2Waves;                      // [kB2Threads] row-group partials
  __shared__ int s_bad;
  if (tid == 0) s_bad = 0;
  __syncthreads();
  for (int64_t e = tid; e < l * k; e += kB2Threads) {
    const int64_t i = e / k, j = e - i * k;
    const double x = C[e];
    if (!isfinite(x)) s_bad = 1;
    Wl[i * kp + j] = x;
  }
  __syncthreads();
  if (tid == 0) sb.info[b] = s_bad ? (int32_t)RE_ERR_NONFINITE : 0;
  for (int c = 0; c < (int)k; ++c) {
    const int len = (int)k - c;
    // column partials of column c: wv = x . W[:, c + j], vv = W[c][c + j].
    // Thread t takes column j = t % len over rows c + g, c + g + G, ...
    // (g = t / len, G groups); the G partials are then summed in order.
    if (len <= kB2Threads) {
      const int G = min(kB2Threads / len, 32);
      const int j = tid % len, g = tid / len;
      if (g < G) {
        double a0 = 0.0, a1 = 0.0;
        int i = c + g;
        for (; i + G < (int)l; i += 2 * G) {
          a0 += Wl[i * kp + c] * Wl[i * kp + c + j];
          a1 += Wl[(i + G) * kp + c] * Wl[(i + G) * kp + c + j];
        }
        if (i < (int)l) a0 += Wl[i * kp + c] * Wl[i * kp + c + j];
        part[g * len + j] = a0 + a1;
      }
      __syncthreads();
      if (tid < len) {
        double t = 0.0;
        for (int q = 0; q < G; ++q) t += part[q * len + tid];
        wv[tid] = t;
        vv[tid] = Wl[c * kp + c + tid];
      }
    } else {
      for (int j = tid; j < len; j += kB2Threads) {
        double a0 = 0.0;
        for (int i = c; i < (int)l; ++i) a0 += Wl[i * kp + c] * Wl[i * kp + c + j];
        wv[j] = a0;
        vv[j] = Wl[c * kp + c + j];
      }
    }
    __syncthreads();
    const double s0 = wv[0], x0 = vv[0];
    const double nx = sqrt(s0);
    const double alpha = nx > 0.0 ? -copysign(nx, x0) : 0.0;
    const double tau = nx > 0.0 ? 1.0 / (s0 - alpha * x0) : 0.0;
    const double u0 = x0 - alpha;
    if (tid == 0) dd[c] = alpha;
    double pp = 0.0;
    for (int64_t j = 1 + tid; j < len; j += kB2Threads) {
      const double row = vv[j];
      const double wj = tau * (wv[j] - alpha * row);
      const double y = row - u0 * wj;
      wv[j] = wj;
      vv[j] = y;
      pp += y * y;
    }
    pp = wave_sum_dpp(pp);
    if (lane == 0) red[wave] = pp;
    __syncthreads();
    double ny2 = 0.0;
#pragma unroll
    for (int v = 0; v < kB2Waves; ++v) ny2 += red[v];
    const double y0 = len > 1 ? vv[1] : 0.0;
    const double ny = sqrt(ny2);
    const double beta = ny > 0.0 ? -copysign(ny, y0) : 0.0;
    const double tau2 = ny > 0.0 ? 1.0 / (ny2 - beta * y0) : 0.0;
    const double v1 = y0 - beta;
    if (tid == 0 && len > 1) ee[c] = beta;
    const int l16 = lane & 15;
    for (int64_t i = c + 1 + 4 * wave + (lane >> 4); i - (lane >> 4) < l; i += 4 * kB2Waves) {
      const bool live = i < l;
      double* row = Wl + (live ? i : 0) * kp + c;
      const double ur = live ? row[0] : 0.0;
      const int64_t jend = live ? len : 0;
      double z0 = 0.0, z1 = 0.0;
      for (int64_t j = 1 + l16; j < jend; j += 32) {
        z0 += (row[j] - ur * wv[j]) * (j == 1 ? v1 : vv[j]);
        if (j + 16 < jend) z1 += (row[j + 16] - ur * wv[j + 16]) * vv[j + 16];
      }
      const double z = row16_sum(z0 + z1) * tau2;
      for (int64_t j = 1 + l16; j < jend; j += 16) row[j] = (row[j] - ur * wv[j]) - z * (j == 1 ? v1 : vv[j]);
    }
    __syncthreads();
  }
}

// ---- bidiagonalisation with the sketch held in registers ----------------
// The same reflectors as above for sketches of up to 16 KT columns and
// 32 RS rows.  Eight wavefronts; each row sits in one row of 16 lanes:
// row i in wavefront (i / 4) mod 8, lanes 16 (i mod 4) .. + 15, slot i / 32,
// and column j in lane j mod 16 of that row, slot j / 16.  So the reflector
// of a row ends in a 16-lane sum, four rows at a time, rather than in a sum
// over the wavefront.  A workgroup needs LDS only for the column partials,
// the Gram row and the pivot row (about 2.5 KT KiB), and two share a CU.  Per
// column two workgroup barriers: the wavefronts' partials of the Gram row
// x . W[:, j] go to LDS, then the first 16 KT threads sum them in wavefront
// order into the Gram row (buffers double-buffered by the parity of c).
// Every wavefront reads the same Gram row and pivot row and so forms the
// same reflectors, and each updates its own rows.
constexpr int kBRWaves = 8, kBRThreads = 64 * kBRWaves;

// Lane `src` (uniform) of a double in every lane.
__device__ __forceinline__ double lane_value(double v, int src) {
  const uint64_t u = __double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)u, src);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), src);
  return __longlong_as_double(((uint64_t)hi << 32) | lo);
}

template <int KT, int RS>
__global__ void __launch_bounds__(kBRThreads) __attribute__((amdgpu_waves_per_eu(KT * RS <= 32 && KT < 8 ? 4 : 1)))
k_bidiag_rows(SmallBatch sb) {
  constexpr int S = 16 * KT;  // LDS row stride of the partials
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int b = blockIdx.x;
  const bool one = sb.C == nullptr;
  const int l = one ? sb.l1 : sb.l[b], k = one ? sb.k1 : sb.k[b];
  const double* __restrict__ C = one ? sb.C1 : sb.C[b];
  double* dd = one ? sb.d1 : sb.d[b];
  double* ee = one ? sb.e1 : sb.e[b];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int q = lane >> 4, l16 = lane & 15;
  const int i0 = 4 * wave + q;  // row of slot 0; slot s holds row i0 + 32 s
  double* part = reinterpret_cast<double*>(smem_raw);  // [2][kBRWaves][S]
  double* rowc = part + 2 * kBRWaves * S;              // [2][S]
  double* gsum = rowc + 2 * S;                         // [2][S]
  double R[RS][KT];
  int bad = 0;
#pragma unroll
  for (int s = 0; s < RS; ++s) {
    const int i = i0 + 32 * s;
#pragma unroll
    for (int t = 0; t < KT; ++t) {
      const int j = l16 + 16 * t;
      const double x = (i < l && j < k) ? C[(int64_t)i * k + j] : 0.0;
      bad |= !isfinite(x);
      R[s][t] = x;
    }
  }
  bad = __syncthreads_or(bad);
  if (tid == 0) sb.info[b] = bad ? (int32_t)RE_ERR_NONFINITE : 0;
#pragma unroll
  for (int tc = 0; tc < KT; ++tc) {
    for (int lc = 0; lc < 16; ++lc) {
      const int c = 16 * tc + lc;
      if (c >= k) break;
      const int buf = c & 1;
      double* pb = part + buf * kBRWaves * S;
      double* rb = rowc + buf * S;
      double* gb = gsum + buf * S;
      const int src = (lane & 48) | lc;  // lane of column c in this row of lanes
      // this wavefront's partials of x . W[:, j] over its rows i >= c, summed
      // over its four rows of lanes, and the pivot row from its owner
      double p[KT];
#pragma unroll
      for (int t = 0; t < KT; ++t) p[t] = 0.0;
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int i = i0 + 32 * s;
        if (4 * wave + 32 * s + 3 >= c && 4 * wave + 32 * s < l) {  // some row of this slot counts
          double xc = __shfl(R[s][tc], src, 64);
          xc = (i >= c && i < l) ? xc : 0.0;
#pragma unroll
          for (int t = 0; t < KT; ++t) p[t] = fma(xc, R[s][t], p[t]);
        }
        if (i == c)
#pragma unroll
          for (int t = 0; t < KT; ++t) rb[l16 + 16 * t] = R[s][t];
      }
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        p[t] += __shfl_xor(p[t], 16, 64);
        p[t] += __shfl_xor(p[t], 32, 64);
        if (q == 0) pb[wave * S + l16 + 16 * t] = p[t];
      }
      __syncthreads();
      // the Gram row, summed over the wavefronts in order once per column
      if (tid < S) {
        double g = 0.0;
#pragma unroll
        for (int w = 0; w < kBRWaves; ++w) g += pb[w * S + tid];
        gb[tid] = g;
      }
      __syncthreads();
      const double s0 = gb[c];
      const double x0 = rb[c];
      const double nx = sqrt(s0);
      const double alpha = nx > 0.0 ? -copysign(nx, x0) : 0.0;
      const double tau = nx > 0.0 ? 1.0 / (s0 - alpha * x0) : 0.0;
      const double u0 = x0 - alpha;
      if (tid == 0) dd[c] = alpha;
      // the pivot row after the left reflector (y, columns j > c) and the
      // left reflector's row factors w
      double wj[KT], v[KT];  // v holds y until the right reflector is formed
      double pp = 0.0;
#pragma unroll
      for (int t = 0; t < KT; ++t) {
        const int j = l16 + 16 * t;
        const double g = gb[j];
        const double row = rb[j];
        const bool live = j > c && j < k;
        wj[t] = live ? tau * (g - alpha * row) : 0.0;
        v[t] = live ? row - u0 * wj[t] : 0.0;
        pp += v[t] * v[t];
      }
      const double ny2 = row16_sum(pp);
      const double ysrc = (lc == 15 && tc + 1 < KT) ? v[tc + 1 < KT ? tc + 1 : tc] : v[tc];
      const double y0 = c + 1 < k ? lane_value(ysrc, (c + 1) & 15) : 0.0;
      const double ny = sqrt(ny2);
      const double beta = ny > 0.0 ? -copysign(ny, y0) : 0.0;
      const double tau2 = ny > 0.0 ? 1.0 / (ny2 - beta * y0) : 0.0;
      const double v1 = y0 - beta;
      if (tid == 0 && c + 1 < k) ee[c] = beta;
#pragma unroll
      for (int t = 0; t < KT; ++t) v[t] = l16 + 16 * t == c + 1 ? v1 : v[t];
      // rows below the pivot: left reflector, then right reflector (rows at
      // or above it take ur = z = 0 and keep their values)
#pragma unroll
      for (int s = 0; s < RS; ++s) {
        const int i = i0 + 32 * s;
        if (4 * wave + 32 * s + 3 > c && 4 * wave + 32 * s < l) {
          const bool live = i > c && i < l;
          double ur = __shfl(R[s][tc], src, 64);
          ur = live ? ur : 0.0;
          double zp = 0.0;
#pragma unroll
          for (int t = 0; t < KT; ++t) {
            R[s][t] = R[s][t] - ur * wj[t];
            zp += R[s][t] * v[t];
          }
          double z = row16_sum(zp) * tau2;
          z = live ? z : 0.0;
#pragma unroll
          for (int t = 0; t < KT; ++t) R[s][t] = R[s][t] - z * v[t];
        }
      }
    }
  }
}

// ---- singular values of the bidiagonal by multisection on Sturm counts ----

// Sturm counts of the Golub-Kahan tridiagonal T of order n = nb + 1 = 2k (zero
// diagonal, off-diagonal b[0..nb), bb[j] = b[j]^2) at a shift x > 0.  The
// number of eigenvalues of T below x, minus its k negative ones, is the
// number of singular values below x; by Sylvester's law of inertia it is the
// number of negative pivots of T - x I, whose LDL^T pivots run top-down as
// q_0 = -x, q_j = -x - bb[j-1] / q_{j-1}.

// The factorisation twisted at row r = k has the same inertia: top-down
// pivots q_0 .. q_r as above, bottom-up p_{n-1} = -x, p_j = -x - bb[j] /
// p_{j+1} down to p_r, and the pivot of row r, g = q_r + p_r + x.
// The same two halves through the leading (trailing) principal minors of
// T - x I instead of the pivots: D_0 = 1, D_1 = -x, D_{j+1} = -x D_j - bb[j-1]
// D_{j-1}, so q_j = D_{j+1} / D_j and the negative pivots are the sign changes
// of D_0 .. D_r.  One FMA per step is on the dependent chain (bb D_{j-1} is
// formed a step ahead) instead of a reciprocal and its Newton correction.
// Each FMA rounds once, which is a relative perturbation of x and of bb[j-1]
// as in the pivot form's error analysis.  The entries come prescaled by a
// power of two so that x <= 2 and bb <= 4: a step grows the pair (D_{j-1},
// D_j) by at most 6x, and shrinks it by no more than x, which the
// multisection keeps above 2^-60 of the bound; the pair is renormalised by a
// power of two every four steps.  Returns the negatives among q_0 .. q_{r-1}
// and the last pivot q_r.
__device__ __forceinline__ void renorm(double& a, double& b) {
  const double mx = fmax(fabs(a), fabs(b));
  if (mx > 0.0) {
    const int e = __builtin_amdgcn_frexp_exp(mx);
    a = __builtin_ldexp(a, -e);
    b = __builtin_ldexp(b, -e);
  }
}

__device__ double minors_top(const double* bb, int r, double x, int& neg) {
  double D0 = 1.0, D1 = -x;
  int ng = r > 0 ? 1 : 0;  // q_0 = -x < 0
  if (r == 0) {
    neg = 0;
    return -x;
  }
  int j = 1;
  for (; j + 3 < r; j += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double D2 = fma(-x, D1, -bb[j + u - 1] * D0);
      ng += (D2 < 0.0) != (D1 < 0.0);
      D0 = D1;
      D1 = D2;
    }
    renorm(D0, D1);
  }
  for (; j < r; ++j) {
    const double D2 = fma(-x, D1, -bb[j - 1] * D0);
    ng += (D2 < 0.0) != (D1 < 0.0);
    D0 = D1;
    D1 = D2;
  }
  neg = ng;
  // q_r = -x - bb[r-1] D_{r-1} / D_r; a zero D_r (q_{r-1} = 0) gives q_r -> +inf
  return D1 != 0.0 ? -x - bb[r - 1] * (D0 / D1) : HUGE_VAL;
}

// Bottom half: E_{n} = 1, E_{n-1} = -x, E_j = -x E_{j+1} - bb[j] E_{j+2}, p_j =
// E_j / E_{j+1}; the negatives among p_{n-1} .. p_{r+1} and the pivot p_r.
__device__ double minors_bottom(const double* bb, int nb, int r, double x, int& neg) {
  const int n = nb + 1;
  double E0 = 1.0, E1 = -x;  // E_{j+2}, E_{j+1} for j = n - 2
  int ng = n - 1 > r ? 1 : 0;  // p_{n-1} = -x < 0
  if (n - 1 <= r) {
    neg = 0;
    return -x;
  }
  int j = n - 2;
  for (; j - 3 > r; j -= 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double E2 = fma(-x, E1, -bb[j - u] * E0);
      ng += (E2 < 0.0) != (E1 < 0.0);
      E0 = E1;
      E1 = E2;
    }
    renorm(E0, E1);
  }
  for (; j > r; --j) {
    const double E2 = fma(-x, E1, -bb[j] * E0);
    ng += (E2 < 0.0) != (E1 < 0.0);
    E0 = E1;
    E1 = E2;
  }
  neg = ng;
  return E1 != 0.0 ? -x - bb[r] * (E0 / E1) : HUGE_VAL;
}

// Singular values of the bidiagonal (d, e) by 64-way multisection on the
// Sturm counts: a pair of wavefronts per value, one running each half of the
// twisted factorisation (the count's dependent chain is issue-bound, so the
// halves go to different SIMDs), meeting in LDS once per multisection round.
__global__ void __launch_bounds__(256) k_bidiag_sv(const double* __restrict__ d, const double* __restrict__ e,
                                                   int64_t k, double scale, const int32_t* __restrict__ info,
                                                   double* __restrict__ sigma) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* b = reinterpret_cast<double*>(smem_raw);  // 2k - 1 off-diagonal entries
  const int nb = (int)(2 * k - 1);
  double* bb = b + nb;                                // their squares
  __shared__ double s_piv[2][64];
  __shared__ int s_neg[2][64];
  __shared__ double s_iv[2][2];
  double bound = 0.0;
  for (int j = threadIdx.x; j < nb; j += blockDim.x) b[j] = (j & 1) ? e[j >> 1] : d[j >> 1];
  __syncthreads();
  for (int j = 0; j < nb; ++j) {  // every thread, same order
    const double left = j > 0 ? fabs(b[j - 1]) : 0.0;
    bound = fmax(bound, fabs(b[j]) + left);
  }
  bound = fmax(bound, nb > 0 ? fabs(b[nb - 1]) : 0.0);
  const bool all_zero = !(bound > 0.0);  // B = 0 (NaN is reported through info)
  bound = bound * (1.0 + 1e-14) + 1e-300;
  // the counts run on the entries scaled by 2^-eb (bound < 2^eb), exactly
  const int eb = __builtin_amdgcn_frexp_exp(bound);
  const double xs = __builtin_ldexp(1.0, -eb);
  __syncthreads();
  for (int j = threadIdx.x; j < nb; j += blockDim.x) {
    const double bs = __builtin_ldexp(b[j], -eb);
    bb[j] = bs * bs;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int slot = wave >> 1, bottom = wave & 1;  // two values per workgroup
  const int r = (nb + 1) >> 1;
  for (int64_t base = 2 * (int64_t)blockIdx.x; base < k; base += 2 * (int64_t)gridDim.x) {
    const int64_t jj = base + slot;
    const bool act = jj < k;
    // jj-th largest singular value: #{sigma < lo} <= k-1-jj < #{sigma < hi}
    const int want = (int)(k - 1 - jj);
    double lo = 0.0, hi = bound;
    for (int it = 0; it < 9; ++it) {  // 65^9 > 2^54: below one ulp of the bound
      const double x = lo + (hi - lo) * (double)(lane + 1) * (1.0 / 65.0);
      int ng = 0;
      double piv = 0.0;
      if (act) piv = bottom ? minors_bottom(bb, nb, r, x * xs, ng) : minors_top(bb, r, x * xs, ng);
      if (bottom) {
        s_piv[slot][lane] = piv;
        s_neg[slot][lane] = ng;
      }
      __syncthreads();
      if (!bottom && act) {
        double g = piv + s_piv[slot][lane] + x * xs;  // the twisted pivot, scaled entries
        if (fabs(g) < 0x1.0p-1020) g = -0x1.0p-1020;
        const int cnt = ng + s_neg[slot][lane] + (g < 0.0) - r;
        const uint64_t le = __ballot(cnt <= want);  // monotone in lane
        const int nle = __popcll(le);               // lanes 0..nle-1 satisfy cnt <= want
        if (lane == 0) {
          s_iv[slot][0] = nle > 0 ? lo + (hi - lo) * (double)nle * (1.0 / 65.0) : lo;
          s_iv[slot][1] = nle < 64 ? lo + (hi - lo) * (double)(nle + 1) * (1.0 / 65.0) : hi;
        }
      }
      __syncthreads();
      lo = s_iv[slot][0];
      hi = s_iv[slot][1];
    }
    if (act && !bottom && lane == 0) sigma[jj] = all_zero ? 0.0 : 0.5 * (lo + hi) * scale;
    __syncthreads();
  }
  (void)info;
}

// r^ = #{ i < r1 : sigma_i > eps sigma_1 } over the descending estimates.
__global__ void __launch_bounds__(256) k_count(const double* __restrict__ sigma, int64_t k, int32_t r1, double eps,
                                              const int32_t* __restrict__ info, int32_t* __restrict__ out) {
  __shared__ int s_bad, s_cnt;
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_cnt = 0;
  }
  __syncthreads();
  const double s1 = k > 0 ? sigma[0] : 0.0;
  const double tau = eps * s1;
  const int64_t lim = r1 < k ? r1 : k;
  int bad = 0, cnt = 0;
  for (int64_t i = threadIdx.x; i < k; i += blockDim.x) {
    const double v = sigma[i];
    bad |= !isfinite(v);
    cnt += (i < lim && v > tau);
  }
  if (bad) atomicOr(&s_bad, 1);
  atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (threadIdx.x != 0) return;
  int32_t st = info ? info[0] : 0;
  if (st == 0 && s_bad) st = RE_ERR_NONFINITE;
  uint32_t flags = 0;
  int32_t r = 0;
  if (st == 0) {
    if (k == 0 || s1 == 0.0) {
      flags |= RE_FLAG_ZERO;
    } else {
      r = s_cnt;
      if (r == r1) flags |= RE_FLAG_NOT_CONVERGED;
    }
  }
  out[0] = r;
  out[1] = (int32_t)flags;
  out[2] = st;
}

// Gap statistics of the descending estimates for a search without a
// tolerance (Sec. 5 after Algorithm 1, Sec. 6.1), over the 1-based i < n =
// min(r1, k) with s_i > 0, ratio_i = s_i / s_{i+1} (infinite when s_{i+1} = 0):
//   g      the largest i with ratio_i >= gamma (0 when none)
//   a      the i of the largest ratio, ties to the smallest i
//   reached  s_n <= floor s_1
// out: int32 {g, a, reached, status}, then doubles {ratio_g, ratio_a, s_1}.
__global__ void __launch_bounds__(256) k_gap(const double* __restrict__ sigma, int64_t k, int32_t r1, double gamma,
                                            double floor_rel, const int32_t* __restrict__ info,
                                            GapOut* __restrict__ out) {
  __shared__ int64_t s_z;
  __shared__ int64_t s_g[256];
  __shared__ double s_q[256];
  __shared__ int64_t s_a[256];
  const int64_t n = r1 < k ? r1 : k;
  if (threadIdx.x == 0) s_z = n;
  __syncthreads();
  // first index (0-based, below n) holding a non-positive estimate
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
    if (!(sigma[j] > 0.0)) atomicMin((unsigned long long*)&s_z, (unsigned long long)j);
  __syncthreads();
  const int64_t z = s_z;
  // ratios for 1 <= i <= min(n - 1, z)
  const int64_t hi = (n - 1) < z ? (n - 1) : z;
  int64_t g = 0, a = 0;
  double qa = -1.0;
  for (int64_t i = 1 + threadIdx.x; i <= hi; i += blockDim.x) {
    const double num = sigma[i - 1], den = sigma[i];
    const double q = den > 0.0 ? num / den : HUGE_VAL;
    if (q >= gamma && i > g) g = i;
    if (q > qa) {  // i increases along a thread's sequence, so strict > keeps its smallest
      qa = q;
      a = i;
    }
  }
  s_g[threadIdx.x] = g;
  s_q[threadIdx.x] = qa;
  s_a[threadIdx.x] = a;
  __syncthreads();
  if (threadIdx.x != 0) return;
  int64_t G = 0, Aix = 0;
  double QA = -1.0;
  for (int t = 0; t < (int)blockDim.x; ++t) {
    if (s_g[t] > G) G = s_g[t];
    if (s_a[t] > 0 && (s_q[t] > QA || (s_q[t] == QA && s_a[t] < Aix))) {
      QA = s_q[t];
      Aix = s_a[t];
    }
  }
  const double s1 = n > 0 ? sigma[0] : 0.0;
  GapOut o{};
  o.status = info ? info[0] : 0;
  if (o.status == 0) {
    for (int64_t j = 0; j < k; ++j)
      if (!isfinite(sigma[j])) o.status = RE_ERR_NONFINITE;
  }
  if (s1 > 0.0 && n >= 2) {
    o.g = (int32_t)G;
    o.a = (int32_t)Aix;
    o.ratio_g = G > 0 ? (sigma[G] > 0.0 ? sigma[G - 1] / sigma[G] : HUGE_VAL) : 0.0;
    o.ratio_a = Aix > 0 ? QA : 0.0;
  }
  o.reached = n > 0 && sigma[n - 1] <= floor_rel * s1;
  o.s1 = s1;
  *out = o;
}

__global__ void k_svd_init(unsigned* bar, int32_t* info) {
  if (threadIdx.x == 0) {
    bar[0] = 0;
    info[0] = 0;
  }
}

int choose_P(int64_t l) {
  int64_t P = l / 32;
  if (P < 1) P = 1;
  if (P > 64) P = 64;
  return (int)P;
}

// LDS-resident bidiagonalisation: the fewest workgroups whose rows fit in
// LDS next to two k+1 vectors; P = 0 when no such launch exists (k > 1025
// or more than 64 workgroups needed), and the global-memory kernel runs.
constexpr size_t kLdsBudget = 156 * 1024;
struct LdsPlan {
  int P, nr_max;
  size_t bytes;
};
int64_t lds_stride(int64_t k) { return k + ((16 - k % 32) + 32) % 32; }

// LDS bytes of the single-workgroup bidiagonalisation of an l x k sketch.
size_t small_lds_bytes(int64_t l, int64_t k) {
  return (size_t)l * lds_stride(k) * 8 + (size_t)(2 * (k + 1) + kB2Waves + kB2Threads) * 8;
}

// The register-held bidiagonalisation for an l x k sketch: kernel and LDS
// bytes, or no kernel when the sketch exceeds 128 columns or 32 x 12 rows
// (32 x 6 rows above 64 columns).
struct RowsKernel {
  const void* fn;
  size_t lds;
};
RowsKernel rows_kernel(int64_t l, int64_t k) {
  const int64_t rs = (l + 31) / 32;
  const void* fn = nullptr;
  int kt = 0;
  if (k <= 64) {
    kt = 4;
    fn = rs <= 2   ? (const void*)k_bidiag_rows<4, 2>
         : rs <= 4 ? (const void*)k_bidiag_rows<4, 4>
         : rs <= 8 ? (const void*)k_bidiag_rows<4, 8>
         : rs <= 12 ? (const void*)k_bidiag_rows<4, 12>
                    : nullptr;
  } else if (k <= 96) {
    kt = 6;
    fn = rs <= 3 ? (const void*)k_bidiag_rows<6, 3> : rs <= 5 ? (const void*)k_bidiag_rows<6, 5> : nullptr;
  } else if (k <= 128) {
    kt = 8;
    fn = rs <= 4 ? (const void*)k_bidiag_rows<8, 4> : rs <= 6 ? (const void*)k_bidiag_rows<8, 6> : nullptr;
  }
  return {fn, (size_t)(2 * kBRWaves + 4) * 16 * kt * sizeof(double)};
}

// Rows per workgroup at most `svd_rows_target()` (fewer rows shorten the
// per-column update; more workgroups lengthen the reduction), overridable
// with RANKEST_SVD_ROWS for tuning.
// Placement of the bidiagonalisation's workgroups (RANKEST_SVD_XCD, default
// 1): all on one XCD (launched eight times over, every eighth workgroup taking
// part), which shortens the device-scope exchanges between them by about 6 %
// at 576 x 384; 0 = consecutive workgroups.
bool svd_one_xcd() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("RANKEST_SVD_XCD");
    v = e ? (atoi(e) != 0) : 1;
  }
  return v == 1;
}

int svd_rows_target() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("RANKEST_SVD_ROWS");
    v = e ? atoi(e) : 48;
    if (v < 1) v = 1;
  }
  return v;
}

// RANKEST_SVD_THREADS=1024 runs the register-cached kernel with 16
// wavefronts for k <= 385 (tuning; 8 measured faster).
bool svd_threads_1024() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("RANKEST_SVD_THREADS");
    v = (e && atoi(e) == 1024) ? 1 : 0;
  }
  return v == 1;
}

// RANKEST_SVD_LEGACY=1 selects the plain LDS-resident kernel (comparisons).
bool svd_legacy_lds() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("RANKEST_SVD_LEGACY");
    v = (e && atoi(e) != 0) ? 1 : 0;
  }
  return v == 1;
}

// RANKEST_SVD_LEGACY_GLOBAL=1 selects the first global-memory kernel for wide
// sketches instead of the register-row one (comparisons).
bool svd_legacy_global() {
  static int v = -1;
  if (v < 0) {
    const char* e = getenv("RANKEST_SVD_LEGACY_GLOBAL");
    v = (e && atoi(e) != 0) ? 1 : 0;
  }
  return v == 1;
}

LdsPlan lds_plan(int64_t l, int64_t k) {
  LdsPlan p{0, 0, 0};
  if (k > 1025) return p;
  const size_t fixed = (size_t)(2 * (k + 1) + kB2Waves) * 8;
  const int P0 = (int)((l + svd_rows_target() - 1) / svd_rows_target());
  for (int P = P0 < 1 ? 1 : (P0 > 64 ? 64 : P0); P <= 64 && P <= l; ++P) {
    const int64_t nr = (l + P - 1) / P;
    const size_t bytes = (size_t)nr * lds_stride(k) * 8 + fixed;
    if (bytes <= kLdsBudget) {
      p.P = P;
      p.nr_max = (int)nr;
      p.bytes = bytes;
      return p;
    }
  }
  return p;
}

// Plan of the register-cached kernel: KPL columns per lane (k <= 64 KPL + 1),
// 512 threads (fewer wavefronts make the per-column barriers cheaper; 1024
// fit the registers only up to KPL = 6); rows per workgroup as lds_plan.
struct RegPlan {
  int P, nr_max, kpl, nt;
  size_t bytes;
};
RegPlan reg_plan(int64_t l, int64_t k) {
  RegPlan p{0, 0, 0, 0, 0};
  const int64_t need = k <= 1 ? 1 : (k - 1 + 63) / 64;
  static const int kpls[] = {1, 2, 4, 6, 8, 12, 16};
  for (int v : kpls)
    if (v >= need) {
      p.kpl = v;
      break;
    }
  if (p.kpl == 0) return p;
  p.nt = (p.kpl <= 6 && svd_threads_1024()) ? 1024 : 512;
  const int nw = p.nt / 64, slots = nw < 8 ? nw : 8;
  const size_t fixed = (size_t)(2 * (k + 1) + nw + slots * (k + 1) + p.nt) * 8;
  const int P0 = (int)((l + svd_rows_target() - 1) / svd_rows_target());
  for (int P = P0 < 1 ? 1 : (P0 > 64 ? 64 : P0); P <= 64 && P <= l; ++P) {
    const int64_t nr = (l + P - 1) / P;
    const size_t bytes = (size_t)nr * lds_stride(k) * 8 + fixed;
    if (bytes <= kLdsBudget) {
      p.P = P;
      p.nr_max = (int)nr;
      p.bytes = bytes;
      return p;
    }
  }
  p.kpl = 0;
  return p;
}

struct SvdLayout {
  size_t W, part, rowbuf, red, d, e, bar, total;
};

SvdLayout svd_layout(int64_t l, int64_t k) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  SvdLayout s{};
  size_t o = 0;
  s.W = o; o += al((size_t)l * k * 8);
  s.part = o; o += al((size_t)2 * kG2MaxP * (k + 1) * 8);
  s.rowbuf = o; o += al((size_t)2 * (k + 1) * 8);
  s.red = o; o += al((size_t)2 * (k + 1) * 8);
  s.d = o; o += al((size_t)k * 8);
  s.e = o; o += al((size_t)k * 8);
  s.bar = o; o += 256;
  s.total = o;
  return s;
}

// Batched counts (problem = blockIdx.x); same arithmetic as k_count.
// Singular values of small bidiagonals, one lane per value: 56 bisection
// steps on the Sturm count (the interval shrinks below 2^-56 of the bound,
// as the 65-way multisection does in 9 rounds) (`one` when desc is NULL).
// A workgroup takes ppw problems: problem
// blockIdx.x ppw + p on lanes p kslot .. p kslot + kslot - 1, so that 96
// values of two problems fill three wavefronts (ppw = 1: the whole workgroup,
// values strided by blockDim.x).  Used for every batched block and for the
// single calls' sketches whose bidiagonalisation fits one workgroup (except
// the plain method on FP64 inputs, which takes the multisection); a lane's
// arithmetic depends only on its problem and value, so a block of a batch
// and the same matrix alone give the same bits.
constexpr int kBisectSteps = 56;
__global__ void __launch_bounds__(256) k_sv_bisect(const SvDesc* __restrict__ desc, SvDesc one, int nprob, int ppw,
                                                   int kslot, int kmax) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int p = ppw > 1 ? (int)threadIdx.x / kslot : 0;
  const int prob = (int)blockIdx.x * ppw + p;
  const bool live = p < ppw && prob < nprob;
  const int k = live ? (desc ? desc[prob].k : one.k) : 0;
  const SvDesc dsc = live ? (desc ? desc[prob] : one) : one;
  const int base = ppw > 1 ? p * kslot : 0, stride = ppw > 1 ? kslot : (int)blockDim.x;
  double* b = reinterpret_cast<double*>(smem_raw) + (size_t)(live ? p : 0) * 4 * kmax;
  const int nb = 2 * k - 1;
  double* bb = b + 2 * kmax;
  for (int j = (int)threadIdx.x - base; j < nb; j += stride) b[j] = (j & 1) ? dsc.e[j >> 1] : dsc.d[j >> 1];
  __syncthreads();
  double bound = 0.0;
  for (int j = 0; j < nb; ++j) {  // every thread, same order
    const double left = j > 0 ? fabs(b[j - 1]) : 0.0;
    bound = fmax(bound, fabs(b[j]) + left);
  }
  bound = fmax(bound, nb > 0 ? fabs(b[nb - 1]) : 0.0);
  const bool all_zero = !(bound > 0.0);
  bound = bound * (1.0 + 1e-14) + 1e-300;
  // the counts run on the entries scaled by 2^-eb (bound < 2^eb), exactly, in
  // the minors form of the factorisation twisted at r = (nb + 1) / 2 (one FMA
  // on each half's dependent chain, the halves independent): the same count as
  // the pivots' signs, as in the one-matrix multisection
  const int eb = __builtin_amdgcn_frexp_exp(bound);
  const double xs = __builtin_ldexp(1.0, -eb);
  __syncthreads();
  for (int j = (int)threadIdx.x - base; j < nb; j += stride) {
    const double bs = __builtin_ldexp(b[j], -eb);
    bb[j] = bs * bs;
  }
  __syncthreads();
  const int r = (nb + 1) >> 1;
  for (int jj = (int)threadIdx.x - base; jj < k; jj += stride) {
    const int want = k - 1 - jj;  // #{sigma < lo} <= want < #{sigma < hi}
    double lo = 0.0, hi = bound;
    for (int it = 0; it < kBisectSteps; ++it) {
      const double x = 0.5 * (lo + hi);
      int nt = 0, nbt = 0;
      const double pt = minors_top(bb, r, x * xs, nt);
      const double pb = minors_bottom(bb, nb, r, x * xs, nbt);
      double g = pt + pb + x * xs;  // the twisted pivot, scaled entries
      if (fabs(g) < 0x1.0p-1020) g = -0x1.0p-1020;
      if (nt + nbt + (g < 0.0) - r <= want) lo = x;
      else hi = x;
    }
    dsc.sigma[jj] = all_zero ? 0.0 : 0.5 * (lo + hi) * dsc.scale;
  }
}

__global__ void __launch_bounds__(256) k_count_batched(const SvDesc* __restrict__ desc) {
  const SvDesc d = desc[blockIdx.x];
  __shared__ int s_bad, s_cnt;
  if (threadIdx.x == 0) {
    s_bad = 0;
    s_cnt = 0;
  }
  __syncthreads();
  const int64_t k = d.k;
  const double s1 = k > 0 ? d.sigma[0] : 0.0;
  const double tau = d.eps * s1;
  const int64_t lim = d.r1 < k ? d.r1 : k;
  int bad = 0, cnt = 0;
  for (int64_t i = threadIdx.x; i < k; i += blockDim.x) {
    const double v = d.sigma[i];
    bad |= !isfinite(v);
    cnt += (i < lim && v > tau);
  }
  if (bad) atomicOr(&s_bad, 1);
  atomicAdd(&s_cnt, cnt);
  __syncthreads();
  if (threadIdx.x != 0) return;
  int32_t st = d.info ? d.info[0] : 0;
  if (st == 0 && s_bad) st = RE_ERR_NONFINITE;
  uint32_t flags = 0;
  int32_t r = 0;
  if (st == 0) {
    if (k == 0 || s1 == 0.0) {
      flags |= RE_FLAG_ZERO;
    } else {
      r = s_cnt;
      if (r == d.r1) flags |= RE_FLAG_NOT_CONVERGED;
    }
  }
  d.out3[0] = r;
  d.out3[1] = (int32_t)flags;
  d.out3[2] = st;
}

}  // namespace

size_t svd_scratch_bytes(int64_t l, int64_t k) { return svd_layout(l, k).total; }

namespace {
// Launch of a kernel whose workgroups meet at grid barriers.  A cooperative
// launch makes the runtime guarantee that they are resident together; when
// it refuses (on this platform, while another process that has made
// cooperative launches on the device is alive, later processes' cooperative
// launches fail), a plain launch is used instead: these grids hold at most
// one workgroup per CU, so on a device not filled by other work they are
// resident together as well, and otherwise the bounded barrier wait ends the
// call with RE_ERR_NO_CONVERGENCE rather than a hang.
// Launch form of the multi-workgroup kernels, whose participants wait for one
// another at grid barriers.  The cooperative form guarantees that they are
// resident together, but this runtime runs cooperative kernels one at a time
// (also across streams), so estimates in flight on other streams cannot
// overlap their small SVDs.  Where the caller allows it, the form pinned to
// one XCD (at most 32 participants, one workgroup per CU; XCDs handed to
// handles in turn) takes a plain launch instead.  The other kernels never wait
// on it, so its participants do become resident, but under a steady stream of
// other kernels a late participant can wait long for a free CU: the plain form
// therefore polls at most 2^15 times per barrier (tens of milliseconds,
// far above a column step's microseconds), and its caller redoes a give-up
// with a plain launch under the default limit (not the cooperative form:
// processes that mixed cooperative launches into plain ones in flight on
// other streams ended with a segmentation fault at exit).  RANKEST_SVD_LAUNCH=coop or =plain forces one
// form for every launch (for comparisons).
static int svd_launch_override() {
  static const int v = [] {
    const char* e = getenv("RANKEST_SVD_LAUNCH");
    if (!e) return 0;
    return strcmp(e, "coop") == 0 ? 1 : strcmp(e, "plain") == 0 ? 2 : 0;
  }();
  return v;
}

// RANKEST_SVD_PLAIN_POLLS overrides the plain form's poll limit (a negative
// value gives up at the first poll: a test of the cooperative redo).
static long plain_polls() {
  static const long v = [] {
    const char* e = getenv("RANKEST_SVD_PLAIN_POLLS");
    return e ? atol(e) : (1l << 15);
  }();
  return v;
}

re_status launch_grid(const void* fn, dim3 grid, dim3 block, void** params, unsigned lds, hipStream_t s,
                      bool plain = false) {
  if (!plain && hipLaunchCooperativeKernel(fn, grid, block, params, lds, s) == hipSuccess) return RE_OK;
  (void)hipGetLastError();
  RE_TRY_HIP(hipLaunchKernel(fn, grid, block, params, lds, s));
  return RE_OK;
}
}  // namespace

re_status launch_svd(hipStream_t s, const double* C, int64_t l, int64_t k, double scale, void* scratch,
                     double* sigma, int32_t* info, long spin_limit, int xcd, int allow_plain, bool* used_plain,
                     bool multisect_small) {
  if (used_plain) *used_plain = false;
  if (k <= 0) return RE_OK;
  const long spins = spin_limit == 0 ? (1l << 26) : spin_limit;
  if (k > l) return RE_ERR_INVALID_ARG;
  const SvdLayout L = svd_layout(l, k);
  char* base = (char*)scratch;
  BidiagArgs a;
  a.C = C;
  a.W = (double*)(base + L.W);
  a.part = (double*)(base + L.part);
  a.rowbuf = (double*)(base + L.rowbuf);
  a.red = (double*)(base + L.red);
  a.d = (double*)(base + L.d);
  a.e = (double*)(base + L.e);
  a.bar = (unsigned*)(base + L.bar);
  a.info = info;
  a.l = l;
  a.k = k;
  a.P = choose_P(l);
  a.spin_limit = spins;
  hipLaunchKernelGGL(k_svd_init, dim3(1), dim3(64), 0, s, a.bar, info);
  const LdsPlan lp = lds_plan(l, k);
  const size_t one_bytes = small_lds_bytes(l, k);
  if (const RowsKernel rk = rows_kernel(l, k); rk.fn) {
    SmallBatch sb{};
    sb.C1 = C;
    sb.d1 = a.d;
    sb.e1 = a.e;
    sb.l1 = (int32_t)l;
    sb.k1 = (int32_t)k;
    sb.info = info;
    void* args[] = {&sb};
    RE_TRY_HIP(hipLaunchKernel(rk.fn, dim3(1), dim3(kBRThreads), args, rk.lds, s));
  } else if (one_bytes <= kLdsBudget) {
    SmallBatch sb{};
    sb.kp = (int)lds_stride(k);
    sb.C1 = C;
    sb.d1 = a.d;
    sb.e1 = a.e;
    sb.l1 = (int32_t)l;
    sb.k1 = (int32_t)k;
    sb.info = info;
    if (one_bytes > 64 * 1024)
      RE_TRY_HIP(hipFuncSetAttribute((const void*)k_bidiag_1wg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)one_bytes));
    hipLaunchKernelGGL(k_bidiag_1wg, dim3(1), dim3(kB2Threads), one_bytes, s, sb);
  } else if (const RegPlan rp = reg_plan(l, k); rp.P > 0 && !svd_legacy_lds()) {
    Bidiag2Args b2;
    b2.C = C;
    b2.part = a.part;
    b2.rowbuf = a.rowbuf;
    b2.d = a.d;
    b2.e = a.e;
    b2.bar = a.bar;
    b2.info = info;
    b2.spin_limit = spins;
    b2.l = l;
    b2.k = k;
    b2.kp = lds_stride(k);
    b2.P = rp.P;
    b2.nr_max = rp.nr_max;
    // all participants on one XCD when eight workgroups per participant fit
    // the device at once (one per CU), else consecutive workgroups
    int dev = 0, ncu = 0;
    RE_TRY_HIP(hipGetDevice(&dev));
    RE_TRY_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    b2.xstride = svd_one_xcd() && 8 * rp.P <= ncu ? 8 : 1;
    b2.xoff = b2.xstride == 8 ? (xcd & 7) : 0;
    const bool t512 = rp.nt == 512;
    const void* fn = rp.kpl == 1   ? (t512 ? (const void*)k_bidiag_reg<1, 512> : (const void*)k_bidiag_reg<1, 1024>)
                     : rp.kpl == 2 ? (t512 ? (const void*)k_bidiag_reg<2, 512> : (const void*)k_bidiag_reg<2, 1024>)
                     : rp.kpl == 4 ? (t512 ? (const void*)k_bidiag_reg<4, 512> : (const void*)k_bidiag_reg<4, 1024>)
                     : rp.kpl == 6 ? (t512 ? (const void*)k_bidiag_reg<6, 512> : (const void*)k_bidiag_reg<6, 1024>)
                     : rp.kpl == 8 ? (const void*)k_bidiag_reg<8, 512>
                     : rp.kpl == 12 ? (const void*)k_bidiag_reg<12, 512>
                                    : (const void*)k_bidiag_reg<16, 512>;
    if (rp.bytes > 64 * 1024)
      RE_TRY_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)rp.bytes));
    const int ov = svd_launch_override();
    const bool plain = ov == 2 || (ov == 0 && allow_plain != 0 && b2.xstride == 8);
    if (plain && spin_limit == 0 && allow_plain == 1) b2.spin_limit = plain_polls();
    if (used_plain) *used_plain = plain;
    void* params2[] = {&b2};
    RE_TRY(launch_grid(fn, dim3(rp.P * b2.xstride), dim3(rp.nt), params2, (unsigned)rp.bytes, s, plain));
  } else if (lp.P > 0) {
    Bidiag2Args b2;
    b2.C = C;
    b2.part = a.part;
    b2.rowbuf = a.rowbuf;
    b2.d = a.d;
    b2.e = a.e;
    b2.bar = a.bar;
    b2.info = info;
    b2.spin_limit = spins;
    b2.l = l;
    b2.k = k;
    b2.kp = lds_stride(k);
    b2.P = lp.P;
    b2.nr_max = lp.nr_max;
    b2.xstride = 1;
    b2.xoff = 0;
    const void* fn = (const void*)k_bidiag_lds;
    if (lp.bytes > 64 * 1024)
      RE_TRY_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lp.bytes));
    void* params2[] = {&b2};
    RE_TRY(launch_grid(fn, dim3(lp.P), dim3(kB2Threads), params2, (unsigned)lp.bytes, s, svd_launch_override() == 2));
  } else if (k <= 48 * 64 && !svd_legacy_global()) {
    // rows in registers: 32 or 48 columns per lane
    const bool t32 = k <= 32 * 64;
    const void* fn = t32 ? (const void*)k_bidiag_g2<32> : (const void*)k_bidiag_g2<48>;
    const size_t lds = (size_t)(2 * (k + 1) + kWaves * 64 * (t32 ? 32 : 48)) * 8;
    if (lds > 64 * 1024) RE_TRY_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    int dev = 0, ncu = 0, per = 0;
    RE_TRY_HIP(hipGetDevice(&dev));
    RE_TRY_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    RE_TRY_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kBidiagThreads, lds));
    int64_t P = (int64_t)ncu * (per > 0 ? per : 0);
    if (P > kG2MaxP) P = kG2MaxP;
    if (P > l) P = l;
    if (P < 1) return RE_ERR_UNSUPPORTED;
    a.P = (int)P;
    void* params[] = {&a};
    RE_TRY(launch_grid(fn, dim3(a.P), dim3(kBidiagThreads), params, (unsigned)lds, s, svd_launch_override() == 2));
  } else {
    const size_t lds = (size_t)(2 * (k + 1) + kWaves * kPartChunk) * 8;
    if (lds > 160 * 1024) return RE_ERR_UNSUPPORTED;
    if (lds > 64 * 1024)
      RE_TRY_HIP(hipFuncSetAttribute((const void*)k_bidiag, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    void* params[] = {&a};
    RE_TRY(launch_grid((const void*)k_bidiag, dim3(a.P), dim3(kBidiagThreads), params, (unsigned)lds, s, svd_launch_override() == 2));
  }
  const size_t lds2 = (size_t)(4 * k) * 8;
  if (lds2 > 160 * 1024) return RE_ERR_UNSUPPORTED;
  if (one_bytes <= kLdsBudget && !multisect_small) {  // the batched form's per-lane bisection
    SvDesc one{};
    one.d = a.d;
    one.e = a.e;
    one.sigma = sigma;
    one.k = (int32_t)k;
    one.scale = scale;
    const int thr = k >= 256 ? 256 : (int)cdiv(k, 64) * 64;
    hipLaunchKernelGGL(k_sv_bisect, dim3(1), dim3(thr), lds2, s, (const SvDesc*)nullptr, one, 1, 1, thr, (int)k);
    RE_TRY_HIP(hipGetLastError());
    return RE_OK;
  }
  if (lds2 > 64 * 1024)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_bidiag_sv, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
  const int blocks = (int)cdiv(k, 2);  // two values per workgroup of four wavefronts
  hipLaunchKernelGGL(k_bidiag_sv, dim3(blocks), dim3(256), lds2, s, a.d, a.e, k, scale, info, sigma);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

size_t batched_svd_lds_bytes(int64_t lmax, int64_t kmax) { return small_lds_bytes(lmax, kmax); }

re_status launch_bidiag_batched(hipStream_t s, const double* const* C, double* const* d, double* const* e,
                                const int32_t* l, const int32_t* k, int32_t* info, int nblk, int64_t lmax,
                                int64_t kmax) {
  if (nblk <= 0) return RE_OK;
  const size_t bytes = small_lds_bytes(lmax, kmax);
  if (bytes > kLdsBudget) return RE_ERR_UNSUPPORTED;
  SmallBatch sb{};
  sb.C = C;
  sb.d = d;
  sb.e = e;
  sb.l = l;
  sb.k = k;
  sb.info = info;
  sb.kp = (int)lds_stride(kmax);
  if (const RowsKernel rk = rows_kernel(lmax, kmax); rk.fn) {
    void* args[] = {&sb};
    RE_TRY_HIP(hipLaunchKernel(rk.fn, dim3((unsigned)nblk), dim3(kBRThreads), args, rk.lds, s));
    return RE_OK;
  }
  if (bytes > 64 * 1024)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_bidiag_1wg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
  hipLaunchKernelGGL(k_bidiag_1wg, dim3((unsigned)nblk), dim3(kB2Threads), bytes, s, sb);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_sv_count_batched(hipStream_t s, const SvDesc* desc, int nblk, int64_t kmax) {
  if (nblk <= 0) return RE_OK;
  // problems per workgroup: as many as 256 lanes hold, one value per lane
  const int ppw = kmax <= 128 ? (int)(256 / kmax) : 1;
  const size_t lds2 = (size_t)ppw * (4 * kmax) * 8;
  if (lds2 > 160 * 1024) return RE_ERR_UNSUPPORTED;
  if (lds2 > 64 * 1024)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_sv_bisect, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
  const int thr = ppw > 1 ? (int)cdiv(ppw * kmax, 64) * 64 : kmax >= 256 ? 256 : (int)cdiv(kmax, 64) * 64;
  hipLaunchKernelGGL(k_sv_bisect, dim3((unsigned)cdiv(nblk, ppw)), dim3(thr), lds2, s, desc, SvDesc{}, nblk, ppw,
                     ppw > 1 ? (int)kmax : thr, (int)kmax);
  hipLaunchKernelGGL(k_count_batched, dim3((unsigned)nblk), dim3(256), 0, s, desc);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_rank_count(hipStream_t s, const double* sigma, int64_t k, int32_t r1, double eps, const int32_t* info,
                            int32_t* out3) {
  hipLaunchKernelGGL(k_count, dim3(1), dim3(256), 0, s, sigma, k, r1, eps, info, out3);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_gap(hipStream_t s, const double* sigma, int64_t k, int32_t r1, double gamma, double floor_rel,
                     const int32_t* info, GapOut* out) {
  hipLaunchKernelGGL(k_gap, dim3(1), dim3(256), 0, s, sigma, k, r1, gamma, floor_rel, info, out);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
