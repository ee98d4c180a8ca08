// Materialisation of the random embeddings of Algorithm 1 (steps 2 and 5):
// Gaussian entries, Rademacher signs and the uniform row sampler of an SRHT.
#include "common.h"

namespace re {

namespace {

constexpr int kSelCap = 4096;      // candidate capacity of the fast selection path
constexpr int kSelThreads = 1024;  // one workgroup finishes a selection

__global__ void k_philox(const uint64_t* __restrict__ ctr, uint64_t seed, int64_t count, uint64_t* __restrict__ out) {
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < count; t += (int64_t)gridDim.x * blockDim.x) {
    const u64x4 w = philox(ctr[4 * t], ctr[4 * t + 1], ctr[4 * t + 2], ctr[4 * t + 3], seed);
    out[4 * t] = w.x;
    out[4 * t + 1] = w.y;
    out[4 * t + 2] = w.z;
    out[4 * t + 3] = w.w;
  }
}

template <typename T>
__device__ __forceinline__ void store_fmt(T* p, double v);
template <>
__device__ __forceinline__ void store_fmt<double>(double* p, double v) { *p = v; }
template <>
__device__ __forceinline__ void store_fmt<float>(float* p, double v) { *p = (float)v; }
template <>
__device__ __forceinline__ void store_fmt<__bf16>(__bf16* p, double v) { *p = (__bf16)(float)v; }
template <>
__device__ __forceinline__ void store_fmt<_Float16>(_Float16* p, double v) { *p = (_Float16)(float)v; }

// The value is rounded once from FP64 to the target format by round_fmt; the
// conversions in store_fmt are then exact.
template <typename T>
__global__ void k_gauss_fill(int fmt, int64_t rows, int64_t cols, uint64_t seed, uint64_t stream, int swap_ab,
                             T* __restrict__ out) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e - i * cols;
    const double z = swap_ab ? gauss01(j, i, stream, seed) : gauss01(i, j, stream, seed);
    store_fmt<T>(out + e, round_fmt(z, fmt));
  }
}

__global__ void k_sign_bits(int64_t npad, uint64_t seed, uint64_t stream, uint32_t* __restrict__ bits) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int neg = (i < npad) ? (int)(philox((uint64_t)i, 0, stream, 0, seed).x & 1u) : 0;
  const uint64_t mask = __ballot(neg);
  if ((threadIdx.x & 63) == 0) {
    const int64_t w0 = i >> 5;
    const int64_t nwords = (npad + 31) >> 5;
    if (w0 < nwords) bits[w0] = (uint32_t)mask;
    if (w0 + 1 < nwords) bits[w0 + 1] = (uint32_t)(mask >> 32);
  }
}

__global__ void k_zero_i32(int32_t* p, int n) {
  if (threadIdx.x < n) p[threadIdx.x] = 0;
}

// Selection, phase 1: every key, plus candidates below a threshold T chosen so
// that, for iid uniform keys, at least k fall below it with overwhelming
// probability.  Phase 2 checks the count and falls back to an exact search.
__global__ void k_sel_keys(int64_t npad, uint64_t seed, uint64_t stream, uint64_t thresh, uint64_t* __restrict__ keys,
                           ulonglong2* __restrict__ cand, int32_t* __restrict__ cnt) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < npad; i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = philox((uint64_t)i, 0, stream, 0, seed).x;
    keys[i] = key;
    if (key < thresh) {
      const int pos = atomicAdd(cnt, 1);
      if (pos < kSelCap) cand[pos] = make_ulonglong2(key, (uint64_t)i);
    }
  }
}

__device__ __forceinline__ bool key_less(uint64_t ka, uint32_t ia, uint64_t kb, uint32_t ib) {
  return ka < kb || (ka == kb && ia < ib);
}

// Exclusive prefix sum over the workgroup of one value per thread.
__device__ int block_exclusive_scan(int v, int* buf, int* total) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {
    const int add = (t >= off) ? buf[t - off] : 0;
    __syncthreads();
    buf[t] += add;
    __syncthreads();
  }
  const int incl = buf[t];
  const int tot = buf[blockDim.x - 1];
  __syncthreads();
  if (total) *total = tot;
  return incl - v;
}

// Exclusive prefix sum over the workgroup of one value per thread, by
// wavefront shuffles and one pass over the wavefront totals.
__device__ int block_exclusive_scan_fast(int v, int* wsum) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  int before = 0;
  for (int w = 0; w < wave; ++w) before += wsum[w];
  (void)nw;
  __syncthreads();
  return before + x - v;
}

__global__ void __launch_bounds__(kSelThreads) k_sel_finish(int64_t npad, int64_t k, uint64_t thresh,
                                                            const uint64_t* __restrict__ keys,
                                                            const ulonglong2* __restrict__ cand,
                                                            const int32_t* __restrict__ cnt, int32_t* __restrict__ out) {
  constexpr int NB = kSelThreads;           // buckets, one per thread
  constexpr int PER = kSelCap / kSelThreads;  // candidates per thread
  __shared__ int hcnt[NB], bstart[NB], bfill[NB];
  __shared__ int slot[kSelCap];
  __shared__ int wsum[kSelThreads / 64];
  __shared__ int scan_buf[kSelThreads];
  __shared__ unsigned hist[256];
  __shared__ uint64_t s_prefix;
  __shared__ int64_t s_rank;
  const int c = *cnt;
  const int t = threadIdx.x;
  if (c >= k && c <= kSelCap) {
    // Fast path: the k smallest (key, index) pairs among the c candidates,
    // written in ascending index order.  Ranks come from a counting sort over
    // monotone buckets (the top bits of the key below thresh, then of the
    // index) followed by comparisons within each bucket.
    int sh = 0;
    while (((thresh - 1) >> sh) >= (uint64_t)NB) ++sh;
    int shi = 0;
    while ((uint64_t)((npad - 1) >> shi) >= (uint64_t)NB) ++shi;
    uint64_t key[PER];
    uint32_t idx[PER];
    int bk[PER];
    hcnt[t] = 0;
    bfill[t] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = t + u * kSelThreads;
      key[u] = 0;
      idx[u] = 0;
      bk[u] = 0;
      if (i < c) {
        const ulonglong2 e = cand[i];
        key[u] = e.x;
        idx[u] = (uint32_t)e.y;
        bk[u] = (int)(e.x >> sh);
        atomicAdd(&hcnt[bk[u]], 1);
      }
    }
    __syncthreads();
    bstart[t] = block_exclusive_scan_fast(hcnt[t], wsum);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = t + u * kSelThreads;
      if (i < c) slot[bstart[bk[u]] + atomicAdd(&bfill[bk[u]], 1)] = i;
    }
    __syncthreads();
    bool keep[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = t + u * kSelThreads;
      keep[u] = false;
      if (i < c) {
        int rank = bstart[bk[u]];
        const int p1 = bstart[bk[u]] + hcnt[bk[u]];
        for (int p = bstart[bk[u]]; p < p1; ++p) {
          const int j = slot[p];
          if (j == i) continue;
          const ulonglong2 o = cand[j];
          rank += key_less(o.x, (uint32_t)o.y, key[u], idx[u]);
        }
        keep[u] = rank < k;
      }
    }
    __syncthreads();
    // the kept indices in ascending order: the same counting sort over index buckets
    hcnt[t] = 0;
    bfill[t] = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      bk[u] = (int)(idx[u] >> shi);
      if (keep[u]) atomicAdd(&hcnt[bk[u]], 1);
    }
    __syncthreads();
    bstart[t] = block_exclusive_scan_fast(hcnt[t], wsum);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (keep[u]) slot[bstart[bk[u]] + atomicAdd(&bfill[bk[u]], 1)] = (int)idx[u];
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      if (!keep[u]) continue;
      int pos = bstart[bk[u]];
      const int p1 = bstart[bk[u]] + hcnt[bk[u]];
      for (int p = bstart[bk[u]]; p < p1; ++p) pos += ((uint32_t)slot[p] < idx[u]);
      out[pos] = (int32_t)idx[u];
    }
    return;
  }
  // Exact path: most-significant-digit radix selection of the k-th smallest
  // key (8 passes of 8 bits), then an index-ordered compaction.
  if (threadIdx.x == 0) {
    s_prefix = 0;
    s_rank = k;  // 1-based rank still to locate among keys matching the prefix
  }
  uint64_t mask = 0;
  for (int shift = 56; shift >= 0; shift -= 8) {
    for (int b = threadIdx.x; b < 256; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    const uint64_t prefix = s_prefix;
    for (int64_t i = threadIdx.x; i < npad; i += blockDim.x) {
      const uint64_t key = keys[i];
      if ((key & mask) == prefix) atomicAdd(&hist[(key >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int64_t rank = s_rank;
      int d = 0;
      for (; d < 256; ++d) {
        if (rank <= (int64_t)hist[d]) break;
        rank -= hist[d];
      }
      s_prefix = prefix | ((uint64_t)d << shift);
      s_rank = rank;
    }
    mask |= (uint64_t)255u << shift;
    __syncthreads();
  }
  const uint64_t kth = s_prefix;
  const int64_t take_eq = s_rank;  // how many keys equal to kth are selected (lowest indices first)
  const int64_t chunk = (npad + blockDim.x - 1) / blockDim.x;
  const int64_t c0 = min((int64_t)threadIdx.x * chunk, npad), c1 = min(c0 + chunk, npad);
  int eq = 0;
  for (int64_t i = c0; i < c1; ++i) eq += (keys[i] == kth);
  int eq_before = block_exclusive_scan(eq, scan_buf, nullptr);
  int sel = 0;
  {
    int e = eq_before;
    for (int64_t i = c0; i < c1; ++i) {
      const uint64_t key = keys[i];
      if (key < kth) ++sel;
      else if (key == kth) { sel += (e < take_eq); ++e; }
    }
  }
  int pos = block_exclusive_scan(sel, scan_buf, nullptr);
  {
    int e = eq_before;
    for (int64_t i = c0; i < c1; ++i) {
      const uint64_t key = keys[i];
      bool take = false;
      if (key < kth) take = true;
      else if (key == kth) { take = (e < take_eq); ++e; }
      if (take) out[pos++] = (int32_t)i;
    }
  }
}

int grid_for(int64_t work, int threads, int cap = 65536) {
  int64_t g = (work + threads - 1) / threads;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

re_status launch_philox(hipStream_t s, const uint64_t* ctr, uint64_t seed, int64_t count, uint64_t* out) {
  if (count <= 0) return RE_OK;
  hipLaunchKernelGGL(k_philox, dim3(grid_for(count, 256)), dim3(256), 0, s, ctr, seed, count, out);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_gauss_fill(hipStream_t s, int fmt, int64_t rows, int64_t cols, uint64_t seed, int stream_id,
                            int swap_ab, void* out) {
  const int64_t total = rows * cols;
  if (total <= 0) return RE_OK;
  const dim3 g(grid_for(total, 256)), b(256);
  switch (fmt) {
    case kF64: hipLaunchKernelGGL(k_gauss_fill<double>, g, b, 0, s, fmt, rows, cols, seed, (uint64_t)stream_id, swap_ab, (double*)out); break;
    case kF32: hipLaunchKernelGGL(k_gauss_fill<float>, g, b, 0, s, fmt, rows, cols, seed, (uint64_t)stream_id, swap_ab, (float*)out); break;
    case kBF16: hipLaunchKernelGGL(k_gauss_fill<__bf16>, g, b, 0, s, fmt, rows, cols, seed, (uint64_t)stream_id, swap_ab, (__bf16*)out); break;
    case kF16: hipLaunchKernelGGL(k_gauss_fill<_Float16>, g, b, 0, s, fmt, rows, cols, seed, (uint64_t)stream_id, swap_ab, (_Float16*)out); break;
    default: return RE_ERR_INVALID_ARG;
  }
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_sign_bits(hipStream_t s, int64_t npad, uint64_t seed, int stream_id, uint32_t* bits) {
  if (npad <= 0) return RE_OK;
  const int64_t padded = (npad + 63) / 64 * 64;
  hipLaunchKernelGGL(k_sign_bits, dim3((unsigned)cdiv(padded, 256)), dim3(256), 0, s, npad, seed, (uint64_t)stream_id, bits);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

size_t select_scratch_bytes(int64_t npad) {
  return (size_t)npad * 8 + (size_t)kSelCap * 16 + 256;
}

re_status launch_select(hipStream_t s, int64_t npad, int64_t k, uint64_t seed, int stream_id, void* scratch,
                        int32_t* idx) {
  if (k <= 0) return RE_OK;
  if (k > npad || npad > (int64_t)INT32_MAX) return RE_ERR_INVALID_ARG;
  uint64_t* keys = (uint64_t*)scratch;
  ulonglong2* cand = (ulonglong2*)((char*)scratch + (size_t)npad * 8);
  int32_t* cnt = (int32_t*)((char*)cand + (size_t)kSelCap * 16);
  // Expected count below T is mu = k + 6 sqrt(k) + 16: short of k with
  // probability ~1e-9, then handled by the exact path.
  const double mu = (double)k + 6.0 * sqrt((double)k) + 16.0;
  const double frac = mu / (double)npad;
  const uint64_t thresh = frac >= 1.0 ? ~0ull : (uint64_t)(frac * 18446744073709551616.0);
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, cnt, 1);
  hipLaunchKernelGGL(k_sel_keys, dim3(grid_for(npad, 256, 1024)), dim3(256), 0, s, npad, seed, (uint64_t)stream_id,
                     thresh, keys, cand, cnt);
  hipLaunchKernelGGL(k_sel_finish, dim3(1), dim3(kSelThreads), 0, s, npad, k, thresh, keys, cand, cnt, idx);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

}  // namespace re
