// Many independent sketches at once (the batched form of Algorithm 1): the
// FP32 Gaussian contraction B_b = A_b X[:n_b] for every block on the matrix
// cores in one persistent launch, then C_b = Y[:, :m_b] B_b, the small SVDs
// and the counts, one workgroup per block.  X (n_max x k) and Y (l x m_max)
// are master sketches: counter-indexed, so block b's leading rows / columns
// are exactly the sketch a single-matrix call with the same seed draws.
#include "common.h"
#include "batch.h"

namespace re {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

// Pointers read from descriptor tables are generic; the casts below let the
// compiler emit global (not flat) memory instructions for them, so that the
// LDS waits of the inner loops do not also wait for in-flight prefetches.
typedef const float __attribute__((address_space(1)))* gcfloat;
typedef float __attribute__((address_space(1)))* gfloat;
typedef double __attribute__((address_space(1)))* gdouble;


// Block of a work item: the last b with desc[b].item0 <= item.
__device__ __forceinline__ int find_block(const GemmDesc* __restrict__ desc, int nblk, int64_t item) {
  int lo = 0, hi = nblk - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].item0 <= item) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Persistent FP32 MFMA contraction.  A workgroup of WAVES wavefronts takes
// items from an atomic queue; an item is 32 MT WAVES rows of one block by up
// to 32 NT columns, swept along K in steps of kBK through double-buffered LDS
// tiles.  Every output is the same sequence of MFMA accumulations whatever
// WAVES, MT and kBK are, so the tile shape never changes the result.
// Wavefront w owns 32 MT rows and MT x NT 32x32 accumulator tiles
// (v_mfma_f32_32x32x2_f32: lane l holds row / column l % 32 and K index l / 32
// of the operands; accumulator q of lane l is row 8 (q/4) + 4 (l/32) + q%4,
// column l % 32).
template <int WAVES, int NT, int kBK, int MT>
__global__ void __launch_bounds__(64 * WAVES) k_gemm_f32_persistent(const GemmDesc* __restrict__ desc, int nblk,
                                                                    const float* __restrict__ X, int64_t k,
                                                                    int64_t total, unsigned* __restrict__ queue) {
  constexpr int BM = 32 * MT * WAVES, BN = 32 * NT, NTH = 64 * WAVES;
  constexpr int kApad = kBK + 1;  // LDS row pitch of the A tile (floats)
  __shared__ float sA[2][BM * kApad];
  __shared__ float sX[2][kBK * BN];
  __shared__ int64_t s_item;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (;;) {
    if (tid == 0) s_item = (int64_t)atomicAdd(queue, 1u);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= total) break;
    const int b = find_block(desc, nblk, item);
    const GemmDesc d = desc[b];
    const int64_t local = item - d.item0;
    const int64_t rt = local / d.ncc, cc = local - rt * d.ncc;
    const int64_t row0 = rt * BM, col0 = cc * BN;
    const int64_t m = d.m, n = d.n;
    const int rows_here = (int)(m - row0 < BM ? m - row0 : BM);
    // 32-bit offsets inside the item (the host keeps BM * lda below 2^31)
    const unsigned lda = (unsigned)d.lda;
    const gcfloat Ab = (gcfloat)(d.A + row0 * d.lda);

    // A: thread t loads PER consecutive K values of tile row ar
    constexpr int PER = BM * kBK / NTH;
    const int ar = (tid * PER) / kBK, ak = (tid * PER) % kBK;
    // X: thread t loads PX consecutive columns of tile row xr
    constexpr int PX = kBK * BN / NTH;
    const int xr = (tid * PX) / BN, xc = (tid * PX) % BN;
    const bool xcols_full = col0 + xc + PX <= k;
    float ra[PER];
    float rx[PX];
    auto load = [&](int64_t k0) {
      const gcfloat sa = Ab + ar * lda + (k0 + ak);
      if (ar < rows_here && k0 + ak + PER <= n) {
#pragma unroll
        for (int q = 0; q < PER; ++q) ra[q] = sa[q];
      } else {
#pragma unroll
        for (int q = 0; q < PER; ++q) ra[q] = (ar < rows_here && k0 + ak + q < n) ? sa[q] : 0.0f;
      }
      const float* __restrict__ sx = X + (k0 + xr) * k + (col0 + xc);
      if (k0 + xr < n && xcols_full) {
#pragma unroll
        for (int q = 0; q < PX; ++q) rx[q] = sx[q];
      } else {
#pragma unroll
        for (int q = 0; q < PX; ++q) rx[q] = (k0 + xr < n && col0 + xc + q < k) ? sx[q] : 0.0f;
      }
    };
    auto store = [&](int buf) {
#pragma unroll
      for (int q = 0; q < PER; ++q) sA[buf][ar * kApad + ak + q] = ra[q];
#pragma unroll
      for (int q = 0; q < PX; ++q) sX[buf][xr * BN + xc + q] = rx[q];
    };
    f32x16 acc[MT][NT];
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 16; ++q) acc[mi][t][q] = 0.0f;
    const int64_t nsteps = (n + kBK - 1) / kBK;
    load(0);
    store(0);
    __syncthreads();
    for (int64_t st = 0; st < nsteps; ++st) {
      const int buf = st & 1;
      if (st + 1 < nsteps) load((st + 1) * kBK);
#pragma unroll
      for (int kk = 0; kk < kBK; kk += 2) {
        float a[MT];
#pragma unroll
        for (int mi = 0; mi < MT; ++mi)
          a[mi] = sA[buf][(32 * (MT * wave + mi) + (lane & 31)) * kApad + kk + (lane >> 5)];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const float xb = sX[buf][(kk + (lane >> 5)) * BN + 32 * t + (lane & 31)];
#pragma unroll
          for (int mi = 0; mi < MT; ++mi)
            acc[mi][t] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[mi], xb, acc[mi][t], 0, 0, 0);
        }
      }
      if (st + 1 < nsteps) store(buf ^ 1);
      __syncthreads();
    }
    const gfloat Bo = (gfloat)d.B;
    const int64_t ldb = d.ldb;
#pragma unroll
    for (int mi = 0; mi < MT; ++mi)
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          const int64_t r = row0 + 32 * (MT * wave + mi) + 8 * (q >> 2) + 4 * (lane >> 5) + (q & 3);
          const int64_t c = col0 + 32 * t + (lane & 31);
          if (r < m && c < k) Bo[r * ldb + c] = acc[mi][t][q];
        }
  }
}

__global__ void k_zero_u32(unsigned* p) {
  if (threadIdx.x == 0) p[0] = 0u;
}

// Writes one descriptor passed by value (stream-ordered, so a host buffer is
// never read after the call returns).
template <typename D>
__global__ void k_put_desc(D v, D* out) {
  if (threadIdx.x == 0) *out = v;
}

// out[i * ld + j] = entry (r0 + i, c0 + j) of a Gaussian sketch in FP32:
// counter (r0 + i, c0 + j), or (c0 + j, r0 + i) when swap_ab (the Y layout).
// Appending rows or columns to a sketch draws exactly the entries a wider
// sketch would hold there.
__global__ void k_gauss_sub(int64_t rows, int64_t cols, int64_t r0, int64_t c0, uint64_t seed, uint64_t stream,
                            int swap_ab, int64_t ld, float* __restrict__ out) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e - i * cols;
    const double z = swap_ab ? gauss01(c0 + j, r0 + i, stream, seed) : gauss01(r0 + i, c0 + j, stream, seed);
    out[i * ld + j] = (float)z;
  }
}

// The same entries in FP64 (the draw is FP64 before any rounding).
__global__ void k_gauss_sub64(int64_t rows, int64_t cols, int64_t r0, int64_t c0, uint64_t seed, uint64_t stream,
                              int swap_ab, int64_t ld, double* __restrict__ out) {
  const int64_t total = rows * cols;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e - i * cols;
    out[i * ld + j] = swap_ab ? gauss01(c0 + j, r0 + i, stream, seed) : gauss01(r0 + i, c0 + j, stream, seed);
  }
}

// Master sketches of a batched call, seed read from the device header so the
// captured graph serves every seed: X[i][j] (n_max x k) from counter (i, j)
// of the X stream and Y[i][j] (l x m_max) from counter (j, i) of the Y
// stream, FP32, the same values the single-matrix draw produces.
__global__ void k_gauss_master(const BatchHeader* __restrict__ hdr, int64_t nmax, int64_t k, int64_t l, int64_t mmax,
                               float* __restrict__ X, float* __restrict__ Y) {
  const uint64_t seed = hdr->seed;
  const int64_t nx = nmax * k, total = nx + l * mmax;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    if (e < nx) {
      const int64_t i = e / k, j = e - i * k;
      X[e] = (float)gauss01(i, j, kXGauss, seed);
    } else {
      const int64_t f = e - nx, i = f / mmax, j = f - i * mmax;
      Y[f] = (float)gauss01(j, i, kYGauss, seed);
    }
  }
}

// C_b (l x k, FP64) = Y[:, :m_b] (FP32, leading dimension ldy) B_b (m_b x k,
// FP32) on the FP64 matrix cores (v_mfma_f64_16x16x4f64: lane q holds
// operand row / column q % 16 at K index q / 16; accumulator r of lane q is
// row q / 16 + 4 r, column q % 16, as measured on gfx950).  One workgroup per
// (block, slab of 48 WR rows of C) runs WR x WC wavefronts; wavefront (i, j)
// owns the 3 x 3 tiles of 16 x 16 at rows 48 i .. 48 i + 47 and columns
// 48 j .. 48 j + 47 of each pass of 48 WC columns.  Six wavefronts (WR = 3,
// WC = 2) at up to 168 VGPRs let two workgroups share a CU, three wavefronts
// on each SIMD.  K runs over m in chunks of 16 staged in LDS as FP64 (the
// FP32 products are exact in FP64).  The sum over m is a sum of groups of
// kYGroup chunks: each group is accumulated on the matrix cores from zero, in
// chunk order, and the group sums are added in group order.  A batch runs the
// groups of a block one after another; a single call with many groups gives
// each its own workgroup (gridDim.z = groups, partials to `parts`) and adds
// the partials in the same order, so both agree.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int kYKC = 16;    // K per chunk
constexpr int kYT = 3;      // 16 x 16 tiles per wavefront along rows and along columns
constexpr int kYApad = kYKC + 1;
constexpr int kYGroup = 32;  // chunks per group (512 rows of m)

template <int WR, int WC>
__global__ void __launch_bounds__(64 * WR * WC) __attribute__((amdgpu_waves_per_eu(WR * WC >= 4 ? 3 : 2))) k_ygemm_mfma(const YDesc* __restrict__ desc,
                                                             const float* __restrict__ Y, int64_t ldy, int64_t l,
                                                             int64_t k, double* __restrict__ parts) {
  constexpr int nth = 64 * WR * WC, rows = 16 * kYT * WR, cols = 16 * kYT * WC, bpad = cols + 4;
  constexpr int perY = rows * kYKC / nth, perB = kYKC * cols / nth;  // staged floats per thread
  static_assert(perY * nth == rows * kYKC && perB * nth == kYKC * cols, "exact staging");
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sY = reinterpret_cast<double*>(smem_raw);  // [2][rows][kYApad]
  double* sB = sY + 2 * rows * kYApad;                // [2][kYKC][bpad]
  const YDesc d = desc[blockIdx.y];
  const int64_t s0 = (int64_t)blockIdx.x * rows;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave / WC, wc = wave % WC;
  const int q16 = lane & 15, kq = lane >> 4;
  const int64_t m = d.m;
  const int64_t nchunks = (m + kYKC - 1) / kYKC;
  const bool split = gridDim.z > 1;  // one group per workgroup, partial to parts[blockIdx.z]
  const int64_t ch_begin = split ? (int64_t)blockIdx.z * kYGroup : 0;
  const int64_t ch_end = split ? (ch_begin + kYGroup < nchunks ? ch_begin + kYGroup : nchunks) : nchunks;
  double* __restrict__ out = split ? parts + (int64_t)blockIdx.z * l * k : d.C;
  // register staging: the next chunk's loads are in flight while the
  // matrix cores work on the current one.  Element e = tid + q nth of the Y
  // tile is row e / 16, K index e % 16 = tid % 16.
  const int yc = tid % kYKC, yr0 = tid / kYKC;
  for (int64_t c0 = 0; c0 < k; c0 += cols) {
    float ry[perY], rb[perB];
    const unsigned ldb = (unsigned)d.ldb;  // 16 rows of B per chunk: 32-bit offsets
    auto load = [&](int64_t i0) {
      const bool col_ok = i0 + yc < m;
#pragma unroll
      for (int q = 0; q < perY; ++q) {
        const int64_t gr = s0 + yr0 + q * (nth / kYKC);
        ry[q] = (col_ok && gr < l) ? Y[gr * ldy + i0 + yc] : 0.0f;
      }
      const gcfloat bch = (gcfloat)(d.B + i0 * d.ldb + c0);
#pragma unroll
      for (int q = 0; q < perB; ++q) {
        const int e = tid + q * nth, r = e / cols, c = e % cols;
        rb[q] = (i0 + r < m && c0 + c < k) ? bch[r * ldb + c] : 0.0f;
      }
    };
    auto store = [&](int buf) {
      double* y = sY + buf * rows * kYApad;
#pragma unroll
      for (int q = 0; q < perY; ++q) y[(yr0 + q * (nth / kYKC)) * kYApad + yc] = (double)ry[q];
      double* bb = sB + buf * kYKC * bpad;
#pragma unroll
      for (int q = 0; q < perB; ++q) {
        const int e = tid + q * nth;
        bb[(e / cols) * bpad + e % cols] = (double)rb[q];
      }
    };
    f64x4 acc[kYT][kYT];
#pragma unroll
    for (int i = 0; i < kYT; ++i)
#pragma unroll
      for (int j = 0; j < kYT; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
    // writes the accumulators to the thread's outputs (or adds them) and
    // clears them.  The row and column of output (i, j, r) are formed from
    // two values made opaque to the optimiser, so that the output addresses
    // are not held across the chunk loop.
    auto put = [&](bool overwrite) {
      int rs = 16 * kYT * wr + kq, cs = 16 * kYT * wc + q16;
      asm volatile("" : "+v"(rs), "+v"(cs));
      const int64_t gs0 = s0 + rs, gc0 = c0 + cs;
      const gdouble obase = (gdouble)out + (gs0 * k + gc0);
#pragma unroll
      for (int i = 0; i < kYT; ++i)
#pragma unroll
        for (int j = 0; j < kYT; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (gs0 + 16 * i + 4 * r < l && gc0 + 16 * j < k) {
              const gdouble o = obase + ((16 * i + 4 * r) * k + 16 * j);
              *o = overwrite ? acc[i][j][r] : *o + acc[i][j][r];
            }
          }
          acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
        }
    };
    bool first = true;
    load(ch_begin * kYKC);
    store(0);
    __syncthreads();
    for (int64_t ch = ch_begin; ch < ch_end; ++ch) {
      const int buf = (ch - ch_begin) & 1;
      if (ch + 1 < ch_end) load((ch + 1) * kYKC);
      const double* y = sY + buf * rows * kYApad + (16 * kYT * wr + q16) * kYApad;
      const double* bb = sB + buf * kYKC * bpad + 16 * kYT * wc + q16;
#pragma unroll 1
      for (int kk = 0; kk < kYKC; kk += 4) {
        double av[kYT], bv[kYT];
#pragma unroll
        for (int i = 0; i < kYT; ++i) av[i] = y[16 * i * kYApad + kk + kq];
#pragma unroll
        for (int j = 0; j < kYT; ++j) bv[j] = bb[(kk + kq) * bpad + 16 * j];
#pragma unroll
        for (int i = 0; i < kYT; ++i)
#pragma unroll
          for (int j = 0; j < kYT; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
      if ((ch + 1) % kYGroup == 0 || ch + 1 == ch_end) {
        // a group ends: its sum goes to the thread's own outputs (first
        // group) or is added to them
        put(first);
        first = false;
      }
      if (ch + 1 < ch_end) store(buf ^ 1);
      __syncthreads();
    }
    if (first) put(true);  // m = 0: the zero accumulators
    __syncthreads();
  }
}

// C = sum of the groups' partial products in group order (the order a batch
// adds them in), for a single call split over m.
__global__ void k_ygemm_reduce(const double* __restrict__ parts, int64_t ngroups, int64_t lk, double* __restrict__ C) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < lk; e += (int64_t)gridDim.x * blockDim.x) {
    double t = parts[e];
    for (int64_t g = 1; g < ngroups; ++g) t += parts[g * lk + e];
    C[e] = t;
  }
}

}  // namespace

re_status launch_gemm_f32_persistent(hipStream_t s, const GemmDesc* desc, int nblk, const float* X, int64_t k,
                                     int64_t total, unsigned* queue, int waves, int grid, int bk, int mt) {
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, queue);
  const int nt = (int)(k >= 128 ? 4 : cdiv(k, 32));
#define RE_GEMM_CASE(W, N, BK, MT)                                                                              \
  if (waves == W && nt == N && bk == BK && mt == MT) {                                                          \
    hipLaunchKernelGGL((k_gemm_f32_persistent<W, N, BK, MT>), dim3(grid), dim3(64 * W), 0, s, desc, nblk, X, k, \
                       total, queue);                                                                           \
    RE_TRY_HIP(hipGetLastError());                                                                              \
    return RE_OK;                                                                                               \
  }
#define RE_GEMM_CASES(BK, MT)                                                                           \
  RE_GEMM_CASE(4, 1, BK, MT) RE_GEMM_CASE(4, 2, BK, MT) RE_GEMM_CASE(4, 3, BK, MT) RE_GEMM_CASE(4, 4, BK, MT) \
  RE_GEMM_CASE(8, 1, BK, MT) RE_GEMM_CASE(8, 2, BK, MT) RE_GEMM_CASE(8, 3, BK, MT) RE_GEMM_CASE(8, 4, BK, MT)
  RE_GEMM_CASES(16, 1)
  RE_GEMM_CASES(32, 1)
  RE_GEMM_CASES(16, 2)
#undef RE_GEMM_CASES
#undef RE_GEMM_CASE
  return RE_ERR_INVALID_ARG;
}

re_status launch_gemm_f32_single(hipStream_t s, const float* A, int64_t m, int64_t n, int64_t lda, const float* X,
                                 int64_t k, float* B, int64_t ldb, GemmDesc* dscratch, unsigned* queue) {
  GemmDesc d;
  d.A = A;
  d.B = B;
  d.m = m;
  d.n = n;
  d.lda = lda;
  d.ldb = ldb;
  d.item0 = 0;
  d.ncc = gemm_col_chunks(k);
  hipLaunchKernelGGL(k_put_desc<GemmDesc>, dim3(1), dim3(64), 0, s, d, dscratch);
  const int64_t total = gemm_items(m, k, 32 * 4);
  const int64_t g = total < 2048 ? total : 2048;
  return launch_gemm_f32_persistent(s, dscratch, 1, X, k, total, queue, 4, (int)g, 32, 1);
}

int64_t ygemm_groups(int64_t m) { return cdiv(cdiv(m, kYKC), kYGroup); }

// a split launch puts the groups on grid dimension z (at most 65535); it is
// taken only while its partial products (groups x l x k doubles) take no more
// memory than B itself (m x k floats), i.e. for l up to about 256: wider Y
// would make the scratch several times B.  The unsplit launch adds the groups
// in the same order in one workgroup and gives the same bits.
bool ygemm_splits(int64_t l, int64_t k, int64_t m) {
  const int64_t g = ygemm_groups(m);
  return g > 1 && g <= 65535 && (double)g * l * k * sizeof(double) <= (double)m * k * sizeof(float);
}

size_t ygemm_split_bytes(int64_t l, int64_t k, int64_t m) {
  return ygemm_splits(l, k, m) ? (size_t)ygemm_groups(m) * l * k * sizeof(double) : 0;
}

re_status launch_ygemm_single(hipStream_t s, const float* B, int64_t m, int64_t k, int64_t ldb, const float* Y,
                              int64_t ldy, int64_t l, double* C, YDesc* dscratch, double* parts) {
  YDesc d;
  d.B = B;
  d.C = C;
  d.m = m;
  d.ldb = ldb;
  hipLaunchKernelGGL(k_put_desc<YDesc>, dim3(1), dim3(64), 0, s, d, dscratch);
  const int64_t g = ygemm_groups(m);
  if (!ygemm_splits(l, k, m) || parts == nullptr) return launch_ygemm_batched(s, dscratch, 1, Y, ldy, l, k);
  RE_TRY(launch_ygemm_grid(s, dscratch, 1, Y, ldy, l, k, (unsigned)g, parts));
  const int64_t lk = l * k;
  hipLaunchKernelGGL(k_ygemm_reduce, dim3((unsigned)(cdiv(lk, 256) < 2048 ? cdiv(lk, 256) : 2048)), dim3(256), 0, s,
                     (const double*)parts, g, lk, C);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_gauss_sub(hipStream_t s, int64_t rows, int64_t cols, int64_t r0, int64_t c0, uint64_t seed,
                           int stream_id, int swap_ab, int64_t ld, float* out) {
  const int64_t total = rows * cols;
  if (total <= 0) return RE_OK;
  const int64_t g = cdiv(total, 256) < 8192 ? cdiv(total, 256) : 8192;
  hipLaunchKernelGGL(k_gauss_sub, dim3((unsigned)g), dim3(256), 0, s, rows, cols, r0, c0, seed, (uint64_t)stream_id,
                     swap_ab, ld, out);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_gauss_sub64(hipStream_t s, int64_t rows, int64_t cols, int64_t r0, int64_t c0, uint64_t seed,
                             int stream_id, int swap_ab, int64_t ld, double* out) {
  const int64_t total = rows * cols;
  if (total <= 0) return RE_OK;
  const int64_t g = cdiv(total, 256) < 8192 ? cdiv(total, 256) : 8192;
  hipLaunchKernelGGL(k_gauss_sub64, dim3((unsigned)g), dim3(256), 0, s, rows, cols, r0, c0, seed, (uint64_t)stream_id,
                     swap_ab, ld, out);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

re_status launch_gauss_master(hipStream_t s, const BatchHeader* hdr, int64_t nmax, int64_t k, int64_t l, int64_t mmax,
                              float* X, float* Y) {
  const int64_t total = nmax * k + l * mmax;
  if (total <= 0) return RE_OK;
  const int64_t g = cdiv(total, 256) < 4096 ? cdiv(total, 256) : 4096;
  hipLaunchKernelGGL(k_gauss_master, dim3((unsigned)g), dim3(256), 0, s, hdr, nmax, k, l, mmax, X, Y);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

int64_t gemm_items(int64_t m, int64_t k, int rows_per_item) {
  const int64_t bm = rows_per_item, bn = k >= 128 ? 128 : 32 * cdiv(k, 32);
  return cdiv(m, bm) * cdiv(k, bn);
}

int gemm_col_chunks(int64_t k) { return (int)cdiv(k, k >= 128 ? 128 : 32 * cdiv(k, 32)); }

re_status launch_ygemm_batched(hipStream_t s, const YDesc* desc, int nblk, const float* Y, int64_t ldy, int64_t l,
                               int64_t k) {
  return launch_ygemm_grid(s, desc, nblk, Y, ldy, l, k, 1, nullptr);
}

template <int WR, int WC>
re_status launch_ygemm_shape(hipStream_t s, const YDesc* desc, int nblk, const float* Y, int64_t ldy, int64_t l,
                             int64_t k, unsigned groups, double* parts) {
  constexpr int rows = 16 * kYT * WR, cols = 16 * kYT * WC;
  const size_t lds = (size_t)(2 * rows * kYApad + 2 * kYKC * (cols + 4)) * sizeof(double);
  if (lds > 64 * 1024)
    RE_TRY_HIP(hipFuncSetAttribute((const void*)k_ygemm_mfma<WR, WC>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds));
  hipLaunchKernelGGL((k_ygemm_mfma<WR, WC>), dim3((unsigned)cdiv(l, rows), (unsigned)nblk, groups),
                     dim3(64 * WR * WC), lds, s, desc, Y, ldy, l, k, parts);
  RE_TRY_HIP(hipGetLastError());
  return RE_OK;
}

// Slabs of 48, 96 or 144 rows (the fewest that cover l, at most three
// wavefront rows) and passes of 48 or 96 columns.
re_status launch_ygemm_grid(hipStream_t s, const YDesc* desc, int nblk, const float* Y, int64_t ldy, int64_t l,
                            int64_t k, unsigned groups, double* parts) {
  if (nblk <= 0 || l <= 0 || k <= 0) return RE_OK;
  const int wr = (int)(cdiv(l, 16 * kYT) < 3 ? cdiv(l, 16 * kYT) : 3);
  const bool wide = k > 16 * kYT;
  switch (wr * 2 + (wide ? 1 : 0)) {
    case 2: return launch_ygemm_shape<1, 1>(s, desc, nblk, Y, ldy, l, k, groups, parts);
    case 3: return launch_ygemm_shape<1, 2>(s, desc, nblk, Y, ldy, l, k, groups, parts);
    case 4: return launch_ygemm_shape<2, 1>(s, desc, nblk, Y, ldy, l, k, groups, parts);
    case 5: return launch_ygemm_shape<2, 2>(s, desc, nblk, Y, ldy, l, k, groups, parts);
    case 6: return launch_ygemm_shape<3, 1>(s, desc, nblk, Y, ldy, l, k, groups, parts);
    default: return launch_ygemm_shape<3, 2>(s, desc, nblk, Y, ldy, l, k, groups, parts);
  }
}

}  // namespace re
