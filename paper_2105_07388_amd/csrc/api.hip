// C ABI of librankest: handle, workspace and the entry points of rankest.h.
#include <math.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <map>
#include <atomic>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "batch.h"
#include "common.h"
#include "hrtt.h"
#include "learned.h"
#include "rangefinder.h"
#include "srct_y.h"

#define RE_API extern "C" __attribute__((visibility("default")))

struct re_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* host = nullptr;  // pinned staging for device-to-host results
  size_t host_bytes = 0;
  bool prof = false;     // record stage events inside re_rank_estimate
  hipEvent_t ev[RE_NUM_STAGES + 1] = {};
  double stage_ms[RE_NUM_STAGES] = {};
  // batched form: captured graph and autotuned tile shapes
  hipStream_t cap = nullptr;
  hipGraphExec_t bexec = nullptr;
  std::string bkey;
  struct Tile {
    int waves, mt, bk, grid;  // wavefronts, 32-row tiles per wavefront, K step, resident workgroups
  };
  std::map<std::string, Tile> tuned;  // shape key -> persistent contraction tile
  // rangefinder: QR and Q^T A workspace (sized once the width is known) and stage times
  void* ws2 = nullptr;
  size_t ws2_bytes = 0;
  double rf_ms[3] = {};
  // re_set_limits: cap on each workspace (0: none) and the small SVD's barrier polls (0: default)
  size_t ws_cap = 0;
  long spin_limit = 0;
  bool relaunched = false;  // the last estimate's small SVD was run again cooperatively
  int xcd = 7;  // XCD of the multi-workgroup small SVD: handles created in turn take XCDs 7, 6, ..., 0 in turn
};

namespace re {
namespace {

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

re_status ensure_ws(re_handle h, size_t bytes) {
  if (bytes <= h->ws_bytes) return RE_OK;
  if (h->ws_cap && bytes > h->ws_cap) return RE_ERR_NO_MEMORY;
  RE_TRY_HIP(hipStreamSynchronize(h->stream));
  if (h->ws) (void)hipFree(h->ws);
  h->ws = nullptr;
  h->ws_bytes = 0;
  const size_t want = al256(bytes + bytes / 8);
  if (hipMalloc(&h->ws, want) != hipSuccess) {
    (void)hipGetLastError();
    h->ws = nullptr;
    return RE_ERR_NO_MEMORY;
  }
  h->ws_bytes = want;
  return RE_OK;
}

re_status ensure_ws2(re_handle h, size_t bytes) {
  if (bytes <= h->ws2_bytes) return RE_OK;
  if (h->ws_cap && bytes > h->ws_cap) return RE_ERR_NO_MEMORY;
  RE_TRY_HIP(hipStreamSynchronize(h->stream));
  if (h->ws2) (void)hipFree(h->ws2);
  h->ws2 = nullptr;
  h->ws2_bytes = 0;
  const size_t want = al256(bytes + bytes / 8);
  if (hipMalloc(&h->ws2, want) != hipSuccess) {
    (void)hipGetLastError();
    h->ws2 = nullptr;
    return RE_ERR_NO_MEMORY;
  }
  h->ws2_bytes = want;
  return RE_OK;
}

re_status ensure_host(re_handle h, size_t bytes) {
  if (bytes <= h->host_bytes) return RE_OK;
  if (h->ws_cap && bytes > h->ws_cap) return RE_ERR_NO_MEMORY;
  RE_TRY_HIP(hipStreamSynchronize(h->stream));
  if (h->host) (void)hipHostFree(h->host);
  h->host = nullptr;
  h->host_bytes = 0;
  if (hipHostMalloc(&h->host, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    h->host = nullptr;
    return RE_ERR_NO_MEMORY;
  }
  h->host_bytes = bytes;
  return RE_OK;
}

// Bump allocator over one workspace region.
struct Carve {
  size_t off = 0;
  size_t take(size_t bytes) {
    const size_t o = off;
    off += al256(bytes);
    return o;
  }
};

int32_t r1_from_k(int32_t k) {
  int32_t r1 = 0;
  for (int32_t r = 1; r <= k; ++r)
    if ((11 * r + 5) / 10 <= k) r1 = r;
  return r1;
}

int elem_size(int fmt) { return fmt == kF64 ? 8 : fmt == kF32 ? 4 : 2; }

// Sketch entry formats: the contraction runs in the storage type of A.
int x_fmt(int32_t dt) { return dt == RE_F64 ? kF64 : kF32; }

struct Resolved {
  int32_t xk, yk;
  int64_t k, l, npad_n, npad_m;
  int fmt_x = -1;     // contraction format of a Gaussian X (kF64, kF32, kBF16, kF16)
  int scale_exp = 0;  // FP16: A is scaled by 2^scale_exp before rounding
  bool lowprec = false;  // a BF16 / FP16 contraction may run (its X tiles need room)
};

// Checks the arguments of one estimate; `sides` selects which embedding's
// sizes are checked (1: X, 2: Y, 3: both).
re_status validate(const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda, const re_sketch* sk, Resolved* rs,
                   int sides = 3) {
  if (!A || !sk) return RE_ERR_INVALID_ARG;
  if (dt != RE_F64 && dt != RE_F32) return RE_ERR_INVALID_ARG;
  if (m < 1 || n < 1 || lda < n) return RE_ERR_INVALID_ARG;
  if (((uintptr_t)A) % (dt == RE_F64 ? 8 : 4) != 0) return RE_ERR_INVALID_ARG;
  if ((sk->x_kind != RE_GAUSSIAN && sk->x_kind != RE_SRHT && sk->x_kind != RE_HRTT && sk->x_kind != RE_SRCT) ||
      (sk->y_kind != RE_GAUSSIAN && sk->y_kind != RE_SRHT && sk->y_kind != RE_SRCT))
    return RE_ERR_INVALID_ARG;
  if (sk->prec < RE_PREC_NATIVE || sk->prec > RE_PREC_AUTO) return RE_ERR_INVALID_ARG;
  rs->xk = sk->x_kind;
  rs->yk = sk->y_kind;
  rs->k = sk->k;
  rs->l = sk->l == 0 ? 2 * (int64_t)sk->k : sk->l;
  rs->npad_n = next_pow2(n);
  rs->npad_m = next_pow2(m);
  const bool dct = rs->xk == RE_HRTT || rs->xk == RE_SRCT;
  const int64_t kmax = rs->xk == RE_SRHT ? rs->npad_n : dct ? hrtt_npad(n) : n;
  const int64_t lmax = rs->yk == RE_SRHT ? rs->npad_m : rs->yk == RE_SRCT ? srct_y_npad(m) : m;
  if (rs->k < 1 || rs->l < rs->k) return RE_ERR_INVALID_ARG;
  if ((sides & 1) && rs->k > kmax) return RE_ERR_INVALID_ARG;
  if ((sides & 2) && rs->l > lmax) return RE_ERR_INVALID_ARG;
  if (rs->k > (int64_t)INT32_MAX / 2) return RE_ERR_INVALID_ARG;
  if (sk->prec != RE_PREC_NATIVE && (dt == RE_F64 || rs->xk != RE_GAUSSIAN)) return RE_ERR_UNSUPPORTED;
  if (dct && (dt != RE_F32 || !dct_x_supported(n, rs->k, rs->xk == RE_HRTT))) return RE_ERR_UNSUPPORTED;
  return RE_OK;
}

// Workspace plan of one estimate.
struct Plan {
  size_t xbits, ybits, xsel, ysel, selscr, X, Y, B, C, svd, sigma, info, out3, stats, gdesc, ydesc, queue, yparts,
      rdiag, hscr, gparts, U, yord, dctws, total;
};

// Sketches the batched form accepts (one workgroup's LDS holds the small SVD).
bool batched_fits(int64_t l, int64_t k) { return k <= 4096 && batched_svd_lds_bytes(l, k) <= 156 * 1024; }

// C = Y B for FP32 B and Y: the batched form's kernel for every sketch the
// batched form accepts (a block of a batch and the same matrix alone then give
// the same bits), the tiled product with a split over m for wider ones.
size_t yb_scratch(int64_t l, int64_t k, int64_t m) {
  return batched_fits(l, k) ? ygemm_split_bytes(l, k, m) : yb_parts_bytes(l, k, m);
}

re_status run_yb(hipStream_t s, const float* B, int64_t m, int64_t k, int64_t ldb, const float* Y, int64_t ldy,
                 int64_t l, double* C, YDesc* yd, void* parts) {
  if (batched_fits(l, k)) return launch_ygemm_single(s, B, m, k, ldb, Y, ldy, l, C, yd, (double*)parts);
  return launch_yb_tiled(s, B, m, k, ldb, Y, ldy, l, C, (double*)parts);
}

Plan plan(int32_t dt, int64_t m, int64_t n, const Resolved& rs) {
  Carve c;
  Plan p{};
  const int fx = x_fmt(dt);
  const size_t be = dt == RE_F64 ? 8 : 4;
  const int64_t brows = rs.yk == RE_SRHT ? (int64_t)srht_cols_rows_alloc(m) : m;
  const int64_t xn = rs.xk == RE_HRTT || rs.xk == RE_SRCT ? hrtt_npad(n) : rs.npad_n;  // X's transform length
  p.xbits = c.take((size_t)cdiv(xn, 32) * 4);
  const int64_t ym = rs.yk == RE_SRCT ? srct_y_npad(m) : rs.npad_m;  // Y's transform length
  p.ybits = c.take((size_t)cdiv(ym, 32) * 4);
  p.xsel = c.take((size_t)rs.k * 4);
  p.ysel = c.take((size_t)rs.l * 4);
  p.selscr = c.take(select_scratch_bytes(xn > ym ? xn : ym));
  const int bdt = dt == RE_F64 && rs.fmt_x != kBF16 && rs.fmt_x != kF16 ? RE_F64 : RE_F32;
  p.U = c.take(rs.yk == RE_SRCT ? srct_y_u_bytes(m, rs.k, dt == RE_F64 ? RE_F64 : bdt) : 0);
  p.yord = c.take(rs.yk == RE_SRCT ? srct_y_order_bytes(rs.l) : 0);
  size_t xb = rs.xk == RE_GAUSSIAN ? (size_t)n * rs.k * (size_t)elem_size(fx) : 0;  // FP32 / FP64 X
  if (rs.xk == RE_GAUSSIAN && rs.lowprec && gemm_lp_x_bytes(n, rs.k) > xb) xb = gemm_lp_x_bytes(n, rs.k);
  p.X = c.take(xb);
  p.Y = c.take(rs.yk == RE_GAUSSIAN ? (size_t)rs.l * m * elem_size(fx) : 0);
  p.B = c.take((size_t)brows * rs.k * be);
  p.C = c.take((size_t)rs.l * rs.k * 8);
  p.svd = c.take(svd_scratch_bytes(rs.l, rs.k));
  p.sigma = c.take((size_t)rs.k * 8);
  p.info = c.take(16);
  p.out3 = c.take(16);
  p.stats = c.take((4 + 2 * 256) * 8);  // sampled statistics and their per-workgroup partials
  p.gdesc = c.take(sizeof(GemmDesc));
  p.ydesc = c.take(sizeof(YDesc));
  p.queue = c.take(16);
  p.yparts = c.take(rs.yk == RE_GAUSSIAN && dt == RE_F32 ? yb_scratch(rs.l, rs.k, m) : 0);
  p.rdiag = c.take((size_t)rs.k * 3 * 8);  // diagonals of the QR passes (step 7 by the QR diagonal)
  if (dt == RE_F64) {  // K-split partial products of the FP64 Gaussian contractions
    const size_t gx = rs.xk == RE_GAUSSIAN ? gemm64_parts_bytes(m, rs.k, n) : 0;
    const size_t gy = rs.yk == RE_GAUSSIAN ? gemm64_parts_bytes(rs.l, rs.k, m) : 0;
    p.gparts = c.take(gx > gy ? gx : gy);
  }
  p.hscr = c.take(rs.xk == RE_HRTT ? hrtt_scratch_bytes(n, rs.k) : 0);
  p.dctws = c.take(rs.xk == RE_HRTT || rs.xk == RE_SRCT ? dct_long_ws_bytes(m, n, rs.xk == RE_HRTT) : 0);
  p.total = c.off;
  return p;
}

char* at(re_handle h, size_t off) { return (char*)h->ws + off; }

void drop_graph(re_handle h) {
  if (h->bexec) (void)hipGraphExecDestroy(h->bexec);
  h->bexec = nullptr;
  h->bkey.clear();
}

void mark(re_handle h, int i) {
  if (h->prof) (void)hipEventRecord(h->ev[i], h->stream);
}

// Algorithm 1 steps 2-3: draw X (stage RE_STAGE_X_DRAW), form B = A X (RE_STAGE_AX).
re_status run_x(re_handle h, const Plan& p, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                const Resolved& rs, uint64_t seed, void* B) {
  hipStream_t s = h->stream;
  if (rs.xk == RE_HRTT) {  // hashed randomized DCT (FP32 A)
    uint32_t* bits = (uint32_t*)at(h, p.xbits);
    RE_TRY(launch_sign_bits(s, hrtt_npad(n), seed, kXSign, bits));
    RE_TRY(launch_hrtt_hash(s, n, rs.k, seed, at(h, p.hscr)));
    mark(h, RE_STAGE_AX);
    return launch_hrtt_rows(s, (const float*)A, m, n, lda, rs.k, bits, at(h, p.hscr), (float*)B, rs.k,
                            at(h, p.dctws));
  }
  if (rs.xk == RE_SRCT) {  // subsampled randomized DCT (FP32 A): the SRHT's signs and sample over N
    const int64_t N = hrtt_npad(n);
    uint32_t* bits = (uint32_t*)at(h, p.xbits);
    int32_t* sel = (int32_t*)at(h, p.xsel);
    RE_TRY(launch_sign_bits(s, N, seed, kXSign, bits));
    RE_TRY(launch_select(s, N, rs.k, seed, kXSel, at(h, p.selscr), sel));
    mark(h, RE_STAGE_AX);
    return launch_srct_rows(s, (const float*)A, m, n, lda, rs.k, bits, sel, (float*)B, rs.k, at(h, p.dctws));
  }
  if (rs.xk == RE_SRHT) {
    uint32_t* bits = (uint32_t*)at(h, p.xbits);
    int32_t* sel = (int32_t*)at(h, p.xsel);
    RE_TRY(launch_sign_bits(s, rs.npad_n, seed, kXSign, bits));
    RE_TRY(launch_select(s, rs.npad_n, rs.k, seed, kXSel, at(h, p.selscr), sel));
    mark(h, RE_STAGE_AX);
    return launch_srht_rows(s, A, dt, m, n, lda, bits, sel, rs.k, B);
  }
  void* X = at(h, p.X);
  if (rs.fmt_x == kBF16 || rs.fmt_x == kF16) {
    RE_TRY(launch_gemm_lp_x(s, rs.fmt_x, n, rs.k, seed, X));
    mark(h, RE_STAGE_AX);
    return launch_gemm_lp(s, rs.fmt_x, (const float*)A, m, n, lda, X, rs.k, rs.scale_exp, (float*)B);
  }
  const int fx = x_fmt(dt);
  RE_TRY(launch_gauss_fill(s, fx, n, rs.k, seed, kXGauss, 0, X));
  mark(h, RE_STAGE_AX);
  if (dt == RE_F32 && lda < kMaxBatchLda)  // FP32: the matrix-core contraction shared with the batched form
    return launch_gemm_f32_single(s, (const float*)A, m, n, lda, (const float*)X, rs.k, (float*)B, rs.k,
                                  (GemmDesc*)at(h, p.gdesc), (unsigned*)at(h, p.queue));
  if (dt == RE_F32)  // rows too far apart for the persistent kernel's descriptors
    return launch_gemm_f64acc(s, m, rs.k, n, A, 1, lda, X, 1, rs.k, B, 1, rs.k);
  return launch_gemm64(s, m, rs.k, n, (const double*)A, lda, (const double*)X, rs.k, (double*)B, rs.k,
                       (double*)at(h, p.gparts));
}

// Algorithm 1 steps 5-6: draw Y (RE_STAGE_Y_DRAW), form C = Y B (RE_STAGE_YB).
re_status run_y(re_handle h, const Plan& p, void* B, int32_t bdt, int64_t m, const Resolved& rs, uint64_t seed,
                double* C) {
  hipStream_t s = h->stream;
  if (rs.yk == RE_SRHT) {
    uint32_t* bits = (uint32_t*)at(h, p.ybits);
    int32_t* sel = (int32_t*)at(h, p.ysel);
    RE_TRY(launch_sign_bits(s, rs.npad_m, seed, kYSign, bits));
    RE_TRY(launch_select(s, rs.npad_m, rs.l, seed, kYSel, at(h, p.selscr), sel));
    mark(h, RE_STAGE_YB);
    return launch_srht_cols(s, B, bdt, m, rs.k, bits, sel, rs.l, C);
  }
  if (rs.yk == RE_SRCT) {  // subsampled randomized DCT: the SRHT's signs and sample over M
    const int64_t M = srct_y_npad(m);
    uint32_t* bits = (uint32_t*)at(h, p.ybits);
    int32_t* sel = (int32_t*)at(h, p.ysel);
    RE_TRY(launch_sign_bits(s, M, seed, kYSign, bits));
    RE_TRY(launch_select(s, M, rs.l, seed, kYSel, at(h, p.selscr), sel));
    mark(h, RE_STAGE_YB);
    RE_TRY(launch_srct_y_lo(s, B, bdt, m, rs.k, rs.k, bits, at(h, p.U), rs.k));
    return launch_srct_y_hi(s, at(h, p.U), bdt, m, rs.k, rs.k, sel, rs.l, (int32_t*)at(h, p.yord), C);
  }
  const int fy = bdt == RE_F64 ? kF64 : kF32;
  void* Y = at(h, p.Y);
  RE_TRY(launch_gauss_fill(s, fy, rs.l, m, seed, kYGauss, 1, Y));
  mark(h, RE_STAGE_YB);
  if (bdt == RE_F32)
    return run_yb(s, (const float*)B, m, rs.k, rs.k, (const float*)Y, m, rs.l, C, (YDesc*)at(h, p.ydesc),
                  at(h, p.yparts));
  return launch_gemm64(s, rs.l, rs.k, m, (const double*)Y, m, (const double*)B, rs.k, C, rs.k,
                       (double*)at(h, p.gparts));
}

}  // namespace
}  // namespace re

using namespace re;

RE_API re_status re_create(re_handle* h, void* hip_stream) {
  if (!h) return RE_ERR_INVALID_ARG;
  re_handle_s* p = new (std::nothrow) re_handle_s();
  if (!p) return RE_ERR_NO_MEMORY;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return RE_ERR_HIP;
  }
  p->stream = (hipStream_t)hip_stream;
  // XCDs in turn from the last one down: workgroup 0 of every launch, and so
  // every one-workgroup kernel of every stream, runs on XCD 0, which the
  // small SVDs of up to seven handles thus avoid
  static std::atomic<unsigned> next_xcd{0};
  p->xcd = (int)(7u - (next_xcd.fetch_add(1, std::memory_order_relaxed) & 7u));
  *h = p;
  return RE_OK;
}

RE_API re_status re_set_profiling(re_handle h, int32_t enable) {
  if (!h) return RE_ERR_INVALID_ARG;
  if (enable && !h->ev[0])
    for (int i = 0; i <= RE_NUM_STAGES; ++i) RE_TRY_HIP(hipEventCreate(&h->ev[i]));
  h->prof = enable != 0;
  return RE_OK;
}

RE_API re_status re_set_limits(re_handle h, int64_t max_workspace_bytes, int64_t barrier_polls) {
  if (!h || max_workspace_bytes < 0) return RE_ERR_INVALID_ARG;
  h->ws_cap = (size_t)max_workspace_bytes;
  h->spin_limit = (long)barrier_polls;
  return RE_OK;
}

RE_API re_status re_last_stage_ms(re_handle h, double* ms) {
  if (!h || !ms || !h->prof) return RE_ERR_INVALID_ARG;
  for (int i = 0; i < RE_NUM_STAGES; ++i) ms[i] = h->stage_ms[i];
  return RE_OK;
}

RE_API re_status re_destroy(re_handle h) {
  if (!h) return RE_OK;
  if (h->stream || h->ws) (void)hipStreamSynchronize(h->stream);
  for (int i = 0; i <= RE_NUM_STAGES; ++i)
    if (h->ev[i]) (void)hipEventDestroy(h->ev[i]);
  drop_graph(h);
  if (h->cap) (void)hipStreamDestroy(h->cap);
  if (h->ws) (void)hipFree(h->ws);
  if (h->ws2) (void)hipFree(h->ws2);
  if (h->host) (void)hipHostFree(h->host);
  delete h;
  return RE_OK;
}

RE_API re_status re_set_stream(re_handle h, void* hip_stream) {
  if (!h) return RE_ERR_INVALID_ARG;
  RE_TRY_HIP(hipStreamSynchronize(h->stream));
  h->stream = (hipStream_t)hip_stream;
  return RE_OK;
}

RE_API re_status re_workspace_bytes(re_handle h, size_t* bytes) {
  if (!h || !bytes) return RE_ERR_INVALID_ARG;
  *bytes = h->ws_bytes;
  return RE_OK;
}

RE_API int32_t re_r1_from_k(int32_t k) { return re::r1_from_k(k); }

RE_API re_status re_gap_rank(const double* sigma, int32_t k, int32_t r1, int32_t* r_out, double* ratio_out) {
  if (!sigma || !r_out || k < 0 || r1 < 0) return RE_ERR_INVALID_ARG;
  const int32_t n = r1 < k ? r1 : k;
  int32_t best_i = 0;
  double best = 0.0;
  if (n >= 2 && sigma[0] > 0.0) {
    best = -1.0;
    for (int32_t i = 1; i < n && sigma[i - 1] > 0.0; ++i) {
      const double q = sigma[i] > 0.0 ? sigma[i - 1] / sigma[i] : HUGE_VAL;
      if (q > best) {
        best = q;
        best_i = i;
      }
    }
  }
  *r_out = best_i;
  if (ratio_out) *ratio_out = best_i > 0 ? best : 0.0;
  return RE_OK;
}

namespace re {
namespace {

// Estimates of the plain method between their launch and their final
// synchronisation, over all handles of the process.  Up to kPlainInFlight of
// them let the small SVD take the plain launch (see launch_svd): with more,
// a steady stream of other estimates' kernels could keep its late
// participants waiting, and the cooperative form is used.
std::atomic<int> g_in_flight{0};
constexpr int kPlainInFlight = 4;

struct InFlight {
  int n;
  InFlight() : n(g_in_flight.fetch_add(1) + 1) {}
  ~InFlight() { g_in_flight.fetch_sub(1); }
};

// One pass of Algorithm 1 with the formats in rs; results left in the
// handle's pinned staging buffer (16 bytes of r, flags, status; then sigma).
re_status run_once(re_handle h, const Plan& p, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                   double eps, const Resolved& rs, uint64_t seed) {
  const InFlight fl;
  void* B = at(h, p.B);
  double* C = (double*)at(h, p.C);
  double* sigma = (double*)at(h, p.sigma);
  int32_t* info = (int32_t*)at(h, p.info);
  int32_t* out3 = (int32_t*)at(h, p.out3);
  const int32_t r1 = r1_from_k((int32_t)rs.k);
  mark(h, RE_STAGE_X_DRAW);
  RE_TRY(run_x(h, p, A, dt, m, n, lda, rs, seed, B));
  mark(h, RE_STAGE_Y_DRAW);
  RE_TRY(run_y(h, p, B, dt, m, rs, seed, C));
  const double scale = 1.0 / sqrt((double)rs.k * (double)rs.l);
  mark(h, RE_STAGE_SVD);
  bool plain = false;
  // FP64 inputs never reach the batched form (FP32 only), so their small
  // sketches take the multisection
  const bool ms = dt == RE_F64;
  RE_TRY(launch_svd(h->stream, C, rs.l, rs.k, scale, at(h, p.svd), sigma, info, h->spin_limit, h->xcd,
                    fl.n <= kPlainInFlight ? 1 : 0, &plain, ms));
  mark(h, RE_STAGE_RANK);
  RE_TRY(launch_rank_count(h->stream, sigma, rs.k, r1, eps, info, out3));
  char* host = (char*)h->host;
  RE_TRY_HIP(hipMemcpyAsync(host, out3, 16, hipMemcpyDeviceToHost, h->stream));
  RE_TRY_HIP(hipMemcpyAsync(host + 64, sigma, (size_t)rs.k * 8, hipMemcpyDeviceToHost, h->stream));
  mark(h, RE_NUM_STAGES);
  RE_TRY_HIP(hipStreamSynchronize(h->stream));
  if (plain && ((const int32_t*)host)[2] == RE_ERR_NO_CONVERGENCE) {
    // a participant of the plain launch waited past its short poll limit: the
    // same step again, plain under the default limit (C is intact; the SVD
    // starts from it afresh)
    RE_TRY(launch_svd(h->stream, C, rs.l, rs.k, scale, at(h, p.svd), sigma, info, h->spin_limit, h->xcd, 2, nullptr,
                      ms));
    RE_TRY(launch_rank_count(h->stream, sigma, rs.k, r1, eps, info, out3));
    RE_TRY_HIP(hipMemcpyAsync(host, out3, 16, hipMemcpyDeviceToHost, h->stream));
    RE_TRY_HIP(hipMemcpyAsync(host + 64, sigma, (size_t)rs.k * 8, hipMemcpyDeviceToHost, h->stream));
    RE_TRY_HIP(hipStreamSynchronize(h->stream));
    h->relaunched = true;
  }
  if (h->prof) {
    for (int i = 0; i < RE_NUM_STAGES; ++i) {
      float ms = 0.f;
      h->stage_ms[i] = hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess ? (double)ms : -1.0;
    }
  }
  return RE_OK;
}

double unit_roundoff(int fmt) { return fmt == kBF16 ? 0x1.0p-8 : fmt == kF16 ? 0x1.0p-11 : 0x1.0p-24; }

}  // namespace
}  // namespace re

RE_API re_status re_rank_estimate(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                                  double eps, const re_sketch* sk, uint64_t seed, int32_t* r_out, double* sigma_out,
                                  int32_t* r1_out, uint32_t* flags_out) {
  if (!h || !r_out || !sigma_out) return RE_ERR_INVALID_ARG;
  if (!(eps > 0.0 && eps < 1.0)) return RE_ERR_INVALID_ARG;
  Resolved rs;
  RE_TRY(validate(A, dt, m, n, lda, sk, &rs));
  rs.fmt_x = x_fmt(dt);
  rs.lowprec = sk->prec != RE_PREC_NATIVE;
  const Plan p = plan(dt, m, n, rs);
  RE_TRY(ensure_ws(h, p.total));
  RE_TRY(ensure_host(h, (size_t)rs.k * 8 + 64 + 32));  // r, flags, status; sigma; the sampled statistics
  const char* host = (const char*)h->host;
  uint32_t extra = 0;
  h->relaunched = false;
  if (sk->prec == RE_PREC_NATIVE) {
    RE_TRY(run_once(h, p, A, dt, m, n, lda, eps, rs, seed));
  } else {
    // sampled ||A||_F^2 and max |a|: FP16 scale and the AUTO acceptance test
    double* st = (double*)at(h, p.stats);
    RE_TRY(launch_sample_stats(h->stream, (const float*)A, m, n, lda, st));
    double* stats = (double*)((char*)h->host + 64 + (size_t)rs.k * 8);  // pinned: the copy stays asynchronous
    RE_TRY_HIP(hipMemcpyAsync(stats, st, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    RE_TRY_HIP(hipStreamSynchronize(h->stream));
    const double frob = sqrt(stats[0] * ((double)m * (double)n / (stats[2] > 0 ? stats[2] : 1.0)));
    const double amax = stats[1];
    const double shape = 1.0 / sqrt((double)rs.k) + 1.0 / sqrt((double)m);
    int tries[3] = {kBF16, kF16, kF32};
    int ntries = 3;
    if (sk->prec == RE_PREC_BF16) { tries[0] = kBF16; ntries = 1; }
    if (sk->prec == RE_PREC_FP16) { tries[0] = kF16; ntries = 1; }
    re_status last = RE_OK;
    for (int t = 0; t < ntries; ++t) {
      rs.fmt_x = tries[t];
      rs.scale_exp = 0;
      if (rs.fmt_x == kF16 && amax > 0.0) {
        int e2 = 0;
        frexp(amax, &e2);   // amax < 2^e2
        rs.scale_exp = 12 - e2;
      }
      last = run_once(h, p, A, dt, m, n, lda, eps, rs, seed);
      const int32_t* o3 = (const int32_t*)host;
      if (rs.fmt_x == kF32) break;
      if (last != RE_OK) return last;
      const double s1 = ((const double*)(host + 64))[0];
      const double phi = unit_roundoff(rs.fmt_x) / sqrt(3.0) * frob * shape;
      const bool resolved = o3[2] == 0 && phi <= eps * s1 / 4.0;
      if (sk->prec != RE_PREC_AUTO) {  // a forced format: report a floor above the threshold
        if (o3[2] == 0 && !resolved) extra |= RE_FLAG_PREC_BELOW_FLOOR;
        break;
      }
      if (resolved) break;  // accepted
      if (t + 1 == ntries - 1) extra |= RE_FLAG_PREC_FALLBACK;
    }
    RE_TRY(last);
    if (rs.fmt_x == kBF16) extra |= RE_FLAG_USED_BF16;
    if (rs.fmt_x == kF16) extra |= RE_FLAG_USED_FP16;
  }
  const int32_t* o3 = (const int32_t*)host;
  if (o3[2] != 0) return (re_status)o3[2];
  *r_out = o3[0];
  memcpy(sigma_out, host + 64, (size_t)rs.k * 8);
  if (r1_out) *r1_out = r1_from_k((int32_t)rs.k);
  if (h->relaunched) extra |= RE_FLAG_SVD_RELAUNCHED;
  if (flags_out) *flags_out = (uint32_t)o3[1] | extra;
  return RE_OK;
}

namespace re {
namespace {

// ---------------------------------------------------------------------------
// Batched form.  Device workspace: [descriptor region | results region |
// sketches and intermediates]; the descriptor region is a byte image of the
// host staging area and is refreshed by one copy before every graph launch,
// the results region comes back by one copy captured in the graph.
// ---------------------------------------------------------------------------
struct BatchPlan {
  // descriptor region (offsets from its start; same in host staging)
  size_t hdr, gdesc, ydesc, sdesc, cptr, dptr, eptr, lv, kv, desc_bytes;
  // results region (offsets from its start)
  size_t out3, sigma, res_bytes;
  // the rest (offsets from the workspace start)
  size_t desc0, res0, X, Y, B, C, d, e, info, queue, total;
};

BatchPlan batch_plan(int nb, int64_t k, int64_t l, int64_t nmax, int64_t mmax, int64_t brows_total) {
  BatchPlan p{};
  Carve a;
  p.hdr = a.take(sizeof(BatchHeader));
  p.gdesc = a.take((size_t)nb * sizeof(GemmDesc));
  p.ydesc = a.take((size_t)nb * sizeof(YDesc));
  p.sdesc = a.take((size_t)nb * sizeof(SvDesc));
  p.cptr = a.take((size_t)nb * 8);
  p.dptr = a.take((size_t)nb * 8);
  p.eptr = a.take((size_t)nb * 8);
  p.lv = a.take((size_t)nb * 4);
  p.kv = a.take((size_t)nb * 4);
  p.desc_bytes = a.off;
  Carve r;
  p.out3 = r.take((size_t)nb * 16);
  p.sigma = r.take((size_t)nb * k * 8);
  p.res_bytes = r.off;
  Carve c;
  p.desc0 = c.take(p.desc_bytes);
  p.res0 = c.take(p.res_bytes);
  p.X = c.take((size_t)nmax * k * 4);
  p.Y = c.take((size_t)l * mmax * 4);
  p.B = c.take((size_t)brows_total * k * 4);  // block b at a 256-byte aligned row offset
  p.C = c.take((size_t)nb * l * k * 8);
  p.d = c.take((size_t)nb * k * 8);
  p.e = c.take((size_t)nb * k * 8);
  p.info = c.take((size_t)nb * 4);
  p.queue = c.take(16);
  p.total = c.off;
  return p;
}

int device_cus(int dev) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
  return cus;
}

// Tile shapes the persistent contraction is instantiated for.
bool tile_ok(int w, int mt, int bk) { return (w == 4 || w == 8) && ((mt == 1 && (bk == 16 || bk == 32)) || (mt == 2 && bk == 16)); }

// Autotuner cache file: one JSON object, one "key": [waves, mt, bk, grid] entry per line.
void load_tune_cache(re_handle h) {
  const char* path = getenv("RANKEST_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    char key[256];
    int w = 0, mt = 0, bk = 0, g = 0;
    if (sscanf(line, " \"%255[^\"]\" : [ %d , %d , %d , %d ]", key, &w, &mt, &bk, &g) == 5 && tile_ok(w, mt, bk) &&
        g > 0)
      h->tuned[key] = {w, mt, bk, g};
  }
  fclose(f);
}

void save_tune_cache(re_handle h) {
  const char* path = getenv("RANKEST_AUTOTUNE_CACHE");
  if (!path) return;
  FILE* f = fopen(path, "w");
  if (!f) return;
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto& kv : h->tuned)
    fprintf(f, "  \"%s\": [%d, %d, %d, %d]%s\n", kv.first.c_str(), kv.second.waves, kv.second.mt, kv.second.bk,
            kv.second.grid, ++i < h->tuned.size() ? "," : "");
  fprintf(f, "}\n");
  fclose(f);
}

// Fills the host image of the descriptor region for tile height 32 * waves;
// returns the total number of work items.
int64_t fill_batch_desc(char* img, const BatchPlan& p, char* ws, const re_block* blocks, int nb, int64_t k, int64_t l,
                        double eps, uint64_t seed, int rows_per_item) {
  BatchHeader* hd = (BatchHeader*)(img + p.hdr);
  hd->seed = seed;
  GemmDesc* gd = (GemmDesc*)(img + p.gdesc);
  YDesc* yd = (YDesc*)(img + p.ydesc);
  SvDesc* sd = (SvDesc*)(img + p.sdesc);
  const double** cp = (const double**)(img + p.cptr);
  double** dp = (double**)(img + p.dptr);
  double** ep = (double**)(img + p.eptr);
  int32_t* lv = (int32_t*)(img + p.lv);
  int32_t* kv = (int32_t*)(img + p.kv);
  char* res = ws + p.res0;
  const int32_t r1 = r1_from_k((int32_t)k);
  const double scale = 1.0 / sqrt((double)k * (double)l);
  int64_t item = 0, brow = 0;
  for (int b = 0; b < nb; ++b) {
    const re_block& bl = blocks[b];
    float* Bb = (float*)(ws + p.B) + brow * k;
    double* Cb = (double*)(ws + p.C) + (size_t)b * l * k;
    double* db = (double*)(ws + p.d) + (size_t)b * k;
    double* eb = (double*)(ws + p.e) + (size_t)b * k;
    gd[b].A = (const float*)bl.A;
    gd[b].B = Bb;
    gd[b].m = bl.m;
    gd[b].n = bl.n;
    gd[b].lda = bl.lda;
    gd[b].ldb = k;
    gd[b].item0 = item;
    gd[b].ncc = gemm_col_chunks(k);
    item += gemm_items(bl.m, k, rows_per_item);
    yd[b].B = Bb;
    yd[b].C = Cb;
    yd[b].m = bl.m;
    yd[b].ldb = k;
    cp[b] = Cb;
    dp[b] = db;
    ep[b] = eb;
    lv[b] = (int32_t)l;
    kv[b] = (int32_t)k;
    sd[b].d = db;
    sd[b].e = eb;
    sd[b].sigma = (double*)(res + p.sigma) + (size_t)b * k;
    sd[b].info = (const int32_t*)(ws + p.info) + b;
    sd[b].out3 = (int32_t*)(res + p.out3) + 4 * b;
    sd[b].k = (int32_t)k;
    sd[b].r1 = r1;
    sd[b].scale = scale;
    sd[b].eps = eps;
    brow += (bl.m + 63) / 64 * 64;
  }
  return item;
}

// The captured sequence: master sketches, persistent A X, batched Y B, small
// SVDs, counts, results to the host.  With profiling on, the same sequence is
// issued directly on the stream with stage events between the launches.
re_status enqueue_batch(re_handle h, hipStream_t s, const BatchPlan& p, int nb, int64_t k, int64_t l, int64_t nmax,
                        int64_t mmax, int64_t total, const re_handle_s::Tile& tl, int grid, void* host_res) {
  char* ws = (char*)h->ws;
  char* dsc = ws + p.desc0;
  float* X = (float*)(ws + p.X);
  float* Y = (float*)(ws + p.Y);
  auto ev = [&](int i) -> re_status {
    if (h->prof) RE_TRY_HIP(hipEventRecord(h->ev[i], s));
    return RE_OK;
  };
  RE_TRY(ev(RE_STAGE_X_DRAW));
  RE_TRY(launch_gauss_master(s, (const BatchHeader*)(dsc + p.hdr), nmax, k, l, mmax, X, Y));
  RE_TRY(ev(RE_STAGE_AX));
  RE_TRY(launch_gemm_f32_persistent(s, (const GemmDesc*)(dsc + p.gdesc), nb, X, k, total, (unsigned*)(ws + p.queue),
                                    tl.waves, grid, tl.bk, tl.mt));
  RE_TRY(ev(RE_STAGE_Y_DRAW));
  RE_TRY(ev(RE_STAGE_YB));
  RE_TRY(launch_ygemm_batched(s, (const YDesc*)(dsc + p.ydesc), nb, Y, mmax, l, k));
  RE_TRY(ev(RE_STAGE_SVD));
  RE_TRY(launch_bidiag_batched(s, (const double* const*)(dsc + p.cptr), (double* const*)(dsc + p.dptr),
                               (double* const*)(dsc + p.eptr), (const int32_t*)(dsc + p.lv),
                               (const int32_t*)(dsc + p.kv), (int32_t*)(ws + p.info), nb, l, k));
  RE_TRY(launch_sv_count_batched(s, (const SvDesc*)(dsc + p.sdesc), nb, k));
  RE_TRY(ev(RE_STAGE_RANK));
  RE_TRY_HIP(hipMemcpyAsync(host_res, ws + p.res0, p.res_bytes, hipMemcpyDeviceToHost, s));
  RE_TRY(ev(RE_NUM_STAGES));
  return RE_OK;
}

}  // namespace
}  // namespace re

RE_API re_status re_rank_estimate_batched(re_handle h, const re_block* blocks, int32_t nblocks, int32_t dt, double eps,
                                          const re_sketch* sk, uint64_t seed, int32_t* r_out, double* sigma_out,
                                          uint32_t* flags_out) {
  if (!h || !sk || nblocks < 0 || (nblocks > 0 && (!blocks || !r_out || !sigma_out))) return RE_ERR_INVALID_ARG;
  if (!(eps > 0.0 && eps < 1.0)) return RE_ERR_INVALID_ARG;
  if (dt != RE_F64 && dt != RE_F32) return RE_ERR_INVALID_ARG;
  if ((sk->x_kind != RE_GAUSSIAN && sk->x_kind != RE_SRHT) || (sk->y_kind != RE_GAUSSIAN && sk->y_kind != RE_SRHT) ||
      sk->prec < RE_PREC_NATIVE || sk->prec > RE_PREC_AUTO)
    return RE_ERR_INVALID_ARG;
  if (dt != RE_F32 || sk->x_kind != RE_GAUSSIAN || sk->y_kind != RE_GAUSSIAN || sk->prec != RE_PREC_NATIVE)
    return RE_ERR_UNSUPPORTED;
  const int64_t k = sk->k, l = sk->l == 0 ? 2 * (int64_t)sk->k : sk->l;
  if (k < 1 || l < k || k > 4096) return RE_ERR_INVALID_ARG;
  if (nblocks == 0) return RE_OK;
  if (!batched_fits(l, k)) return RE_ERR_UNSUPPORTED;
  int64_t nmax = 0, mmax = 0, brows = 0;
  for (int b = 0; b < nblocks; ++b) {
    const re_block& bl = blocks[b];
    if (!bl.A || bl.m < l || bl.n < k || bl.lda < bl.n || bl.lda >= kMaxBatchLda || ((uintptr_t)bl.A) % 4 != 0)
      return RE_ERR_INVALID_ARG;
    if (bl.m > (int64_t)INT32_MAX || bl.n > (int64_t)INT32_MAX) return RE_ERR_INVALID_ARG;
    nmax = bl.n > nmax ? bl.n : nmax;
    mmax = bl.m > mmax ? bl.m : mmax;
    brows += (bl.m + 63) / 64 * 64;
  }
  if (gemm_items(brows, k, 32) >= (int64_t)INT32_MAX) return RE_ERR_INVALID_ARG;
  const BatchPlan p = batch_plan(nblocks, k, l, nmax, mmax, brows);
  const void* old_ws = h->ws;
  RE_TRY(ensure_ws(h, p.total));
  RE_TRY(ensure_host(h, p.desc_bytes + p.res_bytes));
  if (h->ws != old_ws) drop_graph(h);
  char* img = (char*)h->host;
  char* host_res = img + p.desc_bytes;
  char* ws = (char*)h->ws;
  hipStream_t s = h->stream;
  if (!h->cap) {
    RE_TRY_HIP(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
    load_tune_cache(h);
  }

  // autotune the persistent contraction for this size bucket
  const int cus = device_cus(h->device);
  const int64_t items4 = gemm_items(brows, k, 128);
  int lg = 0;
  while ((int64_t(1) << lg) < items4) ++lg;
  char key[128];
  snprintf(key, sizeof(key), "gfx950:f32:k%lld:items2^%d", (long long)k, lg);
  // RANKEST_BATCH_TILE="waves:mt:bk:grid per CU" pins the tile shape (tuning sweeps, tests)
  if (const char* pin = getenv("RANKEST_BATCH_TILE")) {
    int w = 0, mt = 0, bk = 0, gm = 0;
    if (sscanf(pin, "%d:%d:%d:%d", &w, &mt, &bk, &gm) != 4 || !tile_ok(w, mt, bk) || gm < 1 || gm > 64)
      return RE_ERR_INVALID_ARG;
    h->tuned[key] = {w, mt, bk, gm * cus};
  }
  auto it = h->tuned.find(key);
  if (it == h->tuned.end()) {
    const int cand[7][4] = {{4, 1, 16, 2}, {4, 1, 16, 3}, {4, 1, 32, 2}, {8, 1, 16, 2},
                            {4, 2, 16, 2}, {4, 2, 16, 3}, {8, 2, 16, 1}};
    hipEvent_t e0, e1;
    RE_TRY_HIP(hipEventCreate(&e0));
    RE_TRY_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    re_handle_s::Tile pick{4, 1, 16, 2 * cus};
    for (const auto& c : cand) {
      const int64_t tot = fill_batch_desc(img, p, ws, blocks, nblocks, k, l, eps, seed, 32 * c[0] * c[1]);
      const int g = (int)(tot < (int64_t)c[3] * cus ? tot : (int64_t)c[3] * cus);
      RE_TRY_HIP(hipMemcpyAsync(ws + p.desc0, img, p.desc_bytes, hipMemcpyHostToDevice, s));
      RE_TRY(launch_gauss_master(s, (const BatchHeader*)(ws + p.desc0 + p.hdr), nmax, k, l, mmax, (float*)(ws + p.X),
                                 (float*)(ws + p.Y)));
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        RE_TRY_HIP(hipEventRecord(e0, s));
        RE_TRY(launch_gemm_f32_persistent(s, (const GemmDesc*)(ws + p.desc0 + p.gdesc), nblocks, (const float*)(ws + p.X),
                                          k, tot, (unsigned*)(ws + p.queue), c[0], g, c[2], c[1]));
        RE_TRY_HIP(hipEventRecord(e1, s));
        RE_TRY_HIP(hipEventSynchronize(e1));
        RE_TRY_HIP(hipEventElapsedTime(&ms, e0, e1));
      }
      if (ms < best) {
        best = ms;
        pick = {c[0], c[1], c[2], c[3] * cus};
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    h->tuned[key] = pick;
    save_tune_cache(h);
    it = h->tuned.find(key);
  }
  const re_handle_s::Tile tl = it->second;
  const int64_t total = fill_batch_desc(img, p, ws, blocks, nblocks, k, l, eps, seed, 32 * tl.waves * tl.mt);
  const int grid = (int)(total < tl.grid ? total : tl.grid);

  // (re)capture when anything baked into the graph changed
  char gkey[256];
  snprintf(gkey, sizeof(gkey), "%p %p %d %lld %lld %lld %lld %lld %lld %d %d %d %d", (void*)ws, (void*)host_res, nblocks,
           (long long)k, (long long)l, (long long)nmax, (long long)mmax, (long long)brows, (long long)total, tl.waves,
           tl.mt, tl.bk, grid);
  if (h->prof) {  // eager issue of the same launches, stage events in between
    RE_TRY_HIP(hipMemcpyAsync(ws + p.desc0, img, p.desc_bytes, hipMemcpyHostToDevice, s));
    RE_TRY(enqueue_batch(h, s, p, nblocks, k, l, nmax, mmax, total, tl, grid, host_res));
  } else if (!h->bexec || h->bkey != gkey) {
    drop_graph(h);
    RE_TRY_HIP(hipStreamSynchronize(s));
    RE_TRY_HIP(hipStreamBeginCapture(h->cap, hipStreamCaptureModeRelaxed));
    const re_status st = enqueue_batch(h, h->cap, p, nblocks, k, l, nmax, mmax, total, tl, grid, host_res);
    hipGraph_t g = nullptr;
    const hipError_t ce = hipStreamEndCapture(h->cap, &g);
    if (st != RE_OK || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return st != RE_OK ? st : RE_ERR_HIP;
    }
    const hipError_t ie = hipGraphInstantiate(&h->bexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      h->bexec = nullptr;
      return RE_ERR_HIP;
    }
    h->bkey = gkey;
  }
  if (!h->prof) {
    RE_TRY_HIP(hipMemcpyAsync(ws + p.desc0, img, p.desc_bytes, hipMemcpyHostToDevice, s));
    RE_TRY_HIP(hipGraphLaunch(h->bexec, s));
  }
  RE_TRY_HIP(hipStreamSynchronize(s));
  if (h->prof) {
    for (int i = 0; i < RE_NUM_STAGES; ++i) {
      float ms = 0.f;
      h->stage_ms[i] = hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess ? (double)ms : -1.0;
    }
  }
  re_status worst = RE_OK;
  for (int b = 0; b < nblocks; ++b) {
    const int32_t* o3 = (const int32_t*)(host_res + p.out3) + 4 * b;
    r_out[b] = o3[2] == 0 ? o3[0] : -1;
    if (flags_out) flags_out[b] = (uint32_t)o3[1];
    if (o3[2] != 0 && worst == RE_OK) worst = (re_status)o3[2];
  }
  memcpy(sigma_out, host_res + p.sigma, (size_t)nblocks * k * 8);
  return worst;
}

// ---------------------------------------------------------------------------
// Learned sketch-size policy: the network on device buffers, and the adaptive
// driver that appends sketch columns and rows round by round.
// ---------------------------------------------------------------------------
RE_API re_status re_mlp_forward(re_handle h, const float* params_dev, const float* x_dev, int64_t batch, float* y_dev) {
  if (!h || batch < 0 || (batch > 0 && (!params_dev || !x_dev || !y_dev))) return RE_ERR_INVALID_ARG;
  return launch_mlp_forward(h->stream, params_dev, x_dev, batch, y_dev, nullptr, nullptr);
}

RE_API re_status re_mlp_loss_grad(re_handle h, const float* params_dev, const float* x_dev, const float* t_dev,
                                  int64_t batch, float* grad_dev, float* loss_dev) {
  if (!h || batch < 1 || !params_dev || !x_dev || !t_dev || !grad_dev) return RE_ERR_INVALID_ARG;
  RE_TRY(ensure_ws(h, (mlp_scratch_floats(batch) + (size_t)batch) * sizeof(float)));
  return launch_mlp_loss_grad(h->stream, params_dev, x_dev, t_dev, batch, (float*)h->ws, grad_dev, loss_dev);
}

RE_API re_status re_mlp_adam(re_handle h, float* params_dev, const float* grad_dev, float* m_dev, float* v_dev,
                             int64_t n, int32_t step, double lr, double beta1, double beta2, double eps) {
  if (!h || n < 0 || step < 1 || (n > 0 && (!params_dev || !grad_dev || !m_dev || !v_dev))) return RE_ERR_INVALID_ARG;
  if (!(lr > 0.0) || !(beta1 >= 0.0 && beta1 < 1.0) || !(beta2 >= 0.0 && beta2 < 1.0) || !(eps > 0.0))
    return RE_ERR_INVALID_ARG;
  const double c1 = 1.0 / (1.0 - pow(beta1, (double)step)), c2 = 1.0 / (1.0 - pow(beta2, (double)step));
  return launch_mlp_adam(h->stream, params_dev, grad_dev, m_dev, v_dev, n, (float)lr, (float)beta1, (float)beta2,
                         (float)eps, (float)c1, (float)c2);
}

namespace re {
namespace {

int64_t l_for(int64_t k, double ratio, int64_t m) {
  int64_t l = (int64_t)floor(ratio * (double)k + 0.5);
  if (l < k) l = k;
  if (l > m) l = m;
  return l;
}

// Network input from the pilot estimates (same definition as RE_MLP_INPUTS).
void pilot_features(const double* s, int64_t k, int64_t m, int64_t n, double eps, float* f) {
  for (int i = 0; i < 32; ++i) {
    double v = -8.0;
    if (i < k && s[0] > 0.0) {
      const double q = s[i] / s[0];
      v = q > 0.0 ? log10(q) : -8.0;
      if (v < -8.0) v = -8.0;
    }
    f[i] = (float)v;
  }
  f[32] = (float)log10((double)m);
  f[33] = (float)log10((double)n);
  f[34] = (float)log10(eps);
}

struct AdPlan {
  size_t B, Xn, Y, C, svd, sigma, info, out3, gdesc, ydesc, queue, feat, yout, yparts, ybits, ysel, selscr, U, yord,
      total;
};

// Largest Y B scratch over the widths an adaptive run may visit (k0 doubling,
// a proposal rounded to 8, k_max).
size_t yb_scratch_adaptive(int64_t k0, int64_t kmax, double ratio, int64_t m) {
  size_t most = 0;
  for (int64_t k = 8; k <= kmax; k += 8) {
    const size_t b = yb_scratch(l_for(k, ratio, m), k, m);
    most = b > most ? b : most;
  }
  for (int64_t k = k0 < kmax ? k0 : kmax;; k = 2 * k < kmax ? 2 * k : kmax) {
    const size_t b = yb_scratch(l_for(k, ratio, m), k, m);
    most = b > most ? b : most;
    if (k >= kmax) break;
  }
  return most;
}

}  // namespace
}  // namespace re

// The adaptive driver for a Gaussian or an SRHT Y (X Gaussian).  With the SRHT
// Y the first level of its transform along m (signs and blocks of rows) is
// applied once to each new column of A X and kept in place: the stored
// F D A X of Sec. 5 (footnote on growing an SRTT sketch), from which every
// round forms its l sampled rows for all k columns.
static re_status adaptive_impl(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda, double eps,
                        const re_adaptive* ad, int32_t yk, uint64_t seed, int32_t* r_out, double* sigma_out,
                        int32_t* k_out, int32_t* l_out, int32_t* rounds_out, int32_t* k_proposed_out,
                        uint32_t* flags_out) {
  if (!h || !A || !ad || !r_out || !sigma_out) return RE_ERR_INVALID_ARG;
  if (yk != RE_GAUSSIAN && yk != RE_SRHT && yk != RE_SRCT) return RE_ERR_INVALID_ARG;
  if (dt != RE_F64 && dt != RE_F32) return RE_ERR_INVALID_ARG;
  if (dt != RE_F32) return RE_ERR_UNSUPPORTED;
  if (!(eps > 0.0 && eps < 1.0) || m < 1 || n < 1 || lda < n || lda >= kMaxBatchLda || ((uintptr_t)A) % 4 != 0)
    return RE_ERR_INVALID_ARG;
  if (ad->k0 < 1 || !(ad->l_ratio >= 1.0) || ad->k_max < 0 || !isfinite(ad->delta)) return RE_ERR_INVALID_ARG;
  int64_t kmax = m < n ? m : n;
  if (ad->k_max > 0 && ad->k_max < kmax) kmax = ad->k_max;
  if (kmax > RE_MAX_ADAPTIVE_K) kmax = RE_MAX_ADAPTIVE_K;
  const int64_t lmax = l_for(kmax, ad->l_ratio, m);
  const bool srht_y = yk == RE_SRHT, srct_y = yk == RE_SRCT, trig_y = srht_y || srct_y;
  const int64_t npad_m = srct_y ? srct_y_npad(m) : next_pow2(m);
  AdPlan p{};
  Carve c;
  p.B = c.take((size_t)(srht_y ? (int64_t)srht_cols_rows_alloc(m) : m) * kmax * 4);
  p.Xn = c.take((size_t)n * kmax * 4);
  p.Y = c.take(trig_y ? 0 : (size_t)lmax * m * 4);
  p.ybits = c.take(trig_y ? (size_t)cdiv(npad_m, 32) * 4 : 0);
  p.ysel = c.take(trig_y ? (size_t)lmax * 4 : 0);
  p.selscr = c.take(trig_y ? select_scratch_bytes(npad_m) : 0);
  p.U = c.take(srct_y ? srct_y_u_bytes(m, kmax, RE_F32) : 0);
  p.yord = c.take(srct_y ? srct_y_order_bytes(lmax) : 0);
  p.C = c.take((size_t)lmax * kmax * 8);
  p.svd = c.take(svd_scratch_bytes(lmax, kmax));
  p.sigma = c.take((size_t)kmax * 8);
  p.info = c.take(16);
  p.out3 = c.take(16);
  p.gdesc = c.take(sizeof(GemmDesc));
  p.ydesc = c.take(sizeof(YDesc));
  p.queue = c.take(16);
  p.feat = c.take(RE_MLP_INPUTS * 4);
  p.yout = c.take(16);
  p.yparts = c.take(trig_y ? 0 : yb_scratch_adaptive(ad->k0, kmax, ad->l_ratio, m));
  p.total = c.off;
  RE_TRY(ensure_ws(h, p.total));
  RE_TRY(ensure_host(h, 256 + (size_t)kmax * 8));  // out3 | sigma | features
  hipStream_t s = h->stream;
  char* host = (char*)h->host;
  float* B = (float*)at(h, p.B);
  float* Y = (float*)at(h, p.Y);
  double* C = (double*)at(h, p.C);
  double* sigma = (double*)at(h, p.sigma);
  int32_t* info = (int32_t*)at(h, p.info);
  int32_t* out3 = (int32_t*)at(h, p.out3);
  int64_t k_old = 0, l_old = 0, k = ad->k0 < kmax ? ad->k0 : kmax;
  int32_t rounds = 0, kprop = 0;
  for (;;) {
    const int64_t l = l_for(k, ad->l_ratio, m);
    // Algorithm 1 steps 2-6 on the appended part only
    RE_TRY(launch_gauss_sub(s, n, k - k_old, 0, k_old, seed, kXGauss, 0, k - k_old, (float*)at(h, p.Xn)));
    RE_TRY(launch_gemm_f32_single(s, (const float*)A, m, n, lda, (const float*)at(h, p.Xn), k - k_old, B + k_old, kmax,
                                  (GemmDesc*)at(h, p.gdesc), (unsigned*)at(h, p.queue)));
    if (srht_y) {
      uint32_t* ybits = (uint32_t*)at(h, p.ybits);
      int32_t* ysel = (int32_t*)at(h, p.ysel);
      if (k_old == 0) RE_TRY(launch_sign_bits(s, npad_m, seed, kYSign, ybits));
      RE_TRY(launch_srht_cols_lo(s, B + k_old, RE_F32, m, k - k_old, kmax, ybits));  // the new columns of F D A X
      RE_TRY(launch_select(s, npad_m, l, seed, kYSel, at(h, p.selscr), ysel));     // nested in l
      RE_TRY(launch_srht_cols_hi(s, B, RE_F32, m, k, kmax, ysel, l, C));
    } else if (srct_y) {  // the stored first level U of the DCT along m, new columns only
      uint32_t* ybits = (uint32_t*)at(h, p.ybits);
      int32_t* ysel = (int32_t*)at(h, p.ysel);
      float* U = (float*)at(h, p.U);
      if (k_old == 0) RE_TRY(launch_sign_bits(s, npad_m, seed, kYSign, ybits));
      RE_TRY(launch_srct_y_lo(s, B + k_old, RE_F32, m, k - k_old, kmax, ybits, U + k_old, kmax));
      RE_TRY(launch_select(s, npad_m, l, seed, kYSel, at(h, p.selscr), ysel));  // nested in l
      RE_TRY(launch_srct_y_hi(s, U, RE_F32, m, k, kmax, ysel, l, (int32_t*)at(h, p.yord), C));
    } else {
      RE_TRY(launch_gauss_sub(s, l - l_old, m, l_old, 0, seed, kYGauss, 1, m, Y + l_old * m));
      RE_TRY(run_yb(s, B, m, k, kmax, Y, m, l, C, (YDesc*)at(h, p.ydesc), at(h, p.yparts)));
    }
    // steps 7-8
    RE_TRY(launch_svd(s, C, l, k, 1.0 / sqrt((double)k * (double)l), at(h, p.svd), sigma, info, h->spin_limit, h->xcd));
    RE_TRY(launch_rank_count(s, sigma, k, r1_from_k((int32_t)k), eps, info, out3));
    RE_TRY_HIP(hipMemcpyAsync(host, out3, 16, hipMemcpyDeviceToHost, s));
    RE_TRY_HIP(hipMemcpyAsync(host + 64, sigma, (size_t)k * 8, hipMemcpyDeviceToHost, s));
    RE_TRY_HIP(hipStreamSynchronize(s));
    ++rounds;
    const int32_t* o3 = (const int32_t*)host;
    if (o3[2] != 0) return (re_status)o3[2];
    const bool more = (o3[1] & RE_FLAG_NOT_CONVERGED) && k < kmax;
    if (!more) {
      *r_out = o3[0];
      memcpy(sigma_out, host + 64, (size_t)k * 8);
      if (k_out) *k_out = (int32_t)k;
      if (l_out) *l_out = (int32_t)l;
      if (rounds_out) *rounds_out = rounds;
      if (k_proposed_out) *k_proposed_out = kprop;
      if (flags_out) *flags_out = (uint32_t)o3[1];
      return RE_OK;
    }
    k_old = k;
    l_old = l;
    if (rounds == 1 && ad->mlp) {
      float* f = (float*)(host + 64 + (size_t)kmax * 8);
      pilot_features((const double*)(host + 64), k, m, n, eps, f);
      RE_TRY_HIP(hipMemcpyAsync(at(h, p.feat), f, RE_MLP_INPUTS * 4, hipMemcpyHostToDevice, s));
      RE_TRY(launch_mlp_forward(s, ad->mlp, (const float*)at(h, p.feat), 1, (float*)at(h, p.yout), nullptr, nullptr));
      float yv = 0.f;
      RE_TRY_HIP(hipMemcpyAsync(&yv, at(h, p.yout), 4, hipMemcpyDeviceToHost, s));
      RE_TRY_HIP(hipStreamSynchronize(s));
      double e = (double)yv + ad->delta;
      if (!(e < 30.0)) e = 30.0;  // also catches NaN
      int64_t kp = (int64_t)ceil(exp(e));
      kp = (kp + 7) / 8 * 8;
      if (kp < 2 * k_old) kp = 2 * k_old;
      if (kp > kmax) kp = kmax;
      kprop = (int32_t)kp;
      k = kp;
    } else {
      k = 2 * k < kmax ? 2 * k : kmax;
    }
  }
}

// ---- rank without a tolerance: the gap search of Sec. 6.1 -----------------
// Rounds of Algorithm 1 at k0, k0 + dk, ... with a Gaussian X whose new
// columns (and a Gaussian Y's new rows) are drawn and applied per round; an
// SRHT Y keeps its first-level transform of every column of A X (as the
// adaptive driver).  After each round's small SVD the gap statistics are
// formed on the device and the host decides whether to go on.
static re_status gap_impl(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                          const re_gap_search* gs, uint64_t seed, int32_t* r_out, double* ratio_out,
                          int32_t* argmax_out, double* argmax_ratio_out, double* sigma_out, int32_t* k_out,
                          int32_t* l_out, int32_t* rounds_out, double* spectra_out, int32_t spectra_cap,
                          uint32_t* flags_out) {
  if (!h || !A || !gs || !r_out || !sigma_out) return RE_ERR_INVALID_ARG;
  if (dt != RE_F64 && dt != RE_F32) return RE_ERR_INVALID_ARG;
  const size_t be = dt == RE_F64 ? 8 : 4;
  if (m < 1 || n < 1 || lda < n || ((uintptr_t)A) % be != 0) return RE_ERR_INVALID_ARG;
  if (dt == RE_F32 && lda >= kMaxBatchLda) return RE_ERR_UNSUPPORTED;
  if (gs->k0 < 1 || gs->dk < 1 || gs->k_max < 0 || !(gs->l_ratio >= 1.0) || !isfinite(gs->l_ratio)) return RE_ERR_INVALID_ARG;
  if (!(gs->gamma > 1.0) || !(gs->floor >= 0.0) || !isfinite(gs->floor)) return RE_ERR_INVALID_ARG;
  if (gs->y_kind != RE_GAUSSIAN && gs->y_kind != RE_SRHT && gs->y_kind != RE_SRCT) return RE_ERR_INVALID_ARG;
  if (spectra_cap < 0 || (spectra_cap > 0 && !spectra_out)) return RE_ERR_INVALID_ARG;
  int64_t kmax = m < n ? m : n;
  if (gs->k_max > 0 && gs->k_max < kmax) kmax = gs->k_max;
  if (kmax > RE_MAX_ADAPTIVE_K) kmax = RE_MAX_ADAPTIVE_K;
  const int64_t k_first = gs->k0 < kmax ? gs->k0 : kmax;
  const int64_t lmax = l_for(kmax, gs->l_ratio, m);
  const bool srht_y = gs->y_kind == RE_SRHT, srct_y = gs->y_kind == RE_SRCT, trig_y = srht_y || srct_y;
  const int64_t npad_m = srct_y ? srct_y_npad(m) : next_pow2(m);
  const int64_t xcols = k_first > gs->dk ? k_first : gs->dk;  // widest appended block of X
  size_t yparts = 0;
  if (!trig_y && dt == RE_F32) {
    for (int64_t k = k_first;; k = k + gs->dk < kmax ? k + gs->dk : kmax) {
      const size_t b = yb_scratch(l_for(k, gs->l_ratio, m), k, m);
      yparts = b > yparts ? b : yparts;
      if (k >= kmax) break;
    }
  }
  Carve c;
  const size_t oB = c.take((size_t)(srht_y ? (int64_t)srht_cols_rows_alloc(m) : m) * kmax * be);
  const size_t oX = c.take((size_t)n * xcols * be);
  const size_t oY = c.take(trig_y ? 0 : (size_t)lmax * m * be);
  const size_t oybits = c.take(trig_y ? (size_t)cdiv(npad_m, 32) * 4 : 0);
  const size_t oysel = c.take(trig_y ? (size_t)lmax * 4 : 0);
  const size_t oselscr = c.take(trig_y ? select_scratch_bytes(npad_m) : 0);
  const size_t oU = c.take(srct_y ? srct_y_u_bytes(m, kmax, dt) : 0);
  const size_t oyord = c.take(srct_y ? srct_y_order_bytes(lmax) : 0);
  const size_t oC = c.take((size_t)lmax * kmax * 8);
  const size_t osvd = c.take(svd_scratch_bytes(lmax, kmax));
  const size_t osig = c.take((size_t)kmax * 8);
  const size_t oinfo = c.take(16);
  const size_t ogap = c.take(sizeof(GapOut));
  const size_t ogd = c.take(sizeof(GemmDesc));
  const size_t oyd = c.take(sizeof(YDesc));
  const size_t oq = c.take(16);
  const size_t oparts = c.take(yparts);
  size_t gp = 0;  // K-split partials of the FP64 products, the largest over the rounds
  if (dt == RE_F64) {
    for (int64_t k = k_first, ko = 0;; ko = k, k = k + gs->dk < kmax ? k + gs->dk : kmax) {
      const size_t gx = gemm64_parts_bytes(m, k - ko, n);
      const size_t gy = trig_y ? 0 : gemm64_parts_bytes(l_for(k, gs->l_ratio, m), k, m);
      gp = gx > gp ? gx : gp;
      gp = gy > gp ? gy : gp;
      if (k >= kmax) break;
    }
  }
  const size_t ogp = c.take(gp);
  RE_TRY(ensure_ws(h, c.off));
  RE_TRY(ensure_host(h, 64 + (size_t)kmax * 8));
  hipStream_t s = h->stream;
  char* host = (char*)h->host;
  char* B = at(h, oB);
  char* Xn = at(h, oX);
  char* Y = at(h, oY);
  double* C = (double*)at(h, oC);
  double* sigma = (double*)at(h, osig);
  int32_t* info = (int32_t*)at(h, oinfo);
  GapOut* gout = (GapOut*)at(h, ogap);
  int64_t k_old = 0, l_old = 0, k = k_first;
  int32_t rounds = 0, prev_g = -1;
  double acc_ms[RE_NUM_STAGES] = {};  // stage times summed over the rounds (profiling)
  for (;;) {
    const int64_t l = l_for(k, gs->l_ratio, m), dkr = k - k_old;
    // Algorithm 1 steps 2-3 on the appended columns only
    mark(h, RE_STAGE_X_DRAW);
    if (dt == RE_F32) {
      RE_TRY(launch_gauss_sub(s, n, dkr, 0, k_old, seed, kXGauss, 0, dkr, (float*)Xn));
      mark(h, RE_STAGE_AX);
      RE_TRY(launch_gemm_f32_single(s, (const float*)A, m, n, lda, (const float*)Xn, dkr, (float*)B + k_old, kmax,
                                    (GemmDesc*)at(h, ogd), (unsigned*)at(h, oq)));
    } else {
      RE_TRY(launch_gauss_sub64(s, n, dkr, 0, k_old, seed, kXGauss, 0, dkr, (double*)Xn));
      mark(h, RE_STAGE_AX);
      RE_TRY(launch_gemm64(s, m, dkr, n, (const double*)A, lda, (const double*)Xn, dkr, (double*)B + k_old, kmax,
                           (double*)at(h, ogp)));
    }
    // steps 4-6
    mark(h, RE_STAGE_Y_DRAW);
    if (srht_y) {
      uint32_t* ybits = (uint32_t*)at(h, oybits);
      int32_t* ysel = (int32_t*)at(h, oysel);
      if (k_old == 0) RE_TRY(launch_sign_bits(s, npad_m, seed, kYSign, ybits));
      RE_TRY(launch_select(s, npad_m, l, seed, kYSel, at(h, oselscr), ysel));  // nested in l
      mark(h, RE_STAGE_YB);
      RE_TRY(launch_srht_cols_lo(s, B + (size_t)k_old * be, dt, m, dkr, kmax, ybits));
      RE_TRY(launch_srht_cols_hi(s, B, dt, m, k, kmax, ysel, l, C));
    } else if (srct_y) {  // the stored first level U of the DCT along m, new columns only
      uint32_t* ybits = (uint32_t*)at(h, oybits);
      int32_t* ysel = (int32_t*)at(h, oysel);
      char* U = at(h, oU);
      if (k_old == 0) RE_TRY(launch_sign_bits(s, npad_m, seed, kYSign, ybits));
      RE_TRY(launch_select(s, npad_m, l, seed, kYSel, at(h, oselscr), ysel));  // nested in l
      mark(h, RE_STAGE_YB);
      RE_TRY(launch_srct_y_lo(s, B + (size_t)k_old * be, dt, m, dkr, kmax, ybits, U + (size_t)k_old * be, kmax));
      RE_TRY(launch_srct_y_hi(s, U, dt, m, k, kmax, ysel, l, (int32_t*)at(h, oyord), C));
    } else if (dt == RE_F32) {
      RE_TRY(launch_gauss_sub(s, l - l_old, m, l_old, 0, seed, kYGauss, 1, m, (float*)Y + l_old * m));
      mark(h, RE_STAGE_YB);
      RE_TRY(run_yb(s, (const float*)B, m, k, kmax, (const float*)Y, m, l, C, (YDesc*)at(h, oyd), at(h, oparts)));
    } else {
      RE_TRY(launch_gauss_sub64(s, l - l_old, m, l_old, 0, seed, kYGauss, 1, m, (double*)Y + l_old * m));
      mark(h, RE_STAGE_YB);
      RE_TRY(launch_gemm64(s, l, k, m, (const double*)Y, m, (const double*)B, kmax, C, k, (double*)at(h, ogp)));
    }
    // steps 7-8, the gap statistics in place of the count
    const int32_t r1 = r1_from_k((int32_t)k);
    mark(h, RE_STAGE_SVD);
    RE_TRY(launch_svd(s, C, l, k, 1.0 / sqrt((double)k * (double)l), at(h, osvd), sigma, info, h->spin_limit, h->xcd));
    mark(h, RE_STAGE_RANK);
    RE_TRY(launch_gap(s, sigma, k, r1, gs->gamma, gs->floor, info, gout));
    RE_TRY_HIP(hipMemcpyAsync(host, gout, sizeof(GapOut), hipMemcpyDeviceToHost, s));
    RE_TRY_HIP(hipMemcpyAsync(host + 64, sigma, (size_t)k * 8, hipMemcpyDeviceToHost, s));
    mark(h, RE_NUM_STAGES);
    RE_TRY_HIP(hipStreamSynchronize(s));
    if (h->prof) {
      for (int i = 0; i < RE_NUM_STAGES; ++i) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess) acc_ms[i] += (double)ms;
      }
      for (int i = 0; i < RE_NUM_STAGES; ++i) h->stage_ms[i] = acc_ms[i];
    }
    GapOut go;
    memcpy(&go, host, sizeof(go));
    if (go.status != 0) return (re_status)go.status;
    if (spectra_out && rounds < spectra_cap) {
      double* row = spectra_out + (size_t)rounds * kmax;
      memcpy(row, host + 64, (size_t)k * 8);
      for (int64_t j = k; j < kmax; ++j) row[j] = 0.0;
    }
    ++rounds;
    const bool zero = !(go.s1 > 0.0);
    const bool done = !zero && go.g > 0 && go.g == prev_g && go.reached;
    if (zero || done || k >= kmax) {
      *r_out = zero ? 0 : go.g;
      if (ratio_out) *ratio_out = zero ? 0.0 : go.ratio_g;
      if (argmax_out) *argmax_out = zero ? 0 : go.a;
      if (argmax_ratio_out) *argmax_ratio_out = zero ? 0.0 : go.ratio_a;
      memcpy(sigma_out, host + 64, (size_t)k * 8);
      if (k_out) *k_out = (int32_t)k;
      if (l_out) *l_out = (int32_t)l;
      if (rounds_out) *rounds_out = rounds;
      if (flags_out) *flags_out = zero ? (uint32_t)RE_FLAG_ZERO : done ? 0u : (uint32_t)RE_FLAG_NOT_CONVERGED;
      return RE_OK;
    }
    prev_g = go.g;
    k_old = k;
    l_old = l;
    k = k + gs->dk < kmax ? k + gs->dk : kmax;
  }
}

RE_API re_status re_rank_gap(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                             const re_gap_search* gs, uint64_t seed, int32_t* r_out, double* ratio_out,
                             int32_t* argmax_out, double* argmax_ratio_out, double* sigma_out, int32_t* k_out,
                             int32_t* l_out, int32_t* rounds_out, double* spectra_out, int32_t spectra_cap,
                             uint32_t* flags_out) {
  return gap_impl(h, A, dt, m, n, lda, gs, seed, r_out, ratio_out, argmax_out, argmax_ratio_out, sigma_out, k_out,
                  l_out, rounds_out, spectra_out, spectra_cap, flags_out);
}

RE_API re_status re_rank_adaptive(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                                  double eps, const re_adaptive* ad, uint64_t seed, int32_t* r_out, double* sigma_out,
                                  int32_t* k_out, int32_t* l_out, int32_t* rounds_out, int32_t* k_proposed_out,
                                  uint32_t* flags_out) {
  return adaptive_impl(h, A, dt, m, n, lda, eps, ad, RE_GAUSSIAN, seed, r_out, sigma_out, k_out, l_out, rounds_out,
                       k_proposed_out, flags_out);
}

RE_API re_status re_rank_adaptive_y(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                                    double eps, const re_adaptive* ad, int32_t y_kind, uint64_t seed, int32_t* r_out,
                                    double* sigma_out, int32_t* k_out, int32_t* l_out, int32_t* rounds_out,
                                    int32_t* k_proposed_out, uint32_t* flags_out) {
  return adaptive_impl(h, A, dt, m, n, lda, eps, ad, y_kind, seed, r_out, sigma_out, k_out, l_out, rounds_out,
                       k_proposed_out, flags_out);
}

namespace re {
namespace {

// Thin QR of the m x w matrix V (FP32 if v32, else FP64; leading dimension
// ldv) by shifted CholeskyQR3: the kept columns of Q go to Q (ldq), their
// number to *w_eff.  Synchronises the stream once, before the last product.
re_status rf_qr(re_handle h, const void* V, bool v32, int64_t m, int64_t w, int64_t ldv, double* Q, int64_t ldq,
                int32_t* w_eff, double* rdiag3 = nullptr) {
  hipStream_t s = h->stream;
  int64_t gs = 0, grps = 0;
  rf_row_split(m, cdiv(w, 64) * (cdiv(w, 64) + 1) / 2, &gs, &grps);
  Carve c;
  const size_t oQ1 = c.take((size_t)m * w * 8), oQ2 = c.take((size_t)m * w * 8);
  const size_t oG = c.take((size_t)w * w * 8), oRi = c.take((size_t)w * w * 8);
  const size_t oKeep = c.take((size_t)w * 4), oCnt = c.take(16);
  const size_t oParts = c.take((size_t)gs * w * w * 8);
  RE_TRY(ensure_ws2(h, c.off));
  RE_TRY(ensure_host(h, 64));
  char* base = (char*)h->ws2;
  double* Q1 = (double*)(base + oQ1);
  double* Q2 = (double*)(base + oQ2);
  double* G = (double*)(base + oG);
  double* Ri = (double*)(base + oRi);
  int32_t* keep = (int32_t*)(base + oKeep);
  int32_t* cnt = (int32_t*)(base + oCnt);
  double* parts = (double*)(base + oParts);
  const void* Vin[3] = {V, Q1, Q2};
  const int64_t ldin[3] = {ldv, w, w};
  double* Vout[2] = {Q1, Q2};
  for (int pass = 0; pass < 3; ++pass) {
    const bool f32 = pass == 0 && v32;
    RE_TRY(launch_rf_gram(s, Vin[pass], f32, m, w, ldin[pass], gs, grps, parts));
    RE_TRY(launch_rf_sum_parts(s, parts, gs, w, w, true, G, w));
    RE_TRY(launch_rf_chol(s, G, w, pass == 0, m, Ri, keep, cnt, rdiag3 ? rdiag3 + pass * w : nullptr));
    if (pass < 2) {
      RE_TRY(launch_rf_apply(s, Vin[pass], f32, m, w, ldin[pass], Ri, nullptr, Vout[pass], w));
      continue;
    }
    char* host = (char*)h->host;
    RE_TRY_HIP(hipMemcpyAsync(host + 16, cnt, 8, hipMemcpyDeviceToHost, s));
    RE_TRY_HIP(hipStreamSynchronize(s));
    const int32_t* c8 = (const int32_t*)(host + 16);
    if (c8[1] != 0) return (re_status)c8[1];
    *w_eff = c8[0];
    if (Q) RE_TRY(launch_rf_apply(s, Vin[pass], false, m, w, ldin[pass], Ri, keep, Q, ldq));
  }
  return RE_OK;
}

// B (ldb) = Q^T A for the w columns of Q (ldq) and FP32 A (lda).
re_status rf_project(re_handle h, const double* Q, int64_t ldq, int64_t w, const float* A, int64_t m, int64_t n,
                     int64_t lda, double* B, int64_t ldb) {
  hipStream_t s = h->stream;
  const int64_t mc = w >= 128 ? 4 : cdiv(w, 32);
  int64_t qs = 0, qrps = 0;
  rf_row_split(m, cdiv(w, 32 * mc) * rf_qta_col_tiles(n), &qs, &qrps);
  Carve c;
  const size_t oParts = c.take((size_t)qs * w * n * 8), oQ32 = c.take((size_t)m * w * 4);
  RE_TRY(ensure_ws2(h, c.off));
  double* parts = (double*)((char*)h->ws2 + oParts);
  RE_TRY(launch_rf_qta(s, Q, ldq, w, A, m, n, lda, qs, qrps, (float*)((char*)h->ws2 + oQ32), parts));
  return launch_rf_sum_parts(s, parts, qs, w, n, false, B, ldb);
}

}  // namespace
}  // namespace re

RE_API re_status re_rank_estimate_qr(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                                     double eps, const re_sketch* sk, uint64_t seed, int32_t* r_out, double* sigma_out,
                                     int32_t* r1_out, uint32_t* flags_out) {
  if (!h || !r_out || !sigma_out) return RE_ERR_INVALID_ARG;
  if (!(eps > 0.0 && eps < 1.0)) return RE_ERR_INVALID_ARG;
  Resolved rs;
  RE_TRY(validate(A, dt, m, n, lda, sk, &rs));
  if (sk->prec != RE_PREC_NATIVE) return RE_ERR_UNSUPPORTED;
  if (rs.k > 46340) return RE_ERR_INVALID_ARG;
  rs.fmt_x = x_fmt(dt);
  const Plan p = plan(dt, m, n, rs);
  RE_TRY(ensure_ws(h, p.total));
  RE_TRY(ensure_host(h, (size_t)rs.k * 8 + 64));
  hipStream_t s = h->stream;
  void* B = at(h, p.B);
  double* C = (double*)at(h, p.C);
  double* sigma = (double*)at(h, p.sigma);
  int32_t* out3 = (int32_t*)at(h, p.out3);
  double* rdiag3 = (double*)at(h, p.rdiag);
  mark(h, RE_STAGE_X_DRAW);
  RE_TRY(run_x(h, p, A, dt, m, n, lda, rs, seed, B));
  mark(h, RE_STAGE_Y_DRAW);
  RE_TRY(run_y(h, p, B, dt, m, rs, seed, C));
  mark(h, RE_STAGE_SVD);
  int32_t w_eff = 0;
  RE_TRY(rf_qr(h, C, false, rs.l, rs.k, rs.k, nullptr, 0, &w_eff, rdiag3));
  RE_TRY(launch_qr_sigma(s, rdiag3, rs.k, 1.0 / sqrt((double)rs.k * (double)rs.l), sigma));
  mark(h, RE_STAGE_RANK);
  const int32_t r1 = r1_from_k((int32_t)rs.k);
  RE_TRY(launch_rank_count(s, sigma, rs.k, r1, eps, nullptr, out3));
  char* host = (char*)h->host;
  RE_TRY_HIP(hipMemcpyAsync(host, out3, 16, hipMemcpyDeviceToHost, s));
  RE_TRY_HIP(hipMemcpyAsync(host + 64, sigma, (size_t)rs.k * 8, hipMemcpyDeviceToHost, s));
  mark(h, RE_NUM_STAGES);
  RE_TRY_HIP(hipStreamSynchronize(s));
  if (h->prof) {
    for (int i = 0; i < RE_NUM_STAGES; ++i) {
      float ms = 0.f;
      h->stage_ms[i] = hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess ? (double)ms : -1.0;
    }
  }
  const int32_t* o3 = (const int32_t*)host;
  if (o3[2] != 0) return (re_status)o3[2];
  *r_out = o3[0];
  memcpy(sigma_out, host + 64, (size_t)rs.k * 8);
  if (r1_out) *r1_out = r1;
  if (flags_out) *flags_out = (uint32_t)o3[1];
  return RE_OK;
}

RE_API re_status re_rangefinder(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda, double eps,
                                int32_t p, const re_adaptive* ad, double norm_a, uint64_t seed, double* Q, int64_t ldq,
                                double* Bq, int64_t ldb, int32_t* r_out, int32_t* w_out, double* sigma_out,
                                int32_t* k_out, uint32_t* flags_out) {
  if (!h || !A || !ad || !Q || !Bq || !r_out || !w_out || !sigma_out) return RE_ERR_INVALID_ARG;
  if (dt != RE_F64 && dt != RE_F32) return RE_ERR_INVALID_ARG;
  if (dt != RE_F32 || ad->mlp) return RE_ERR_UNSUPPORTED;
  if (!(eps > 0.0 && eps < 1.0) || m < 1 || n < 1 || lda < n || lda >= kMaxBatchLda || ((uintptr_t)A) % 4 != 0)
    return RE_ERR_INVALID_ARG;
  if (ad->k0 < 1 || !(ad->l_ratio >= 1.0) || ad->k_max < 0 || !isfinite(norm_a) || norm_a < 0.0)
    return RE_ERR_INVALID_ARG;
  int64_t kmax = m < n ? m : n;
  if (ad->k_max > 0 && ad->k_max < kmax) kmax = ad->k_max;
  if (kmax > RE_MAX_ADAPTIVE_K) kmax = RE_MAX_ADAPTIVE_K;
  if (p < 2 || p >= kmax || ldq < kmax || ldb < n) return RE_ERR_INVALID_ARG;
  const int64_t lmax = l_for(kmax, ad->l_ratio, m);
  AdPlan pl{};
  Carve c;
  pl.B = c.take((size_t)m * kmax * 4);
  pl.Xn = c.take((size_t)n * kmax * 4);
  pl.Y = c.take((size_t)lmax * m * 4);
  pl.C = c.take((size_t)lmax * kmax * 8);
  pl.svd = c.take(svd_scratch_bytes(lmax, kmax));
  pl.sigma = c.take((size_t)kmax * 8);
  pl.info = c.take(16);
  pl.out3 = c.take(16);
  pl.gdesc = c.take(sizeof(GemmDesc));
  pl.ydesc = c.take(sizeof(YDesc));
  pl.queue = c.take(16);
  pl.yparts = c.take(yb_scratch_adaptive(ad->k0, kmax, ad->l_ratio, m));
  const size_t oTail = c.take((size_t)(kmax + 1) * 8);
  pl.total = c.off;
  RE_TRY(ensure_ws(h, pl.total));
  RE_TRY(ensure_host(h, 256 + (size_t)kmax * 8));
  hipStream_t s = h->stream;
  char* host = (char*)h->host;
  float* B = (float*)at(h, pl.B);
  float* Y = (float*)at(h, pl.Y);
  double* C = (double*)at(h, pl.C);
  double* sigma = (double*)at(h, pl.sigma);
  int32_t* info = (int32_t*)at(h, pl.info);
  int32_t* out4 = (int32_t*)at(h, pl.out3);
  mark(h, 0);
  // 1-2: rank estimation with appended sketches until the width rule finds r
  int64_t k_old = 0, l_old = 0, k = ad->k0 < kmax ? ad->k0 : kmax;
  const int32_t* o4 = (const int32_t*)host;
  for (;;) {
    const int64_t l = l_for(k, ad->l_ratio, m);
    RE_TRY(launch_gauss_sub(s, n, k - k_old, 0, k_old, seed, kXGauss, 0, k - k_old, (float*)at(h, pl.Xn)));
    RE_TRY(launch_gemm_f32_single(s, (const float*)A, m, n, lda, (const float*)at(h, pl.Xn), k - k_old, B + k_old, kmax,
                                  (GemmDesc*)at(h, pl.gdesc), (unsigned*)at(h, pl.queue)));
    RE_TRY(launch_gauss_sub(s, l - l_old, m, l_old, 0, seed, kYGauss, 1, m, Y + l_old * m));
    RE_TRY(run_yb(s, B, m, k, kmax, Y, m, l, C, (YDesc*)at(h, pl.ydesc), at(h, pl.yparts)));
    RE_TRY(launch_svd(s, C, l, k, 1.0 / sqrt((double)k * (double)l), at(h, pl.svd), sigma, info, h->spin_limit, h->xcd));
    RE_TRY(launch_rf_width(s, sigma, k, r1_from_k((int32_t)k), n, eps, p, norm_a, info, (double*)at(h, oTail), out4));
    RE_TRY_HIP(hipMemcpyAsync(host, out4, 16, hipMemcpyDeviceToHost, s));
    RE_TRY_HIP(hipMemcpyAsync(host + 64, sigma, (size_t)k * 8, hipMemcpyDeviceToHost, s));
    RE_TRY_HIP(hipStreamSynchronize(s));
    if (o4[2] != 0) return (re_status)o4[2];
    if (o4[0] >= 0 || k >= kmax) break;
    k_old = k;
    l_old = l;
    k = 2 * k < kmax ? 2 * k : kmax;
  }
  const int32_t r = o4[0];
  uint32_t flags = (uint32_t)o4[3];
  int32_t w_eff = 0;
  mark(h, 1);
  if (r > 0) {
    const int64_t w = o4[1];
    RE_TRY(rf_qr(h, B, true, m, w, kmax, Q, ldq, &w_eff));  // 3: thin QR of A X[:, :w]
    if (w_eff < w) flags |= RE_FLAG_COLUMNS_DROPPED;
    mark(h, 2);
    if (w_eff > 0) RE_TRY(rf_project(h, Q, ldq, w_eff, (const float*)A, m, n, lda, Bq, ldb));  // 4: B = Q^T A
  } else {
    mark(h, 2);
  }
  mark(h, 3);
  RE_TRY_HIP(hipStreamSynchronize(s));
  if (h->prof) {
    for (int i = 0; i < 3; ++i) {
      float ms = 0.f;
      h->rf_ms[i] = hipEventElapsedTime(&ms, h->ev[i], h->ev[i + 1]) == hipSuccess ? (double)ms : -1.0;
    }
  }
  *r_out = r;
  *w_out = w_eff;
  memcpy(sigma_out, host + 64, (size_t)k * 8);
  if (k_out) *k_out = (int32_t)k;
  if (flags_out) *flags_out = flags;
  return RE_OK;
}

RE_API re_status re_thin_qr(re_handle h, const void* W, int32_t dt, int64_t m, int64_t w, int64_t ldw, double* Q,
                            int64_t ldq, int32_t* w_out, uint32_t* flags_out) {
  if (!h || !W || !Q || !w_out) return RE_ERR_INVALID_ARG;
  if (dt != RE_F64 && dt != RE_F32) return RE_ERR_INVALID_ARG;
  if (w < 1 || m < w || ldw < w || ldq < w || w > 46340 || ((uintptr_t)W) % (dt == RE_F64 ? 8 : 4) != 0)
    return RE_ERR_INVALID_ARG;
  int32_t we = 0;
  RE_TRY(rf_qr(h, W, dt == RE_F32, m, w, ldw, Q, ldq, &we));
  RE_TRY_HIP(hipStreamSynchronize(h->stream));
  *w_out = we;
  if (flags_out) *flags_out = we < w ? RE_FLAG_COLUMNS_DROPPED : 0u;
  return RE_OK;
}

RE_API re_status re_project(re_handle h, const double* Q, int64_t ldq, int64_t w, const void* A, int32_t dt, int64_t m,
                            int64_t n, int64_t lda, double* B, int64_t ldb) {
  if (!h || !Q || !A || !B) return RE_ERR_INVALID_ARG;
  if (dt != RE_F64 && dt != RE_F32) return RE_ERR_INVALID_ARG;
  if (dt != RE_F32) return RE_ERR_UNSUPPORTED;
  if (w < 1 || m < 1 || n < 1 || ldq < w || lda < n || ldb < n || ((uintptr_t)A) % 4 != 0) return RE_ERR_INVALID_ARG;
  return rf_project(h, Q, ldq, w, (const float*)A, m, n, lda, B, ldb);
}

RE_API re_status re_rangefinder_stage_ms(re_handle h, double* ms) {
  if (!h || !ms || !h->prof) return RE_ERR_INVALID_ARG;
  for (int i = 0; i < 3; ++i) ms[i] = h->rf_ms[i];
  return RE_OK;
}

RE_API re_status re_philox(re_handle h, const uint64_t* ctr, uint64_t seed, int64_t count, uint64_t* out) {
  if (!h || count < 0 || (count > 0 && (!ctr || !out))) return RE_ERR_INVALID_ARG;
  return launch_philox(h->stream, ctr, seed, count, out);
}

RE_API re_status re_gauss_fill(re_handle h, int32_t fmt, int64_t rows, int64_t cols, uint64_t seed, int32_t stream_id,
                               int32_t swap_ab, void* out) {
  if (!h || rows < 0 || cols < 0 || fmt < 0 || fmt > 3 || (rows * cols > 0 && !out)) return RE_ERR_INVALID_ARG;
  return launch_gauss_fill(h->stream, fmt, rows, cols, seed, stream_id, swap_ab, out);
}

RE_API re_status re_srht_signs(re_handle h, int64_t npad, uint64_t seed, int32_t stream_id, uint32_t* bits) {
  if (!h || npad < 0 || (npad > 0 && !bits)) return RE_ERR_INVALID_ARG;
  return launch_sign_bits(h->stream, npad, seed, stream_id, bits);
}

RE_API re_status re_srht_select(re_handle h, int64_t npad, int64_t k, uint64_t seed, int32_t stream_id, int32_t* idx) {
  if (!h || npad < 1 || k < 0 || k > npad || npad > (int64_t)INT32_MAX || (k > 0 && !idx)) return RE_ERR_INVALID_ARG;
  RE_TRY(ensure_ws(h, select_scratch_bytes(npad)));
  return launch_select(h->stream, npad, k, seed, stream_id, h->ws, idx);
}

RE_API re_status re_sketch_x(re_handle h, const void* A, int32_t dt, int64_t m, int64_t n, int64_t lda,
                             const re_sketch* sk, uint64_t seed, void* B) {
  if (!h || !B) return RE_ERR_INVALID_ARG;
  Resolved rs;
  RE_TRY(validate(A, dt, m, n, lda, sk, &rs, 1));
  if (sk->prec == RE_PREC_AUTO) return RE_ERR_INVALID_ARG;  // the stage call needs an explicit format
  rs.fmt_x = sk->prec == RE_PREC_BF16 ? kBF16 : sk->prec == RE_PREC_FP16 ? kF16 : x_fmt(dt);
  rs.lowprec = rs.fmt_x == kBF16 || rs.fmt_x == kF16;
  const Plan p = plan(dt, m, n, rs);
  RE_TRY(ensure_ws(h, p.total));
  if (rs.fmt_x == kF16) {
    double* st = (double*)at(h, p.stats);
    RE_TRY(launch_sample_stats(h->stream, (const float*)A, m, n, lda, st));
    RE_TRY(ensure_host(h, 32));
    double* stats = (double*)h->host;  // pinned: the copy stays asynchronous
    RE_TRY_HIP(hipMemcpyAsync(stats, st, 3 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    RE_TRY_HIP(hipStreamSynchronize(h->stream));
    if (stats[1] > 0.0) {
      int e2 = 0;
      frexp(stats[1], &e2);
      rs.scale_exp = 12 - e2;
    }
  }
  return run_x(h, p, A, dt, m, n, lda, rs, seed, B);
}

RE_API int64_t re_sketch_y_rows(int64_t m) { return (int64_t)srht_cols_rows_alloc(m); }

RE_API re_status re_sketch_y(re_handle h, void* B, int32_t bdt, int64_t m, int64_t k, const re_sketch* sk,
                             uint64_t seed, double* C) {
  if (!h || !B || !C || !sk || m < 1 || k < 1 || sk->k != k) return RE_ERR_INVALID_ARG;
  Resolved rs;
  // validate the Y side only: a stand-in A of m x k with lda = k
  RE_TRY(validate(B, bdt, m, k, k, sk, &rs, 2));
  const Plan p = plan(bdt, m, k, rs);
  RE_TRY(ensure_ws(h, p.total));
  return run_y(h, p, B, bdt, m, rs, seed, C);
}

RE_API re_status re_singular_values(re_handle h, const double* C, int64_t l, int64_t k, double scale, double* sigma) {
  if (!h || !C || !sigma || k < 1 || l < k) return RE_ERR_INVALID_ARG;
  const size_t need = al256(svd_scratch_bytes(l, k)) + 256;
  RE_TRY(ensure_ws(h, need));
  RE_TRY(ensure_host(h, 64));
  int32_t* info = (int32_t*)((char*)h->ws + al256(svd_scratch_bytes(l, k)));
  RE_TRY(launch_svd(h->stream, C, l, k, scale, h->ws, sigma, info, h->spin_limit, h->xcd));
  // the device status (NaN / Inf in C, a grid barrier that gave up)
  RE_TRY_HIP(hipMemcpyAsync(h->host, info, sizeof(int32_t), hipMemcpyDeviceToHost, h->stream));
  RE_TRY_HIP(hipStreamSynchronize(h->stream));
  return (re_status) * (const int32_t*)h->host;
}

// ---- allocation-free singular values ------------------------------------
// The working memory of re_singular_values_noalloc: one fixed array per GPU
// (each device holds its own copy of a __device__ variable).  Host code uses
// the device address obtained from hipGetSymbolAddress on each device, never
// the name of the array itself.
__device__ __align__(256) unsigned char scratch[RE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxNoallocDevices = 64;
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kMaxNoallocDevices] = {};

size_t noalloc_need(int64_t l, int64_t k) { return al256(svd_scratch_bytes(l, k)) + 256; }

// Device address of `scratch` on the current device, looked up once per device.
re_status noalloc_scratch(char** out) {
  int dev = 0;
  RE_TRY_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxNoallocDevices) return RE_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    RE_TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RE_ERR_HIP;
    g_noalloc_ptr[dev] = (char*)p;
  }
  *out = g_noalloc_ptr[dev];
  return RE_OK;
}
}  // namespace

RE_API int32_t re_singular_values_noalloc_fits(int64_t l, int64_t k) {
  if (k < 1 || l < k) return 0;
  if ((double)l * (double)k * 8.0 > (double)RE_NOALLOC_SCRATCH_BYTES) return 0;
  return noalloc_need(l, k) <= RE_NOALLOC_SCRATCH_BYTES ? 1 : 0;
}

RE_API re_status re_singular_values_noalloc(void* hip_stream, const double* C, int64_t l, int64_t k, double scale,
                                            double* sigma) {
  if (!C || !sigma || k < 1 || l < k) return RE_ERR_INVALID_ARG;
  if (!re_singular_values_noalloc_fits(l, k)) return RE_ERR_SCRATCH_LIMIT;
  char* base = nullptr;
  RE_TRY(noalloc_scratch(&base));
  int32_t* info = (int32_t*)(base + al256(svd_scratch_bytes(l, k)));
  // launch_svd clears its barrier counter and status word with a kernel before
  // use, so what an earlier call left in the array does not matter.
  return launch_svd((hipStream_t)hip_stream, C, l, k, scale, base, sigma, info);
}

RE_API re_status re_rank_count(re_handle h, const double* sigma, int64_t k, int32_t r1, double eps, int32_t* out) {
  if (!h || !sigma || !out || k < 1 || r1 < 1 || !(eps > 0.0 && eps < 1.0)) return RE_ERR_INVALID_ARG;
  return launch_rank_count(h->stream, sigma, k, r1, eps, nullptr, out);
}

RE_API const char* re_status_string(re_status s) {
  switch (s) {
    case RE_OK: return "ok";
    case RE_ERR_INVALID_ARG: return "invalid argument";
    case RE_ERR_UNSUPPORTED: return "unsupported combination";
    case RE_ERR_NO_MEMORY: return "out of device or pinned memory";
    case RE_ERR_HIP: return "HIP runtime error";
    case RE_ERR_NONFINITE: return "non-finite values in the input or the sketch";
    case RE_ERR_NO_CONVERGENCE: return "small SVD did not complete";
    case RE_ERR_SCRATCH_LIMIT: return "input larger than the fixed scratch of the allocation-free call";
    default: return "unknown status";
  }
}
