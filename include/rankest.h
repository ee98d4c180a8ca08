/*
 * rankest.h — C ABI of librankest, an MI355X (gfx950) implementation of the
 * two-sided sketched numerical-rank estimator of M. Meier and Y. Nakatsukasa,
 * "Fast Randomized Numerical Rank Estimation for Numerically Low-Rank
 * Matrices" (arXiv 2105.07388), Algorithm 1 (Sec. 5).
 *
 * Given an m x n matrix A in device memory, a relative tolerance eps and a
 * sketch width k = round(1.1 r1) (r1 = the rank upper bound of Algorithm 1),
 * the library forms the sketch Y A X (X: n x k, Y: l x m random embeddings),
 * computes its singular values in FP64, scales them by 1/sqrt(k l) (the
 * embedding normalisations of Sec. 1, X = G/sqrt(k), and Eq. (Theta)), and
 * counts those above eps * sigma_1 among the first r1 (Def. 1, Algorithm 1
 * steps 7-8).
 *
 * Conventions for every entry point:
 *   - Matrices are row-major with a leading dimension in elements.
 *   - "device" pointers are memory allocated on the handle's GPU; "host"
 *     pointers are ordinary host memory.  The caller owns all pointers it
 *     passes; the library owns only the workspace inside the handle.
 *   - Calls enqueue work on the handle's stream.  Entry points that write to
 *     host memory synchronise that stream before returning; entry points that
 *     write only device memory return without synchronising.
 *   - Every call returns a re_status.  On error nothing has been written to
 *     the host outputs; device outputs may hold partial results.  No entry
 *     point prints, aborts or throws.
 *   - A handle is not thread-safe: use one handle per host thread.
 */
#ifndef RANKEST_H
#define RANKEST_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RE_OK = 0,
  RE_ERR_INVALID_ARG = -1,   /* an argument is out of range or a pointer is NULL */
  RE_ERR_UNSUPPORTED = -2,   /* a valid combination this build does not implement */
  RE_ERR_NO_MEMORY = -3,     /* a workspace allocation failed */
  RE_ERR_HIP = -4,           /* a HIP runtime call failed */
  RE_ERR_NONFINITE = -5,     /* A (or the sketch) holds NaN or Inf */
  RE_ERR_NO_CONVERGENCE = -6, /* the small SVD did not converge */
  RE_ERR_SCRATCH_LIMIT = -7   /* the input needs more than the fixed scratch of an allocation-free call */
} re_status;

/* Storage type of A. */
typedef enum { RE_F64 = 0, RE_F32 = 1 } re_dtype;

/* Random embedding families (Sec. 3.3, Sec. 4): a Gaussian embedding, or a
 * subsampled randomized Hadamard transform sqrt(N/k) S H D (Eq. (Theta), with
 * the Hadamard matrix as the trigonometric transform and N = the dimension
 * zero-padded to a power of two, any N up to 2^30 for either storage type),
 * or (X only) a hashed randomized DCT H F D
 * (Sec. 3.3: a CountSketch H in place of the sampling S, F the orthonormal
 * DCT-II of length N = max(2, next power of two >= n); the paper's
 * experimental X) or the subsampled randomized DCT sqrt(N/k) S F D (the
 * SRHT's signs D and sample S over that N), as X or as Y (Sec. 6 uses it for
 * Theta = Y; along the m rows of B = A X, M = max(2, next power of two >= m),
 * the Y stream's signs and sample, any storage type of A).  As X the two DCT
 * kinds need FP32 A with N <= 2^20, k <= 16384 for the hashed DCT when
 * N > 16384, and native precision (else RE_ERR_UNSUPPORTED); the hashed DCT
 * as a Y is rejected (RE_ERR_INVALID_ARG). */
typedef enum { RE_GAUSSIAN = 0, RE_SRHT = 1, RE_HRTT = 2, RE_SRCT = 3 } re_kind;

/* Arithmetic of the A X contraction.  NATIVE: the storage type of A.
 * BF16 / FP16: A (FP32 only) and a Gaussian X rounded to that format on the
 * matrix cores, FP32 accumulation; FP16 first scales A by an exact power of
 * two so that its sampled largest entry sits near 2^12.
 * AUTO: BF16, then FP16, then FP32, keeping the first whose rounding floor
 * phi = (u / sqrt(3)) ||A||_F (1/sqrt(k) + 1/sqrt(m)) (||A||_F from a sample
 * of A's entries) is at most eps * sigma_1 / 4, with sigma_1 the estimate the
 * sketch itself returns; a rejected format costs one more pass over A. */
typedef enum { RE_PREC_NATIVE = 0, RE_PREC_BF16 = 1, RE_PREC_FP16 = 2, RE_PREC_AUTO = 3 } re_prec;

/* The sketch of Algorithm 1: X is n x k (k = round(1.1 r1), step 1) and Y is
 * l x m (l = r2, step 4; 0 selects the paper's r2 = 2k). */
typedef struct {
  int32_t x_kind; /* re_kind of X */
  int32_t y_kind; /* re_kind of Y */
  int32_t k;      /* columns of X, 1 <= k <= n (n rounded up to a power of two for SRHT) */
  int32_t l;      /* rows of Y, k <= l <= m (m rounded up for SRHT); 0 means 2k */
  int32_t prec;   /* re_prec */
} re_sketch;

/* Result flags. */
enum {
  RE_FLAG_NOT_CONVERGED = 1u, /* all of the first r1 estimates exceed eps*sigma_1: rank >= r1 (Algorithm 1 step 8) */
  RE_FLAG_ZERO = 2u,          /* sigma_1 of the sketch is zero */
  RE_FLAG_PREC_FALLBACK = 4u, /* AUTO could not use a low-precision format */
  RE_FLAG_USED_BF16 = 8u,     /* the A X contraction ran in BF16 */
  RE_FLAG_USED_FP16 = 16u,    /* the A X contraction ran in FP16 */
  RE_FLAG_COLUMNS_DROPPED = 32u, /* re_rangefinder: columns of A X dependent at FP64 precision were left out of Q */
  RE_FLAG_PREC_BELOW_FLOOR = 64u, /* a forced BF16 / FP16 contraction: its error floor phi_f exceeds eps*sigma_1/4, so
                                    estimates near the threshold are not resolved (AUTO would have moved on) */
  RE_FLAG_SVD_RELAUNCHED = 128u  /* re_rank_estimate: the small SVD, launched without the cooperative form so
                                    that estimates on other streams could overlap it, waited past its short poll
                                    limit for a free CU and was run again with the default limit (same result,
                                    more time) */
};

typedef struct re_handle_s* re_handle;

/* Create a handle bound to the current HIP device and to `hip_stream`
 * (a hipStream_t; NULL = the default stream).  *h receives the handle. */
re_status re_create(re_handle* h, void* hip_stream);

/* Release the handle and all of its workspace.  NULL is accepted. */
re_status re_destroy(re_handle h);

/* Rebind the handle to another stream of the same device. */
re_status re_set_stream(re_handle h, void* hip_stream);

/* Bytes of device workspace the handle currently holds. */
re_status re_workspace_bytes(re_handle h, size_t* bytes);

/* Stages of re_rank_estimate timed by re_set_profiling: drawing X, the A X
 * pass, drawing Y, the Y B pass, the small SVD, and the count with the copy
 * of the results to the host (Algorithm 1 steps 2, 3, 5, 6, 7, 8). */
enum {
  RE_STAGE_X_DRAW = 0,
  RE_STAGE_AX = 1,
  RE_STAGE_Y_DRAW = 2,
  RE_STAGE_YB = 3,
  RE_STAGE_SVD = 4,
  RE_STAGE_RANK = 5,  /* the count plus the copy of the results to the host */
  RE_NUM_STAGES = 6
};

/* enable != 0: record HIP events on the handle's stream around each stage of
 * every later re_rank_estimate call (adds seven event records per call). */
re_status re_set_profiling(re_handle h, int32_t enable);

/* Limits for callers that must bound the library, and hooks for tests of the
 * error paths:
 *   max_workspace_bytes  > 0: no workspace of the handle (device workspaces
 *                        and the pinned host staging) may grow past this many
 *                        bytes; a call that needs more returns
 *                        RE_ERR_NO_MEMORY, as a failed allocation would,
 *                        and leaves the handle usable.  0 removes the cap.
 *   barrier_polls        polls of a grid barrier of the multi-workgroup small
 *                        SVD (sketches too large for one workgroup) before it
 *                        gives up and the call returns RE_ERR_NO_CONVERGENCE;
 *                        0 restores the default (2^26); a negative value
 *                        gives up at the first poll, which makes that error
 *                        happen on purpose (every workgroup still exits).
 * Errors: RE_ERR_INVALID_ARG for a NULL handle or a negative byte cap. */
re_status re_set_limits(re_handle h, int64_t max_workspace_bytes, int64_t barrier_polls);

/* Durations in milliseconds of the stages of the last re_rank_estimate call
 * (ms: host array of RE_NUM_STAGES doubles, indexed by RE_STAGE_*).
 * Requires profiling enabled. */
re_status re_last_stage_ms(re_handle h, double* ms);

/*
 * Algorithm 1 of the paper on one matrix.
 *   A_dev      device, m x n row-major with leading dimension lda >= n, type dt;
 *              read only; aligned to its element size (16-byte alignment with lda % 4 == 0 enables the vector-load kernels).
 *   eps        relative tolerance, 0 < eps < 1 (Def. 1).
 *   sk         sketch description (host).
 *   seed       key of the counter-based generator defining X and Y.
 *   r_out      host: the rank estimate r^ (number of the first r1 estimates
 *              strictly above eps * sigma_1).
 *   sigma_out  host, k doubles: sigma_i(Y A X) / sqrt(k l), descending.
 *   r1_out     host or NULL: r1, the largest r with round(1.1 r) <= k.
 *   flags_out  host or NULL: RE_FLAG_* bits.
 * Errors: RE_ERR_INVALID_ARG for bad sizes or pointers, RE_ERR_UNSUPPORTED for
 * low precision with an FP64 A or an SRHT X, RE_ERR_NONFINITE when A holds
 * NaN/Inf, RE_ERR_NO_CONVERGENCE when the small SVD fails.
 * Synchronises the handle's stream.
 */
re_status re_rank_estimate(re_handle h, const void* A_dev, int32_t dt, int64_t m, int64_t n, int64_t lda, double eps,
                           const re_sketch* sk, uint64_t seed, int32_t* r_out, double* sigma_out, int32_t* r1_out,
                           uint32_t* flags_out);

/*
 * Algorithm 1 with the alternative step 7 of Sec. 5: the estimates are the
 * magnitudes of the diagonal of R in a QR factorisation Y A X = Q R (an
 * unpivoted QR of a sketch whose right singular vectors are randomised is rank
 * revealing with high probability), here from the library's shifted
 * CholeskyQR3 in FP64 (R = R3 R2 R1, |R_jj| = |R3_jj R2_jj R1_jj|), sorted in
 * descending order and scaled by 1/sqrt(k l); the count is step 8's.  A column
 * of Y A X dependent on the earlier ones at FP64 precision gives 0.
 * Arguments, outputs and errors as re_rank_estimate (sigma_out: the k sorted
 * diagonal magnitudes); RE_ERR_UNSUPPORTED unless sk->prec = RE_PREC_NATIVE.
 * Stage times: the QR takes the place of the SVD (RE_STAGE_SVD).
 */
re_status re_rank_estimate_qr(re_handle h, const void* A_dev, int32_t dt, int64_t m, int64_t n, int64_t lda,
                              double eps, const re_sketch* sk, uint64_t seed, int32_t* r_out, double* sigma_out,
                              int32_t* r1_out, uint32_t* flags_out);

/* One block of a batched call: caller-owned device matrix, m x n row-major
 * with leading dimension n <= lda < 2^23 (FP32, 4-byte aligned). */
typedef struct {
  const void* A;
  int64_t m, n, lda;
} re_block;

/*
 * Algorithm 1 on many independent blocks (for example the off-diagonal blocks
 * of a hierarchical matrix) in one graph launch.  Gaussian X and Y only, FP32
 * blocks, native precision.  X and Y are master sketches of n_max x k and
 * l x m_max drawn once per call; block b uses X's first n_b rows and Y's
 * first m_b columns, so every block gets exactly the estimate that
 * re_rank_estimate with the same seed returns for it.  The A X contraction of
 * all blocks is one persistent matrix-core kernel fed by an atomic queue of
 * (block, row tile, column chunk) items; the Y B products, small SVDs and
 * counts run one workgroup per block.  The work is captured once into a HIP
 * graph (re-captured when the shapes or the workspace change) and the tile
 * shape of the persistent kernel (wavefronts per workgroup, 32-row tiles per
 * wavefront, K step, resident workgroups) is chosen by timing the candidates
 * on the first call for a size bucket (cached in the handle, and in the JSON
 * file named by RANKEST_AUTOTUNE_CACHE when that variable is set;
 * RANKEST_BATCH_TILE = "waves:tiles:kstep:workgroups per CU" pins it).  With profiling on, the same
 * launches are issued directly on the stream so that stage events separate
 * them.
 *   blocks     host array of nblocks descriptors (k <= n_b, l <= m_b each)
 *   r_out      host, nblocks: rank estimates
 *   sigma_out  host, nblocks * k: estimates of block b at b * k
 *   flags_out  host or NULL, nblocks: RE_FLAG_* bits
 * Argument errors as re_rank_estimate (every block checked before any work;
 * outputs untouched); RE_ERR_UNSUPPORTED for SRHT sketches, FP64 blocks, low
 * precision, or an l x k sketch too large for one workgroup.  When a block's
 * sketch is not finite, the outputs of all blocks are written, that block's
 * r is -1, and the call returns RE_ERR_NONFINITE.  Synchronises the handle's
 * stream.
 */
re_status re_rank_estimate_batched(re_handle h, const re_block* blocks, int32_t nblocks, int32_t dt, double eps,
                                   const re_sketch* sk, uint64_t seed, int32_t* r_out, double* sigma_out,
                                   uint32_t* flags_out);

/*
 * Stage entry points.  Each runs one step of Algorithm 1 on device buffers,
 * enqueued on the handle's stream without synchronising, so that a caller can
 * run, time or check the steps one at a time.
 */

/* Philox4x64-10 of the sketch specification: out[4i..4i+3] = Philox(ctr[4i..4i+3],
 * key = (seed, 0)).  ctr_dev and out_dev are device arrays of 4*count uint64. */
re_status re_philox(re_handle h, const uint64_t* ctr_dev, uint64_t seed, int64_t count, uint64_t* out_dev);

/* Gaussian sketch entries (Sec. 1: iid N(0,1), scale applied at the end):
 * out[i*cols + j] = round_fmt(z(a, b)) with (a, b) = (i, j), or (j, i) when
 * swap_ab != 0, drawn from counter stream `stream_id` (1 for X, 2 for Y).
 * fmt: 0 FP64, 1 FP32, 2 BF16, 3 FP16 (elements of 8, 4, 2, 2 bytes). */
re_status re_gauss_fill(re_handle h, int32_t fmt, int64_t rows, int64_t cols, uint64_t seed, int32_t stream_id,
                        int32_t swap_ab, void* out_dev);

/* Rademacher diagonal D of an SRHT (Eq. (Theta)): bit i of word i/32 of
 * bits_dev (device, npad/32 words rounded up) is set when d_i = -1.
 * stream_id 3 for X, 4 for Y. */
re_status re_srht_signs(re_handle h, int64_t npad, uint64_t seed, int32_t stream_id, uint32_t* bits_dev);

/* Row sampler S of an SRHT (uniform sampling without replacement, Appendix A.1):
 * the k indices of [0, npad) with the smallest 64-bit keys (ties by index),
 * written in ascending order to idx_dev (device, k int32).  stream_id 5 (X) or 6 (Y). */
re_status re_srht_select(re_handle h, int64_t npad, int64_t k, uint64_t seed, int32_t stream_id, int32_t* idx_dev);

/* Algorithm 1 step 3, B = A X without the 1/sqrt(k) scale.  A_dev as in
 * re_rank_estimate; B_dev device, m x k row-major, FP64 when dt = RE_F64 and
 * FP32 otherwise.  For SRHT this is B[i][t] = (H (d .* [a_i, 0]))[S_t]. */
re_status re_sketch_x(re_handle h, const void* A_dev, int32_t dt, int64_t m, int64_t n, int64_t lda,
                      const re_sketch* sk, uint64_t seed, void* B_dev);

/* Algorithm 1 step 6, C = Y B without the 1/sqrt(l) scale.  B_dev device,
 * m x k row-major of type bdt (RE_F64 or RE_F32); it is used as scratch and
 * overwritten, and must provide re_sketch_y_rows(m) rows.  C_dev device,
 * l x k row-major FP64. */
re_status re_sketch_y(re_handle h, void* B_dev, int32_t bdt, int64_t m, int64_t k, const re_sketch* sk,
                      uint64_t seed, double* C_dev);
int64_t re_sketch_y_rows(int64_t m);

/* Algorithm 1 step 7: the k singular values of the l x k FP64 row-major
 * device matrix C_dev (k <= l), multiplied by `scale`, descending, into
 * sigma_dev (device, k doubles).  C_dev is not modified.  Synchronises the
 * handle's stream to read the device status: RE_ERR_NONFINITE when C_dev
 * holds NaN/Inf, RE_ERR_NO_CONVERGENCE when a grid barrier of the
 * multi-workgroup bidiagonalisation gives up (see re_set_limits). */
re_status re_singular_values(re_handle h, const double* C_dev, int64_t l, int64_t k, double scale,
                             double* sigma_dev);

/* Allocation-free form of re_singular_values, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  It takes no handle and calls no hipMalloc / hipFree
 * or allocating library routine: its working memory is a fixed static device
 * array of RE_NOALLOC_SCRATCH_BYTES (16 MiB) per GPU, held from the first call
 * on that GPU until the process ends.  The work is enqueued on `hip_stream`
 * (NULL = the default stream of the current device) and the call does not
 * synchronise.  Arguments and results as re_singular_values: C_dev device,
 * l x k row-major FP64 (k <= l), not modified; sigma_dev device, k doubles.
 * Returns RE_ERR_SCRATCH_LIMIT when the sketch's working set exceeds the
 * array (l k up to about 1.9e6 at k = 384, 1.5e6 at k = 1024; see
 * re_singular_values_noalloc_fits).  All calls on one GPU share that GPU's
 * array and leave their contents in it: calls that overlap in time on one GPU
 * (different streams or host threads) race and must be serialised by the
 * caller.  Being asynchronous, it does not report the device status
 * (NaN/Inf in C_dev): sigma_dev is then undefined. */
#define RE_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
re_status re_singular_values_noalloc(void* hip_stream, const double* C_dev, int64_t l, int64_t k, double scale,
                                     double* sigma_dev);
/* 1 when an l x k sketch fits the allocation-free call's scratch, else 0. */
int32_t re_singular_values_noalloc_fits(int64_t l, int64_t k);

/* Algorithm 1 step 8 on device: out_dev[0] = r^, out_dev[1] = flags for the
 * descending sigma_dev[0..k) with r1 and eps (strict inequality of Def. 1). */
re_status re_rank_count(re_handle h, const double* sigma_dev, int64_t k, int32_t r1, double eps, int32_t* out_dev);

/* ------------------------------------------------------------------------
 * Adaptive sketch width.  When r1 is too small (r^ = r1) the paper reruns
 * Algorithm 1 with a larger r1, appending columns to X and rows to Y and
 * keeping what was computed (Sec. 5, with the update r1 := 2 r1, whose
 * overhead for Gaussian sketches is at most a factor 2).  Sec. 7 leaves open
 * how to pick the new r1 from the first run; the learned policy below (an
 * addition of this library, not a claim of the paper) lets a small network
 * read the pilot sketch and propose the width, with doubling as fallback.
 * ------------------------------------------------------------------------ */
#define RE_MLP_INPUTS 35   /* log10(s_i/s_1), i < 32 (clamped at -8), log10 m, log10 n, log10 eps */
#define RE_MLP_PARAMS 6529 /* W1 (64x35), b1 (64), W2 (64x64), b2 (64), w3 (64), b3 (1), row-major */

/* Largest sketch width of the adaptive drivers (re_rank_adaptive,
 * re_rangefinder): the widest small SVD the library forms in one call. */
#define RE_MAX_ADAPTIVE_K 5120

typedef struct {
  int32_t k0;          /* pilot width (e.g. 32); the pilot uses l = l_for(k0) rows */
  int32_t k_max;       /* largest width; 0 means min(m, n); capped at RE_MAX_ADAPTIVE_K */
  double l_ratio;      /* rows of Y per column of X: l = clamp(round(l_ratio k), k, m) */
  const float* mlp;    /* device, RE_MLP_PARAMS floats, or NULL for plain doubling */
  double delta;        /* margin added to the network output (natural log of the width) */
} re_adaptive;

/*
 * Rank estimate with an adaptive width, FP32 A and Gaussian X and Y.  Round 1
 * runs Algorithm 1 at k0.  While r^ = r1(k) and k < k_max: the next width is
 * the network's proposal after round 1 when `mlp` is given (ceil(exp(y +
 * delta)) rounded up to a multiple of 8, clamped to [2 k0, k_max]), and 2k
 * otherwise.  Each round draws only the new columns of X and rows of Y, forms
 * only the new columns of A X (one more pass over A), recomputes Y B, its SVD
 * and the count; the final estimate equals re_rank_estimate at the final
 * (k, l) with the same seed.
 *   sigma_out   host, k_max doubles: the final round's estimates (k_out of them)
 *   k_out, l_out, rounds_out, k_proposed_out (0 when no proposal), flags_out:
 *               host, may be NULL
 * Errors as re_rank_estimate; RE_ERR_UNSUPPORTED unless dt = RE_F32.
 */
re_status re_rank_adaptive(re_handle h, const void* A_dev, int32_t dt, int64_t m, int64_t n, int64_t lda, double eps,
                           const re_adaptive* ad, uint64_t seed, int32_t* r_out, double* sigma_out, int32_t* k_out,
                           int32_t* l_out, int32_t* rounds_out, int32_t* k_proposed_out, uint32_t* flags_out);

/*
 * re_rank_adaptive with the kind of Y chosen: RE_GAUSSIAN (as re_rank_adaptive),
 * RE_SRHT or RE_SRCT (X stays Gaussian).  Sec. 5's footnote on growing r1 with an SRTT
 * sketch: the transform F D A X is kept and only subsampled again.  Here each
 * new column of A X gets the signs and the first level of the Walsh-Hadamard
 * transform along m (blocks of 256 or fewer rows) once, in place in the
 * workspace, and every round forms the l sampled rows of the full transform
 * from those blocks for all k columns; the samples nest in l.  The final
 * estimate equals re_rank_estimate with Gaussian X and SRHT Y at the final
 * (k, l) and the same seed, bit for bit.
 *   y_kind   RE_GAUSSIAN, RE_SRHT or RE_SRCT (else RE_ERR_INVALID_ARG).  With the
 *            subsampled DCT the kept first level is the 32-point DFTs of the
 *            column pieces of the DCT along m (the DFT of length M split as
 *            (M / 32) x 32), formed once per new column; each round forms the
 *            l sampled outputs from them.
 * Other arguments, outputs and errors as re_rank_adaptive.
 */
re_status re_rank_adaptive_y(re_handle h, const void* A_dev, int32_t dt, int64_t m, int64_t n, int64_t lda,
                             double eps, const re_adaptive* ad, int32_t y_kind, uint64_t seed, int32_t* r_out,
                             double* sigma_out, int32_t* k_out, int32_t* l_out, int32_t* rounds_out,
                             int32_t* k_proposed_out, uint32_t* flags_out);

/* ------------------------------------------------------------------------
 * Rank without a tolerance (Sec. 5 after Algorithm 1; Sec. 6.1).  With no eps
 * the sketched spectrum itself shows where the gaps are: Sec. 6.1 grows a
 * Gaussian X by 100 columns per round from 110 until the gap of its test
 * matrix shows.  A gap at i (1-based, i < r1, over the estimates that are
 * kept after discarding the oversampled ones) is a ratio s_i / s_{i+1} >=
 * gamma (infinite when s_{i+1} = 0 < s_i).  Round j uses k_j = k0 + j dk
 * (capped at k_max) and l_j = clamp(round(l_ratio k_j), k_j, m); its estimates
 * are Algorithm 1's at (k_j, l_j) with the same seed, X and Y only being
 * appended to.  The search stops after the first round whose first r1
 * estimates reach below floor * s_1 (the spectrum has been followed down to
 * the floor) and whose deepest gap (largest such i) is the previous round's;
 * at k_max without that, it stops with RE_FLAG_NOT_CONVERGED; when s_1 = 0
 * it stops at once with RE_FLAG_ZERO and r^ = 0.
 * ------------------------------------------------------------------------ */
typedef struct {
  int32_t k0;      /* first width of X (Sec. 6.1: 110) */
  int32_t dk;      /* columns appended per round (Sec. 6.1: 100) */
  int32_t k_max;   /* largest width; 0 means min(m, n); capped at RE_MAX_ADAPTIVE_K */
  int32_t y_kind;  /* RE_GAUSSIAN (rows appended), RE_SRHT or RE_SRCT (stored first-level transform) */
  double l_ratio;  /* rows of Y per column of X, >= 1 */
  double gamma;    /* gap threshold on s_i / s_{i+1}, > 1 */
  double floor;    /* relative level s_{r1} <= floor s_1 the estimates must reach before stopping, >= 0 */
} re_gap_search;

/*
 * The search above on an FP32 or FP64 A (device, row-major, lda >= n; 4- or
 * 8-byte aligned), Gaussian X.  Each round draws the new columns of X (and
 * rows of a Gaussian Y), forms only the new columns of A X (one more pass
 * over A), then C = Y B, its singular values and the gap statistics on the
 * device; the host reads 48 bytes and the estimates to decide.
 *   r_out        host: the deepest gap of the last round (0: none)
 *   ratio_out    host, may be NULL: its ratio s_r / s_{r+1}
 *   argmax_out, argmax_ratio_out  host, may be NULL: Sec. 5's measure on the
 *                last round, the i of the largest ratio (ties to the smallest)
 *   sigma_out    host, k_max doubles: the last round's k estimates
 *   k_out, l_out, rounds_out, flags_out  host, may be NULL
 *   spectra_out  host, may be NULL: row j (stride k_max) receives round j's k_j
 *                estimates, zero-padded, for j < spectra_cap
 * Errors: RE_ERR_INVALID_ARG (arguments, including gamma <= 1, floor < 0,
 * y_kind), RE_ERR_NONFINITE, RE_ERR_NO_CONVERGENCE (small SVD), RE_ERR_NO_MEMORY.
 * Synchronises the handle's stream once per round.  With profiling on
 * (re_set_profiling), re_last_stage_ms gives each stage summed over the rounds.
 */
re_status re_rank_gap(re_handle h, const void* A_dev, int32_t dt, int64_t m, int64_t n, int64_t lda,
                      const re_gap_search* gs, uint64_t seed, int32_t* r_out, double* ratio_out, int32_t* argmax_out,
                      double* argmax_ratio_out, double* sigma_out, int32_t* k_out, int32_t* l_out, int32_t* rounds_out,
                      double* spectra_out, int32_t spectra_cap, uint32_t* flags_out);

/* The network, FP32, on device buffers (training and inference).
 * x_dev: batch x RE_MLP_INPUTS row-major; y_dev, t_dev: batch. */
re_status re_mlp_forward(re_handle h, const float* params_dev, const float* x_dev, int64_t batch, float* y_dev);
/* grad_dev (RE_MLP_PARAMS) = gradient of (1/batch) sum (y - t)^2; loss_dev
 * (1 float, may be NULL) = that loss.  Deterministic. */
re_status re_mlp_loss_grad(re_handle h, const float* params_dev, const float* x_dev, const float* t_dev,
                           int64_t batch, float* grad_dev, float* loss_dev);
/* One Adam step (Kingma & Ba) on n parameters; step counts from 1; m_dev and
 * v_dev start at zero. */
re_status re_mlp_adam(re_handle h, float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, int64_t n,
                      int32_t step, double lr, double beta1, double beta2, double eps);

/* Rank without a tolerance: the largest gap among the first r1 estimates
 * (Sec. 5 after Algorithm 1 suggests argmax_i s_i / s_{i+1}; Sec. 6.1 reads
 * the gap of its test matrix off the sketched spectrum).  Host-only, on the
 * descending estimates re_rank_estimate returns.
 *   sigma     host, k descending values
 *   r_out     host: the 1-based i in 1..min(r1, k)-1 with the largest
 *             s_i / s_{i+1} (ties to the smallest i; a zero s_{i+1} after a
 *             positive s_i counts as an infinite ratio); 0 when s_1 = 0 or
 *             min(r1, k) < 2
 *   ratio_out host or NULL: that ratio (0 when r_out is 0)
 * RE_ERR_INVALID_ARG for NULL sigma / r_out or negative sizes. */
re_status re_gap_rank(const double* sigma, int32_t k, int32_t r1, int32_t* r_out, double* ratio_out);

/* --------------------------------------------------------------------------
 * Rank estimation combined with the randomized rangefinder (Algorithm 3,
 * Sec. 5.1): a fixed-precision QB factorisation A ~ Q B with
 * ||A - Q B||_F <~ eps ||A||.
 *
 * 1. Rank estimation with appended sketches exactly as re_rank_adaptive with
 *    mlp = NULL (Gaussian X and Y, k0, 2 k0, ... up to k_max, each round one
 *    more pass over A for the new columns of X only), stopping at the first
 *    width k for which step 2 finds an r.
 * 2. With s_i the estimates of that round, i <= r1 = r1(k), extended by
 *    s_i = s_{r1} for r1 < i <= n: r = the smallest r >= 1 with r + p <= k and
 *    (1 + r/(p-1))^(1/2) (sum_{j>r} s_j^2)^(1/2) <= eps ||A||  (Eq. errRFfro;
 *    the a priori bound of Halko, Martinsson and Tropp 2011, Thm. 10.5),
 *    ||A|| = norm_a if norm_a > 0, else s_1.
 * 3. Q = orthonormal basis of the first w = r + p columns of A X (thin QR by
 *    shifted CholeskyQR3 in FP64; columns numerically dependent at FP64
 *    precision are left out, setting RE_FLAG_COLUMNS_DROPPED and w < r + p).
 * 4. B = Q^T A (one more pass over A: FP32 matrix-core products with Q
 *    rounded to FP32, FP64 sums across every 256 rows of A).
 *
 *   A_dev      device, m x n FP32 row-major, lda >= n, lda < 2^23, 4-byte aligned
 *   eps        0 < eps < 1
 *   p          oversampling, 2 <= p < k_max
 *   ad         host: k0, k_max, l_ratio as in re_rank_adaptive; mlp must be NULL
 *   norm_a     ||A|| (spectral norm) if known and > 0; otherwise 0
 *   Q_dev      device, FP64, m x k_max capacity row-major (ldq >= k_max, k_max
 *              after clamping to min(m, n)); the first w columns are written
 *   B_dev      device, FP64, k_max x n capacity (ldb >= n); the first w rows
 *              are written
 *   r_out      host: r; 0 when the sketch is zero (A = 0); -1 when no r with
 *              r + p <= k_max qualifies (RE_FLAG_NOT_CONVERGED).  Q and B are
 *              written only when r > 0.
 *   w_out      host: columns of Q (0 unless r > 0)
 *   sigma_out  host, k_max doubles: the final round's estimates (k_out of them)
 *   k_out      host or NULL: the final width k;  flags_out: host or NULL
 * Errors: RE_ERR_INVALID_ARG for bad sizes or pointers, RE_ERR_UNSUPPORTED
 * unless dt = RE_F32 and mlp = NULL, RE_ERR_NONFINITE when the sketch or the
 * QR meets NaN/Inf, RE_ERR_NO_CONVERGENCE when the small SVD fails.
 * Synchronises the handle's stream before returning.
 */
re_status re_rangefinder(re_handle h, const void* A_dev, int32_t dt, int64_t m, int64_t n, int64_t lda, double eps,
                         int32_t p, const re_adaptive* ad, double norm_a, uint64_t seed, double* Q_dev, int64_t ldq,
                         double* B_dev, int64_t ldb, int32_t* r_out, int32_t* w_out, double* sigma_out, int32_t* k_out,
                         uint32_t* flags_out);

/* Step 3 of re_rangefinder alone (Algorithm 3, the thin QR of the kept
 * sketch columns; Algorithm 2 step 2): an orthonormal basis of the columns of W.
 *   W_dev      device, m x w row-major (ldw >= w), FP32 or FP64 (dt), m >= w >= 1
 *   Q_dev      device, FP64, m x w capacity (ldq >= w); the first w_out columns are
 *              written: Q R = W with diag(R) > 0 over the kept columns
 *   w_out      host: kept columns (w unless some are numerically dependent at
 *              FP64 precision; then RE_FLAG_COLUMNS_DROPPED).  After the
 *              first, shifted pass a column whose pivot is below 16 u (u = 2^-53)
 *              of the largest counts as dependent: directions of W with
 *              singular values below about 4 u^(1/2) (11 (m w + w (w+1)) u)^(1/2)
 *              ||W||_F are left out (about 1e-12 ||W||_F at m = 4000, w = 120).
 *   flags_out  host or NULL
 * Errors: RE_ERR_INVALID_ARG, RE_ERR_NONFINITE.  Synchronises the stream. */
re_status re_thin_qr(re_handle h, const void* W_dev, int32_t dt, int64_t m, int64_t w, int64_t ldw, double* Q_dev,
                     int64_t ldq, int32_t* w_out, uint32_t* flags_out);

/* Step 4 of re_rangefinder alone (Algorithm 3, B = Q^T A; Algorithm 2 step 3):
 * Q_dev FP64 m x w (ldq >= w), A_dev FP32 m x n (lda >= n), B_dev FP64 w x n
 * (ldb >= n).  FP32 matrix-core products with Q rounded to FP32, FP64 sums
 * across every 256 rows.  RE_ERR_UNSUPPORTED unless dt = RE_F32.  Does not
 * synchronise. */
re_status re_project(re_handle h, const double* Q_dev, int64_t ldq, int64_t w, const void* A_dev, int32_t dt,
                     int64_t m, int64_t n, int64_t lda, double* B_dev, int64_t ldb);

/* Durations in milliseconds of the three stages of the last re_rangefinder
 * call with profiling enabled: ms[0] rank estimation (every round and the
 * width rule), ms[1] the thin QR, ms[2] B = Q^T A. */
re_status re_rangefinder_stage_ms(re_handle h, double* ms);

/* r1 derived from the sketch width k (Algorithm 1 step 1 inverted). */
int32_t re_r1_from_k(int32_t k);

/* Human-readable text for a status code. */
const char* re_status_string(re_status s);

#ifdef __cplusplus
}
#endif

#endif /* RANKEST_H */
