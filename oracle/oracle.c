/*
 * oracle.c — plain, slow, FP64 CPU oracle for the two-sided sketched
 * numerical-rank estimator of Meier & Nakatsukasa, "Fast Randomized Numerical
 * Rank Estimation for Numerically Low-Rank Matrices" (arXiv 2105.07388).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and
 * the CPU-baseline leg of the benchmark may load this library.  The product
 * path (the HIP library under paper_2105_07388_amd/) never links, imports or
 * calls it, and this file shares no code, header, table or helper with it.
 *
 * What it computes, in the paper's order (Sec. 5, Algorithm 1):
 *   step 1   r~1 = round(1.1 r1)   -> here: r1 is derived from the sketch width k
 *   step 2/3 draw the n x k embedding X, form B = A X
 *   step 4-6 draw the l x m embedding Y (Theta), form C = Y B
 *   step 7   singular values of C (one-sided Jacobi, Hestenes)
 *   step 8   r^ = number of the first r1 estimates strictly above eps * s1
 * The embeddings are defined by a counter-based generator (Philox4x64-10 of
 * Salmon et al., SC'11) so that the oracle and the GPU library, written
 * independently, draw the same sketch from the same seed.
 *
 * Every floating-point step is FP64, summed in the plain index order written
 * below.  No blocking, no reordering, no fusion.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EXPORT __attribute__((visibility("default")))

/* Status codes (mirrors of the library's, kept separately on purpose). */
enum { OR_OK = 0, OR_ERR_INVALID_ARG = -1, OR_ERR_UNSUPPORTED = -2, OR_ERR_NO_MEMORY = -3,
       OR_ERR_NONFINITE = -5, OR_ERR_NO_CONVERGENCE = -6 };
enum { OR_FLAG_NOT_CONVERGED = 1u, OR_FLAG_ZERO = 2u };
enum { OR_FMT_F64 = 0, OR_FMT_F32 = 1, OR_FMT_BF16 = 2, OR_FMT_F16 = 3 };
enum { OR_GAUSSIAN = 0, OR_SRHT = 1 };

/* Counter streams of the sketch specification. */
enum { OR_STREAM_XGAUSS = 1, OR_STREAM_YGAUSS = 2, OR_STREAM_XSIGN = 3, OR_STREAM_YSIGN = 4,
       OR_STREAM_XSEL = 5, OR_STREAM_YSEL = 6 };

/* ------------------------------------------------------------------------ */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11, Sec. 4 and Table 2).    */
/* Written from the published round function:                                */
/*   (c0,c1,c2,c3) <- (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,  */
/*                     lo(M0*c0)),  key bumped by the Weyl constants between */
/*   rounds, ten rounds.                                                      */
/* ------------------------------------------------------------------------ */
OR_EXPORT void or_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0;
        uint64_t n1 = lo1;
        uint64_t n2 = hi0 ^ c3 ^ k1;
        uint64_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint64_t a, uint64_t b, uint64_t stream, uint64_t blk, uint64_t out[4]) {
    const uint64_t ctr[4] = {a, b, stream, blk};
    const uint64_t key[2] = {seed, 0};
    or_philox4x64_10(ctr, key, out);
}

/* Standard normal by the Box-Muller transform of two uniforms taken from the
 * top 53 bits of two Philox words: u1 in (0,1], u2 in [0,1). */
OR_EXPORT double or_gauss(uint64_t seed, uint64_t a, uint64_t b, uint64_t stream, uint64_t blk) {
    uint64_t w[4];
    draw(seed, a, b, stream, blk, w);
    double u1 = ((double)((w[0] >> 11) + 1)) * 0x1.0p-53;
    double u2 = ((double)(w[1] >> 11)) * 0x1.0p-53;
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* Round-to-nearest-even of an FP64 value to a format with `sig` significant
 * bits whose smallest normal binade has frexp exponent `emin`.  Division and
 * multiplication by a power of two are exact, nearbyint() rounds to even. */
static double round_sig(double v, int sig, int emin) {
    if (v == 0.0 || !isfinite(v)) return v;
    int e;
    (void)frexp(v, &e);
    if (e < emin) e = emin;
    double q = ldexp(1.0, e - sig);
    return nearbyint(v / q) * q;
}

OR_EXPORT double or_round_to(double v, int fmt) {
    switch (fmt) {
    case OR_FMT_F64: return v;
    case OR_FMT_F32: return (double)(float)v;
    case OR_FMT_BF16: return round_sig(v, 8, -125);
    case OR_FMT_F16: return round_sig(v, 11, -13);
    default: return NAN;
    }
}

/* The Gaussian embedding written out as a dense rows x cols matrix (row-major),
 * each entry rounded to the contraction format: G[i][j] = round_fmt(gauss(i, j))
 * for X (swap = 0); Y's entry (s, i) takes the counter (i, s), so swap = 1
 * gives G[s][i] = round_fmt(gauss(i, s)).  Counters do not depend on the
 * matrix size, so a smaller matrix is a leading block of a larger one. */
OR_EXPORT void or_gauss_matrix(uint64_t seed, int64_t rows, int64_t cols, uint64_t stream, uint64_t blk, int fmt,
                               int swap, double* G) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < rows; ++i)
        for (int64_t j = 0; j < cols; ++j)
            G[i * cols + j] = or_round_to(swap ? or_gauss(seed, (uint64_t)j, (uint64_t)i, stream, blk)
                                               : or_gauss(seed, (uint64_t)i, (uint64_t)j, stream, blk), fmt);
}

/* Rademacher sign d_i = 1 - 2 * (lowest bit of the first Philox word). */
OR_EXPORT int or_sign(uint64_t seed, uint64_t i, uint64_t stream, uint64_t blk) {
    uint64_t w[4];
    draw(seed, i, 0, stream, blk, w);
    return 1 - 2 * (int)(w[0] & 1u);
}

OR_EXPORT uint64_t or_select_key(uint64_t seed, uint64_t i, uint64_t stream, uint64_t blk) {
    uint64_t w[4];
    draw(seed, i, 0, stream, blk, w);
    return w[0];
}

typedef struct { uint64_t key; int64_t idx; } keyed_t;

static int cmp_keyed(const void* pa, const void* pb) {
    const keyed_t* a = (const keyed_t*)pa;
    const keyed_t* b = (const keyed_t*)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int cmp_i64(const void* pa, const void* pb) {
    int64_t a = *(const int64_t*)pa, b = *(const int64_t*)pb;
    return (a > b) - (a < b);
}

/* Uniform sampling of k of npad indices without replacement (the row sampler
 * S of the SRTT, Appendix A.1: uniform sampling without replacement): the k
 * indices whose iid 64-bit keys are smallest, ties broken by index, returned
 * in ascending index order. */
OR_EXPORT int or_select(uint64_t seed, int64_t npad, int64_t k, uint64_t stream, uint64_t blk, int64_t* idx) {
    if (k < 0 || k > npad) return OR_ERR_INVALID_ARG;
    keyed_t* all = (keyed_t*)malloc(sizeof(keyed_t) * (size_t)(npad > 0 ? npad : 1));
    if (!all) return OR_ERR_NO_MEMORY;
    for (int64_t i = 0; i < npad; ++i) { all[i].key = or_select_key(seed, (uint64_t)i, stream, blk); all[i].idx = i; }
    qsort(all, (size_t)npad, sizeof(keyed_t), cmp_keyed);
    for (int64_t t = 0; t < k; ++t) idx[t] = all[t].idx;
    qsort(idx, (size_t)k, sizeof(int64_t), cmp_i64);
    free(all);
    return OR_OK;
}

/* Unnormalised Walsh-Hadamard transform in Sylvester (natural) order,
 * y[p] = sum_q (-1)^popcount(p & q) x[q]; n must be a power of two. */
OR_EXPORT void or_fwht(double* x, int64_t n) {
    for (int64_t h = 1; h < n; h *= 2) {
        for (int64_t i = 0; i < n; i += 2 * h) {
            for (int64_t j = i; j < i + h; ++j) {
                double a = x[j], b = x[j + h];
                x[j] = a + b;
                x[j + h] = a - b;
            }
        }
    }
}

OR_EXPORT int64_t or_next_pow2(int64_t v) {
    int64_t p = 1;
    while (p < v) p *= 2;
    return p;
}

/* Algorithm 1 step 1 sets k = round(1.1 r1).  The oracle works from the
 * sketch width k and takes the largest r1 whose rounded 1.1 r1 (halves
 * rounded up, computed in integers) still fits in k. */
OR_EXPORT int or_r1_from_k(int k) {
    int r1 = 0;
    for (int r = 1; r <= k; ++r)
        if ((11 * r + 5) / 10 <= k) r1 = r;
    return r1;
}

/* Def. 1: relative eps-rank of a descending spectrum, i with
 * s_i > eps * s_1 >= s_{i+1}; min(m,n) (= len) when no such i exists. */
OR_EXPORT int or_rank_def(const double* s, int len, double eps) {
    if (len <= 0) return 0;
    double tau = eps * s[0];
    for (int i = 0; i < len; ++i)
        if (!(s[i] > tau)) return i;
    return len;
}

static double load_a(const void* A, int dtype, int64_t i, int64_t j, int64_t lda) {
    return dtype == OR_FMT_F64 ? ((const double*)A)[i * lda + j] : (double)((const float*)A)[i * lda + j];
}

/* Algorithm 1 steps 2-3: B = A X, B is m x k row-major FP64.
 * Gaussian X[j,t] = round_fmt(gauss(j, t, stream 1)), applied as plain sums;
 * SRHT X = D H S^T applied per row: w = d .* [a_i, 0], w <- H w, B[i,t] = w[S_t].
 * Embedding scale factors (1/sqrt(k)) are applied once to the final singular
 * values, not here. */
OR_EXPORT int or_apply_x(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, int xkind, int64_t k,
                         int fmt_x, uint64_t seed, uint64_t blk, double* B) {
    if (xkind == OR_GAUSSIAN) {
        double* X = (double*)malloc(sizeof(double) * (size_t)(n * k));
        if (!X) return OR_ERR_NO_MEMORY;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t t = 0; t < k; ++t)
                X[j * k + t] = or_round_to(or_gauss(seed, (uint64_t)j, (uint64_t)t, OR_STREAM_XGAUSS, blk), fmt_x);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t t = 0; t < k; ++t) {
                double acc = 0.0;
                for (int64_t j = 0; j < n; ++j) acc += load_a(A, dtype, i, j, lda) * X[j * k + t];
                B[i * k + t] = acc;
            }
        }
        free(X);
        return OR_OK;
    }
    if (xkind != OR_SRHT) return OR_ERR_INVALID_ARG;
    int64_t npad = or_next_pow2(n);
    int64_t* S = (int64_t*)malloc(sizeof(int64_t) * (size_t)k);
    double* d = (double*)malloc(sizeof(double) * (size_t)npad);
    if (!S || !d) { free(S); free(d); return OR_ERR_NO_MEMORY; }
    int st = or_select(seed, npad, k, OR_STREAM_XSEL, blk, S);
    if (st != OR_OK) { free(S); free(d); return st; }
    for (int64_t j = 0; j < npad; ++j) d[j] = (double)or_sign(seed, (uint64_t)j, OR_STREAM_XSIGN, blk);
    int fail = 0;
#pragma omp parallel
    {
        double* w = (double*)malloc(sizeof(double) * (size_t)npad);
        if (!w) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(static)
        for (int64_t i = 0; i < m; ++i) {
            if (!w) continue;
            for (int64_t j = 0; j < npad; ++j) w[j] = j < n ? d[j] * load_a(A, dtype, i, j, lda) : 0.0;
            or_fwht(w, npad);
            for (int64_t t = 0; t < k; ++t) B[i * k + t] = w[S[t]];
        }
        free(w);
    }
    free(S); free(d);
    return fail ? OR_ERR_NO_MEMORY : OR_OK;
}

/* Algorithm 1 steps 4-6: C = Y B, C is l x k row-major FP64.
 * Gaussian Y[s,i] = round_fmt(gauss(i, s, stream 2)) (plain sums over i);
 * SRHT Y = S H D applied per column of B along m. */
OR_EXPORT int or_apply_y(const double* B, int64_t m, int64_t k, int ykind, int64_t l, int fmt_y,
                         uint64_t seed, uint64_t blk, double* C) {
    if (ykind == OR_GAUSSIAN) {
        double* Y = (double*)malloc(sizeof(double) * (size_t)(l * m));
        if (!Y) return OR_ERR_NO_MEMORY;
        for (int64_t s = 0; s < l; ++s)
            for (int64_t i = 0; i < m; ++i)
                Y[s * m + i] = or_round_to(or_gauss(seed, (uint64_t)i, (uint64_t)s, OR_STREAM_YGAUSS, blk), fmt_y);
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < l; ++s) {
            for (int64_t t = 0; t < k; ++t) {
                double acc = 0.0;
                for (int64_t i = 0; i < m; ++i) acc += Y[s * m + i] * B[i * k + t];
                C[s * k + t] = acc;
            }
        }
        free(Y);
        return OR_OK;
    }
    if (ykind != OR_SRHT) return OR_ERR_INVALID_ARG;
    int64_t mpad = or_next_pow2(m);
    int64_t* S = (int64_t*)malloc(sizeof(int64_t) * (size_t)l);
    double* d = (double*)malloc(sizeof(double) * (size_t)mpad);
    if (!S || !d) { free(S); free(d); return OR_ERR_NO_MEMORY; }
    int st = or_select(seed, mpad, l, OR_STREAM_YSEL, blk, S);
    if (st != OR_OK) { free(S); free(d); return st; }
    for (int64_t i = 0; i < mpad; ++i) d[i] = (double)or_sign(seed, (uint64_t)i, OR_STREAM_YSIGN, blk);
    int fail = 0;
#pragma omp parallel
    {
        double* v = (double*)malloc(sizeof(double) * (size_t)mpad);
        if (!v) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(static)
        for (int64_t t = 0; t < k; ++t) {
            if (!v) continue;
            for (int64_t i = 0; i < mpad; ++i) v[i] = i < m ? d[i] * B[i * k + t] : 0.0;
            or_fwht(v, mpad);
            for (int64_t s = 0; s < l; ++s) C[s * k + t] = v[S[s]];
        }
        free(v);
    }
    free(S); free(d);
    return fail ? OR_ERR_NO_MEMORY : OR_OK;
}

static int cmp_desc(const void* pa, const void* pb) {
    double a = *(const double*)pa, b = *(const double*)pb;
    return (a < b) - (a > b);
}

/* Algorithm 1 step 7: singular values of the l x k matrix C (row-major) by
 * the one-sided Jacobi method of Hestenes (Demmel-Veselic form): cyclic
 * sweeps over column pairs p < q in row order; a pair is rotated when
 * |c_p . c_q| > tol * |c_p| |c_q| with tol = l * 2^-53; the rotation
 * zeroes c_p . c_q exactly in exact arithmetic.  Stops after a sweep without
 * rotations.  Returns the column norms in descending order (unscaled). */
OR_EXPORT int or_jacobi_sv(const double* C, int64_t l, int64_t k, int max_sweeps, double* sigma, int* sweeps_out) {
    double* W = (double*)malloc(sizeof(double) * (size_t)(l * k > 0 ? l * k : 1));
    if (!W) return OR_ERR_NO_MEMORY;
    for (int64_t t = 0; t < k; ++t)
        for (int64_t s = 0; s < l; ++s) W[t * l + s] = C[s * k + t];
    const double tol = (double)l * 0x1.0p-53;
    int sweep = 0, converged = 0;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        int rotated = 0;
        for (int64_t p = 0; p + 1 < k; ++p) {
            for (int64_t q = p + 1; q < k; ++q) {
                double* cp = W + p * l;
                double* cq = W + q * l;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t s = 0; s < l; ++s) {
                    alpha += cp[s] * cp[s];
                    beta += cq[s] * cq[s];
                    gamma += cp[s] * cq[s];
                }
                if (alpha == 0.0 || beta == 0.0) continue;
                if (fabs(gamma) <= tol * sqrt(alpha) * sqrt(beta)) continue;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double t;
                if (fabs(zeta) > 1e150) t = 1.0 / (2.0 * zeta);
                else t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double sn = c * t;
                for (int64_t s = 0; s < l; ++s) {
                    double a = cp[s], b = cq[s];
                    cp[s] = c * a - sn * b;
                    cq[s] = sn * a + c * b;
                }
                rotated = 1;
            }
        }
        if (!rotated) { converged = 1; break; }
    }
    for (int64_t t = 0; t < k; ++t) {
        double acc = 0.0;
        for (int64_t s = 0; s < l; ++s) acc += W[t * l + s] * W[t * l + s];
        sigma[t] = sqrt(acc);
    }
    qsort(sigma, (size_t)k, sizeof(double), cmp_desc);
    free(W);
    if (sweeps_out) *sweeps_out = converged ? sweep + 1 : sweep;
    return converged ? OR_OK : OR_ERR_NO_CONVERGENCE;
}

/* Algorithm 1 step 8 with Def. 1's strict inequality: tau = eps * s1,
 * r^ = #{ i <= r1 : s_i > tau } over the descending estimates; r^ = r1 means
 * no i <= r1 had s_{i+1} <= tau, so the rank is only bounded below. */
OR_EXPORT int or_rank_count(const double* sigma, int k, int r1, double eps, int* r_out, unsigned* flags_out) {
    unsigned flags = 0;
    for (int i = 0; i < k; ++i)
        if (!isfinite(sigma[i])) return OR_ERR_NONFINITE;
    int r = 0;
    if (k == 0 || sigma[0] == 0.0) {
        flags |= OR_FLAG_ZERO;
    } else {
        double tau = eps * sigma[0];
        int lim = r1 < k ? r1 : k;
        while (r < lim && sigma[r] > tau) ++r;
        if (r == r1) flags |= OR_FLAG_NOT_CONVERGED;
    }
    *r_out = r;
    *flags_out = flags;
    return OR_OK;
}

/* Sketch value formats used by the contraction, by storage type of A and
 * requested contraction precision (0 native, 1 bf16, 2 fp16). */
OR_EXPORT int or_x_format(int dtype, int prec) {
    if (dtype == OR_FMT_F64) return OR_FMT_F64;
    if (prec == 1) return OR_FMT_BF16;
    if (prec == 2) return OR_FMT_F16;
    return OR_FMT_F32;
}

OR_EXPORT int or_y_format(int dtype) { return dtype == OR_FMT_F64 ? OR_FMT_F64 : OR_FMT_F32; }

/* The whole of Algorithm 1 for one matrix.  A is m x n row-major with leading
 * dimension lda (dtype 0 = FP64, 1 = FP32).  sigma_out receives the k
 * estimates s_i = sigma_i(C) / sqrt(k l) in descending order. */
OR_EXPORT int or_rank_estimate(const void* A, int dtype, int64_t m, int64_t n, int64_t lda, double eps,
                               int xkind, int ykind, int64_t k, int64_t l, int prec, uint64_t seed,
                               uint64_t blk, int* r_out, double* sigma_out, int* r1_out, unsigned* flags_out,
                               int* sweeps_out) {
    if (!A || m < 1 || n < 1 || lda < n || !(eps > 0.0 && eps < 1.0) || k < 1 || l < k) return OR_ERR_INVALID_ARG;
    if (dtype != OR_FMT_F64 && dtype != OR_FMT_F32) return OR_ERR_INVALID_ARG;
    int64_t nmax = xkind == OR_SRHT ? or_next_pow2(n) : n;
    int64_t mmax = ykind == OR_SRHT ? or_next_pow2(m) : m;
    if (k > nmax || l > mmax) return OR_ERR_INVALID_ARG;
    if (dtype == OR_FMT_F64 && prec != 0) return OR_ERR_UNSUPPORTED;
    if (xkind == OR_SRHT && prec != 0) return OR_ERR_UNSUPPORTED;
    for (int64_t i = 0; i < m; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (!isfinite(load_a(A, dtype, i, j, lda))) return OR_ERR_NONFINITE;
    double* B = (double*)malloc(sizeof(double) * (size_t)(m * k));
    double* C = (double*)malloc(sizeof(double) * (size_t)(l * k));
    if (!B || !C) { free(B); free(C); return OR_ERR_NO_MEMORY; }
    int st = or_apply_x(A, dtype, m, n, lda, xkind, k, or_x_format(dtype, prec), seed, blk, B);
    if (st == OR_OK) st = or_apply_y(B, m, k, ykind, l, or_y_format(dtype), seed, blk, C);
    if (st == OR_OK) {
        st = or_jacobi_sv(C, l, k, 60, sigma_out, sweeps_out);
        double scale = 1.0 / sqrt((double)k * (double)l);
        for (int64_t t = 0; t < k; ++t) sigma_out[t] *= scale;
    }
    free(B); free(C);
    if (st != OR_OK) return st;
    int r1 = or_r1_from_k((int)k);
    st = or_rank_count(sigma_out, (int)k, r1, eps, r_out, flags_out);
    if (r1_out) *r1_out = r1;
    return st;
}

OR_EXPORT int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
