"""FP64 oracle of the hashed randomized DCT sketch (HRTT) for X, test
infrastructure only (only tests/, the package smoke check and the benchmark's
CPU-baseline leg may import it).

Sec. 3.3: a hashed randomized trigonometric transform replaces the sampling
matrix S of the subsampled transform S F D by a hashing matrix H (CountSketch:
each transformed coordinate goes to one of k buckets with a random sign), the
paper's experimental X (Sec. 3.3, Sec. 6) with F a DCT.  Here, per row a of A
(zero-padded to N = the next power of two >= max(n, 2), as for the Hadamard
transform):  B[i, b] = sqrt(k) sum_{j : h(j) = b} s(j) (F D a_i)_j  with D the
random signs of the SRHT's X (Philox stream 3), F the orthonormal DCT-II of
length N (scipy's, a library FFT serving as the transform step), h(j) in
[0, k) and s(j) in {+1, -1} from Philox4x64-10 at counter (j, 0, 7, 0):
h(j) = floor(w0 k / 2^64), s(j) = +1 if the lowest bit of w1 is 0.  The factor
sqrt(k) lets every X kind share the 1/sqrt(k) scale of the estimates.

The subsampled randomized DCT (SRCT, Sec. 3.3 with F a DCT, and Sec. 4) keeps
the sampling S of the subsampled transform instead:
B[i, b] = sqrt(N) (F D a_i)_{s_b}, with s the SRHT's X sample (the k smallest
Philox keys of stream 5 over the N coordinates, sorted); sqrt(N) plays the part
of the unnormalised Hadamard matrix's scale, so that E ||a X||^2 = k ||a||^2
as for the other kinds.

The subsampled randomized DCT as Y (SRCT Y: Sec. 4 with F a DCT; Sec. 6 uses it
for Theta = Y) acts on the columns of B = A X (m x k, zero-padded to M = the
next power of two >= max(m, 2)):  C[s, t] = sqrt(M) (F D_Y b_t)_{q_s}, with
D_Y the SRHT's Y signs (Philox stream 4) and q the SRHT's Y sample (the l
smallest stream-6 keys over the M coordinates, sorted), so E ||Y b||^2 =
l ||b||^2 as for the Gaussian and SRHT Y.
"""
import math

import numpy as np
import scipy.fft as sf

from . import pyoracle as _o

STREAM_XHASH = 7


def npad(n):
    return max(2, _o.next_pow2(int(n)))


def hash_table(seed, N, k, blk=0):
    """(bucket[N], sign[N]) of the CountSketch."""
    b = np.zeros(N, dtype=np.int64)
    s = np.zeros(N, dtype=np.float64)
    for j in range(N):
        w = _o.philox4x64_10([j, 0, STREAM_XHASH, blk], [seed, 0])
        b[j] = (int(w[0]) * int(k)) >> 64
        s[j] = 1.0 - 2.0 * float(int(w[1]) & 1)
    return b, s


def signs(seed, N, blk=0):
    return np.array([_o.sign(seed, j, _o.STREAM_XSIGN, blk) for j in range(N)], dtype=np.float64)


def dct_matrix(N):
    """Orthonormal DCT-II by its definition: F[q, j] = c_q sqrt(2/N) cos(pi q (2j+1) / (2N))."""
    q = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    F = math.sqrt(2.0 / N) * np.cos(np.pi * q * (2 * j + 1) / (2 * N))
    F[0] /= math.sqrt(2.0)
    return F


def apply_x(A, k, seed=0, blk=0):
    """B = A X for the HRTT X (m x k, FP64)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    N = npad(n)
    Z = np.zeros((m, N))
    Z[:, :n] = A
    Z *= signs(seed, N, blk)[None, :]
    Yt = sf.dct(Z, type=2, norm="ortho", axis=1)
    b, s = hash_table(seed, N, k, blk)
    H = np.zeros((N, k))
    H[np.arange(N), b] = s
    return math.sqrt(k) * (Yt @ H)


def apply_x_srct(A, k, seed=0, blk=0):
    """B = A X for the SRCT X (m x k, FP64)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    N = npad(n)
    Z = np.zeros((m, N))
    Z[:, :n] = A
    Z *= signs(seed, N, blk)[None, :]
    Yt = sf.dct(Z, type=2, norm="ortho", axis=1)
    sel = _o.select(seed, N, k, _o.STREAM_XSEL, blk)
    return math.sqrt(N) * Yt[:, sel]


def signs_y(seed, M, blk=0):
    return np.array([_o.sign(seed, i, _o.STREAM_YSIGN, blk) for i in range(M)], dtype=np.float64)


def apply_y_srct(B, l, seed=0, blk=0):
    """C = Y B for the SRCT Y (l x k, FP64): the orthonormal DCT-II along the
    (signed, zero-padded) columns of B, the l sampled outputs, times sqrt(M)."""
    B = np.asarray(B, dtype=np.float64)
    m, k = B.shape
    M = npad(m)
    Z = np.zeros((M, k))
    Z[:m] = B
    Z *= signs_y(seed, M, blk)[:, None]
    Ft = sf.dct(Z, type=2, norm="ortho", axis=0)
    sel = _o.select(seed, M, l, _o.STREAM_YSEL, blk)
    return math.sqrt(M) * Ft[sel, :]


def apply_x_any(A, x, k, seed=0):
    """B = A X for x in gaussian / srht (oracle.c, X in A's storage format as
    the plain oracle draws it), hrtt, srct."""
    if x == "hrtt":
        return apply_x(A, k, seed=seed)
    if x == "srct":
        return apply_x_srct(A, k, seed=seed)
    return _o.apply_x(A, _o.SRHT if x == "srht" else _o.GAUSSIAN, k, seed=seed)


def rank_estimate_any(A, eps, x="gaussian", y="srct", k=40, l=None, seed=0):
    """Algorithm 1 with any X kind and a Gaussian, SRHT or SRCT Y: (r, sigma[k],
    r1, flags).  Gaussian / SRHT Y as the plain oracle draws them (A's storage
    format)."""
    A = np.ascontiguousarray(A)
    l = 2 * k if l is None else l
    B = apply_x_any(A, x, k, seed=seed)
    if y == "srct":
        Cm = apply_y_srct(B, l, seed=seed)
    else:
        fmt = _o.FMT_F64 if A.dtype == np.float64 else _o.FMT_F32
        Cm = _o.apply_y(B, _o.SRHT if y == "srht" else _o.GAUSSIAN, l, fmt_y=fmt, seed=seed)
    s, _, st = _o.jacobi_sv(Cm)
    if st != 0:
        raise _o.OracleError(st)
    s = s / math.sqrt(k * l)
    r1 = _o.r1_from_k(k)
    r, flags = _o.rank_count(s, r1, eps)
    return r, s, r1, flags


def rank_estimate(A, eps, k=40, l=None, ykind=_o.GAUSSIAN, seed=0, x="hrtt"):
    """Algorithm 1 with the HRTT (x="hrtt") or SRCT (x="srct") X: (r, sigma[k],
    r1, flags); Y Gaussian or SRHT in A's storage format, as the plain oracle
    draws it."""
    A = np.ascontiguousarray(A)
    l = 2 * k if l is None else l
    fmt = _o.FMT_F64 if A.dtype == np.float64 else _o.FMT_F32
    B = apply_x(A, k, seed=seed) if x == "hrtt" else apply_x_srct(A, k, seed=seed)
    Cm = _o.apply_y(B, ykind, l, fmt_y=fmt, seed=seed)
    s, _, st = _o.jacobi_sv(Cm)
    if st != 0:
        raise _o.OracleError(st)
    s = s / math.sqrt(k * l)
    r1 = _o.r1_from_k(k)
    r, flags = _o.rank_count(s, r1, eps)
    return r, s, r1, flags
