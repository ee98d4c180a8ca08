"""ctypes wrapper around oracle/liboracle.so (test infrastructure only).

Each function mirrors one step of Algorithm 1 of Meier & Nakatsukasa
(arXiv 2105.07388) as implemented in oracle.c; see that file for the
citations.  Arrays are numpy, FP64 unless stated.
"""
import ctypes as C
import os

import numpy as np

from .build import LIB
from .build import build as _build_lib

GAUSSIAN, SRHT = 0, 1
FMT_F64, FMT_F32, FMT_BF16, FMT_F16 = 0, 1, 2, 3
FLAG_NOT_CONVERGED, FLAG_ZERO = 1, 2
STREAM_XGAUSS, STREAM_YGAUSS, STREAM_XSIGN, STREAM_YSIGN, STREAM_XSEL, STREAM_YSEL = 1, 2, 3, 4, 5, 6

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build_lib()
        L = C.CDLL(LIB)
        u64, i64, i32, dbl, vp = C.c_uint64, C.c_int64, C.c_int, C.c_double, C.c_void_p
        L.or_philox4x64_10.argtypes = [vp, vp, vp]
        L.or_gauss.argtypes = [u64, u64, u64, u64, u64]
        L.or_gauss.restype = dbl
        L.or_round_to.argtypes = [dbl, i32]
        L.or_round_to.restype = dbl
        L.or_sign.argtypes = [u64, u64, u64, u64]
        L.or_sign.restype = i32
        L.or_select_key.argtypes = [u64, u64, u64, u64]
        L.or_select_key.restype = u64
        L.or_select.argtypes = [u64, i64, i64, u64, u64, vp]
        L.or_select.restype = i32
        L.or_fwht.argtypes = [vp, i64]
        L.or_next_pow2.argtypes = [i64]
        L.or_next_pow2.restype = i64
        L.or_r1_from_k.argtypes = [i32]
        L.or_r1_from_k.restype = i32
        L.or_rank_def.argtypes = [vp, i32, dbl]
        L.or_rank_def.restype = i32
        L.or_apply_x.argtypes = [vp, i32, i64, i64, i64, i32, i64, i32, u64, u64, vp]
        L.or_apply_x.restype = i32
        L.or_apply_y.argtypes = [vp, i64, i64, i32, i64, i32, u64, u64, vp]
        L.or_apply_y.restype = i32
        L.or_jacobi_sv.argtypes = [vp, i64, i64, i32, vp, vp]
        L.or_jacobi_sv.restype = i32
        L.or_rank_count.argtypes = [vp, i32, i32, dbl, vp, vp]
        L.or_rank_count.restype = i32
        L.or_x_format.argtypes = [i32, i32]
        L.or_x_format.restype = i32
        L.or_y_format.argtypes = [i32]
        L.or_y_format.restype = i32
        L.or_rank_estimate.argtypes = [vp, i32, i64, i64, i64, dbl, i32, i32, i64, i64, i32, u64, u64,
                                       vp, vp, vp, vp, vp]
        L.or_rank_estimate.restype = i32
        L.or_num_threads.restype = i32
        L.or_gauss_matrix.argtypes = [u64, i64, i64, u64, u64, i32, i32, vp]
        L.or_gauss_matrix.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(C.c_void_p)


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def _check(st):
    if st != 0:
        raise OracleError(st)


def philox4x64_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gauss(seed, a, b, stream, blk=0):
    return lib().or_gauss(seed, a, b, stream, blk)


def round_to(v, fmt):
    return lib().or_round_to(float(v), fmt)


def sign(seed, i, stream, blk=0):
    return lib().or_sign(seed, i, stream, blk)


def select_key(seed, i, stream, blk=0):
    return lib().or_select_key(seed, i, stream, blk)


def select(seed, npad, k, stream, blk=0):
    idx = np.zeros(max(k, 1), dtype=np.int64)
    _check(lib().or_select(seed, npad, k, stream, blk, _ptr(idx)))
    return idx[:k]


def fwht(x):
    y = np.array(x, dtype=np.float64, copy=True)
    lib().or_fwht(_ptr(y), y.size)
    return y


def next_pow2(v):
    return lib().or_next_pow2(v)


def r1_from_k(k):
    return lib().or_r1_from_k(k)


def rank_def(sigma, eps):
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    return lib().or_rank_def(_ptr(s), s.size, eps)


def _a_dtype(A):
    if A.dtype == np.float64:
        return FMT_F64
    if A.dtype == np.float32:
        return FMT_F32
    raise TypeError("A must be float32 or float64")


def apply_x(A, xkind, k, fmt_x=None, seed=0, blk=0):
    A = np.ascontiguousarray(A)
    m, n = A.shape
    dt = _a_dtype(A)
    if fmt_x is None:
        fmt_x = dt
    B = np.zeros((m, k), dtype=np.float64)
    _check(lib().or_apply_x(_ptr(A), dt, m, n, n, xkind, k, fmt_x, seed, blk, _ptr(B)))
    return B


def apply_y(B, ykind, l, fmt_y=FMT_F64, seed=0, blk=0):
    B = np.ascontiguousarray(B, dtype=np.float64)
    m, k = B.shape
    Cm = np.zeros((l, k), dtype=np.float64)
    _check(lib().or_apply_y(_ptr(B), m, k, ykind, l, fmt_y, seed, blk, _ptr(Cm)))
    return Cm


def jacobi_sv(Cm, max_sweeps=60):
    Cm = np.ascontiguousarray(Cm, dtype=np.float64)
    l, k = Cm.shape
    s = np.zeros(max(k, 1), dtype=np.float64)
    sw = C.c_int(0)
    st = lib().or_jacobi_sv(_ptr(Cm), l, k, max_sweeps, _ptr(s), C.byref(sw))
    return s[:k], sw.value, st


def rank_count(sigma, r1, eps):
    s = np.ascontiguousarray(sigma, dtype=np.float64)
    r = C.c_int(0)
    fl = C.c_uint(0)
    _check(lib().or_rank_count(_ptr(s), s.size, r1, eps, C.byref(r), C.byref(fl)))
    return r.value, fl.value


def x_format(dtype_code, prec):
    return lib().or_x_format(dtype_code, prec)


def rank_estimate(A, eps, xkind=GAUSSIAN, ykind=GAUSSIAN, k=40, l=None, prec=0, seed=0, blk=0):
    """Algorithm 1 end to end; returns (r, sigma[k], r1, flags, sweeps)."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    if l is None:
        l = 2 * k
    dt = _a_dtype(A)
    s = np.zeros(k, dtype=np.float64)
    r = C.c_int(0)
    r1 = C.c_int(0)
    fl = C.c_uint(0)
    sw = C.c_int(0)
    _check(lib().or_rank_estimate(_ptr(A), dt, m, n, n, eps, xkind, ykind, k, l, prec, seed, blk,
                                  C.byref(r), _ptr(s), C.byref(r1), C.byref(fl), C.byref(sw)))
    return r.value, s, r1.value, fl.value, sw.value


def gauss_matrix(seed, rows, cols, stream, fmt, swap=False, blk=0):
    """The Gaussian embedding as a dense FP64 matrix of its rounded entries
    (oracle.c or_gauss_matrix): X = gauss_matrix(seed, n, k, 1, fmt) and
    Y = gauss_matrix(seed, l, m, 2, fmt, swap=True)."""
    G = np.zeros((rows, cols), dtype=np.float64)
    lib().or_gauss_matrix(seed, rows, cols, stream, blk, fmt, int(bool(swap)), _ptr(G))
    return G


def rank_estimate_gemm(A, eps, xkind=GAUSSIAN, ykind=GAUSSIAN, k=40, l=None, prec=0, seed=0, blk=0,
                       X=None, Y=None):
    """Algorithm 1 (Sec. 5) as rank_estimate, with the Gaussian products of
    steps 3 and 6 taken by numpy's FP64 matrix product (a library primitive)
    instead of oracle.c's plain loops, so that the oracle finishes at the
    workloads' full sizes.  The embeddings are the same rounded entries
    (gauss_matrix); an SRHT side runs oracle.c's transform.  X (n x k) and Y
    (l x m) may be passed in as leading blocks of larger master draws.
    Returns (r, sigma[k], r1, flags, sweeps)."""
    A = np.ascontiguousarray(A)
    m, n = A.shape
    if l is None:
        l = 2 * k
    dt = _a_dtype(A)
    if xkind == GAUSSIAN:
        if X is None:
            X = gauss_matrix(seed, n, k, STREAM_XGAUSS, x_format(dt, prec), blk=blk)
        B = A.astype(np.float64) @ X[:n, :k]
    else:
        if prec != 0:
            raise OracleError(-2)
        B = apply_x(A, xkind, k, seed=seed, blk=blk)
    if ykind == GAUSSIAN:
        if Y is None:
            Y = gauss_matrix(seed, l, m, STREAM_YGAUSS, lib().or_y_format(dt), swap=True, blk=blk)
        Cm = Y[:l, :m] @ B
    else:
        Cm = apply_y(B, ykind, l, seed=seed, blk=blk)
    s, sw, st = jacobi_sv(Cm)
    _check(st)
    s = s / np.sqrt(float(k) * float(l))
    r1 = r1_from_k(k)
    r, fl = rank_count(s, r1, eps)
    return r, s, r1, fl, sw


def num_threads():
    return lib().or_num_threads()
