"""FP64 oracle of the QR-diagonal alternative to step 7 of Algorithm 1 (test
infrastructure only: only tests/, the package smoke check and the benchmark's
CPU-baseline leg may import it).

Sec. 5, after Algorithm 1: instead of the singular values of the sketch C = Y A X
one may take the magnitudes of the diagonal of R in a QR factorisation C = Q R;
with randomised right singular vectors an unpivoted QR is rank revealing with
high probability.  Here: Householder QR (numpy), |R_jj| sorted in descending
order (read as estimates of the ordered singular values), scaled by 1/sqrt(k l)
as the singular values are, then the count of Algorithm 1 step 8.
"""
import math

import numpy as np

from . import pyoracle as _o


def qr_diag(C):
    """|diag R| of the thin Householder QR of C (l x k, l >= k), descending."""
    R = np.linalg.qr(np.asarray(C, dtype=np.float64), mode="r")
    return np.sort(np.abs(np.diagonal(R)))[::-1].copy()


def sketch(A, xkind, ykind, k, l, seed=0):
    """C = Y A X with the formats of Algorithm 1's oracle: X rounded to A's
    storage format, Y to FP32 for an FP32 A, products in FP64."""
    A = np.ascontiguousarray(A)
    fmt = _o.FMT_F64 if A.dtype == np.float64 else _o.FMT_F32
    B = _o.apply_x(A, xkind, k, seed=seed)
    return _o.apply_y(B, ykind, l, fmt_y=fmt, seed=seed)


def rank_estimate_qr(A, eps, xkind=_o.GAUSSIAN, ykind=_o.GAUSSIAN, k=40, l=None, seed=0):
    """Algorithm 1 with step 7 by the QR diagonal: (r, d[k], r1, flags)."""
    l = 2 * k if l is None else l
    d = qr_diag(sketch(A, xkind, ykind, k, l, seed)) / math.sqrt(k * l)
    r1 = _o.r1_from_k(k)
    r, flags = _o.rank_count(d, r1, eps)
    return r, d, r1, flags
