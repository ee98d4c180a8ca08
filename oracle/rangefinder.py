"""FP64 oracle of Algorithm 3 (rank estimation followed by the randomized
rangefinder), test infrastructure only: only tests/, the package smoke check
and the benchmark's CPU-baseline leg may import it.

Steps in the paper's order (Sec. 5.1, Algorithm 3):
  1. rank estimation: the estimates s_i of Algorithm 1 (`pyoracle.rank_estimate`,
     Gaussian X and Y, s_i = sigma_i(Y A X) / sqrt(k l)) for i <= r1;
  2. extend them with s_i = s_{r1} for r1 < i <= n;
  3. r = the smallest integer whose a priori Frobenius bound (Halko, Martinsson
     and Tropp 2011, Thm. 10.5, with the estimates in place of the true values)
     (1 + r / (p - 1))^(1/2) (sum_{j>r} s_j^2)^(1/2) is at most eps ||A||, with
     ||A|| estimated by s_1 unless given; when no r with r + p <= k exists the
     estimation is repeated with a larger r1 (k doubled, appended sketches);
  4. keep the first w = r + p columns of A X;
  5. thin QR of them (Householder, numpy), signs fixed so that diag(R) > 0;
  6. B = Q^T A.
"""
import math

import numpy as np

from . import pyoracle as _o
from .learned import l_for


def tail_bound(sigma, r1, n, r, p):
    """(1 + r/(p-1))^(1/2) (sum_{j>r} s_j^2)^(1/2) over the extended estimates."""
    s = np.asarray(sigma, dtype=np.float64)[:r1]
    head = float(np.sum(s[r:] ** 2)) if r < r1 else 0.0
    extra = (n - max(r, r1)) * s[r1 - 1] ** 2
    return math.sqrt(1.0 + r / (p - 1)) * math.sqrt(head + extra)


def choose_rank(sigma, r1, n, eps, p, norm_a=None):
    """The smallest r >= 1 with tail_bound <= eps ||A|| among r + p <= len(sigma),
    0 when s_1 = 0 (a zero sketch), None when no width qualifies."""
    s = np.asarray(sigma, dtype=np.float64)
    r1 = min(int(r1), len(s))
    if not s[0] > 0.0:
        return 0
    target = eps * (s[0] if norm_a is None else norm_a)
    for r in range(1, len(s) - p + 1):
        if tail_bound(s, r1, n, r, p) <= target:
            return r
    return None


def thin_qr(W):
    """Householder thin QR of W (rows >= cols), columns signed so diag(R) >= 0."""
    Q, R = np.linalg.qr(np.asarray(W, dtype=np.float64))
    d = np.sign(np.diagonal(R))
    d[d == 0] = 1.0
    return Q * d, R * d[:, None]


def rangefinder(A, eps, p, k0=32, kmax=None, l_ratio=2.0, norm_a=None, seed=0):
    """Algorithm 3 on A (numpy, FP32 or FP64).  Returns dict(r, w, k, l, rounds,
    r1, sigma, Q, B); r is None (Q, B None) when no width up to kmax qualifies."""
    A = np.asarray(A)
    m, n = A.shape
    kmax = min(m, n, kmax or min(m, n))
    k = min(k0, kmax)
    rounds = 0
    while True:
        l = l_for(k, l_ratio, m)
        _, sigma, r1, _, _ = _o.rank_estimate(A, 0.5, _o.GAUSSIAN, _o.GAUSSIAN, k=k, l=l, seed=seed)
        rounds += 1
        r = choose_rank(sigma, r1, n, eps, p, norm_a)
        if r is not None or k >= kmax:
            break
        k = min(2 * k, kmax)
    out = dict(r=r, w=None, k=k, l=l, rounds=rounds, r1=r1, sigma=sigma, Q=None, B=None)
    if r is None or r == 0:
        out["w"] = 0 if r == 0 else None
        return out
    w = r + p
    AX = _o.apply_x(A, _o.GAUSSIAN, k, seed=seed)[:, :w]
    Q, _ = thin_qr(AX)
    out.update(w=w, Q=Q, B=Q.T @ A.astype(np.float64))
    return out
