"""Gap-based rank without a tolerance (test infrastructure only).

When no eps is given, Sec. 5 (after Algorithm 1) suggests reading the gap off
the sketched spectrum, e.g. r^ = argmax_i s_i / s_{i+1}; Sec. 6.1 uses the
sketched singular values this way to reveal the gaps of its test matrix A_G,
growing a Gaussian X by 100 columns per round from 110 (an SRTT Y) until the
gap shows.  Only the first r1 estimates are used (the oversampled ones are
discarded, Sec. 3.2).

Plain definitions (1-based i, over 1 <= i < r1 with s_i > 0; a zero s_{i+1}
after a positive s_i is an infinite ratio):
  gap_rank:      the i with the largest s_i / s_{i+1}, ties to the smallest i
                 (Sec. 5's measure); 0 when s_1 = 0 or r1 < 2.
  deepest_gap:   the largest i with s_i / s_{i+1} >= gamma; 0 when none.
The search (gap_search) follows Sec. 6.1 with these readings: round j uses
the width k_j = k0 + j dk (capped at k_max) and l = round(l_ratio k) rows; the
sketches nest, so round j's estimates are Algorithm 1's at (k_j, l_j) with the
same seed.  It stops after the first round whose first r1 estimates reach
below floor * s_1 (the spectrum has been followed down to the floor) and
whose deepest gap equals the previous round's; or at k_max (flag
NOT_CONVERGED unless that holds there), or when s_1 = 0 (flag ZERO, r^ = 0).
r^ is the deepest gap of the last round.
"""
import math

import numpy as np


from . import pyoracle as _o

FLAG_NOT_CONVERGED, FLAG_ZERO = 1, 2


def _ratios(sigma, r1):
    """(i, s_i / s_{i+1}) for 1 <= i < r1 while s_i > 0."""
    s = [float(v) for v in sigma]
    r1 = min(int(r1), len(s))
    out = []
    for i in range(1, r1):
        a, b = s[i - 1], s[i]
        if not a > 0.0:
            break  # everything after a zero estimate is zero
        out.append((i, math.inf if b <= 0.0 else a / b))
    return out


def gap_rank(sigma, r1):
    """Returns (r^, ratio s_r / s_{r+1}) with r^ the argmax of the ratios."""
    s0 = float(sigma[0]) if len(sigma) else 0.0
    if min(int(r1), len(sigma)) < 2 or not s0 > 0.0:
        return 0, 0.0
    best_i, best = 0, -1.0
    for i, q in _ratios(sigma, r1):
        if q > best:
            best_i, best = i, q
    return best_i, best


def deepest_gap(sigma, r1, gamma):
    """Returns (g, ratio s_g / s_{g+1}): the largest i < r1 with ratio >= gamma."""
    g, q_g = 0, 0.0
    for i, q in _ratios(sigma, r1):
        if q >= gamma:
            g, q_g = i, q
    return g, q_g


def l_for(k, l_ratio, m):
    return int(min(max(int(math.floor(l_ratio * k + 0.5)), k), m))


def widths(k0, dk, kmax):
    """k0, k0 + dk, ..., capped at kmax (which is always the last width)."""
    k = min(k0, kmax)
    while True:
        yield k
        if k >= kmax:
            return
        k = min(k + dk, kmax)


def estimates(A, k, l, ykind, seed):
    """Algorithm 1's k scaled estimates at (k, l) with a Gaussian X (FP64
    library products of the rounded draws) and a Gaussian, SRHT or (ykind =
    "srct") subsampled randomized DCT Y."""
    if ykind == "srct":
        from . import hrtt
        Xg = _o.gauss_matrix(seed, A.shape[1], k, _o.STREAM_XGAUSS, _o.x_format(_o._a_dtype(A), 0))
        Cm = hrtt.apply_y_srct(np.asarray(A, dtype=np.float64) @ Xg, l, seed=seed)
        s, _, st = _o.jacobi_sv(Cm)
        if st != 0:
            raise _o.OracleError(st)
        return s / math.sqrt(float(k) * float(l))
    _, s, _, _, _ = _o.rank_estimate_gemm(A, 0.5, _o.GAUSSIAN, ykind, k=k, l=l, seed=seed)
    return s


def gap_search(A, k0=110, dk=100, kmax=None, l_ratio=1.5, gamma=100.0, floor=1e-13, ykind=_o.GAUSSIAN, seed=0):
    """The search of Sec. 6.1 as described in the module docstring.  Returns a
    dict with r (deepest gap of the last round), ratio, argmax (Sec. 5's
    measure on the last round) and its ratio, k, l, rounds, the spectra of
    every round (list of arrays), the deepest gap of every round, and flags."""
    m, n = A.shape
    if kmax is None:
        kmax = min(m, n)
    kmax = min(int(kmax), m, n)
    spectra, gaps = [], []
    prev = None
    for k in widths(int(k0), int(dk), kmax):
        l = l_for(k, l_ratio, m)
        s = estimates(A, k, l, ykind, seed)
        r1 = _o.r1_from_k(k)
        spectra.append(s)
        out = {"k": k, "l": l, "rounds": len(spectra), "spectra": spectra, "gaps": gaps}
        if not s[0] > 0.0:
            gaps.append(0)
            out.update(r=0, ratio=0.0, argmax=0, argmax_ratio=0.0, flags=FLAG_ZERO)
            return out
        g, q = deepest_gap(s, r1, gamma)
        gaps.append(g)
        a, qa = gap_rank(s, r1)
        out.update(r=g, ratio=q, argmax=a, argmax_ratio=qa)
        reached = s[min(r1, len(s)) - 1] <= floor * s[0]
        done = g > 0 and g == prev and reached
        if done or k >= kmax:
            out["flags"] = 0 if done else FLAG_NOT_CONVERGED
            return out
        prev = g
