"""Gap-based rank without a tolerance (test infrastructure only).

When no eps is given, Sec. 5 (after Algorithm 1) suggests reading the gap off
the sketched spectrum, e.g. r^ = argmax_i s_i / s_{i+1}; Sec. 6.1 uses the
sketched singular values this way to reveal the gap of its test matrix.  Only
the first r1 estimates are used (the oversampled ones are discarded, Sec.
3.2).  Plain definition: the 1-based i in 1..r1-1 with the largest ratio
s_i / s_{i+1} (a zero s_{i+1} after a positive s_i is an infinite ratio;
ties go to the smallest i); r^ = 0 when s_1 = 0 or r1 < 2.
"""
import math


def gap_rank(sigma, r1):
    """Returns (r^, ratio s_r / s_{r+1})."""
    s = [float(v) for v in sigma]
    r1 = min(int(r1), len(s))
    if r1 < 2 or not s[0] > 0.0:
        return 0, 0.0
    best_i, best = 0, -1.0
    for i in range(1, r1):  # ratio s_i / s_{i+1}, 1-based i
        a, b = s[i - 1], s[i]
        if not a > 0.0:
            break  # everything after a zero estimate is zero
        q = math.inf if b <= 0.0 else a / b
        if q > best:
            best_i, best = i, q
    return best_i, best
