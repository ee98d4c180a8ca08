"""Pins of the gap statistics and of the tolerance-free search of Sec. 6.1
(oracle/gap.py) against closed forms: planted jumps in geometric sequences, the
reduced A_G of Sec. 6 (blocks at 1, 1e-4, 1e-8, 1e-12, 1e-16) whose rounds,
widths and gaps follow from which gaps lie inside the first r1 estimates, an
exact-rank matrix, gaps spaced wider than the growth step, the zero matrix and
a gap-free spectrum.  No GPU needed."""
import math

import numpy as np
import pytest

from paper_2105_07388_amd import inputs


def _geom(n, q, jumps):
    """s_i = q^(i-1), divided by J after index g for every (g, J) in jumps."""
    s = q ** np.arange(n, dtype=np.float64)
    for g, J in jumps:
        s[g:] /= J
    return s


def test_statistics_on_planted_jumps(orc):
    gp = orc.gap
    s = _geom(50, 0.9, [(12, 1e3)])
    # every ratio is 1/0.9 except s_12 / s_13 = 1e3 / 0.9
    assert gp.gap_rank(s, 40) == (12, pytest.approx(1e3 / 0.9, rel=1e-12))
    assert gp.deepest_gap(s, 40, 100.0)[0] == 12
    assert gp.deepest_gap(s, 12, 100.0) == (0, 0.0)  # the jump needs s_13, the 13th estimate
    assert gp.deepest_gap(s, 13, 100.0)[0] == 12
    s2 = _geom(60, 0.9, [(10, 1e6), (30, 1e3)])
    assert gp.gap_rank(s2, 50)[0] == 10  # the largest ratio
    assert gp.deepest_gap(s2, 50, 100.0)[0] == 30  # the last ratio above gamma
    assert gp.deepest_gap(s2, 50, 2e6)[0] == 0
    # ties go to the smallest index; an exact zero after a positive value is infinite
    assert gp.gap_rank(np.array([4.0, 2.0, 1.0, 0.5]), 4)[0] == 1
    z = np.array([3.0, 2.0, 0.0, 0.0])
    assert gp.gap_rank(z, 4) == (2, math.inf) and gp.deepest_gap(z, 4, 10.0) == (2, math.inf)
    assert gp.gap_rank(np.zeros(5), 5) == (0, 0.0) and gp.deepest_gap(np.zeros(5), 5, 10.0) == (0, 0.0)


def test_widths_and_rows(orc):
    gp = orc.gap
    assert list(gp.widths(110, 100, 500)) == [110, 210, 310, 410, 500]
    assert list(gp.widths(22, 20, 122)) == [22, 42, 62, 82, 102, 122]
    assert list(gp.widths(50, 10, 30)) == [30]
    assert gp.l_for(110, 1.5, 10**6) == 165 and gp.l_for(41, 1.5, 10**6) == 62 and gp.l_for(100, 1.5, 120) == 120


def _ag(m, block, dense=False):
    s = inputs.spectrum_gap(m, block)
    if dense:  # the same spectrum with Haar singular vectors, so B = A X has no coherent rows
        return inputs.planted(m, m, s, 606).numpy()
    return inputs.diagonal(m, m, s).numpy()


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("ykind,dense", [(0, False), (0, True), (1, True)])
def test_reduced_ag_rounds_in_closed_form(orc, seed, ykind, dense):
    """A_G with blocks of 20 (400 x 400, FP64; diagonal as in Sec. 6, or with
    Haar singular vectors), k0 = 22, dk = 20.  r1(k) = 20, 38, 56, 74, 93, 111
    for k = 22 ... 122, so round j reveals every planted gap below r1 (20, 40,
    60, 80): deepest gaps 0, 20, 40, 60, 80; the estimates past 80 sit at the
    1e-16 level (below the floor 1e-13) from k = 102 on, and k = 122 repeats
    the gap at 80: six rounds."""
    out = orc.gap.gap_search(_ag(400, 20, dense), k0=22, dk=20, gamma=100.0, floor=1e-13, ykind=ykind, seed=seed)
    assert [orc.r1_from_k(k) for k in (22, 42, 62, 82, 102, 122)] == [20, 38, 56, 74, 93, 111]
    assert out["gaps"] == [0, 20, 40, 60, 80, 80]
    assert (out["r"], out["k"], out["l"], out["rounds"], out["flags"]) == (80, 122, 183, 6, 0)
    assert out["ratio"] >= 100.0
    s = out["spectra"][-1]
    # the estimates keep the orders of magnitude of the blocks (Sec. 3: sketched
    # singular values within modest factors of the true ones)
    for b, lev in enumerate((1.0, 1e-4, 1e-8, 1e-12)):
        blk = s[20 * b:20 * (b + 1)]
        assert np.all(blk > lev / 30) and np.all(blk < lev * 30), (b, blk.min(), blk.max())
    assert out["argmax"] in (20, 40, 60, 80)


def test_srht_y_on_the_diagonal_ag_misplaces_a_gap(orc):
    """The coherent case of Sec. 6.2: on the diagonal A_G, B = A X keeps the
    block structure in its rows, and a subsampled Hadamard Y restricted to the
    first 40 rows has too few distinct rows (its columns below 64 depend on the
    low six bits of the sampled row index only), so it shows fewer than 20
    values of the second block and reports a gap inside it; a Gaussian Y sees
    the block whole."""
    A = _ag(400, 20)
    s_h = orc.gap.estimates(A, 42, 63, 1, 0)
    s_g = orc.gap.estimates(A, 42, 63, 0, 0)
    assert 20 < orc.gap.deepest_gap(s_h, 38, 100.0)[0] < 38
    assert orc.gap.deepest_gap(s_g, 38, 100.0)[0] == 20
    assert np.count_nonzero(s_g[20:40] > 1e-6) == 20 > np.count_nonzero(s_h[20:40] > 1e-6)


def test_exact_rank_stops_after_two_rounds(orc):
    A = inputs.exact_rank(300, 200, 15, 5).numpy()
    out = orc.gap.gap_search(A, k0=20, dk=20, gamma=100.0, floor=1e-13, seed=3)
    assert (out["r"], out["rounds"], out["k"], out["flags"]) == (15, 2, 40, 0)
    assert out["spectra"][0][15] <= 1e-13 * out["spectra"][0][0]


def test_floor_keeps_searching_past_a_stable_shallow_gap(orc):
    """Gaps at 10 (1 -> 1e-5) and 60 (1e-5 -> 1e-16), dk = 10: the gap at 10 is
    stable from k = 22 on, but the estimates stay above the floor until r1 > 60;
    r1 = 65 at k = 72 reveals 60 and k = 82 repeats it."""
    s = np.full(300, 1e-16)
    s[:10] = 1.0
    s[10:60] = 1e-5
    A = inputs.diagonal(300, 300, s).numpy()
    out = orc.gap.gap_search(A, k0=12, dk=10, gamma=100.0, floor=1e-13, seed=4)
    assert out["gaps"][:2] == [10, 10] and out["gaps"][-2:] == [60, 60]
    assert (out["r"], out["k"], out["rounds"], out["flags"]) == (60, 82, 8, 0)
    loose = orc.gap.gap_search(A, k0=12, dk=10, gamma=100.0, floor=1.0, seed=4)
    assert (loose["r"], loose["k"], loose["rounds"]) == (10, 22, 2)


def test_zero_matrix_and_no_gap(orc):
    out = orc.gap.gap_search(np.zeros((64, 48)), k0=8, dk=8, seed=1)
    assert (out["r"], out["rounds"], out["flags"]) == (0, 1, orc.gap.FLAG_ZERO)
    A = inputs.diagonal(200, 200, 0.97 ** np.arange(200)).numpy()
    out = orc.gap.gap_search(A, k0=16, dk=16, kmax=64, gamma=100.0, seed=2)
    assert (out["r"], out["k"], out["rounds"], out["flags"]) == (0, 64, 4, orc.gap.FLAG_NOT_CONVERGED)


def test_round_estimates_match_the_plain_oracle(orc):
    """The search's per-round estimates (numpy FP64 products of the oracle's
    draws) equal oracle.c's plain-loop Algorithm 1 at the same (k, l, seed)."""
    A = _ag(160, 8)
    for k, l in ((12, 18), (22, 33)):
        got = orc.gap.estimates(A, k, l, 1, 7)
        _, want, _, _, _ = orc.rank_estimate(A, 0.5, orc.GAUSSIAN, orc.SRHT, k=k, l=l, seed=7)
        assert np.all(np.abs(got - want) <= 1e-12 * want[0])
