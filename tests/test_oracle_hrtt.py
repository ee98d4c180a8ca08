"""Pins of the HRTT sketch oracle (oracle/hrtt.py): the DCT step against its
definition, the hashing step against an explicit matrix, the whole X against
the product D F^T H^T written out, uniform buckets, the expected isometry, and
the paper's remark that the hashed transform handles a diagonal (coherent)
matrix where the subsampled one does not."""
import math

import numpy as np
import pytest
import scipy.stats as st

from paper_2105_07388_amd import inputs


def test_dct_step_is_the_orthonormal_dct(orc):
    H = orc.hrtt
    for N in (2, 4, 16, 64):
        F = H.dct_matrix(N)
        assert np.allclose(F @ F.T, np.eye(N), atol=1e-13)
        x = np.random.default_rng(N).standard_normal(N)
        import scipy.fft as sf
        assert np.allclose(sf.dct(x, type=2, norm="ortho"), F @ x, atol=1e-13)


def test_whole_x_is_the_written_out_product(orc):
    H = orc.hrtt
    rng = np.random.default_rng(5)
    m, n, k, seed = 7, 13, 5, 11
    A = rng.standard_normal((m, n))
    N = H.npad(n)
    D = np.diag(H.signs(seed, N))
    b, s = H.hash_table(seed, N, k)
    Hm = np.zeros((k, N))
    Hm[b, np.arange(N)] = s
    X = (D @ H.dct_matrix(N).T @ Hm.T)[:n] * math.sqrt(k)  # n x k
    assert np.allclose(H.apply_x(A, k, seed=seed), A @ X, atol=1e-12)
    # the hash is the published Philox draw: bucket = floor(w0 k / 2^64), sign from w1
    w = orc.philox4x64_10([3, 0, 7, 0], [seed, 0])
    assert b[3] == (int(w[0]) * k) >> 64 and s[3] == (1.0 if int(w[1]) % 2 == 0 else -1.0)


def test_buckets_uniform_and_isometry_in_expectation(orc):
    H = orc.hrtt
    b, s = H.hash_table(1, 8192, 64)
    counts = np.bincount(b, minlength=64)
    assert st.chisquare(counts).pvalue > 1e-3
    assert abs(np.mean(s)) < 4 / math.sqrt(8192)
    # E ||Theta x||^2 = ||x||^2 for the CountSketch of an orthogonal transform
    x = np.random.default_rng(2).standard_normal((1, 100))
    r = [np.sum(H.apply_x(x, 16, seed=t) ** 2) / 16 / np.sum(x ** 2) for t in range(60)]
    assert abs(np.mean(r) - 1.0) < 4 * np.std(r) / math.sqrt(60)


def test_diagonal_matrix_hashed_beats_subsampled(orc):
    # Sec. 3.3 / 3.4: on a diagonal (maximally coherent) matrix with a gap at 30
    # the hashed DCT keeps the gap, while a subsampled transform can miss
    # coordinates and understate the rank
    n = 512
    s = np.concatenate([np.ones(30), 1e-8 * np.ones(n - 30)])
    A = np.diag(s)
    r, sig, r1, fl = orc.hrtt.rank_estimate(A, 1e-4, k=64, l=128, seed=3)
    assert r == 30
    rs, _, _, _, _ = orc.rank_estimate(A, 1e-4, orc.SRHT, orc.GAUSSIAN, k=64, l=128, seed=3)
    assert rs < 30


def test_srct_is_the_written_out_product(orc):
    H = orc.hrtt
    rng = np.random.default_rng(8)
    m, n, k, seed = 6, 21, 9, 4
    A = rng.standard_normal((m, n))
    N = H.npad(n)
    D = np.diag(H.signs(seed, N))
    sel = orc.select(seed, N, k, orc.STREAM_XSEL)
    S = np.zeros((k, N))
    S[np.arange(k), sel] = 1.0
    X = (D @ H.dct_matrix(N).T @ S.T)[:n] * math.sqrt(N)  # n x k
    assert np.allclose(H.apply_x_srct(A, k, seed=seed), A @ X, atol=1e-12)
    # the sample nests in k and is the SRHT's
    assert np.array_equal(np.sort(sel), sel)
    assert set(orc.select(seed, N, k // 2, orc.STREAM_XSEL)) <= set(sel)


def test_srct_full_sample_is_orthogonal(orc):
    # k = N and l = m' sample every coordinate: both embeddings are sqrt(N) resp.
    # sqrt(m') times an orthogonal matrix, so the scaled estimates are sigma(A)
    rng = np.random.default_rng(3)
    m, n = 64, 32
    A = rng.standard_normal((m, 5)) @ rng.standard_normal((5, n)) + 1e-3 * rng.standard_normal((m, n))
    r, s, r1, fl = orc.hrtt.rank_estimate(A, 1e-2, k=n, l=m, ykind=orc.SRHT, seed=2, x="srct")
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s, sv, rtol=0, atol=1e-12 * sv[0])
    assert r == orc.rank_def(sv[:r1], 1e-2)


def test_srct_isometry_in_expectation(orc):
    x = np.random.default_rng(4).standard_normal((1, 100))
    r = [np.sum(orc.hrtt.apply_x_srct(x, 16, seed=t) ** 2) / 16 / np.sum(x ** 2) for t in range(80)]
    assert abs(np.mean(r) - 1.0) < 4 * np.std(r) / math.sqrt(80)


# --- the subsampled randomized DCT as Y -------------------------------------------------

def test_srct_y_is_the_written_out_product(orc):
    """C = sqrt(M) S F D_Y [B; 0] with F the DCT-II written out, D_Y the SRHT's Y
    signs and S the SRHT's Y sample (streams 4 and 6)."""
    H = orc.hrtt
    rng = np.random.default_rng(9)
    m, k, l, seed = 37, 6, 11, 5
    B = rng.standard_normal((m, k))
    M = H.npad(m)
    D = np.diag(H.signs_y(seed, M))
    sel = orc.select(seed, M, l, orc.STREAM_YSEL)
    S = np.zeros((l, M))
    S[np.arange(l), sel] = 1.0
    Y = (S @ H.dct_matrix(M) @ D)[:, :m] * math.sqrt(M)  # l x m
    assert np.allclose(H.apply_y_srct(B, l, seed=seed), Y @ B, atol=1e-12)
    assert np.array_equal(D.diagonal(), [orc.sign(seed, i, orc.STREAM_YSIGN) for i in range(M)])
    assert set(orc.select(seed, M, l // 2, orc.STREAM_YSEL)) <= set(sel)


def test_srct_y_full_sample_is_orthogonal(orc):
    """An SRHT X with k = N and an SRCT Y with l = M sample every coordinate: both
    are sqrt(N) resp. sqrt(M) times orthogonal maps, so the scaled estimates are
    sigma(A) and the rank is Def. 1's."""
    rng = np.random.default_rng(13)
    m, n = 48, 32
    A = rng.standard_normal((m, 4)) @ rng.standard_normal((4, n)) + 1e-3 * rng.standard_normal((m, n))
    r, s, r1, fl = orc.hrtt.rank_estimate_any(A, 1e-2, x="srht", y="srct", k=n, l=64, seed=3)
    sv = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s, sv, rtol=0, atol=1e-12 * sv[0])
    assert r == orc.rank_def(sv[:r1], 1e-2)


def test_srct_y_isometry_in_expectation(orc):
    b = np.random.default_rng(6).standard_normal((100, 1))
    r = [np.sum(orc.hrtt.apply_y_srct(b, 16, seed=t) ** 2) / 16 / np.sum(b ** 2) for t in range(80)]
    assert abs(np.mean(r) - 1.0) < 4 * np.std(r) / math.sqrt(80)


def test_srct_y_sees_the_coherent_block_the_srht_y_misses(orc):
    """The diagonal A_G (400 x 400, blocks of 20) with a Gaussian X of 42
    columns: B = A X keeps the blocks in its rows.  The subsampled Hadamard Y
    shows fewer than 20 values of the second block (its columns below 64
    depend on the low six bits of the sampled row only); the subsampled DCT Y,
    Sec. 6's choice for this matrix, shows all of them and no gap inside."""
    A = inputs.diagonal(400, 400, inputs.spectrum_gap(400, 20)).numpy()
    s_c = orc.gap.estimates(A, 42, 63, "srct", 0)
    s_h = orc.gap.estimates(A, 42, 63, orc.SRHT, 0)
    assert orc.gap.deepest_gap(s_c, 38, 100.0)[0] == 20
    assert np.count_nonzero(s_c[20:40] > 1e-6) == 20 > np.count_nonzero(s_h[20:40] > 1e-6)
    out = orc.gap.gap_search(A, k0=22, dk=20, gamma=100.0, floor=1e-13, ykind="srct", seed=1)
    assert out["gaps"] == [0, 20, 40, 60, 80, 80] and out["r"] == 80
