"""GPU tests of the hashed randomized DCT sketch (HRTT X) against the oracle
(oracle/hrtt.py).

Tolerance of B = A X, per row: the FP32 FFT's normwise error (6 log2 N + 6) u32
||a|| (Cooley-Tukey with twiddles within 2 ulp, Higham Thm. 24.2, plus the
post-twiddle), through the CountSketch (norm sqrt(max bucket)), plus the
rounding of each bucket's sum (max bucket^(3/2) u32 ||a||), times sqrt(k).
Estimates: that error through Y, |d sigma| <= 1.1 (sqrt m + sqrt l) ||dB||_F /
sqrt(k l).  Ranks compared on gaps.
"""
import math

import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_
from paper_2105_07388_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"
U32 = 2.0 ** -24


def _row_tol(orc, n, k, seed, anorm):
    N = orc.hrtt.npad(n)
    lg = int(math.log2(N))
    b, _ = orc.hrtt.hash_table(seed, N, k)
    bmax = int(np.bincount(b, minlength=k).max())
    return math.sqrt(k) * (math.sqrt(bmax) * (6 * lg + 6) + bmax ** 1.5) * U32 * anorm


@pytest.mark.parametrize("m,n,k", [(300, 1000, 64), (257, 1024, 7), (64, 2049, 384), (50, 1, 1), (33, 2, 2),
                                   (40, 3, 4), (128, 16384, 384), (90, 700, 700), (70, 2048, 100), (66, 4096, 300),
                                   (40, 8192, 1000), (48, 64, 64), (48, 512, 33)])
def test_sketch_x_matches_oracle(orc, m, n, k):
    A = inputs.gaussian(m, n, 100 + n, torch.float32)
    seed = 17 + k
    Bg = re_.sketch_x(A.to(DEV), k=k, x="hrtt", seed=seed).cpu().numpy().astype(np.float64)
    Bo = orc.hrtt.apply_x(A.numpy(), k, seed=seed)
    err = np.linalg.norm(Bg - Bo, axis=1)
    tol = np.array([_row_tol(orc, n, k, seed, float(np.linalg.norm(a))) for a in A.double().numpy()])
    assert np.all(err <= tol), float(np.max(err / tol))


@pytest.mark.parametrize("off,pad", [(1, 3), (0, 4), (2, 5)])
def test_sketch_x_row_views(orc, off, pad):
    # rows of a wider matrix: a pointer off the 16-byte grid or a row stride
    # that is not a multiple of 4 takes the scalar loads, the rest the vector ones
    m, n, k = 96, 1024, 100
    S = inputs.gaussian(m, n + pad, 77 + off, torch.float32)
    A = S[:, off:off + n]
    seed = 5
    Bg = re_.sketch_x(S.to(DEV)[:, off:off + n], k=k, x="hrtt", seed=seed).cpu().numpy().astype(np.float64)
    Bo = orc.hrtt.apply_x(A.numpy(), k, seed=seed)
    err = np.linalg.norm(Bg - Bo, axis=1)
    tol = np.array([_row_tol(orc, n, k, seed, float(np.linalg.norm(a))) for a in A.double().numpy()])
    assert np.all(err <= tol), float(np.max(err / tol))


def test_rank_estimate_matches_oracle_on_a_gap(orc):
    A = inputs.planted(1500, 1000, inputs.spectrum_step(1000, 20, 1.0, 1e-8), 31, torch.float32)
    k, l = 40, 60
    for y, ykind in (("gaussian", orc.GAUSSIAN), ("srht", orc.SRHT)):
        r, s, info = re_.rank_estimate(A.to(DEV), 1e-5, k=k, l=l, x="hrtt", y=y, seed=6)
        ro, so, r1, fl = orc.hrtt.rank_estimate(A.numpy(), 1e-5, k=k, l=l, ykind=ykind, seed=6)
        assert r == ro == 20 and info["flags"] == fl
        dB = math.sqrt(sum(_row_tol(orc, 1000, k, 6, float(np.linalg.norm(a))) ** 2 for a in A.double().numpy()))
        tol = 1.1 * (math.sqrt(1500) + math.sqrt(l)) * dB / math.sqrt(k * l) + 1e-12 * so[0]
        assert np.all(np.abs(s - so) <= tol), (float(np.max(np.abs(s - so))), tol)


def test_coherent_diagonal_matrix(orc):
    # Sec. 3.3: the hashed transform keeps the gap of a diagonal matrix, the
    # subsampled Hadamard transform does not (the same on both sides)
    n = 512
    A = torch.diag(torch.cat([torch.ones(30), 1e-8 * torch.ones(n - 30)])).float()
    r, _, _ = re_.rank_estimate(A.to(DEV), 1e-4, k=64, l=128, x="hrtt", seed=3)
    ro, _, _, _ = orc.hrtt.rank_estimate(A.numpy(), 1e-4, k=64, l=128, seed=3)
    assert r == ro == 30
    rs, _, _ = re_.rank_estimate(A.to(DEV), 1e-4, k=64, l=128, x="srht", seed=3)
    rso, _, _, _, _ = orc.rank_estimate(A.numpy(), 1e-4, orc.SRHT, orc.GAUSSIAN, k=64, l=128, seed=3)
    assert rs == rso < 30


def test_repeatable_and_errors():
    A = inputs.gaussian(400, 3000, 9, torch.float32).to(DEV)
    b1 = re_.sketch_x(A, k=100, x="hrtt", seed=2)
    b2 = re_.sketch_x(A, k=100, x="hrtt", seed=2)
    assert torch.equal(b1, b2)
    with pytest.raises(re_.RankEstError) as e:
        re_.sketch_x(A.double(), k=10, x="hrtt")
    assert e.value.status == re_._binding.RE_ERR_UNSUPPORTED
    W = torch.zeros(2, (1 << 20) + 1, device=DEV)  # N = 2^21: past the longest transform
    with pytest.raises(re_.RankEstError) as e:
        re_.sketch_x(W, k=10, x="hrtt")
    assert e.value.status == re_._binding.RE_ERR_UNSUPPORTED
    W = torch.zeros(2, 20000, device=DEV)  # chunked bucket lists hold at most 16384 buckets
    with pytest.raises(re_.RankEstError) as e:
        re_.sketch_x(W, k=16385, x="hrtt")
    assert e.value.status == re_._binding.RE_ERR_UNSUPPORTED
    with pytest.raises(re_.RankEstError) as e:
        re_.rank_estimate(A, 1e-3, k=10, x="hrtt", precision="bf16")
    assert e.value.status == re_._binding.RE_ERR_UNSUPPORTED
    with pytest.raises(re_.RankEstError) as e:
        re_.rank_estimate(A, 1e-3, k=10, y="hrtt")
    assert e.value.status == re_._binding.RE_ERR_INVALID_ARG


# The subsampled randomized DCT X (SRCT): B = sqrt(N) (F D a)[sel].  The k
# sampled entries' error is at most the whole transform's, (6 lg N + 6) u32 ||a||
# normwise, times sqrt(N).
def _srct_tol(n, anorm):
    import oracle.hrtt as oh
    N = oh.npad(n)
    return math.sqrt(N) * (6 * math.log2(N) + 6) * U32 * anorm


@pytest.mark.parametrize("m,n,k,off", [(300, 1000, 64, 0), (50, 1, 1, 0), (33, 2, 2, 0), (40, 3, 4, 0),
                                       (128, 16384, 384, 0), (90, 700, 700, 0), (64, 2049, 384, 0),
                                       (96, 1024, 100, 1), (70, 2048, 100, 0), (66, 4096, 300, 0),
                                       (40, 8192, 1000, 0), (48, 64, 64, 0), (48, 512, 33, 0)])
def test_srct_sketch_x_matches_oracle(orc, m, n, k, off):
    S = inputs.gaussian(m, n + off, 300 + n, torch.float32)
    A = S[:, off:off + n]
    seed = 23 + k
    Bg = re_.sketch_x(S.to(DEV)[:, off:off + n], k=k, x="srct", seed=seed).cpu().numpy().astype(np.float64)
    Bo = orc.hrtt.apply_x_srct(A.numpy(), k, seed=seed)
    err = np.linalg.norm(Bg - Bo, axis=1)
    tol = np.array([_srct_tol(n, float(np.linalg.norm(a))) for a in A.double().numpy()])
    assert np.all(err <= tol), float(np.max(err / tol))


def test_srct_full_sample_gives_the_singular_values(orc):
    # k = N and l = m' make both embeddings orthogonal up to scale: the estimates
    # are sigma(A) up to the FP32 transforms' rounding
    m, n = 256, 128
    A = inputs.planted(m, n, inputs.spectrum_step(n, 12, 1.0, 1e-3), 8, torch.float32)
    r, s, info = re_.rank_estimate(A.to(DEV), 1e-2, k=n, l=m, x="srct", y="srht", seed=4)
    sv = np.linalg.svd(A.double().numpy(), compute_uv=False)
    assert r == 12
    assert np.max(np.abs(s - sv)) <= 1e-5 * sv[0]


def test_srct_rank_estimate_matches_oracle_on_a_gap(orc):
    A = inputs.planted(1500, 1000, inputs.spectrum_step(1000, 20, 1.0, 1e-8), 31, torch.float32)
    k, l = 40, 60
    for y, ykind in (("gaussian", orc.GAUSSIAN), ("srht", orc.SRHT)):
        r, s, info = re_.rank_estimate(A.to(DEV), 1e-5, k=k, l=l, x="srct", y=y, seed=6)
        ro, so, r1, fl = orc.hrtt.rank_estimate(A.numpy(), 1e-5, k=k, l=l, ykind=ykind, seed=6, x="srct")
        assert r == ro == 20 and info["flags"] == fl
        dB = math.sqrt(sum(_srct_tol(1000, float(np.linalg.norm(a))) ** 2 for a in A.double().numpy()))
        tol = 1.1 * (math.sqrt(1500) + math.sqrt(l)) * dB / math.sqrt(k * l) + 1e-12 * so[0]
        assert np.all(np.abs(s - so) <= tol), (float(np.max(np.abs(s - so))), tol)


def test_srct_repeatable_and_errors():
    A = inputs.gaussian(400, 3000, 9, torch.float32).to(DEV)
    assert torch.equal(re_.sketch_x(A, k=100, x="srct", seed=2), re_.sketch_x(A, k=100, x="srct", seed=2))
    for kw, st in ((dict(x="srct", y="hrtt"), re_._binding.RE_ERR_INVALID_ARG),
                   (dict(x="srct", precision="bf16"), re_._binding.RE_ERR_UNSUPPORTED)):
        with pytest.raises(re_.RankEstError) as e:
            re_.rank_estimate(A, 1e-3, k=10, **kw)
        assert e.value.status == st
    with pytest.raises(re_.RankEstError) as e:
        re_.sketch_x(A.double(), k=10, x="srct")
    assert e.value.status == re_._binding.RE_ERR_UNSUPPORTED


@pytest.mark.parametrize("x", ["hrtt", "srct"])
def test_dct_kinds_full_size_sampled_rows(orc, x):
    # the benchmark's shape and launch configuration (512 workgroups, rows
    # r = w + 512 t): rows at workgroup and pass boundaries against the oracle
    m, n, k = 65536, 16384, 384
    A = inputs.c2_matrix(device=DEV)
    seed = 21
    B = re_.sketch_x(A, k=k, x=x, seed=seed)
    rows = np.array([0, 1, 511, 512, 513, 1023, 32767, 32768, 65023, 65535])
    An = A[torch.as_tensor(rows, device=DEV)].cpu().numpy()
    got = B[torch.as_tensor(rows, device=DEV)].cpu().numpy().astype(np.float64)
    if x == "hrtt":
        want = orc.hrtt.apply_x(An, k, seed=seed)
        tol = np.array([_row_tol(orc, n, k, seed, float(np.linalg.norm(a))) for a in An.astype(np.float64)])
    else:
        want = orc.hrtt.apply_x_srct(An, k, seed=seed)
        tol = np.array([_srct_tol(n, float(np.linalg.norm(a))) for a in An.astype(np.float64)])
    err = np.linalg.norm(got - want, axis=1)
    assert np.all(err <= tol), float(np.max(err / tol))


# --- rows past 16384 coordinates: the four-step split M = M1 x 8192 ---------------------------
# The M1-term bracket sums (M1 - 1 additions and a table twiddle of at most 2 ulp
# per term, normwise (M1 + 8) u32 relative) come on top of the FFT's bound, so
# the per-row tolerances take 6 lg N + 14 + M1 in place of 6 lg N + 6.

def _long_levels(N):
    M1 = max(1, N // 2 // 8192)
    return 6 * math.log2(N) + 14 + M1


@pytest.mark.parametrize("m,n,k,off", [(24, 20000, 384, 0), (16, 32768, 512, 0), (8, 65536, 300, 0),
                                       (5, 70000, 100, 0), (6, 131072, 2000, 0), (7, 40000, 64, 1),
                                       (70, 600000, 40, 0)])
def test_srct_long_rows_match_oracle(orc, m, n, k, off):
    """(70, 600000): N = 2^20, two passes of rows through the workspace; off = 1:
    a row stride and pointer off the 16-byte grid (clamped scalar loads)."""
    S = inputs.gaussian(m, n + off, 500 + n, torch.float32)
    A = S[:, off:off + n]
    seed = 31 + k
    Bg = re_.sketch_x(S.to(DEV)[:, off:off + n], k=k, x="srct", seed=seed).cpu().numpy().astype(np.float64)
    Bo = orc.hrtt.apply_x_srct(np.ascontiguousarray(A.numpy()), k, seed=seed)
    N = orc.hrtt.npad(n)
    err = np.linalg.norm(Bg - Bo, axis=1)
    tol = math.sqrt(N) * _long_levels(N) * U32 * np.linalg.norm(A.double().numpy(), axis=1)
    assert np.all(err <= tol), float(np.max(err / tol))


@pytest.mark.parametrize("m,n,k,off", [(24, 20000, 384, 0), (12, 65536, 1000, 0), (5, 100000, 64, 0),
                                       (9, 40000, 333, 2), (3, 32768, 16384, 0)])
def test_hrtt_long_rows_match_oracle(orc, m, n, k, off):
    S = inputs.gaussian(m, n + off, 700 + n, torch.float32)
    A = S[:, off:off + n]
    seed = 41 + k
    Bg = re_.sketch_x(S.to(DEV)[:, off:off + n], k=k, x="hrtt", seed=seed).cpu().numpy().astype(np.float64)
    Bo = orc.hrtt.apply_x(np.ascontiguousarray(A.numpy()), k, seed=seed)
    N = orc.hrtt.npad(n)
    b, _ = orc.hrtt.hash_table(seed, N, k)
    bmax = int(np.bincount(b, minlength=k).max())
    err = np.linalg.norm(Bg - Bo, axis=1)
    tol = (math.sqrt(k) * (math.sqrt(bmax) * _long_levels(N) + bmax ** 1.5) * U32
           * np.linalg.norm(A.double().numpy(), axis=1))
    assert np.all(err <= tol), float(np.max(err / tol))


def test_long_rows_repeatable_and_rank_on_a_gap(orc):
    """Bit-identical repeats, and the rank of a planted gap through both DCT kinds at n = 65536."""
    m, n, r = 600, 65536, 12
    s = np.concatenate([np.ones(r), 1e-7 * np.ones(64 - r)])
    A = inputs.planted(m, n, s, 3, torch.float32, 0.0, DEV)
    for x in ("srct", "hrtt"):
        b1 = re_.sketch_x(A, k=48, x=x, seed=7)
        b2 = re_.sketch_x(A, k=48, x=x, seed=7)
        assert torch.equal(b1, b2)
        rk, sig, _ = re_.rank_estimate(A, 1e-4, k=48, l=72, x=x, seed=7)
        assert rk == r, (x, rk, sig[:16])
