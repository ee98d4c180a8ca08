"""GPU parity: every step of the HIP path against the CPU oracle on the same
seeded inputs (run on an MI355X; calls go through the C ABI via the binding).

Tolerances
  integer / bit work (Philox words, signs, sampled indices): bit-exact;
  FP64 paths: |d sigma_i| <= 1e-10 sigma_1, and <= 1e-10 sigma_i when
      sigma_i >= 1e-4 sigma_1;
  FP32 SRHT paths: |d sigma_i| <= 1e-5 sigma_1;
  FWHT rows in FP32: |d B_it| <= log2(N) 2^-24 ||a_i||_1 (a rounding bound of the
      log2(N) butterfly additions), exact for small-integer inputs;
  rank: identical whenever no oracle estimate among the first r1 lies within the
      sigma tolerance of tau = eps sigma_1; otherwise within the number that do.
"""
import math

import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_
from paper_2105_07388_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _np(t):
    return t.detach().cpu().numpy()


# --- sketch specification -----------------------------------------------------------------------

def test_philox_bit_exact(orc):
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**63, size=(4096, 4), dtype=np.int64)
    for seed in [0, 5, 2**63 + 11]:
        got = _np(re_.philox(torch.from_numpy(ctr).to(DEV), seed)).view(np.uint64)
        for t in range(0, 4096, 97):
            want = orc.philox4x64_10(ctr[t].view(np.uint64), np.array([seed % 2**64, 0], dtype=np.uint64))
            assert np.array_equal(got[t], want), t


@pytest.mark.parametrize("fmt,ofmt", [("f64", 0), ("f32", 1), ("bf16", 2), ("f16", 3)])
def test_gauss_fill_matches_oracle(orc, fmt, ofmt):
    rows, cols = 257, 41
    for swap, stream in [(False, 1), (True, 2)]:
        got = _np(re_.gauss_fill(fmt, rows, cols, 99, stream, swap).to(torch.float64))
        want = np.array([[orc.round_to(orc.gauss(99, j if swap else i, i if swap else j, stream), ofmt)
                          for j in range(cols)] for i in range(rows)])
        if fmt == "f64":
            np.testing.assert_allclose(got, want, rtol=4 * 2.0**-52, atol=1e-300)
        else:
            # identical after rounding unless the FP64 values straddle a rounding boundary
            mism = np.count_nonzero(got != want)
            assert mism <= 1, mism


def test_signs_bit_exact(orc):
    for npad, stream in [(64, 3), (1000, 4), (16384, 3), (65536, 4)]:
        bits = _np(re_.srht_signs(npad, 17, stream)).view(np.uint32)
        d = np.array([(int(bits[i >> 5]) >> (i & 31)) & 1 for i in range(npad)], dtype=np.int64)
        want = np.array([orc.sign(17, i, stream) for i in range(npad)])
        assert np.array_equal(1 - 2 * d, want)


# (65536, 5000): more candidates below the threshold than the fast path holds (4096): the exact path
@pytest.mark.parametrize("npad,k", [(1, 1), (16, 5), (1024, 40), (16384, 384), (65536, 576), (1024, 1024),
                                    (4096, 3000), (8192, 1), (65536, 5000)])
def test_select_exact(orc, npad, k):
    for seed, stream in [(3, 5), (4, 6)]:
        got = _np(re_.srht_select(npad, k, seed, stream)).astype(np.int64)
        assert np.array_equal(got, orc.select(seed, npad, k, stream))


# --- AX -----------------------------------------------------------------------------------------

def _row_tol(A, N, levels=None):
    levels = math.log2(max(N, 2)) if levels is None else levels
    return levels * 2.0**-24 * np.abs(A.astype(np.float64)).sum(axis=1)[:, None] * 1.01 + 1e-30


def _long_row_levels(N, sub):
    """Rounding levels of a row longer than one transform of length sub: the
    N / sub chunk sums are accumulated one after another (N / sub - 1
    additions), then log2(sub) butterfly stages."""
    return N // sub - 1 + math.log2(sub)


@pytest.mark.parametrize("m,n,k", [(37, 1000, 40), (64, 16384, 384), (5, 3, 2), (130, 4096, 200), (3, 32768, 17),
                                   # the register-tiled row transforms, N = 2^11 .. 2^15, exact and zero-padded,
                                   # k above and below the thread count
                                   (200, 2048, 100), (90, 3000, 256), (77, 8192, 384), (41, 12000, 500),
                                   (33, 20000, 512), (40, 32768, 1024), (9, 16000, 384), (5, 2049, 7)])
def test_srht_x_fp32(orc, m, n, k):
    A = inputs.gaussian(m, n, m + n, dtype=torch.float32)
    B = _np(re_.sketch_x(A.to(DEV), k=k, x="srht", y="srht", l=k, seed=8))
    want = orc.apply_x(A.numpy(), orc.SRHT, k, seed=8)
    N = 1 << (n - 1).bit_length()
    assert np.all(np.abs(B - want) <= _row_tol(A.numpy(), N))


@pytest.mark.parametrize("m,n,k", [(50, 16384, 384), (40, 2048, 300), (30, 8192, 384), (20, 32768, 700),
                                   (25, 5000, 96)])
def test_srht_x_integer_exact(orc, m, n, k):
    A = inputs.small_integers(m, n, 3, -100, 100)
    B = _np(re_.sketch_x(A.to(DEV), k=k, x="srht", y="srht", l=k, seed=1))
    assert np.array_equal(B.astype(np.float64), orc.apply_x(A.numpy(), orc.SRHT, k, seed=1))


# rows past 2^15 (FP32) / 2^14 (FP64): chunk sums over H = N / 2^15 (or 2^14) sub-rows,
# exact and zero-padded N, H = 2 .. 8, k above and below the thread count
@pytest.mark.parametrize("m,n,k", [(24, 40000, 384), (16, 65536, 1500), (9, 70000, 600), (4, 140000, 300),
                                   (11, 65537, 33)])
def test_srht_x_fp32_long_rows(orc, m, n, k):
    A = inputs.gaussian(m, n, m + n, dtype=torch.float32)
    B = _np(re_.sketch_x(A.to(DEV), k=k, x="srht", y="srht", l=k, seed=8))
    want = orc.apply_x(A.numpy(), orc.SRHT, k, seed=8)
    N = 1 << (n - 1).bit_length()
    assert np.all(np.abs(B - want) <= _row_tol(A.numpy(), N, _long_row_levels(N, 1 << 15)))


@pytest.mark.parametrize("m,n,k", [(12, 65536, 700), (7, 100000, 256)])
def test_srht_x_long_rows_integer_exact(orc, m, n, k):
    A = inputs.small_integers(m, n, 5, -100, 100)
    B = _np(re_.sketch_x(A.to(DEV), k=k, x="srht", y="srht", l=k, seed=4))
    assert np.array_equal(B.astype(np.float64), orc.apply_x(A.numpy(), orc.SRHT, k, seed=4))


def test_srht_x_fp32_long_rows_unaligned_view(orc):
    """A row stride that is not a multiple of 4 takes the LDS chunk-sum kernel."""
    m, n, k = 10, 40000, 200
    Abig = inputs.gaussian(m, n + 1, 77, dtype=torch.float32)
    A = Abig[:, :n]
    B = _np(re_.sketch_x(Abig.to(DEV)[:, :n], k=k, x="srht", y="srht", l=k, seed=6))
    want = orc.apply_x(np.ascontiguousarray(A.numpy()), orc.SRHT, k, seed=6)
    N = 1 << (n - 1).bit_length()
    assert np.all(np.abs(B - want) <= _row_tol(A.numpy(), N, _long_row_levels(N, 1 << 15)))


@pytest.mark.parametrize("m,n,k", [(6, 20000, 128), (5, 40000, 300), (3, 16385, 17)])
def test_srht_x_fp64_long_rows(orc, m, n, k):
    A = inputs.gaussian(m, n, 3 + n, dtype=torch.float64)
    B = _np(re_.sketch_x(A.to(DEV), k=k, x="srht", y="srht", l=k, seed=2))
    want = orc.apply_x(A.numpy(), orc.SRHT, k, seed=2)
    N = 1 << (n - 1).bit_length()
    # both sides round in FP64: the GPU's chunk sums and stages plus the oracle's log2(N) stages
    tol = (_long_row_levels(N, 1 << 14) + math.log2(N)) * 2.0**-53 * np.abs(A.numpy()).sum(axis=1)[:, None] * 1.01
    assert np.all(np.abs(B - want) <= tol)


def test_srht_x_fp64(orc):
    A = inputs.gaussian(20, 3000, 9, dtype=torch.float64)
    B = _np(re_.sketch_x(A.to(DEV), k=64, x="srht", y="srht", l=64, seed=2))
    want = orc.apply_x(A.numpy(), orc.SRHT, 64, seed=2)
    np.testing.assert_allclose(B, want, rtol=0, atol=1e-12 * np.abs(A.numpy()).sum(axis=1).max())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gaussian_x(orc, dtype):
    A = inputs.gaussian(150, 333, 12, dtype=dtype)
    B = _np(re_.sketch_x(A.to(DEV), k=40, seed=5)).astype(np.float64)
    want = orc.apply_x(A.numpy(), orc.GAUSSIAN, 40, seed=5)
    Xabs = np.abs(np.array([[orc.round_to(orc.gauss(5, j, t, 1), 0 if dtype == torch.float64 else 1)
                             for t in range(40)] for j in range(333)]))
    bound = np.abs(A.numpy().astype(np.float64)) @ Xabs
    if dtype == torch.float64:  # FP64 accumulation, FP64 result
        tol = 4 * 333 * 2.0**-53 * bound + 2.0**-53 * np.abs(want)
    else:  # FP32 accumulation of 333 products on the matrix cores, FP32 result
        tol = (333 + 2) * 2.0**-24 * bound
    assert np.all(np.abs(B - want) <= tol)


# --- Y B -----------------------------------------------------------------------------------------

@pytest.mark.parametrize("m,k,l", [(65536, 8, 576), (1000, 40, 60), (300, 7, 9), (4096, 96, 144)])
def test_srht_y_fp32(orc, m, k, l):
    Bm = inputs.gaussian(m, k, m + k, dtype=torch.float32)
    Cm = _np(re_.sketch_y(Bm.to(DEV), l=l, y="srht", seed=6))
    want = orc.apply_y(Bm.numpy().astype(np.float64), orc.SRHT, l, seed=6)
    tol = 8 * 2.0**-24 * np.abs(Bm.numpy().astype(np.float64)).sum(axis=0)[None, :] * 1.01
    assert np.all(np.abs(Cm - want) <= tol)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_gaussian_y(orc, dtype):
    m, k, l = 2000, 40, 60
    Bm = inputs.gaussian(m, k, 3, dtype=dtype)
    Cm = _np(re_.sketch_y(Bm.to(DEV), l=l, y="gaussian", seed=7))
    fmt = 0 if dtype == torch.float64 else 1
    want = orc.apply_y(Bm.numpy().astype(np.float64), orc.GAUSSIAN, l, fmt_y=fmt, seed=7)
    np.testing.assert_allclose(Cm, want, rtol=0, atol=1e-12 * np.abs(want).max())


# --- small SVD --------------------------------------------------------------------------------------

def _svd_cases():
    rng = np.random.default_rng(5)
    out = []
    for l, k in [(1, 1), (2, 2), (60, 40), (144, 96), (576, 384), (33, 33), (768, 512), (100, 3), (700, 600),
                 (160, 128), (150, 65), (17, 17), (129, 129), (161, 64)]:
        out.append((f"rand{l}x{k}", rng.standard_normal((l, k))))
    l, k = 200, 120
    U, _ = np.linalg.qr(rng.standard_normal((l, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    out.append(("graded", (U * 10.0 ** -np.linspace(0, 15, k)) @ V.T))
    Z = rng.standard_normal((90, 60))
    Z[:, 20:] = 0
    out.append(("rankdef", Z))
    out.append(("zero", np.zeros((10, 4))))
    out.append(("diag", np.diag([3.0, -7.0, 0.5, 0.0])))
    return out


@pytest.mark.parametrize("name,Cm", _svd_cases(), ids=[c[0] for c in _svd_cases()])
def test_singular_values(orc, name, Cm):
    got = _np(re_.singular_values(torch.from_numpy(Cm).to(DEV), 1.0))
    want, _, st = orc.jacobi_sv(Cm)
    assert st == 0
    s1 = max(want[0], 1e-300)
    assert np.all(np.abs(got - want) <= 1e-12 * s1), np.abs(got - want).max() / s1
    big = want >= 1e-4 * s1
    assert np.all(np.abs(got - want)[big] <= 1e-10 * want[big])


@pytest.mark.parametrize("l,k", [(1100, 1030), (2600, 2400), (1400, 700)])
def test_singular_values_global_memory_path(l, k):
    """Large sketches: k > 1025 runs the global-memory bidiagonalisation
    (column partials in chunks of 1024); 1400 x 700 is too tall for the
    register-cached kernel's LDS plan and runs the plain LDS-resident one.
    Checked against LAPACK (the oracle's Jacobi is pinned to it and would
    take minutes at these sizes)."""
    rng = np.random.default_rng(11)
    Cm = rng.standard_normal((l, k)) * (10.0 ** -np.linspace(0, 6, k))[None, :]
    got = _np(re_.singular_values(torch.from_numpy(Cm).to(DEV), 1.0))
    want = np.linalg.svd(Cm, compute_uv=False)
    assert np.all(np.abs(got - want) <= 1e-12 * want[0]), np.abs(got - want).max() / want[0]


def test_rank_count_cases():
    s = torch.tensor([2.0, 1.0, 2e-6, 1e-6, 1e-7, 1e-8], dtype=torch.float64, device=DEV)
    assert re_.rank_count(s, 5, 1e-6) == (2, 0, 0)
    assert re_.rank_count(s, 5, 4e-7) == (4, 0, 0)
    assert re_.rank_count(s, 3, 1e-9) == (3, 1, 0)
    assert re_.rank_count(torch.zeros(4, dtype=torch.float64, device=DEV), 3, 1e-3) == (0, 2, 0)
    assert re_.rank_count(torch.tensor([1.0, float("nan")], dtype=torch.float64, device=DEV), 1, 1e-3)[2] == -5


# --- Algorithm 1 end to end ----------------------------------------------------------------------------

def _compare(orc_out, got_r, got_s, got_info, eps, tol_rel):
    r_o, s_o, r1_o, fl_o, _ = orc_out
    s1 = s_o[0]
    assert got_info["r1"] == r1_o
    assert np.all(np.abs(got_s - s_o) <= tol_rel * s1), np.abs(got_s - s_o).max() / s1
    tau = eps * s1
    band = int(np.count_nonzero(np.abs(s_o[:r1_o] - tau) <= 2 * tol_rel * s1))
    assert abs(got_r - r_o) <= band, (got_r, r_o, band)
    if band == 0:
        assert got_info["flags"] == fl_o


def test_c1_plain_method(orc):
    """FP64 2000 x 1000 planted step spectrum, Gaussian 40/60, eps 1e-6: rank 20
    on 100 sketch seeds, each against the oracle's full estimate."""
    A = inputs.c1_matrix()
    Ad = A.to(DEV)
    for seed in range(100):
        r, s, info = re_.rank_estimate(Ad, 1e-6, k=40, l=60, seed=seed)
        out = orc.rank_estimate(A.numpy(), 1e-6, orc.GAUSSIAN, orc.GAUSSIAN, k=40, l=60, seed=seed)
        assert r == out[0] == 20
        assert re_.gap_rank(s, info["r1"])[0] == 20  # no eps needed: the largest gap (Sec. 5, Sec. 6.1)
        s_o = out[1]
        assert np.all(np.abs(s - s_o) <= 1e-10 * s_o[0])
        big = s_o >= 1e-4 * s_o[0]
        assert np.all(np.abs(s - s_o)[big] <= 1e-10 * s_o[big])


def test_gap_rank_on_planted_gap(orc):
    """A graded spectrum 10^(-i/20) with one jump of 1e-4 after 37 values: the
    largest ratio of the first r1 sketched estimates sits at the jump, and
    matches the oracle's definition applied to the oracle's estimates."""
    spec = 10.0 ** (-np.arange(300) / 20.0)
    spec[37:] *= 1e-4
    A = inputs.planted(3000, 1500, spec, 77, torch.float32)
    for xk, yk in (("srht", "srht"), ("gaussian", "gaussian")):
        r, s, info = re_.rank_estimate(A.to(DEV), 1e-3, k=96, l=144, x=xk, y=yk, seed=4)
        g = re_.gap_rank(s, info["r1"])
        out = orc.rank_estimate(A.numpy(), 1e-3, {"srht": 1, "gaussian": 0}[xk], {"srht": 1, "gaussian": 0}[yk],
                                k=96, l=144, seed=4)
        assert g[0] == 37 == orc.gap.gap_rank(out[1], out[2])[0]
        assert g[1] > 1e3


@pytest.mark.parametrize("m,n,xk,yk,dtype", [
    (4096, 2048, "srht", "srht", torch.float32),
    (3000, 1500, "srht", "gaussian", torch.float32),
    (1000, 700, "gaussian", "srht", torch.float64),
    (777, 513, "srht", "srht", torch.float64),
])
def test_mixed_sketches(orc, m, n, xk, yk, dtype):
    spec = inputs.c2_spectrum(min(m, n) // 2)
    A = inputs.planted(m, n, spec, 50 + m, dtype)
    k, l = 96, 144
    for eps in [1e-3, 1e-5]:
        r, s, info = re_.rank_estimate(A.to(DEV), eps, k=k, l=l, x=xk, y=yk, seed=3)
        out = orc.rank_estimate(A.numpy(), eps, {"srht": 1, "gaussian": 0}[xk], {"srht": 1, "gaussian": 0}[yk],
                                k=k, l=l, seed=3)
        _compare(out, r, s, info, eps, 1e-10 if dtype == torch.float64 else 1e-5)


def test_edge_shapes(orc):
    for (m, n, k, l, xk, yk) in [(1, 1, 1, 1, "gaussian", "gaussian"), (5, 3, 2, 4, "srht", "srht"),
                                 (17, 9, 9, 17, "gaussian", "gaussian"), (9, 17, 4, 9, "srht", "gaussian")]:
        A = inputs.gaussian(m, n, m * n, dtype=torch.float64)
        r, s, info = re_.rank_estimate(A.to(DEV), 1e-3, k=k, l=l, x=xk, y=yk, seed=1)
        out = orc.rank_estimate(A.numpy(), 1e-3, {"srht": 1, "gaussian": 0}[xk], {"srht": 1, "gaussian": 0}[yk],
                                k=k, l=l, seed=1)
        _compare(out, r, s, info, 1e-3, 1e-10)


def test_errors_and_flags():
    A = torch.zeros(64, 32, dtype=torch.float32, device=DEV)
    r, s, info = re_.rank_estimate(A, 1e-3, k=8, l=12, x="srht", y="srht")
    assert r == 0 and info["flags"] & re_.FLAG_ZERO and np.all(s == 0)
    A[3, 5] = float("nan")
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_estimate(A, 1e-3, k=8, l=12, x="srht", y="srht")
    assert ei.value.status == -5
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_estimate(torch.ones(8, 8, device=DEV), 0.0, k=2, l=2)
    assert ei.value.status == -1
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_estimate(torch.ones(8, 8, device=DEV), 1e-3, k=4, l=3)
    assert ei.value.status == -1
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_estimate(torch.ones(8, 8, device=DEV, dtype=torch.float64), 1e-3, k=4, l=4, precision="bf16")
    assert ei.value.status == -2


def test_plain_method_full_size(orc):
    """The benchmark's own matrix and launch configuration: FP32 65536 x 16384,
    s_i = 10^(-i/20) + 1e-9 noise, SRHT X 384 and Y 576.  The oracle runs the
    same estimate in FP64 on the whole matrix.  Tolerance: the FP32-SRHT bar
    |d sigma_i| <= 1e-5 sigma_1 (the observed maximum is about 2e-9 sigma_1: the
    rounding errors of the FP32 sketch largely cancel in the estimates); sampled
    rows of A X entrywise within the FWHT bound.  The spectrum has no gap at
    either eps (ties at 61 and 101), so the ranks may differ by the oracle
    estimates that lie inside that band around tau."""
    A = inputs.c2_matrix(device=DEV)
    An = A.cpu().numpy()
    k, l = 384, 576
    for eps, seed in ((1e-3, 3), (1e-5, 4)):
        r, s, info = re_.rank_estimate(A, eps, k=k, l=l, x="srht", y="srht", seed=seed)
        ro, so, r1, fl, _ = orc.rank_estimate(An, eps, orc.SRHT, orc.SRHT, k=k, l=l, seed=seed)
        tol = 1e-5 * so[0]
        print(f"plain method full size, eps {eps}: max |d sigma| / sigma_1 = {np.max(np.abs(s - so)) / so[0]:.3e}, "
              f"ranks {r} / {ro}")
        assert np.max(np.abs(s - so)) <= tol, float(np.max(np.abs(s - so)) / so[0])
        band = int(np.count_nonzero(np.abs(so[:r1] - eps * so[0]) <= tol))
        assert abs(r - ro) <= band, (eps, r, ro, band)
        assert (41 <= r <= 80) if eps == 1e-3 else (81 <= r <= 120)  # the desiderata windows of Sec. 1.1
    B = _np(re_.sketch_x(A, k=k, x="srht", y="srht", l=k, seed=8))
    rows = np.array([0, 1, 255, 256, 4095, 4096, 32767, 32768, 65534, 65535])
    want = orc.apply_x(An[rows], orc.SRHT, k, seed=8)
    assert np.all(np.abs(B[rows] - want) <= _row_tol(An[rows], 16384))
