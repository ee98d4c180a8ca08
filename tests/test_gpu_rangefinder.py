"""GPU tests of rank estimation followed by the randomized rangefinder
(re_rangefinder, Algorithm 3) against the FP64 oracle (oracle/rangefinder.py).

What is compared, and to which tolerance:
  - r and the final width k (so the number of doubling rounds): among the
    outcomes the oracle's estimates allow when each moves by its FP32
    tolerance (the rule is monotone in every estimate), and equal to the
    oracle's where that leaves one outcome (a spectrum with a gap); w = r + p;
  - the estimates: within 8 2^-24 sqrt(n) s_1 (FP32 Gaussian contraction);
  - Q: orthonormal to 64 w u64, and spanning the oracle's A X[:, :w] up to
    ||dW||_F <= (n + 2) u32 || |A| |X| ||_F (the worst-case error of the FP32
    contraction forming the device's sketch) plus 64 w u64 ||W||_F;
  - ||A - Q B||_F: at most twice the oracle's plus 8 u32 sqrt(w) ||A||_F.
The two steps after the estimate are also compared alone, on inputs both
sides share exactly (re_thin_qr, re_project):
  - thin QR: Q within the first-order perturbation bound (Sun, BIT 1991)
    2 (1 + sqrt 2) kappa_2(W) eta, with the backward error eta = 8 m w u64
    ||W||_F / ||W||_2 allowed for shifted CholeskyQR3;
  - B = Q^T A: every entry within 260 u32 (|Q|^T |A|) (Q rounded to FP32,
    FP32 sums over at most 256 rows, FP64 sums across them).
"""
import math

import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_
from paper_2105_07388_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"
U32, U64 = 2.0 ** -24, 2.0 ** -53


def _gpu(A, eps, p, **kw):
    Q, B, info = re_.rangefinder(A.to(DEV), eps, p, **kw)
    torch.cuda.synchronize()
    return Q.cpu().numpy(), B.cpu().numpy(), info


def _outcomes(orc, A, eps, p, k0, seed, kmax=None):
    """Admissible (k, r) of the device for the oracle's doubling when every
    estimate may move by the FP32 tolerance d = 8 u32 sqrt(n) s_1.  The rule is
    monotone in each estimate (and in ||A|| = s_1), so at width k the device's r
    lies between the choices for the optimistic (s - d, s_1 + d) and the
    pessimistic (s + d, s_1 - d) estimates; it stops at a width whose optimistic
    choice exists, at the latest at the first whose pessimistic one does.
    Returns {k: (r_lo, r_hi, sigma_k)}."""
    m, n = A.shape
    F = orc.rangefinder
    kmax = min(m, n, kmax or min(m, n))
    k = min(k0, kmax)
    out = {}
    while True:
        l = orc.learned.l_for(k, 2.0, m)
        _, s, r1, _, _ = orc.rank_estimate(A, 0.5, orc.GAUSSIAN, orc.GAUSSIAN, k=k, l=l, seed=seed)
        d = 8 * U32 * math.sqrt(n) * s[0]
        lo = F.choose_rank(np.maximum(s - d, 0.0), r1, n, eps, p, norm_a=s[0] + d)
        hi = F.choose_rank(s + d, r1, n, eps, p, norm_a=s[0] - d)
        if lo is not None:
            out[k] = (lo, hi if hi is not None else k - p, s)
        if hi is not None or k >= kmax:
            return out
        k = min(2 * k, kmax)


def _compare(orc, A32, eps, p, k0, seed, k_max=0, exact=False):
    m, n = A32.shape
    A = A32.numpy()
    A64 = A.astype(np.float64)
    ok = _outcomes(orc, A, eps, p, k0, seed, k_max or None)
    Qg, Bg, got = _gpu(A32, eps, p, k0=k0, k_max=k_max, seed=seed)
    k, r, w = got["k"], got["r"], got["w"]
    assert k in ok, (k, list(ok))
    lo, hi, sig = ok[k]
    assert lo <= r <= hi and w == r + p and got["flags"] == 0, (got, lo, hi)
    if exact:  # the decisions do not depend on the FP32 perturbation
        want = orc.rangefinder.rangefinder(A, eps, p, k0=k0, kmax=k_max or None, seed=seed)
        assert len(ok) == 1 and lo == hi and (k, r, w) == (want["k"], want["r"], want["w"])
    s_tol = 8 * U32 * math.sqrt(n) * sig[0]
    assert np.all(np.abs(got["sigma"] - sig) <= s_tol)
    # Q orthonormal
    assert np.abs(Qg.T @ Qg - np.eye(w)).max() <= 64 * w * U64
    # Q spans the oracle's A X[:, :w] up to the FP32 contraction error of the
    # device sketch: (I - Q Q^T) W_o = (I - Q Q^T)(W_o - W_gpu) + FP64 QR error
    X = orc.apply_x(np.eye(n, dtype=np.float32), orc.GAUSSIAN, w, seed=seed)  # FP32-rounded X, as drawn
    Wo = A64 @ X
    dW = (n + 2) * U32 * np.linalg.norm(np.abs(A64) @ np.abs(X))
    off = np.linalg.norm(Wo - Qg @ (Qg.T @ Wo))
    assert off <= dW + 64 * w * U64 * np.linalg.norm(Wo), (off, dW)
    # the factorisation error against the oracle's at the same width
    Qo, _ = orc.rangefinder.thin_qr(Wo)
    err_g = np.linalg.norm(A64 - Qg @ Bg)
    err_o = np.linalg.norm(A64 - Qo @ (Qo.T @ A64))
    assert err_g <= 2 * err_o + 8 * U32 * math.sqrt(w) * np.linalg.norm(A64), (err_g, err_o)
    return got, Qg, Bg


def test_step_spectrum_one_round(orc):
    # 20 unit values then 1e-8: r = 20, w = 25, one 64-column tile, LDS factorisation
    A = inputs.planted(2000, 1000, inputs.spectrum_step(1000, 20, 1.0, 1e-8), 11, torch.float32)
    got, Qg, Bg = _compare(orc, A, 3e-3, 5, 32, 3, exact=True)
    assert got["r"] == 20 and got["w"] == 25
    assert np.linalg.norm(A.numpy() - Qg @ Bg) <= 1e-5 * np.linalg.norm(A.numpy(), 2)


def test_exponential_decay_with_doubling(orc):
    # ragged shape, two rounds (k = 48, 96): r = 41, w = 51
    A = inputs.planted(3001, 1100, 10.0 ** (-np.arange(400) / 20.0), 12, torch.float32)
    got, _, _ = _compare(orc, A, 0.03, 10, 48, 5, exact=True)
    assert got["k"] == 96 and got["w"] == 51


def test_two_gram_tiles(orc):
    # three rounds (k = 64, 128, 256): r = 94, w = 104 spans two 64-column tiles
    A = inputs.planted(2500, 1500, 10.0 ** (-np.arange(600) / 40.0), 14, torch.float32)
    got, _, _ = _compare(orc, A, 0.03, 10, 64, 7, exact=True)
    assert got["k"] == 256 and got["w"] == 104


def test_wide_basis_global_factorisation(orc):
    # w above the LDS-resident factorisation (136): the global-memory path
    A = inputs.planted(2500, 1500, 10.0 ** (-np.arange(800) / 60.0), 14, torch.float32)
    got, _, _ = _compare(orc, A, 0.03, 10, 96, 7)
    assert got["k"] == 384 and got["w"] > 136


def test_wide_matrix_and_capped_width(orc):
    # m < n: k is capped by m; k0 above k_max starts at k_max
    A = inputs.planted(700, 1900, inputs.spectrum_step(700, 30, 1.0, 1e-7), 17, torch.float32)
    got, _, _ = _compare(orc, A, 1e-2, 8, 500, 9, k_max=64, exact=True)
    assert got["k"] == 64 and got["r"] == 30 and got["w"] == 38


def _geometric(m, w, cond, seed, dtype=torch.float64):
    return inputs.planted(m, w, np.geomspace(1.0, 1.0 / cond, w), seed, dtype)


@pytest.mark.parametrize("m,w,cond,dtype", [(3001, 150, 1e4, torch.float64), (777, 40, 1e2, torch.float64),
                                            (2048, 64, 1e6, torch.float32), (5000, 200, 1e3, torch.float64),
                                            (1000, 1, 1.0, torch.float64), (1500, 136, 1e3, torch.float64),
                                            (1500, 137, 1e3, torch.float64), (2600, 1100, 1e2, torch.float64),
                                            (2600, 1101, 1e2, torch.float64), (2400, 2200, 1e2, torch.float64),
                                            (2400, 2201, 1e2, torch.float64)])
def test_thin_qr_matches_oracle(orc, m, w, cond, dtype):
    W = _geometric(m, w, cond, 31 + w, dtype)
    Qg, flags = re_.thin_qr(W.to(DEV))
    Qg = Qg.cpu().numpy()
    W64 = W.double().numpy()
    Qo, _ = orc.rangefinder.thin_qr(W64)
    assert Qg.shape == (m, w) and flags == 0
    sv = np.linalg.svd(W64, compute_uv=False)
    eta = 8 * m * w * U64 * np.linalg.norm(W64) / sv[0]
    tol = 2 * (1 + math.sqrt(2)) * (sv[0] / sv[-1]) * eta
    assert np.linalg.norm(Qg - Qo) <= tol, (np.linalg.norm(Qg - Qo), tol)
    assert np.abs(Qg.T @ Qg - np.eye(w)).max() <= 64 * w * U64


def test_thin_qr_ill_conditioned_and_dependent_columns():
    # kappa = 1e11 (the smallest singular value above the resolution of the
    # unshifted passes, about 1e-12 ||W||_F at this size): all columns kept,
    # orthonormal, and spanning W to FP64 precision
    W = _geometric(4000, 120, 1e11, 41).to(DEV)
    Q, flags = re_.thin_qr(W)
    assert Q.shape[1] == 120 and flags == 0
    eye = torch.eye(120, dtype=torch.float64, device=DEV)
    assert float((Q.T @ Q - eye).abs().max()) <= 64 * 120 * U64
    assert float(torch.linalg.norm(W - Q @ (Q.T @ W))) <= 64 * 120 * U64 * float(torch.linalg.norm(W))
    # kappa = 1e14: the directions below that resolution are left out; Q
    # stays orthonormal and the rest of W is captured
    W = _geometric(4000, 120, 1e14, 42).to(DEV)
    Q, flags = re_.thin_qr(W)
    w = Q.shape[1]
    assert 90 <= w < 120 and flags & re_.FLAG_COLUMNS_DROPPED
    eye = torch.eye(w, dtype=torch.float64, device=DEV)
    assert float((Q.T @ Q - eye).abs().max()) <= 64 * w * U64
    assert float(torch.linalg.norm(W - Q @ (Q.T @ W))) <= 1e-9 * float(torch.linalg.norm(W))
    # columns 1 and 3 repeat column 0 (times 2): two kept columns span all four
    v = torch.randn(900, 1, dtype=torch.float64, device=DEV)
    u = torch.randn(900, 1, dtype=torch.float64, device=DEV)
    W = torch.cat([v, v, u, 2 * v], 1)
    Q, flags = re_.thin_qr(W)
    assert Q.shape[1] == 2 and flags & re_.FLAG_COLUMNS_DROPPED
    assert float(torch.linalg.norm(W - Q @ (Q.T @ W))) <= 1e-13 * float(torch.linalg.norm(W))


@pytest.mark.parametrize("m,n,w", [(3001, 1100, 150), (999, 257, 33), (4100, 130, 96), (513, 700, 1),
                                   (2000, 128, 64)])
def test_project_matches_oracle(orc, m, n, w):
    Qo, _ = orc.rangefinder.thin_qr(np.random.default_rng(w).standard_normal((m, w)))
    A = inputs.gaussian(m, n, 50 + w, torch.float32)
    B = re_.project(torch.from_numpy(Qo).to(DEV), A.to(DEV)).cpu().numpy()
    A64 = A.double().numpy()
    want = Qo.T @ A64
    tol = 260 * U32 * (np.abs(Qo).T @ np.abs(A64))
    assert np.all(np.abs(B - want) <= tol)


def test_repeatable_bits():
    A = inputs.planted(1500, 900, 10.0 ** (-np.arange(300) / 20.0), 14, torch.float32).to(DEV)
    Q1, B1, i1 = re_.rangefinder(A, 1e-3, 5, k0=32, seed=9)
    Q2, B2, i2 = re_.rangefinder(A, 1e-3, 5, k0=32, seed=9)
    assert i1["w"] == i2["w"] and torch.equal(Q1, Q2) and torch.equal(B1, B2)


def test_estimates_equal_the_adaptive_driver():
    # the rank-estimation stage is the adaptive driver's doubling, bit for bit
    A = inputs.planted(1800, 1000, 10.0 ** (-np.arange(300) / 20.0), 15, torch.float32).to(DEV)
    _, _, info = re_.rangefinder(A, 1e-4, 10, k0=32, seed=4)
    _, sigma, ai = re_.rank_adaptive(A, 0.5, k0=info["k"], l_ratio=2.0, seed=4)
    assert ai["k"] == info["k"] and np.array_equal(sigma, info["sigma"])


def test_rank_one_identical_rows_drops_dependent_columns():
    # every row equal: A X has rank one exactly, so Q keeps one column
    A = torch.ones(1000, 700, dtype=torch.float32)
    Qg, Bg, info = _gpu(A, 1e-3, 5, k0=16, seed=2)
    assert info["r"] == 1 and info["w"] == 1
    assert info["flags"] & re_.FLAG_COLUMNS_DROPPED
    assert np.allclose(np.abs(Qg[:, 0]), 1 / math.sqrt(1000), rtol=1e-12)
    # only B's rounding remains: Q rounded to FP32, FP32 sums of 256 rows
    A64 = A.double().numpy()
    assert np.linalg.norm(A64 - Qg @ Bg) <= 260 * U32 * np.linalg.norm(np.abs(Qg).T @ A64)


def test_zero_matrix_and_no_admissible_width():
    A = torch.zeros(300, 200, dtype=torch.float32, device=DEV)
    Q = torch.full((300, 200), 7.0, dtype=torch.float64, device=DEV)
    _, _, info = re_.rangefinder(A, 1e-3, 5, k0=16, seed=1, Q=Q)
    assert info["r"] == 0 and info["w"] == 0 and info["flags"] & re_.FLAG_ZERO
    assert bool((Q == 7.0).all())  # untouched
    S = inputs.planted(600, 400, inputs.spectrum_step(400, 20, 1.0, 1e-8), 16, torch.float32).to(DEV)
    _, _, info = re_.rangefinder(S, 1e-5, 5, k0=8, k_max=24, seed=1)
    assert info["r"] == -1 and info["w"] == 0 and info["flags"] & re_.FLAG_NOT_CONVERGED and info["k"] == 24


def test_argument_errors():
    A = torch.randn(300, 200, device=DEV)
    with pytest.raises(re_.RankEstError) as e:
        re_.rangefinder(A.double(), 1e-3, 5)
    assert e.value.status == re_._binding.RE_ERR_UNSUPPORTED
    for kw in ({"p": 1}, {"p": 200}):
        with pytest.raises(re_.RankEstError) as e:
            re_.rangefinder(A, 1e-3, kw["p"], k0=16)
        assert e.value.status == re_._binding.RE_ERR_INVALID_ARG
    with pytest.raises(re_.RankEstError):
        re_.rangefinder(A, 1.5, 5)
    with pytest.raises(re_.RankEstError):
        re_.rangefinder(A, 1e-3, 5, norm_a=-1.0)
    Q = torch.empty(300, 100, dtype=torch.float64, device=DEV)
    with pytest.raises(ValueError):
        re_.rangefinder(A, 1e-3, 5, k_max=150, Q=Q)


def test_full_size_properties():
    # 65536 x 16384 FP32, s_i = 10^(-i/20) + 1e-9 noise: orthonormal Q, B = Q^T A
    # on sampled columns (FP64 on the device), the rule's error bound met on
    # sampled columns of A - Q B
    A = inputs.c2_matrix(device=DEV)
    eps, p = 1e-3, 10
    Q, B, info = re_.rangefinder(A, eps, p, k0=128, k_max=256, seed=21)
    w = info["w"]
    assert info["r"] > 0 and w == info["r"] + p and w <= info["k"] <= 256
    G = Q.T @ Q
    assert float((G - torch.eye(w, dtype=torch.float64, device=DEV)).abs().max()) <= 64 * w * U64
    cols = torch.from_numpy(np.random.default_rng(3).choice(A.shape[1], 64, replace=False)).to(DEV)
    Ac = A[:, cols].double()
    want = Q.T @ Ac
    tol = 258 * U32 * ((Q.abs().T @ Ac.abs()))
    assert bool(((B[:, cols] - want).abs() <= tol + 1e-300).all())
    # column-sampled Frobenius error, scaled to the whole matrix
    R = Ac - Q @ B[:, cols]
    err = float(torch.linalg.norm(R)) * math.sqrt(A.shape[1] / 64)
    assert err <= 2 * eps * info["sigma"][0]
