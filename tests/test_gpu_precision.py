"""GPU parity of the low-precision A X contraction (BF16/FP16 MFMA with FP32
accumulation) and of the precision selection, against the CPU oracle.

The oracle keeps A exact (FP64 of the FP32 input) and uses the same rounded X, so
the GPU result differs by the rounding of A (the precision floor) plus FP32
accumulation:
  |d B_it| <= (u_f + n 2^-24) (|A| |X|)_it              (entrywise),
  |d sigma_i| <= 2 phi_f,  phi_f = (u_f / sqrt 3) ||A||_F (1/sqrt k + 1/sqrt m).
With small-integer A (exact in the format) only the accumulation term remains,
which pins the MFMA operand and accumulator layouts.
"""
import math

import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_
from paper_2105_07388_amd import inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"
U = {"bf16": 2.0**-8, "fp16": 2.0**-11}
OFMT = {"bf16": 2, "fp16": 3}
OPREC = {"bf16": 1, "fp16": 2}


def _x(orc, seed, n, k, fmt):
    return np.array([[orc.round_to(orc.gauss(seed, j, t, 1), OFMT[fmt]) for t in range(k)] for j in range(n)])


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("m,n,k", [(130, 96, 40), (64, 1000, 200), (70, 333, 300), (257, 600, 512)])
def test_lowprec_x_integer_layout(orc, fmt, m, n, k):
    A = inputs.small_integers(m, n, m * 7 + n, -100, 100)
    B = re_.sketch_x(A.to(DEV), k=k, l=k, precision=fmt, seed=4).cpu().numpy().astype(np.float64)
    X = _x(orc, 4, n, k, fmt)
    want = orc.apply_x(A.numpy(), orc.GAUSSIAN, k, fmt_x=OFMT[fmt], seed=4)
    np.testing.assert_allclose(want, A.numpy().astype(np.float64) @ X, rtol=1e-12, atol=1e-9)
    bound = (n * 2.0**-24) * (np.abs(A.numpy()) @ np.abs(X)) + 1e-30
    assert np.all(np.abs(B - want) <= bound), float(np.max(np.abs(B - want) / bound))


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
@pytest.mark.parametrize("scale", [1.0, 1e-6, 3e5])
def test_lowprec_x_gaussian_and_scaling(orc, fmt, scale):
    m, n, k = 200, 700, 96
    A = inputs.gaussian(m, n, 21, dtype=torch.float32) * scale
    B = re_.sketch_x(A.to(DEV), k=k, l=k, precision=fmt, seed=9).cpu().numpy().astype(np.float64)
    X = _x(orc, 9, n, k, fmt)
    want = orc.apply_x(A.numpy(), orc.GAUSSIAN, k, fmt_x=OFMT[fmt], seed=9)
    bound = (U[fmt] + n * 2.0**-24) * (np.abs(A.numpy().astype(np.float64)) @ np.abs(X))
    assert np.all(np.abs(B - want) <= bound)
    assert np.isfinite(B).all()


def _phi(fmt, A, k, m):
    fro = float(torch.linalg.norm(A.double()))
    return U[fmt] / math.sqrt(3) * fro * (1 / math.sqrt(k) + 1 / math.sqrt(m))


@pytest.mark.parametrize("fmt,eps", [("bf16", 1e-2), ("fp16", 1e-3)])
def test_precision_form_reduced(orc, fmt, eps):
    """Planted step spectrum (200 values at 1, then 1e-4 decaying geometrically) at
    reduced size: clear gap, so the rank is exactly 200 in either format."""
    m, n, k, l = 4096, 2048, 256, 384
    A = inputs.planted(m, n, inputs.c3_spectrum(1024), 1003, torch.float32)
    r, s, info = re_.rank_estimate(A.to(DEV), eps, k=k, l=l, x="gaussian", y="srht", precision=fmt, seed=2)
    ro, so, r1o, flo, _ = orc.rank_estimate(A.numpy(), eps, orc.GAUSSIAN, orc.SRHT, k=k, l=l, prec=OPREC[fmt], seed=2)
    assert r == ro == 200
    phi = _phi(fmt, A, k, m)
    err = np.abs(s - so)
    assert np.all(err <= 2 * phi), (float(err.max()), phi)
    assert info["flags"] & (re_.FLAG_USED_BF16 if fmt == "bf16" else re_.FLAG_USED_FP16)


def test_precision_auto_choice(orc):
    """AUTO keeps BF16 at eps 1e-2 and moves to FP16 at 1e-3 (the floors are
    1.6e-3 and 2.0e-4 of sigma_1 for this spectrum and sketch)."""
    m, n, k, l = 4096, 2048, 256, 384
    A = inputs.planted(m, n, inputs.c3_spectrum(1024), 1003, torch.float32).to(DEV)
    r, s, info = re_.rank_estimate(A, 1e-2, k=k, l=l, y="srht", precision="auto", seed=2)
    assert r == 200 and info["flags"] & re_.FLAG_USED_BF16
    r, s, info = re_.rank_estimate(A, 1e-3, k=k, l=l, y="srht", precision="auto", seed=2)
    assert r == 200 and info["flags"] & re_.FLAG_USED_FP16
    r, s, info = re_.rank_estimate(A, 1e-7, k=k, l=l, y="srht", precision="auto", seed=2)
    assert info["flags"] & re_.FLAG_PREC_FALLBACK
    assert not info["flags"] & (re_.FLAG_USED_BF16 | re_.FLAG_USED_FP16)


def test_precision_form_full_size(orc):
    """FP32 32768 x 8192, Gaussian X of 512 columns in BF16 (eps 1e-2) and FP16
    (eps 1e-3), SRHT Y of 768 rows: rank 200 both ways; sampled rows of A X match
    the oracle's rows within the entrywise bound."""
    A = inputs.c3_matrix(device=DEV)
    m, n = A.shape
    k, l = 512, 768
    for fmt, eps in [("bf16", 1e-2), ("fp16", 1e-3)]:
        r, s, info = re_.rank_estimate(A, eps, k=k, l=l, y="srht", precision=fmt, seed=11)
        assert r == 200, (fmt, r)
        assert s[199] > 0.1 and s[200] < eps * s[0] / 4  # the gap around tau
        B = re_.sketch_x(A, k=k, l=k, precision=fmt, seed=11)
        rows = np.array([0, 1, 4097, 20000, m - 1])
        Arows = A[rows].cpu().numpy()
        X = np.array([[orc.round_to(orc.gauss(11, j, t, 1), OFMT[fmt]) for t in range(k)] for j in range(n)])
        want = Arows.astype(np.float64) @ X
        got = B[rows].cpu().numpy().astype(np.float64)
        bound = (U[fmt] + n * 2.0**-24) * (np.abs(Arows.astype(np.float64)) @ np.abs(X))
        assert np.all(np.abs(got - want) <= bound)


def test_precision_form_full_size_every_sigma(orc):
    """Every one of the 512 estimates at the workload's size (FP32 32768 x 8192,
    Gaussian X 512 in BF16 at eps 1e-2 and FP16 at eps 1e-3, SRHT Y 768) against
    the FP64 oracle run on the same FP32 A with the same rounded X: the error
    stays within 2 phi_f, and the rank is 200 on both sides."""
    A = inputs.c3_matrix(device=DEV)
    m, n = A.shape
    k, l = 512, 768
    An = A.cpu().numpy()
    phi = {f: _phi(f, A, k, m) for f in ("bf16", "fp16")}
    for fmt, eps, seed in [("bf16", 1e-2, 11), ("fp16", 1e-3, 12)]:
        r, s, info = re_.rank_estimate(A, eps, k=k, l=l, y="srht", precision=fmt, seed=seed)
        ro, so, r1o, flo, _ = orc.rank_estimate_gemm(An, eps, orc.GAUSSIAN, orc.SRHT, k=k, l=l, prec=OPREC[fmt],
                                                     seed=seed)
        err = np.abs(s - so)
        print(f"precision form full size, {fmt} at eps {eps}: max |d sigma| = {err.max():.3e} "
              f"({err.max() / phi[fmt]:.3f} phi_f, {err.max() / so[0]:.3e} sigma_1), ranks {r} / {ro}")
        assert r == ro == 200, (fmt, r, ro)
        assert np.all(err <= 2 * phi[fmt]), (fmt, float(err.max()), phi[fmt])
