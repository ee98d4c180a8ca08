"""Pins of the QR-diagonal estimates (oracle/qrdiag.py): exact cases where the
diagonal of R is known, the determinant identity, and the rank-revealing
behaviour the paper relies on for sketches with randomised right singular
vectors."""
import math

import numpy as np
import pytest

from paper_2105_07388_amd import inputs


def test_orthogonal_columns_give_their_norms(orc):
    # C = U diag(s) with orthonormal U: R = diag(s) up to signs
    s = np.array([3.0, 0.5, 2.0, 1e-9, 7.0])
    U, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((40, 5)))
    d = orc.qrdiag.qr_diag(U * s)
    assert np.allclose(d, np.sort(s)[::-1], rtol=1e-12, atol=1e-15)


def test_triangular_and_determinant(orc):
    rng = np.random.default_rng(2)
    T = np.triu(rng.standard_normal((6, 6))) + 3 * np.eye(6)
    assert np.allclose(orc.qrdiag.qr_diag(T), np.sort(np.abs(np.diagonal(T)))[::-1], rtol=1e-13)
    C = rng.standard_normal((9, 9))
    # prod |R_jj| = |det C| = prod sigma_j
    assert math.isclose(np.prod(orc.qrdiag.qr_diag(C)), abs(np.linalg.det(C)), rel_tol=1e-10)
    assert math.isclose(np.prod(orc.qrdiag.qr_diag(C)), np.prod(np.linalg.svd(C, compute_uv=False)), rel_tol=1e-10)


def test_rank_revealing_on_randomised_right_singular_vectors(orc):
    # C = U diag(s) V^T with Haar V: the diagonal of an unpivoted QR tracks the
    # singular values within a modest factor, and a gap shows up at its index
    rng = np.random.default_rng(3)
    k = 60
    s = np.concatenate([np.geomspace(1, 0.1, 25), 1e-7 * np.geomspace(1, 0.1, k - 25)])
    U, _ = np.linalg.qr(rng.standard_normal((90, k)))
    V, _ = np.linalg.qr(rng.standard_normal((k, k)))
    d = orc.qrdiag.qr_diag((U * s) @ V.T)
    assert np.all(d[:25] > 1e-3) and np.all(d[25:] < 1e-6)
    assert np.all(d[:25] <= s[0] * (1 + 1e-12))
    assert np.max(np.abs(np.log10(d[:25] / s[:25]))) < 2.5


def test_planted_gap_rank(orc):
    A = inputs.c1_matrix().numpy()
    r, d, r1, flags = orc.qrdiag.rank_estimate_qr(A, 1e-6, k=40, l=60, seed=0)
    assert r == 20 and r1 == 36 and flags == 0
    # the same sketch's singular values bound the diagonal's product
    rs, s, _, _, _ = orc.rank_estimate(A, 1e-6, k=40, l=60, seed=0)
    assert rs == 20
    assert math.isclose(np.sum(np.log(d)), np.sum(np.log(s)), rel_tol=1e-9)
