"""Pins of the Algorithm 3 oracle (oracle/rangefinder.py): the width rule in
closed form and against its definition, the step-spectrum case where the rule
must land on the gap, and the QB factorisation against Eckart-Young and the
Halko-Martinsson-Tropp expectation bound on matrices of known spectrum."""
import math

import numpy as np
import pytest

from paper_2105_07388_amd import inputs


def test_width_rule_closed_form(orc):
    F = orc.rangefinder
    # ten unit values, then 1e-3: for r = 10 the extended tail is
    # 26 (1e-3)^2 over j = 11..36 plus 964 (1e-3)^2 beyond r1 = 36, so the
    # bound is sqrt(1 + 10/4) sqrt(990e-6) = 0.058864...
    s = np.array([1.0] * 10 + [1e-3] * 30)
    r1, n, p = 36, 1000, 5
    assert F.tail_bound(s, r1, n, 10, p) == pytest.approx(math.sqrt(3.5) * math.sqrt(990e-6), rel=1e-14)
    assert F.choose_rank(s, r1, n, 0.06, p) == 10
    assert F.choose_rank(s, r1, n, 0.9, p) == 10
    # r = 9 leaves one unit value: sqrt(1 + 9/4) sqrt(1 + 990e-6) = 1.8037 <= 2
    assert F.choose_rank(s, r1, n, 2.0, p) == 9
    # the factor (1 + r/4)^(1/2) grows faster than the flat tail shrinks
    assert F.choose_rank(s, r1, n, 0.05, p) is None
    assert F.choose_rank(s, r1, n, 1e-9, p) is None
    # a given ||A|| replaces s_1: 0.12 * 0.5 = 0.06 admits r = 10, 0.12 * 0.45 not
    assert F.choose_rank(s, r1, n, 0.12, p, norm_a=0.5) == 10
    assert F.choose_rank(s, r1, n, 0.12, p, norm_a=0.45) is None
    assert F.choose_rank(np.zeros(5), 4, 10, 0.1, 2) == 0


def test_width_rule_is_the_first_admissible_width(orc):
    F = orc.rangefinder
    rng = np.random.default_rng(1)
    s = np.sort(rng.random(60))[::-1] ** 6
    r1, n, p, eps = 54, 500, 4, 1e-2
    r = F.choose_rank(s, r1, n, eps, p)
    ext = np.concatenate([s[:r1], np.full(n - r1, s[r1 - 1])])

    def bound(rr):  # the rule written out over the extended sequence
        return math.sqrt(1 + rr / (p - 1)) * math.sqrt(np.sum(ext[rr:] ** 2))

    assert r is not None
    assert bound(r) <= eps * s[0] and all(bound(q) > eps * s[0] for q in range(1, r))


def test_step_spectrum_lands_on_the_gap(orc):
    # 20 unit values then 1e-8 (the workload with a planted gap): every r < 20
    # leaves a unit value in the tail, r = 20 leaves only 1e-8 values
    A = inputs.c1_matrix().numpy()
    out = orc.rangefinder.rangefinder(A, 1e-5, p=5, k0=32, seed=3)
    assert out["r"] == 20 and out["w"] == 25 and out["rounds"] == 1


def test_doubling_until_a_width_qualifies(orc):
    spec = 10.0 ** (-np.arange(200) / 20.0)
    A = inputs.planted(300, 240, spec, 5).numpy()
    out = orc.rangefinder.rangefinder(A, 1e-3, p=5, k0=16, seed=6)
    # rank_1e-3 is about 61, so k = 16 and 32 cannot hold r + p; k = 64 may not
    assert out["k"] in (64, 128) and out["rounds"] == int(math.log2(out["k"] // 16)) + 1
    assert out["r"] + 5 <= out["k"]
    # k capped below any admissible width: no r, nothing formed
    none = orc.rangefinder.rangefinder(A, 1e-3, p=5, k0=16, kmax=40, seed=6)
    assert none["r"] is None and none["Q"] is None and none["k"] == 40


def test_qb_recovers_an_exact_low_rank_matrix(orc):
    A = inputs.exact_rank(300, 200, 15, 3).numpy()
    out = orc.rangefinder.rangefinder(A, 1e-6, p=5, k0=40, seed=2)
    assert out["r"] == 15 and out["w"] == 20
    Q, B = out["Q"], out["B"]
    assert np.allclose(Q.T @ Q, np.eye(20), atol=1e-12)
    assert np.linalg.norm(A - Q @ B) <= 1e-10 * np.linalg.norm(A)


def test_thin_qr_signs_and_factorisation(orc):
    W = np.random.default_rng(4).standard_normal((50, 7))
    Q, R = orc.rangefinder.thin_qr(W)
    assert np.all(np.diagonal(R) > 0) and np.allclose(np.triu(R), R)
    assert np.allclose(Q @ R, W, atol=1e-13) and np.allclose(Q.T @ Q, np.eye(7), atol=1e-14)


def test_qb_error_between_eckart_young_and_the_expectation_bound(orc):
    spec = 10.0 ** (-np.arange(150) / 20.0)
    A = inputs.planted(400, 300, spec, 9).numpy()
    p, errs, bounds = 5, [], []
    for seed in range(6):
        out = orc.rangefinder.rangefinder(A, 1e-2, p=p, k0=96, seed=seed)
        w, r = out["w"], out["r"]
        err = np.linalg.norm(A - out["Q"] @ out["B"])
        # no rank-w factorisation beats the truncated SVD (Eckart-Young)
        assert err >= math.sqrt(np.sum(spec[w:] ** 2)) * (1 - 1e-9)
        errs.append(err)
        bounds.append(math.sqrt(1 + r / (p - 1)) * math.sqrt(np.sum(spec[r:] ** 2)))
    # the expectation bound with the true values, on the average over draws
    assert np.mean(errs) <= np.mean(bounds)
