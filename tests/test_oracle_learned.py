"""Pins of the adaptive-driver and MLP oracle (oracle/learned.py) against what
the mathematics fixes: central finite differences for the gradient, a
hand-evaluated network, Adam's first step in closed form, and the doubling
schedule's convergence point on planted step spectra (the first k on the
doubling grid with r1(k) above the planted rank, Sec. 5)."""
import math

import numpy as np
import pytest
import torch

from paper_2105_07388_amd import inputs


@pytest.fixture(scope="module")
def L(orc):
    return orc.learned


def _rand_problem(L, seed, B=7):
    rng = np.random.default_rng(seed)
    p = L.init_params(seed) + rng.normal(0, 0.05, L.N_PARAMS)
    X = rng.normal(0, 1, (B, L.N_IN))
    t = rng.normal(0, 1, B)
    return p, X, t


def test_gradient_matches_central_differences(L):
    for seed in (1, 2):
        p, X, t = _rand_problem(L, seed)
        g = L.grad(p, X, t)
        rng = np.random.default_rng(seed + 10)
        idx = np.concatenate([rng.choice(L.N_PARAMS, 60, replace=False), [L.N_PARAMS - 1, 0, 2240, 2304]])
        h = 1e-6
        for i in idx:
            e = np.zeros(L.N_PARAMS)
            e[i] = h
            fd = (L.loss(p + e, X, t) - L.loss(p - e, X, t)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_forward_hand_evaluated(L):
    rng = np.random.default_rng(3)
    p = np.zeros(L.N_PARAMS)
    w = L.unpack(p)
    w["W1"][...] = rng.normal(0, 1, (64, 35))
    w["W2"][...] = np.eye(64)
    w["w3"][...] = 1.0
    w["b3"][0] = 0.25
    X = rng.normal(0, 1, (5, 35))
    want = np.array([sum(max(0.0, float(np.dot(w["W1"][i], x))) for i in range(64)) for x in X]) + 0.25
    y, _, _ = L.forward(p, X)
    assert np.allclose(y, want, rtol=1e-14, atol=1e-14)
    # at the targets the loss and its gradient vanish
    assert L.loss(p, X, y) == 0.0 and np.abs(L.grad(p, X, y)).max() == 0.0


def test_adam_first_steps_closed_form(L):
    rng = np.random.default_rng(4)
    p = rng.normal(0, 1, 50)
    g = rng.normal(0, 1, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    p1, m, v = L.adam_step(p, g, m, v, 1, 1e-3)
    # first step: m^ = g, v^ = g^2, so the step is lr g / (|g| + eps)
    assert np.allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    p2, m, v = L.adam_step(p1, g, m, v, 2, 1e-3)  # constant gradient: same step again
    assert np.allclose(p2 - p1, p1 - p, rtol=1e-12, atol=1e-16)


def test_features_and_proposal(L):
    s = 10.0 ** -np.arange(32, dtype=np.float64) * 3.0
    f = L.features(s, 4096, 1024, 1e-3)
    assert np.allclose(f[:9], -np.arange(9), atol=1e-12) and np.all(f[9:32] == -8.0)
    assert np.allclose(f[32:], [math.log10(4096), math.log10(1024), -3.0])
    f = L.features(np.zeros(32), 100, 25, 1e-6)
    assert np.all(f[:32] == -8.0)
    assert L.proposal(math.log(100.0), 0.0, 32, 1000) == 104
    assert L.proposal(math.log(10.0), 0.0, 32, 1000) == 64      # at least 2 k0
    assert L.proposal(math.log(5000.0), 0.0, 32, 1000) == 1000  # at most kmax
    assert L.l_for(64, 1.5, 1000) == 96 and L.l_for(64, 1.5, 80) == 80


@pytest.mark.parametrize("rank,rounds,kfinal", [(20, 1, 32), (50, 2, 64), (120, 4, 256)])
def test_doubling_converges_at_first_sufficient_width(L, orc, rank, rounds, kfinal):
    A = inputs.planted(600, 400, inputs.spectrum_step(400, rank, 1.0, 1e-10), 60 + rank).numpy()
    out = L.doubling(A, 1e-6, seed=5)
    assert (out["rounds"], out["k"], out["r"]) == (rounds, kfinal, rank)
    # the closed form: the first k = 32 2^t with r1(k) > rank
    k = 32
    while orc.r1_from_k(k) <= rank:
        k *= 2
    assert k == kfinal


@pytest.mark.parametrize("rank,rounds,kfinal", [(50, 2, 64), (120, 4, 256)])
def test_doubling_with_an_srht_y(L, orc, rank, rounds, kfinal):
    # the same closed form with the SRHT Y (m = 600: padded to 1024 rows), and
    # the final round is Algorithm 1 at that width
    A = inputs.planted(600, 400, inputs.spectrum_step(400, rank, 1.0, 1e-10), 60 + rank).numpy()
    out = L.doubling(A, 1e-6, seed=5, ykind=orc.SRHT)
    assert (out["rounds"], out["k"], out["r"]) == (rounds, kfinal, rank)
    r, s, r1, fl, _ = orc.rank_estimate(A, 1e-6, orc.GAUSSIAN, orc.SRHT, k=out["k"], l=out["l"], seed=5)
    assert r == out["r"] and np.array_equal(s, out["sigma"])


def test_learned_round_uses_the_proposal(L):
    A = inputs.planted(600, 400, inputs.spectrum_step(400, 120, 1.0, 1e-10), 180).numpy()
    p = np.zeros(L.N_PARAMS)
    L.unpack(p)["b3"][0] = math.log(197.5)  # constant network: proposes 200
    out = L.doubling(A, 1e-6, seed=5, params=p)
    assert (out["rounds"], out["k"], out["r"], out["k_proposed"]) == (2, 200, 120, 200)
    L.unpack(p)["b3"][0] = math.log(97.5)  # too small: doubling continues from 104
    out = L.doubling(A, 1e-6, seed=5, params=p)
    assert (out["rounds"], out["k"], out["r"], out["k_proposed"]) == (3, 208, 120, 104)


# --- gap-based rank (Sec. 5 after Algorithm 1, Sec. 6.1) ---------------------------

def test_gap_rank_definition(orc):
    G = orc.gap
    s = [1.0] * 20 + [1e-8] * 20
    assert G.gap_rank(s, 36) == (20, 1e8)
    assert G.gap_rank(s, 15) == (1, 1.0)      # no gap inside the first r1: ties go to i = 1
    assert G.gap_rank([3.0, 1.0, 0.5, 0.0, 0.0], 5) == (3, math.inf)
    assert G.gap_rank([0.0, 0.0], 2) == (0, 0.0)
    assert G.gap_rank([2.0], 1) == (0, 0.0)
    # graded spectrum 10^(-i/20) with one planted jump of 1e-4 after 37 values
    s = [10.0 ** (-i / 20) for i in range(60)]
    s = s[:37] + [v * 1e-4 for v in s[37:]]
    r, q = G.gap_rank(s, 54)
    assert r == 37 and abs(q - 10.0 ** (1 / 20) * 1e4) < 1e-6 * q


def test_evaluation_acceptance_rule():
    """Sec. 1.1's goal for an estimate of the eps-rank, on a hand-checked
    spectrum: r^ is acceptable when sigma_{r^+1} < 10 eps sigma_1 and
    sigma_{r^} > 0.1 eps sigma_1; step spectra need the exact planted rank."""
    from paper_2105_07388_amd import learned
    s = np.array([1.0, 0.2, 0.05, 3e-3, 1.5e-3, 5e-4, 2e-4, 9e-5, 1e-6])
    eps = 1e-3
    # sigma_{r+1} < 1e-2 needs r >= 3 (sigma_4 = 1.5e-3); sigma_r > 1e-4 needs r <= 7 (sigma_7 = 2e-4, sigma_8 = 9e-5)
    got = [learned.acceptable(s, r, eps) for r in range(0, 10)]
    assert got == [False, False, False, True, True, True, True, True, False, False]
    # r = 0 only when sigma_1 is already below 10 eps
    assert learned.acceptable(np.array([1.0, 1e-9]), 1, 1e-3) and not learned.acceptable(np.array([1.0]), 0, 1e-3)
    p = dict(R=40, r=12, eps=1e-4, decay="step", m=400, n=100, seed=3)
    assert learned.agrees(p, 12) and not learned.agrees(p, 11) and not learned.agrees(p, 13)
    p = dict(p, decay="exp")
    sig = __import__("paper_2105_07388_amd").inputs.learned_spectrum(p)
    ok = [r for r in range(0, 41) if learned.agrees(p, r)]
    assert 12 in ok and ok == list(range(ok[0], ok[-1] + 1))
    assert sig[ok[0]] < 10 * p["eps"] and sig[ok[-1] - 1] > 0.1 * p["eps"]
