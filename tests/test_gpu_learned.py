"""GPU tests of the learned sketch-width policy: the network kernels against
the FP64 oracle (forward, gradient, Adam, a short training run), the adaptive
driver against the oracle's doubling driver and against single calls, and the
trained network's gain over plain doubling.

Tolerances: FP32 network arithmetic over at most 64-term dot products and a
batch sum, against FP64: outputs |dy| <= 1e-4 (1 + |y|); gradients
|dg| <= 2e-4 max|g|; Adam parameters 1e-6 absolute.  Adaptive runs: the same
final width and rounds as the oracle, sigma within the FP32 Gaussian bound
8 2^-24 sqrt(n) sigma_1, ranks equal away from the eps threshold.
"""
import math
import os

import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_
from paper_2105_07388_amd import inputs, learned

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _problem(L, seed, B=300):
    rng = np.random.default_rng(seed)
    p = L.init_params(seed) + rng.normal(0, 0.05, L.N_PARAMS)
    X = rng.normal(0, 1, (B, L.N_IN))
    X[:, 32:] = rng.uniform(-6, 5, (B, 3))
    t = rng.normal(4, 1, B)
    return p, X, t


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def test_mlp_forward_matches_oracle(orc):
    L = orc.learned
    p, X, t = _problem(L, 1)
    # the oracle works in FP64 on the FP32-rounded inputs
    p32, X32 = p.astype(np.float32).astype(np.float64), X.astype(np.float32).astype(np.float64)
    want, _, _ = L.forward(p32, X32)
    got = re_.mlp_forward(_dev(p), _dev(X)).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - want) <= 1e-4 * (1 + np.abs(want)))


def test_mlp_gradient_matches_oracle(orc):
    L = orc.learned
    for seed, B in ((2, 300), (3, 1), (4, 1000)):
        p, X, t = _problem(L, seed, B)
        p32, X32, t32 = (a.astype(np.float32).astype(np.float64) for a in (p, X, t))
        want = L.grad(p32, X32, t32)
        g, loss = re_.mlp_loss_grad(_dev(p), _dev(X), _dev(t))
        g = g.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(g - want) <= 2e-4 * np.abs(want).max()), np.abs(g - want).max() / np.abs(want).max()
        assert abs(float(loss.item()) - L.loss(p32, X32, t32)) <= 1e-4 * L.loss(p32, X32, t32)
        # deterministic: the same call gives the same bits
        g2, _ = re_.mlp_loss_grad(_dev(p), _dev(X), _dev(t))
        assert np.array_equal(g2.cpu().numpy(), g.astype(np.float32))


def test_adam_and_short_training_match_oracle(orc):
    L = orc.learned
    p, X, t = _problem(L, 5, 64)
    pd, md, vd = _dev(p), torch.zeros(L.N_PARAMS, device=DEV), torch.zeros(L.N_PARAMS, device=DEV)
    po = p.astype(np.float32).astype(np.float64)
    mo, vo = np.zeros(L.N_PARAMS), np.zeros(L.N_PARAMS)
    Xd, td = _dev(X), _dev(t)
    X32, t32 = X.astype(np.float32).astype(np.float64), t.astype(np.float32).astype(np.float64)
    for step in range(1, 6):
        g, _ = re_.mlp_loss_grad(pd, Xd, td)
        re_.mlp_adam(pd, g, md, vd, step, 1e-3)
        po, mo, vo = L.adam_step(po, L.grad(po, X32, t32), mo, vo, step, 1e-3)
    # each Adam step moves a parameter by about lr; FP32 gradients only change its sign
    # where the gradient is near zero, so compare where the oracle's steps were decisive
    diff = np.abs(pd.cpu().numpy() - po)
    assert np.quantile(diff, 0.99) <= 1e-5 and diff.max() <= 1e-2


def _planted32(m, n, rank, seed, decay="step"):
    s = inputs.spectrum_step(n, rank, 1.0, 1e-9) if decay == "step" else inputs.c2_spectrum(n)
    return inputs.planted(m, n, s, seed, torch.float32)


@pytest.mark.parametrize("rank", [20, 50, 120])
def test_adaptive_doubling_matches_oracle(orc, rank):
    A = _planted32(800, 400, rank, 70 + rank)
    r, s, info = re_.rank_adaptive(A.to(DEV), 1e-6, seed=5)
    out = orc.learned.doubling(A.numpy(), 1e-6, seed=5)
    assert (info["k"], info["l"], info["rounds"]) == (out["k"], out["l"], out["rounds"])
    assert r == out["r"] == rank
    tol = 8 * 2.0**-24 * math.sqrt(400) * out["sigma"][0]
    assert np.all(np.abs(s - out["sigma"]) <= tol)


def test_adaptive_equals_single_call_at_final_width():
    A = _planted32(1500, 700, 90, 11, decay="geo").to(DEV)
    for eps in (1e-2, 1e-4):
        r, s, info = re_.rank_adaptive(A, eps, seed=9)
        r1, s1, info1 = re_.rank_estimate(A, eps, k=info["k"], l=info["l"], seed=9)
        assert r == r1 and np.array_equal(s, s1) and info["flags"] == info1["flags"]


def test_adaptive_learned_round_with_constant_network(orc):
    A = _planted32(800, 400, 120, 190)
    L = orc.learned
    # outputs away from the multiple-of-8 rounding edges: 197.5 -> 200, 97.5 -> 104
    for kp, want_rounds, want_k in ((197.5, 2, 200), (97.5, 3, 208)):
        p = np.zeros(L.N_PARAMS)
        L.unpack(p)["b3"][0] = math.log(kp)
        p = p.astype(np.float32).astype(np.float64)  # the network runs in FP32
        r, s, info = re_.rank_adaptive(A.to(DEV), 1e-6, mlp=_dev(p), seed=5)
        out = L.doubling(A.numpy(), 1e-6, seed=5, params=p)
        assert (info["rounds"], info["k"], info["k_proposed"]) == (out["rounds"], out["k"], out["k_proposed"])
        assert (info["rounds"], info["k"], r) == (want_rounds, want_k, 120)


def test_adaptive_limits_and_errors():
    A = _planted32(300, 100, 95, 3).to(DEV)
    r, s, info = re_.rank_adaptive(A, 1e-6, seed=1)  # rank 95 of n = 100: stops at k = n unconverged
    assert info["k"] == 100 and info["flags"] & re_.FLAG_NOT_CONVERGED and r == re_.r1_from_k(100)
    r, s, info = re_.rank_adaptive(A, 1e-6, k_max=48, seed=1)
    assert info["k"] == 48 and info["rounds"] == 2
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_adaptive(A.double(), 1e-6)
    assert ei.value.status == -2
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_adaptive(A, 0.0)
    assert ei.value.status == -1


@pytest.mark.parametrize("m,n,rank", [(800, 400, 50), (1000, 500, 120), (3000, 1200, 250)])
def test_adaptive_srht_y_matches_oracle_and_single_call(orc, m, n, rank):
    # the SRHT Y grown from its stored first-level transform (Sec. 5 footnote):
    # the final round equals one call at the final width, bit for bit
    A = _planted32(m, n, rank, 40 + rank)
    Ad = A.to(DEV)
    r, s, info = re_.rank_adaptive(Ad, 1e-6, seed=5, y="srht")
    out = orc.learned.doubling(A.numpy(), 1e-6, seed=5, ykind=orc.SRHT)
    assert (info["k"], info["l"], info["rounds"]) == (out["k"], out["l"], out["rounds"])
    assert r == out["r"] == rank
    tol = 8 * 2.0**-24 * math.sqrt(n) * out["sigma"][0]
    assert np.all(np.abs(s - out["sigma"]) <= tol)
    r1, s1, info1 = re_.rank_estimate(Ad, 1e-6, k=info["k"], l=info["l"], x="gaussian", y="srht", seed=5)
    assert r == r1 and np.array_equal(s, s1) and info["flags"] == info1["flags"]


def test_adaptive_srht_y_unaligned_store_equals_single_call():
    # k_max = 130 gives the stored transform a leading dimension that is not a
    # multiple of 4, so the growth takes the one-element-per-thread Y kernels;
    # the single call at the final k = 64 takes the four-column vector kernels.
    # Both perform the same butterflies and block sums in the same order.
    A = _planted32(2000, 800, 50, 77).to(DEV)
    r, s, info = re_.rank_adaptive(A, 1e-6, k_max=130, seed=9, y="srht")
    assert info["k"] == 64 and info["rounds"] == 2 and r == 50
    r1, s1, info1 = re_.rank_estimate(A, 1e-6, k=64, l=info["l"], x="gaussian", y="srht", seed=9)
    assert r == r1 and np.array_equal(s, s1) and info["flags"] == info1["flags"]


def test_adaptive_srht_y_limits_and_errors():
    A = _planted32(300, 100, 95, 3).to(DEV)
    r, s, info = re_.rank_adaptive(A, 1e-6, seed=1, y="srht")
    assert info["k"] == 100 and info["flags"] & re_.FLAG_NOT_CONVERGED
    r, s, info = re_.rank_adaptive(A, 1e-6, k_max=48, seed=1, y="srht")
    assert info["k"] == 48 and info["rounds"] == 2
    r1, s1, _ = re_.rank_estimate(A, 1e-6, k=48, l=info["l"], x="gaussian", y="srht", seed=1)
    assert r == r1 and np.array_equal(s, s1)
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_adaptive(A, 1e-6, y="hrtt")
    assert ei.value.status == -1


def test_trained_policy_beats_doubling():
    """The committed network against plain doubling on unseen matrices: fewer
    rounds on average, and at least the same agreement (the exact planted rank
    on step spectra, Sec. 1.1's conditions on poly and exp spectra)."""
    if not os.path.exists(learned.DEFAULT_WEIGHTS):
        pytest.skip("no trained weights committed")
    policy, delta = learned.load_policy()
    params = inputs.learned_params(16, seed=3005, m_lo=4096, m_hi=8192)  # the training range's small end
    out = learned.compare(params, policy, delta, log=lambda s: None)
    assert out["learned"]["mean_rounds"] < out["doubling"]["mean_rounds"]
    assert out["learned"]["agreement"] >= out["doubling"]["agreement"] - 1.0 / 16
    if out["step_same_rank"] is not None:
        assert out["step_same_rank"] == 1.0


def test_adaptive_srht_y_full_size_equals_single_call():
    # the stored-transform growth on the benchmark's 65536 x 16384 matrix
    A = inputs.c2_matrix(device=DEV)
    for eps in (1e-3, 1e-5):
        r, s, info = re_.rank_adaptive(A, eps, seed=31, y="srht")
        r1, s1, info1 = re_.rank_estimate(A, eps, k=info["k"], l=info["l"], x="gaussian", y="srht", seed=31)
        assert info["rounds"] >= 2 and r == r1 and np.array_equal(s, s1) and info["flags"] == info1["flags"]
