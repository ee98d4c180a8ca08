"""FP64 oracle of the adaptive sketch-size driver and of its MLP (test
infrastructure only: only tests/, the package smoke check and the benchmark's
CPU-baseline leg may import it; the product library never does).

What the paper fixes (Sec. 5, the paragraphs after Algorithm 1 and their
footnote): when the estimate reaches the sketch's capacity (r^ = r1, the
NOT_CONVERGED case) the algorithm is rerun with a larger r1, reusing the work
done by appending columns to X and rows to Y; with Gaussian sketches the
update r1 := 2 r1 costs at most a factor 2 over knowing r1 in advance.
Because every sketch entry here is a function of its index only, the k-column
X and l-row Y of a round are the leading columns / rows of every larger
round's, so `doubling` below simply reruns the plain estimator with k doubled.

What the paper leaves open (Sec. 7: choosing a new r1 from the first run) and
this project adds: a small multilayer perceptron reads features of a cheap
pilot sketch and proposes the sketch width; doubling takes over when the
proposal turns out too small.  The network here is the plain FP64 reference
of the GPU kernels: 35 inputs -> 64 ReLU -> 64 ReLU -> 1 output, mean squared
error, Adam (Kingma & Ba, ICLR 2015, Algorithm 1).

Parameter vector layout (6529 values): W1 (64 x 35, row-major), b1 (64),
W2 (64 x 64), b2 (64), w3 (64), b3 (1).
"""
import math

import numpy as np

from . import pyoracle as _o

N_IN, N_H = 35, 64
SIZES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)), ("w3", (N_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 6529


def unpack(p):
    """Views of the parameter vector by name."""
    out, o = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = p[o:o + size].reshape(shape)
        o += size
    return out


def forward(p, X):
    """Outputs y (batch) and the hidden pre-activations z1, z2 (batch x 64)."""
    w = unpack(np.asarray(p, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w["w3"] + w["b3"][0]
    return y, z1, z2


def loss(p, X, t):
    """Mean squared error (1/B) sum (y_s - t_s)^2."""
    y, _, _ = forward(p, X)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def grad(p, X, t):
    """Gradient of `loss` by the chain rule, layer by layer."""
    w = unpack(np.asarray(p, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    y, z1, z2 = forward(p, X)
    h1, h2 = np.maximum(z1, 0.0), np.maximum(z2, 0.0)
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / B  # dL/dy_s
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, w["w3"]) * (z2 > 0.0)
    g["W2"] = dz2.T @ h1
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ w["W2"]) * (z1 > 0.0)
    g["W1"] = dz1.T @ X
    g["b1"] = dz1.sum(axis=0)
    return np.concatenate([g[name].ravel() for name, _ in SIZES])


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def init_params(seed):
    """He-uniform weights, zero biases (the starting point used for training)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(N_PARAMS)
    w = unpack(p)
    for name, fan_in in (("W1", N_IN), ("W2", N_H), ("w3", N_H)):
        lim = math.sqrt(6.0 / fan_in)
        w[name][...] = rng.uniform(-lim, lim, w[name].shape)
    return p


def features(sigma, m, n, eps):
    """Network input from a pilot sketch: log10(s_i / s_1) for the first 32
    estimates (clamped below at -8; missing ones count as -8), then log10 m,
    log10 n, log10 eps."""
    s = np.asarray(sigma, dtype=np.float64)[:32]
    f = np.full(N_IN, -8.0)
    if s.size and s[0] > 0:
        with np.errstate(divide="ignore"):
            r = np.log10(np.maximum(s / s[0], 0.0))
        f[:s.size] = np.maximum(r, -8.0)
    f[32], f[33], f[34] = math.log10(m), math.log10(n), math.log10(eps)
    return f


def proposal(y, delta, k0, kmax):
    """Sketch width proposed by network output y (natural log of the width):
    ceil(exp(y + delta)) rounded up to a multiple of 8, within [2 k0, kmax]."""
    k = int(math.ceil(math.exp(y + delta)))
    k = (k + 7) // 8 * 8
    return int(min(max(k, 2 * k0), kmax))


def l_for(k, l_ratio, m):
    """Rows of Y for a k-column X: round(l_ratio k), at least k, at most m."""
    return int(min(max(int(math.floor(l_ratio * k + 0.5)), k), m))


def doubling(A, eps, seed=0, k0=32, l_ratio=1.5, kmax=None, params=None, delta=0.0, ykind=_o.GAUSSIAN):
    """The adaptive driver: pilot at k0, then (with `params`) one round at the
    network's proposal, then doubling until r^ < r1(k) or k reaches kmax.
    X is Gaussian, Y Gaussian or SRHT (`ykind`); the sketches nest in (k, l),
    so each round is Algorithm 1 at that width (Sec. 5: rerun with a larger
    r1 by appending to X and Y).  Returns dict(r, k, l, rounds, sigma, flags,
    k_proposed)."""
    m, n = A.shape
    kmax = min(n, kmax or n)
    k = min(k0, kmax)
    rounds, kprop = 0, 0
    while True:
        l = l_for(k, l_ratio, m)
        r, s, r1, flags, _ = _o.rank_estimate(A, eps, _o.GAUSSIAN, ykind, k=k, l=l, seed=seed)
        rounds += 1
        if not (flags & _o.FLAG_NOT_CONVERGED) or k >= kmax:
            return dict(r=r, k=k, l=l, rounds=rounds, sigma=s, flags=flags, k_proposed=kprop)
        if rounds == 1 and params is not None:
            y, _, _ = forward(params, features(s, m, n, eps)[None, :])
            kprop = proposal(float(y[0]), delta, k0, kmax)
            k = kprop
        else:
            k = min(2 * k, kmax)
