"""Seeded synthetic test matrices (no part of the estimator's arithmetic).

Shared by the tests, the benchmark and the smoke check, for both the GPU library
and the CPU oracle.  Every matrix is synthetic with a prescribed spectrum, as in
the paper's experiments (Sec. 6: diagonal test matrices with gaps, polynomial and
exponential decay).  Dense planted matrices A = U diag(s) V^T use thin Haar factors
(QR of a seeded Gaussian, columns multiplied by sign(diag R), Mezzadri 2007), are
formed in FP64 and rounded once to the storage type.

All generation goes through ``torch`` so that large inputs can be produced directly
in device memory; a given (seed, device type) always yields the same bytes.
"""
from __future__ import annotations

import numpy as np
import torch


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def haar(rows: int, cols: int, seed: int, device="cpu") -> torch.Tensor:
    """Thin Haar-distributed factor with orthonormal columns (rows >= cols), FP64."""
    g = _gen(seed, device)
    G = torch.randn(rows, cols, generator=g, dtype=torch.float64, device=device)
    Q, R = torch.linalg.qr(G, mode="reduced")
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    return Q * d


def haar_cholqr2(rows: int, cols: int, seed: int, device="cpu") -> torch.Tensor:
    """The same factor as ``haar`` (the Q of the QR with a positive diagonal
    of the same seeded Gaussian, which is unique) computed by two Cholesky-QR
    passes: Q1 = G L1^-T with L1 L1^T = G^T G, then Q = Q1 L2^-T with
    L2 L2^T = Q1^T Q1.  A tall Gaussian is well conditioned (kappa near
    (1 + sqrt(c/r)) / (1 - sqrt(c/r))), so two passes give orthogonality and
    agreement with ``haar`` at the FP64 rounding level, at a fraction of the
    cost of a Householder QR on the GPU."""
    g = _gen(seed, device)
    G = torch.randn(rows, cols, generator=g, dtype=torch.float64, device=device)
    eye = torch.eye(cols, dtype=torch.float64)
    for _ in range(2):
        # the small cols x cols factorisation and inverse on the host (LAPACK);
        # the products on the device
        L = torch.linalg.cholesky((G.T @ G).cpu())
        Linv = torch.linalg.solve_triangular(L, eye, upper=False)
        G = G @ Linv.T.to(device)
    return G


def planted(m: int, n: int, sigma, seed: int, dtype=torch.float64, noise: float = 0.0,
            device="cpu", chunk_rows: int = 4096, factor=None) -> torch.Tensor:
    """A = U diag(sigma) V^T (+ noise * N(0,1)) rounded once to ``dtype``.

    U is m x R and V is n x R thin Haar with R = len(sigma) <= min(m, n),
    from ``factor`` (default ``haar``; ``haar_cholqr2`` gives the same factors
    faster).
    """
    factor = haar if factor is None else factor
    s = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    R = s.numel()
    if R > min(m, n):
        raise ValueError("len(sigma) must not exceed min(m, n)")
    U = factor(m, R, seed, device)
    V = factor(n, R, seed + 7919, device)
    W = (V * s).T.contiguous()  # R x n
    A = torch.empty(m, n, dtype=dtype, device=device)
    gn = _gen(seed + 104729, device) if noise else None
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        blk = U[r0:r1] @ W
        if noise:
            blk += noise * torch.randn(r1 - r0, n, generator=gn, dtype=torch.float64, device=device)
        A[r0:r1] = blk.to(dtype)
        del blk
    return A


def diagonal(m: int, n: int, sigma, dtype=torch.float64, device="cpu") -> torch.Tensor:
    """The test matrices of Sec. 6: the singular values on the diagonal of an
    m x n matrix (decreasing), stored dense."""
    s = np.asarray(sigma, dtype=np.float64)
    d = min(m, n, s.size)
    A = torch.zeros(m, n, dtype=dtype, device=device)
    idx = torch.arange(d, device=device)
    A[idx, idx] = torch.as_tensor(s[:d], device=device).to(dtype)
    return A


def exact_rank(m: int, n: int, r: int, seed: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    """A = B C with Gaussian B (m x r) and C (r x n): rank exactly r (a.s.)."""
    g = _gen(seed, device)
    Bm = torch.randn(m, r, generator=g, dtype=torch.float64, device=device)
    Cm = torch.randn(r, n, generator=g, dtype=torch.float64, device=device)
    return (Bm @ Cm).to(dtype)


def gaussian(m: int, n: int, seed: int, dtype=torch.float64, device="cpu") -> torch.Tensor:
    g = _gen(seed, device)
    return torch.randn(m, n, generator=g, dtype=torch.float64, device=device).to(dtype)


def small_integers(m: int, n: int, seed: int, lo: int = -8, hi: int = 8, dtype=torch.float32,
                   device="cpu") -> torch.Tensor:
    """Integer-valued entries: every sum of products stays exact in FP32/FP64."""
    g = _gen(seed, device)
    return torch.randint(lo, hi + 1, (m, n), generator=g, device=device).to(dtype)


# --- spectra ------------------------------------------------------------------

def spectrum_gap(n: int, block: int = 100, levels=(1.0, 1e-4, 1e-8, 1e-12, 1e-16)) -> np.ndarray:
    """Sec. 6, matrix A_G: constant blocks of `block` values at each level."""
    s = np.full(n, levels[-1], dtype=np.float64)
    for b, v in enumerate(levels):
        s[b * block:(b + 1) * block] = v
    return s[:n]


def spectrum_poly(n: int, p: float) -> np.ndarray:
    """Sec. 6, A_SP (p = 1) and A_FP (p = 3): s_i = i^-p."""
    return np.arange(1, n + 1, dtype=np.float64) ** (-p)


def spectrum_exp(n: int, q: float) -> np.ndarray:
    """Sec. 6, A_SE (q = 0.01) and A_FE (q = 0.5): s_i = 10^(-q (i-1))."""
    return 10.0 ** (-q * np.arange(n, dtype=np.float64))


def spectrum_step(n: int, r: int, hi: float = 1.0, lo: float = 1e-8) -> np.ndarray:
    s = np.full(n, lo, dtype=np.float64)
    s[:r] = hi
    return s


# --- the workload shapes ----------------------------------------------------------

def c1_matrix(seed: int = 1001, device="cpu") -> torch.Tensor:
    """FP64 2000 x 1000, s = 1 (x20) then 1e-8 (x980): eps = 1e-6 gives rank 20."""
    return planted(2000, 1000, spectrum_step(1000, 20, 1.0, 1e-8), seed, torch.float64, 0.0, device)


def c2_spectrum(R: int = 1024) -> np.ndarray:
    """s_i = 10^(-i/20), i = 1..R."""
    return 10.0 ** (-np.arange(1, R + 1, dtype=np.float64) / 20.0)


def c2_matrix(m: int = 65536, n: int = 16384, R: int = 1024, seed: int = 1002, device="cpu") -> torch.Tensor:
    """FP32 m x n = U diag(10^(-i/20)) V^T + 1e-9 N, rounded once to FP32."""
    return planted(m, n, c2_spectrum(R), seed, torch.float32, 1e-9, device)


def c3_spectrum(R: int = 1024, r: int = 200) -> np.ndarray:
    """1 for the first r values, then 1e-4 decaying by a factor 10 every 100 values."""
    i = np.arange(1, R + 1, dtype=np.float64)
    s = 1e-4 * 10.0 ** (-(i - (r + 1)) / 100.0)
    s[:r] = 1.0
    return s


def c3_matrix(m: int = 32768, n: int = 8192, R: int = 1024, seed: int = 1003, device="cpu") -> torch.Tensor:
    return planted(m, n, c3_spectrum(R), seed, torch.float32, 0.0, device)



# --- kernel blocks of a hierarchical matrix ----------------------------------------

def kernel_block_params(nblocks: int, seed: int = 1004, size_lo: int = 256, size_hi: int = 4096,
                        gap_lo: float = 0.08, gap_hi: float = 3.0) -> list[dict]:
    """Shapes and cluster gaps of `nblocks` off-diagonal blocks: m, n uniform
    integers in [size_lo, size_hi], the gap g log-uniform in [gap_lo, gap_hi],
    one point seed per block.  Calibrated with full SVDs: at eps = 1e-6 the
    rank is about 63 for 4096 x 4096 at g = 0.08, 37 for 256 x 256 at g = 0.1
    and 6 at g = 3 for any size, so the ranks span about 6 to 63."""
    rng = np.random.default_rng(seed)
    m = rng.integers(size_lo, size_hi + 1, nblocks)
    n = rng.integers(size_lo, size_hi + 1, nblocks)
    g = np.exp(rng.uniform(np.log(gap_lo), np.log(gap_hi), nblocks))
    ps = rng.integers(0, 2**62, nblocks)
    return [dict(m=int(m[b]), n=int(n[b]), gap=float(g[b]), seed=int(ps[b])) for b in range(nblocks)]


def kernel_block_points(p: dict) -> tuple[torch.Tensor, torch.Tensor]:
    """FP32 target points (m x 2) uniform in [1+g, 2+g] x [0, 1] and source
    points (n x 2) uniform in [0, 1]^2, drawn on the CPU."""
    gen = torch.Generator(device="cpu")
    gen.manual_seed(p["seed"])
    t = torch.rand(p["m"], 2, generator=gen, dtype=torch.float32)
    t[:, 0] += 1.0 + p["gap"]
    s = torch.rand(p["n"], 2, generator=gen, dtype=torch.float32)
    return t, s


def kernel_block(p: dict, device="cpu", out: torch.Tensor | None = None) -> torch.Tensor:
    """A[i, j] = 1 / |t_i - s_j|, evaluated in FP64 from the FP32 points (one
    operation per kernel, so no fused multiply-add) and rounded once to FP32."""
    t, s = kernel_block_points(p)
    t = t.to(device=device, dtype=torch.float64)
    s = s.to(device=device, dtype=torch.float64)
    dx = t[:, 0:1] - s[:, 0].unsqueeze(0)
    dy = t[:, 1:2] - s[:, 1].unsqueeze(0)
    r2 = dx * dx
    r2 += dy * dy
    del dx, dy
    A = (1.0 / torch.sqrt(r2)).to(torch.float32)
    if out is None:
        return A
    out.copy_(A)
    return out


def kernel_blocks(nblocks: int, seed: int = 1004, device="cpu", **kw) -> tuple[torch.Tensor, list, list[dict]]:
    """All blocks in one flat FP32 buffer, each block contiguous (lda = n) and
    256-byte aligned.  Returns (buffer, list of m x n views, parameters)."""
    params = kernel_block_params(nblocks, seed, **kw)
    offs, off = [], 0
    for p in params:
        offs.append(off)
        off += (p["m"] * p["n"] + 63) // 64 * 64
    buf = torch.empty(max(off, 1), dtype=torch.float32, device=device)
    views = []
    for p, o in zip(params, offs):
        v = buf[o:o + p["m"] * p["n"]].view(p["m"], p["n"])
        kernel_block(p, device, out=v)
        views.append(v)
    return buf, views, params


# --- the learned sketch-size set --------------------------------------------------

def learned_params(count: int, seed: int = 1005, m_lo: int = 4096, m_hi: int = 65536,
                   r_cap: int = 2000) -> list[dict]:
    """Matrix recipes for the learned policy: m log-uniform in [m_lo, m_hi]
    (a multiple of 256), n = m / 4, decay uniform over {poly, exp, step}, a
    target eps log-uniform in [1e-6, 1e-2] and a target rank r log-uniform in
    [10, min(r_cap, n / 4)] that the spectrum realises at that eps."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        m = int(np.exp(rng.uniform(np.log(m_lo), np.log(m_hi))) // 256 * 256)
        m = max(m, 256)
        n = m // 4
        rmax = max(10, min(r_cap, n // 4))
        r = int(round(np.exp(rng.uniform(np.log(10), np.log(rmax)))))
        eps = float(np.exp(rng.uniform(np.log(1e-6), np.log(1e-2))))
        decay = ("poly", "exp", "step")[int(rng.integers(0, 3))]
        out.append(dict(m=m, n=n, r=r, eps=eps, decay=decay, R=min(n, 2 * r + 64), seed=int(seed * 100003 + i)))
    return out


def learned_spectrum(p: dict) -> np.ndarray:
    """sigma_1 = 1 and rank_eps = r exactly: poly s_i = i^-a with
    a = -ln(eps) / ln(r + 1/2); exp s_i = 10^(-q (i - 1)) with
    q = -log10(eps) / (r - 1/2); step: 1 for i <= r, then 1e-3 eps."""
    R, r, eps = p["R"], p["r"], p["eps"]
    i = np.arange(1, R + 1, dtype=np.float64)
    if p["decay"] == "poly":
        return i ** (np.log(eps) / np.log(r + 0.5))
    if p["decay"] == "exp":
        return 10.0 ** (np.log10(eps) / (r - 0.5) * (i - 1))
    s = np.full(R, 1e-3 * eps)
    s[:r] = 1.0
    return s


def learned_matrix(p: dict, device="cpu") -> torch.Tensor:
    """FP32 m x n = U diag(learned_spectrum(p)) V^T (Haar factors by
    Cholesky-QR, see ``haar_cholqr2``)."""
    return planted(p["m"], p["n"], learned_spectrum(p), p["seed"], torch.float32, 0.0, device, factor=haar_cholqr2)
