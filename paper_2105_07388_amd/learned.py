"""Learned sketch-width policy: labels, training and evaluation.

Algorithm 1 needs the sketch width up front; when it is too small the
estimate saturates at r1 and the paper reruns with r1 doubled, appending to
the sketches (Sec. 5).  Sec. 7 asks whether the first run could suggest the
right width instead.  This module trains the library's small network (35 ->
64 -> 64 -> 1, FP32, forward / gradient / Adam kernels in librankest) to do
that from a 32-column pilot sketch, and compares the resulting adaptive runs
(re_rank_adaptive with the network) with plain doubling.  Everything that
touches a matrix runs in the HIP library; this file only prepares labels,
drives training and keeps the bookkeeping.

  python -m paper_2105_07388_amd.learned label --shard 0/4 --out shard0.npz   (x4: 10^4 recipes)
  python -m paper_2105_07388_amd.learned fit shard*.npz          (split 8000 / 1000 / 1000 by matrix)
  python -m paper_2105_07388_amd.learned evaluate                (the 1000 test matrices)

Defaults follow the learned form's configuration: 10^4 planted FP32 matrices,
m log-uniform in [4096, 65536], n = m / 4, poly / exp / step decay, ranks in
[10, 2000].
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import _binding as B
from . import inputs

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "data", "mlp_sketch_width.npz")
K0, L_RATIO, GRID = 32, 1.5, 8


def features(sigma: np.ndarray, m: int, n: int, eps: float) -> np.ndarray:
    """Network input: log10(s_i / s_1) of the first 32 pilot estimates (at
    least -8; missing ones -8), then log10 m, log10 n, log10 eps."""
    f = np.full(B.MLP_INPUTS, -8.0)
    s = np.asarray(sigma, dtype=np.float64)[:32]
    if s.size and s[0] > 0:
        q = s / s[0]
        with np.errstate(divide="ignore"):
            f[:s.size] = np.maximum(np.where(q > 0, np.log10(np.where(q > 0, q, 1.0)), -8.0), -8.0)
    f[32], f[33], f[34] = math.log10(m), math.log10(n), math.log10(eps)
    return f


def l_for(k: int, m: int) -> int:
    return int(min(max(int(math.floor(L_RATIO * k + 0.5)), k), m))


def converged(A, eps, k, seed, handle) -> bool:
    r, _, info = B.rank_estimate(A, eps, k=k, l=l_for(k, A.shape[0]), seed=seed, handle=handle)
    return not (info["flags"] & B.FLAG_NOT_CONVERGED)


def label(A, eps, seed, handle, kmax) -> int:
    """k*: the smallest multiple of 8 (>= 32) at which the plain estimator
    with this seed converges, by doubling then bisection on the grid
    (convergence is taken to be monotone in k; kmax when never)."""
    k = K0
    while k < kmax and not converged(A, eps, k, seed, handle):
        k = min(2 * k, kmax)
    if k == K0:
        return K0
    lo, hi = k // 2, k  # lo fails, hi converges (or is kmax)
    while hi - lo > GRID:
        mid = (lo + hi) // 2 // GRID * GRID
        if mid <= lo:
            break
        if converged(A, eps, mid, seed, handle):
            hi = mid
        else:
            lo = mid
    return hi


def build_dataset(params: list[dict], ids=None, seed: int = 7, eps_per_matrix: int = 2, log=print) -> dict:
    """Features and labels from runs of the plain estimator on the GPU: for
    each matrix its target eps and further random ones (drawn from the
    matrix id, so shards are reproducible on their own)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    h = B.Handle(dev)
    ids = list(range(len(params))) if ids is None else list(ids)
    X, y, meta = [], [], []
    t0 = time.time()
    for i, p in zip(ids, params):
        rng = np.random.default_rng([seed, i])
        A = inputs.learned_matrix(p, device=dev)
        m, n = A.shape
        kmax = min(n, 4096)
        epss = [p["eps"]] + [float(np.exp(rng.uniform(np.log(1e-6), np.log(1e-2)))) for _ in range(eps_per_matrix - 1)]
        for eps in epss:
            _, s, info = B.rank_estimate(A, eps, k=K0, l=l_for(K0, m), seed=seed + i, handle=h)
            ks = label(A, eps, seed + i, h, kmax)
            X.append(features(s, m, n, eps))
            y.append(math.log(ks))
            meta.append(dict(i=i, m=m, n=n, eps=eps, decay=p["decay"], k_star=ks,
                             pilot_converged=not (info["flags"] & B.FLAG_NOT_CONVERGED)))
        del A
        done = len(meta) // eps_per_matrix
        if done % 25 == 0 or done == len(params):
            log(f"[learned] labelled {done}/{len(params)} matrices, {time.time() - t0:.0f} s")
    return dict(X=np.array(X, dtype=np.float32), y=np.array(y, dtype=np.float32), meta=meta)


def train(X: np.ndarray, y: np.ndarray, *, steps: int = 4000, batch: int = 256, lr: float = 1e-3, seed: int = 0,
          Xval=None, yval=None, log=print) -> tuple[torch.Tensor, list]:
    """Adam on the mean squared error of log k*, all on the GPU through the
    library's kernels.  Returns (parameters, loss history)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    h = B.Handle(dev)
    p = torch.from_numpy(init_params(seed)).to(dev)
    mom = torch.zeros_like(p)
    var = torch.zeros_like(p)
    Xd = torch.from_numpy(np.ascontiguousarray(X)).to(dev)
    yd = torch.from_numpy(np.ascontiguousarray(y)).to(dev)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(seed)
    hist = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, X.shape[0], (min(batch, X.shape[0]),), generator=gen).to(dev)
        g, loss = B.mlp_loss_grad(p, Xd[idx], yd[idx], handle=h)
        B.mlp_adam(p, g, mom, var, step, lr, handle=h)
        if step % 500 == 0 or step == steps:
            rec = {"step": step, "train_mse": float(loss.item())}
            if Xval is not None:
                pv = B.mlp_forward(p, torch.from_numpy(Xval).to(dev), handle=h).cpu().numpy()
                rec["val_mse"] = float(np.mean((pv - yval) ** 2))
            hist.append(rec)
            log(f"[learned] {rec}")
    return p, hist


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero hidden biases, output bias log(64)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(B.MLP_PARAMS, dtype=np.float32)
    for lo, hi, fan_in in ((0, 2240, 35), (2304, 6400, 64), (6464, 6528, 64)):  # W1, W2, w3
        lim = math.sqrt(6.0 / fan_in)
        p[lo:hi] = rng.uniform(-lim, lim, hi - lo)
    p[6528] = math.log(64.0)
    return p


def simulate_rounds(kprop: np.ndarray, kstar: np.ndarray, kmax: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Rounds and final width of the learned driver given the labels: pilot,
    then the proposal, then doubling until the width reaches k*."""
    rounds = np.ones_like(kstar)
    kfin = np.full_like(kstar, K0)
    for i in range(len(kstar)):
        if kstar[i] <= K0:
            continue
        k, r = int(kprop[i]), 2
        while k < kstar[i] and k < kmax[i]:
            k, r = min(2 * k, int(kmax[i])), r + 1
        rounds[i], kfin[i] = r, k
    return rounds, kfin


def proposals(yhat: np.ndarray, delta: float, kmax: np.ndarray) -> np.ndarray:
    k = np.ceil(np.exp(np.minimum(yhat.astype(np.float64) + delta, 30.0))).astype(np.int64)
    k = (k + 7) // 8 * 8
    return np.minimum(np.maximum(k, 2 * K0), kmax)


def choose_delta(yhat: np.ndarray, kstar: np.ndarray, kmax: np.ndarray, max_overshoot: float = 1.5) -> float:
    """Margin on the validation set: the fewest mean rounds among the margins
    whose mean final width stays within max_overshoot times k* (a larger
    margin always saves rounds but pays for the extra columns)."""
    best = None
    for delta in np.arange(0.0, 1.01, 0.05):
        r, kf = simulate_rounds(proposals(yhat, delta, kmax), kstar, kmax)
        over = float(np.mean(kf / kstar))
        if over > max_overshoot and delta > 0.0:
            continue
        score = (float(np.mean(r)), over)
        if best is None or score < best[0]:
            best = (score, float(delta))
    return best[1]


def load_policy(path: str = DEFAULT_WEIGHTS, device=None) -> tuple[torch.Tensor, float]:
    """Trained parameters (device float32) and margin delta."""
    with np.load(path, allow_pickle=False) as z:
        p = torch.from_numpy(z["params"].astype(np.float32))
        delta = float(z["delta"])
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    return p.to(dev), delta


def acceptable(sigma: np.ndarray, r: int, eps: float) -> bool:
    """Sec. 1.1's goal for an estimate r^ of the eps-rank: not a severe
    underestimate, sigma_{r^+1} < 10 eps ||A||, and not a severe overestimate,
    sigma_{r^} > 0.1 eps ||A|| (sigma_0 = infinity; values past the planted
    ones are zero; ||A|| = sigma_1)."""
    s = np.asarray(sigma, dtype=np.float64)
    nxt = s[r] if r < s.size else 0.0
    cur = s[r - 1] if 1 <= r <= s.size else (np.inf if r == 0 else 0.0)
    return bool(nxt < 10.0 * eps * s[0] and cur > 0.1 * eps * s[0])


def agrees(p: dict, r: int) -> bool:
    """The acceptance rule of the evaluation: on step spectra (a clear gap at
    eps) the exact planted rank; on poly and exp spectra (no gap) Sec. 1.1's
    two conditions on the planted singular values."""
    sig = inputs.learned_spectrum(p)
    if p["decay"] == "step":
        return r == int(np.count_nonzero(sig > p["eps"] * sig[0]))
    return acceptable(sig, r, p["eps"])


def compare(params: list[dict], policy, delta: float, seed: int = 99, log=print) -> dict:
    """Doubling vs the learned policy on the same matrices and seeds: rounds,
    time (ms, synchronised around each call) and agreement of r^ (``agrees``:
    the exact planted rank on step spectra, Sec. 1.1's conditions on poly and
    exp spectra), also the plain equality with the planted eps-rank."""
    dev = torch.device("cuda", torch.cuda.current_device())
    h = B.Handle(dev)
    rows = []
    for i, p in enumerate(params):
        A = inputs.learned_matrix(p, device=dev)
        kmax = min(A.shape[1], 4096)
        rank_true = int(np.count_nonzero(inputs.learned_spectrum(p) > p["eps"]))
        res = {}
        for name, mlp in (("doubling", None), ("learned", policy)):
            B.rank_adaptive(A, p["eps"], k_max=kmax, mlp=mlp, delta=delta, seed=seed + i, handle=h)  # warm
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r, _, info = B.rank_adaptive(A, p["eps"], k_max=kmax, mlp=mlp, delta=delta, seed=seed + i, handle=h)
            torch.cuda.synchronize()
            res[name] = dict(r=r, ms=1e3 * (time.perf_counter() - t0), rounds=info["rounds"], k=info["k"],
                             kprop=info["k_proposed"])
        for name in res:
            res[name]["ok"] = agrees(p, res[name]["r"])
        rows.append(dict(m=p["m"], n=p["n"], decay=p["decay"], eps=p["eps"], rank=rank_true, **{
            f"{a}_{b}": v for a in res for b, v in res[a].items()}))
        del A
        if (i + 1) % 50 == 0 or i + 1 == len(params):
            log(f"[learned] compared {i + 1}/{len(params)} matrices")
    out = {"count": len(rows)}
    for name in ("doubling", "learned"):
        out[name] = {
            "mean_rounds": float(np.mean([r[f"{name}_rounds"] for r in rows])),
            "mean_ms": float(np.mean([r[f"{name}_ms"] for r in rows])),
            "total_ms": float(np.sum([r[f"{name}_ms"] for r in rows])),
            "agreement": float(np.mean([r[f"{name}_ok"] for r in rows])),
            "rank_equals_planted": float(np.mean([r[f"{name}_r"] == r["rank"] for r in rows])),
            "mean_k_final": float(np.mean([r[f"{name}_k"] for r in rows])),
        }
        for d in ("step", "poly", "exp"):
            sub = [r for r in rows if r["decay"] == d]
            if sub:
                out[name][d] = {"count": len(sub), "agreement": float(np.mean([r[f"{name}_ok"] for r in sub])),
                                "mean_rounds": float(np.mean([r[f"{name}_rounds"] for r in sub])),
                                "mean_ms": float(np.mean([r[f"{name}_ms"] for r in sub]))}
    out["same_rank_both"] = float(np.mean([r["doubling_r"] == r["learned_r"] for r in rows]))
    step = [r for r in rows if r["decay"] == "step"]
    out["step_same_rank"] = float(np.mean([r["doubling_r"] == r["learned_r"] == r["rank"] for r in step])) if step else None
    out["rows"] = rows
    log(f"[learned] compare: " + json.dumps({k: v for k, v in out.items() if k != "rows"}))
    return out


def _split(meta, frac_train=0.8, frac_val=0.1):
    """Split by matrix (never by sample): train / validation / test masks."""
    mi = np.array([r["i"] for r in meta])
    nmat = int(mi.max()) + 1 if len(mi) else 0
    ntr, nva = int(frac_train * nmat), int(frac_val * nmat)
    return mi < ntr, (mi >= ntr) & (mi < ntr + nva), mi >= ntr + nva


def fit(ds: dict, steps: int, out: str, extra: dict, log=print) -> dict:
    """Train on the training split, pick delta on validation, report the
    simulated rounds on the test split, save weights and summary."""
    tr, va, te = _split(ds["meta"])
    # the network is only consulted when the pilot did not converge
    used = ~np.array([r["pilot_converged"] for r in ds["meta"]])
    trn, van = tr & used, va & used
    p, hist = train(ds["X"][trn], ds["y"][trn], steps=steps, Xval=ds["X"][van], yval=ds["y"][van], log=log)
    dev = p.device
    kst = np.array([r["k_star"] for r in ds["meta"]])
    kmx = np.array([min(r["n"], 4096) for r in ds["meta"]])
    yv = B.mlp_forward(p, torch.from_numpy(ds["X"][van]).to(dev)).cpu().numpy()
    delta = choose_delta(yv, kst[van], kmx[van])
    yt = B.mlp_forward(p, torch.from_numpy(ds["X"][te]).to(dev)).cpu().numpy()
    r_l, k_l = simulate_rounds(proposals(yt, delta, kmx[te]), kst[te], kmx[te])
    r_d, k_d = simulate_rounds(np.minimum(2 * K0, kmx[te]), kst[te], kmx[te])
    summary = dict(extra, samples=int(len(ds["y"])), train=int(trn.sum()), val=int(van.sum()), test=int(te.sum()),
                   pilot_converged=float(1.0 - used.mean()), delta=delta, history=hist,
                   test_mse_network_used=float(np.mean((yt - ds["y"][te])[used[te]] ** 2)),
                   test_mean_rounds_learned_simulated=float(np.mean(r_l)),
                   test_mean_rounds_doubling_simulated=float(np.mean(r_d)),
                   test_mean_kfinal_over_kstar_learned=float(np.mean(k_l / kst[te])),
                   test_mean_kfinal_over_kstar_doubling=float(np.mean(k_d / kst[te])))
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.savez(out, params=p.cpu().numpy(), delta=np.float64(delta), summary=json.dumps(summary))
    log(f"[learned] saved {out}: " + json.dumps({k: v for k, v in summary.items() if k != "history"}))
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    lb = sub.add_parser("label", help="features and labels of one shard of the matrix recipes")
    lb.add_argument("--count", type=int, default=10000)
    lb.add_argument("--shard", default="0/1", help="i/N: recipes i, i+N, i+2N, ...")
    lb.add_argument("--m-lo", type=int, default=4096)
    lb.add_argument("--m-hi", type=int, default=65536)
    lb.add_argument("--r-cap", type=int, default=2000)
    lb.add_argument("--out", required=True)
    ft = sub.add_parser("fit", help="train on labelled shards")
    ft.add_argument("data", nargs="+")
    ft.add_argument("--steps", type=int, default=6000)
    ft.add_argument("--out", default=DEFAULT_WEIGHTS)
    e = sub.add_parser("evaluate", help="doubling vs learned on the test split (or on unseen recipes)")
    e.add_argument("--count", type=int, default=10000, help="recipes of the labelled set (test split: the last 10%%)")
    e.add_argument("--unseen", type=int, default=0, help="evaluate on this many recipes of another seed instead")
    e.add_argument("--limit", type=int, default=0, help="only the first LIMIT evaluation matrices")
    e.add_argument("--m-lo", type=int, default=4096)
    e.add_argument("--m-hi", type=int, default=65536)
    e.add_argument("--r-cap", type=int, default=2000)
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--report", default=None)
    a = ap.parse_args(argv)
    log = lambda s: print(s, file=sys.stderr, flush=True)  # noqa: E731
    if a.cmd == "label":
        i, nsh = (int(v) for v in a.shard.split("/"))
        params = inputs.learned_params(a.count, seed=1005, m_lo=a.m_lo, m_hi=a.m_hi, r_cap=a.r_cap)
        mine = list(range(i, a.count, nsh))
        ds = build_dataset([params[j] for j in mine], ids=mine, log=log)
        np.savez(a.out, X=ds["X"], y=ds["y"], meta=json.dumps(ds["meta"]),
                 recipe=json.dumps(dict(count=a.count, m_lo=a.m_lo, m_hi=a.m_hi, r_cap=a.r_cap)))
        log(f"[learned] wrote {a.out}: {len(ds['y'])} samples")
    elif a.cmd == "fit":
        X, y, meta, recipe = [], [], [], None
        for f in a.data:
            with np.load(f, allow_pickle=False) as z:
                X.append(z["X"])
                y.append(z["y"])
                meta += json.loads(str(z["meta"]))
                recipe = json.loads(str(z["recipe"]))
        ds = dict(X=np.concatenate(X), y=np.concatenate(y), meta=meta)
        fit(ds, a.steps, a.out, dict(recipe=recipe), log=log)
    else:
        policy, delta = load_policy(a.weights)
        if a.unseen:
            params = inputs.learned_params(a.unseen, seed=2005, m_lo=a.m_lo, m_hi=a.m_hi, r_cap=a.r_cap)
        else:  # the test split of the labelled recipes (matrices never trained or validated on)
            params = inputs.learned_params(a.count, seed=1005, m_lo=a.m_lo, m_hi=a.m_hi, r_cap=a.r_cap)
            params = params[int(0.9 * a.count):]
        if a.limit:
            params = params[:a.limit]
        out = compare(params, policy, delta, log=log)
        if a.report:
            with open(a.report, "w") as fh:
                json.dump(out, fh)
        print(json.dumps({k: v for k, v in out.items() if k != "rows"}), flush=True)


if __name__ == "__main__":
    main()
