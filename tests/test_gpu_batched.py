"""GPU tests of the batched form (many blocks in one graph launch).

Every block of a batched call must give exactly (bit for bit) what a
single-matrix call with the same seed gives, whatever tile shape the autotuner
picks, and must agree with the CPU oracle to the FP32 Gaussian tolerance
|d sigma_i| <= 8 2^-24 sqrt(n) sigma_1 (FP32 contraction of n terms, the
sketch entries rounded to FP32 on both sides).  Ranks agree except for
estimates that lie within that tolerance of eps sigma_1.
"""
import math
import os

import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_
from paper_2105_07388_amd import inputs

pytestmark = pytest.mark.gpu

DEV = "cuda"
K, L = 96, 144


def _single(A, eps, seed, h, k=K, l=L):
    return re_.rank_estimate(A, eps, k=k, l=l, x="gaussian", y="gaussian", seed=seed, handle=h)


def _oracle_check(orc, A, eps, seed, r, s, k=K, l=L):
    An = A.cpu().numpy()
    r_o, s_o, r1_o, fl_o, _ = orc.rank_estimate(An, eps, orc.GAUSSIAN, orc.GAUSSIAN, k=k, l=l, seed=seed)
    tol = 8 * 2.0**-24 * math.sqrt(A.shape[1]) * s_o[0]
    assert np.all(np.abs(s - s_o) <= tol), (np.abs(s - s_o).max() / s_o[0], A.shape)
    band = int(np.count_nonzero(np.abs(s_o[:r1_o] - eps * s_o[0]) <= 2 * tol))
    assert abs(r - r_o) <= band, (r, r_o, band)
    return r_o


def test_batched_equals_single_calls(orc):
    buf, views, params = inputs.kernel_blocks(10, seed=11, device=DEV, size_lo=150, size_hi=900)
    h = re_.Handle()
    for seed in (3, 4):  # the second call replays the captured graph with a new seed
        r, s, fl = re_.rank_estimate_batched(views, 1e-6, k=K, l=L, seed=seed, handle=h)
        for b, A in enumerate(views):
            r1, s1, info = _single(A, 1e-6, seed, h)
            assert r[b] == r1 and fl[b] == info["flags"], (b, r[b], r1)
            assert np.array_equal(s[b], s1), (b, np.abs(s[b] - s1).max())
    # a smaller batch of other shapes re-captures
    r, s, fl = re_.rank_estimate_batched(views[3:6], 1e-6, k=K, l=L, seed=9, handle=h)
    for b, A in enumerate(views[3:6]):
        r1, s1, info = _single(A, 1e-6, 9, h)
        assert r[b] == r1 and np.array_equal(s[b], s1)
    for b in (0, 4):
        _oracle_check(orc, views[b], 1e-6, 3, *re_.rank_estimate_batched([views[b]], 1e-6, k=K, l=L, seed=3,
                                                                          handle=h)[:2])


def test_batched_oracle_parity_and_ranks(orc):
    buf, views, params = inputs.kernel_blocks(6, seed=21, device=DEV, size_lo=200, size_hi=1200)
    r, s, fl = re_.rank_estimate_batched(views, 1e-6, k=K, l=L, seed=17)
    for b, A in enumerate(views):
        r_o = _oracle_check(orc, A, 1e-6, 17, r[b], s[b])
        assert 3 <= r_o < re_.r1_from_k(K)


@pytest.mark.parametrize("tile", ["4:1:16:2", "4:1:32:1", "8:1:16:1", "8:1:32:3", "4:2:16:2", "8:2:16:1"])
def test_batched_tile_shapes_agree(tile, monkeypatch):
    buf, views, params = inputs.kernel_blocks(7, seed=31, device=DEV, size_lo=150, size_hi=700)
    ref = re_.rank_estimate_batched(views, 1e-6, k=K, l=L, seed=2, handle=re_.Handle())
    monkeypatch.setenv("RANKEST_BATCH_TILE", tile)
    got = re_.rank_estimate_batched(views, 1e-6, k=K, l=L, seed=2, handle=re_.Handle())
    assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1]) and np.array_equal(ref[2], got[2])


@pytest.mark.parametrize("k,l", [(8, 12), (33, 50), (64, 96), (100, 120), (112, 128)])
def test_batched_other_sketch_sizes(k, l):
    buf, views, params = inputs.kernel_blocks(5, seed=41 + k, device=DEV, size_lo=max(l, 200), size_hi=640)
    views.append(torch.randn(l, k, device=DEV))        # the smallest legal block
    views.append(torch.randn(l + 7, 3 * k, device=DEV)[:, 5:5 + k + 1])  # a strided view
    h = re_.Handle()
    r, s, fl = re_.rank_estimate_batched(views, 1e-5, k=k, l=l, seed=8, handle=h)
    for b, A in enumerate(views):
        r1, s1, info = _single(A, 1e-5, 8, h, k, l)
        assert r[b] == r1 and np.array_equal(s[b], s1), b


def test_batched_autotune_cache(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("RANKEST_AUTOTUNE_CACHE", str(path))
    buf, views, params = inputs.kernel_blocks(4, seed=51, device=DEV, size_lo=150, size_hi=400)
    a = re_.rank_estimate_batched(views, 1e-6, k=K, l=L, seed=1, handle=re_.Handle())
    text = path.read_text()
    assert "gfx950:f32:k96:" in text and text.strip().startswith("{")
    b = re_.rank_estimate_batched(views, 1e-6, k=K, l=L, seed=1, handle=re_.Handle())  # read back from the file
    assert np.array_equal(a[1], b[1])


def test_batched_errors():
    A = torch.randn(200, 120, device=DEV)
    assert re_.rank_estimate_batched([], 1e-6, k=K, l=L)[0].shape == (0,)
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_estimate_batched([A, torch.randn(100, 120, device=DEV)], 1e-6, k=K, l=L)  # m < l
    assert ei.value.status == -1
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_estimate_batched([A], 1e-6, k=K, l=80)  # l < k
    assert ei.value.status == -1
    with pytest.raises(ValueError):
        re_.rank_estimate_batched([A.double()], 1e-6, k=K, l=L)
    with pytest.raises(re_.RankEstError) as ei:  # an l x k sketch beyond one workgroup's LDS
        re_.rank_estimate_batched([torch.randn(300, 200, device=DEV)], 1e-6, k=200, l=256)
    assert ei.value.status == -2
    # SRHT sketches and low precision are not offered by the batched form
    import ctypes as C
    tab = re_.make_blocks([A])
    for sk in (re_._binding.make_sketch(K, L, "srht", "gaussian"), re_._binding.make_sketch(K, L, "gaussian", "gaussian", "bf16")):
        r = np.zeros(1, np.int32)
        s = np.zeros(K)
        st = re_.lib().re_rank_estimate_batched(re_.default_handle().bind(), C.cast(tab, C.c_void_p), 1, 1, 1e-6,
                                                C.byref(sk), 0, r.ctypes.data_as(C.c_void_p),
                                                s.ctypes.data_as(C.c_void_p), None)
        assert st == -2
    # a non-finite block fails the call, the others still get their ranks
    B = A.clone()
    B[7, 9] = float("inf")
    with pytest.raises(re_.RankEstError) as ei:
        re_.rank_estimate_batched([A, B], 1e-6, k=K, l=L)
    assert ei.value.status == -5


def test_long_single_call_split_over_m(orc):
    # m = 20000: the single call's Y B runs 40 groups of 512 rows on separate
    # workgroups and adds their partials in order; the same matrix as a
    # one-block batch adds the groups one after another.  Same bits, and the
    # oracle's FP64 estimate within the FP32 bound.
    A = inputs.planted(20000, 500, np.geomspace(1.0, 1e-7, 200), 41, torch.float32).to(DEV)
    h = re_.Handle()
    r1, s1, info = _single(A, 1e-5, 6, h)
    r, s, fl = re_.rank_estimate_batched([A], 1e-5, k=K, l=L, seed=6, handle=h)
    assert r[0] == r1 and np.array_equal(s[0], s1)
    _oracle_check(orc, A, 1e-5, 6, r1, s1)


def test_wide_y_single_call_unsplit(orc):
    """k = 8 and l = 300 on m = 20000: the split over m would need partials of
    40 x 300 x 8 doubles, more than B itself, so the single call keeps one
    workgroup per block (the unsplit launch): the same bits as the one-block
    batch, and the oracle's estimate within the FP32 bound."""
    A = inputs.planted(20000, 500, np.geomspace(1.0, 1e-7, 200), 43, torch.float32).to(DEV)
    h = re_.Handle()
    r1, s1, info = re_.rank_estimate(A, 1e-5, k=8, l=300, seed=9, handle=h)
    r, s, fl = re_.rank_estimate_batched([A], 1e-5, k=8, l=300, seed=9, handle=h)
    assert r[0] == r1 and np.array_equal(s[0], s1)
    ro, so, r1o, flo, _ = orc.rank_estimate_gemm(A.cpu().numpy(), 1e-5, orc.GAUSSIAN, orc.GAUSSIAN, k=8, l=300,
                                                 seed=9)
    assert np.max(np.abs(s1 - so)) <= 8 * 2.0**-24 * math.sqrt(500) * so[0]


def test_batched_full_size_sampled(orc):
    """4096 kernel blocks (m, n in [256, 4096], ~79 GB of FP32) in one call; the
    oracle checks a stratified sample of 64 blocks (evenly spaced in the order of
    block size, from the smallest to the largest), and a few of them are checked
    bit for bit against single calls.  The oracle's Gaussian products run as FP64
    library products on master draws of X (4096 x 96) and Y (144 x 4096), whose
    leading blocks are each block's sketch."""
    free, _ = torch.cuda.mem_get_info()
    if free < 100 * 2**30:
        pytest.skip("needs ~100 GB of free device memory")
    buf, views, params = inputs.kernel_blocks(4096, device=DEV)
    h = re_.Handle()
    r, s, fl = re_.rank_estimate_batched(views, 1e-6, k=K, l=L, seed=77, handle=h)
    sizes = np.array([p["m"] * p["n"] for p in params])
    order = np.argsort(sizes, kind="stable")
    picks = np.unique(np.round(np.linspace(0, len(order) - 1, 64)).astype(int))
    sample = [int(order[i]) for i in picks]
    assert len(sample) == 64 and sample[-1] == int(order[-1]) and sample[0] == int(order[0])
    for b in (sample[0], sample[1], sample[32], sample[-1]):
        r1, s1, info = _single(views[b], 1e-6, 77, h)
        assert r[b] == r1 and np.array_equal(s[b], s1)
    X = orc.gauss_matrix(77, 4096, K, orc.STREAM_XGAUSS, orc.FMT_F32)
    Y = orc.gauss_matrix(77, L, 4096, orc.STREAM_YGAUSS, orc.FMT_F32, swap=True)
    worst = 0.0
    for b in sample:
        An = views[b].cpu().numpy()
        r_o, s_o, r1_o, fl_o, _ = orc.rank_estimate_gemm(An, 1e-6, orc.GAUSSIAN, orc.GAUSSIAN, k=K, l=L, seed=77,
                                                         X=X, Y=Y)
        tol = 8 * 2.0**-24 * math.sqrt(An.shape[1]) * s_o[0]
        err = float(np.max(np.abs(s[b] - s_o)))
        worst = max(worst, err / tol)
        assert err <= tol, (b, An.shape, err / s_o[0])
        band = int(np.count_nonzero(np.abs(s_o[:r1_o] - 1e-6 * s_o[0]) <= 2 * tol))
        assert abs(int(r[b]) - r_o) <= band, (b, int(r[b]), r_o, band)
    print(f"batched full size: 64 stratified blocks, worst |d sigma| / tolerance {worst:.3g}")
    assert 3 <= int(np.min(r)) and int(np.max(r)) < re_.r1_from_k(K)
    del buf, views
