"""The allocation-free singular values (re_singular_values_noalloc, fixed
per-GPU scratch) against re_singular_values on the same sketches: two calls in
a row on one GPU, the second smaller than the first, so the second runs on the
scratch the first left behind.  Both entry points run the same kernels on the
same input, so the results agree bit for bit (within the FP64 parity bar of
1e-10 sigma_1 at the least)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _sketch(l, k, seed):
    g = torch.Generator().manual_seed(seed)
    U, _ = torch.linalg.qr(torch.randn(l, k, generator=g, dtype=torch.float64))
    V, _ = torch.linalg.qr(torch.randn(k, k, generator=g, dtype=torch.float64))
    s = 10.0 ** (-torch.arange(k, dtype=torch.float64) / 40.0)
    return ((U * s) @ V.T).contiguous()


def _noalloc(Cd, scale):
    l, k = Cd.shape
    sig = torch.full((k,), float("nan"), dtype=torch.float64, device=DEV)
    lib = re_.lib()
    st = torch.cuda.current_stream().cuda_stream
    rc = lib.re_singular_values_noalloc(ctypes.c_void_p(st), ctypes.c_void_p(Cd.data_ptr()), l, k, float(scale),
                                        ctypes.c_void_p(sig.data_ptr()))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return sig.cpu().numpy()


@pytest.mark.parametrize("shapes", [((576, 384), (144, 96)), ((768, 512), (60, 40))])
def test_noalloc_matches_singular_values(shapes):
    for i, (l, k) in enumerate(shapes):
        print(f"noalloc case {l} x {k}", flush=True)
        C = _sketch(l, k, 100 * l + k + i)
        Cd = C.to(DEV)
        scale = 1.0 / np.sqrt(k * l)
        got = _noalloc(Cd, scale)
        want = re_.singular_values(Cd, scale).cpu().numpy()
        assert np.all(np.isfinite(got))
        assert np.abs(got - want).max() <= 1e-10 * want[0]
        assert np.array_equal(got, want)
        # and both match the exact singular values of the input
        ref = torch.linalg.svdvals(C).numpy() * scale
        assert np.abs(got - ref).max() <= 1e-12 * ref[0]


def test_noalloc_wrapper_and_limit():
    C = _sketch(130, 100, 5).to(DEV)
    sig = torch.empty(100, dtype=torch.float64, device=DEV)
    re_.singular_values_noalloc(C, sig, 0.5)
    torch.cuda.synchronize()
    assert np.array_equal(sig.cpu().numpy(), re_.singular_values(C, 0.5).cpu().numpy())
    big = torch.zeros(4096, 1024, dtype=torch.float64, device=DEV)
    with pytest.raises(re_.RankEstError) as ei:
        re_.singular_values_noalloc(big, torch.empty(1024, dtype=torch.float64, device=DEV))
    assert ei.value.status == -7  # RE_ERR_SCRATCH_LIMIT
