"""Error paths forced from the host (every kernel still exits normally):
a cap on the handle's workspace stands in for a failed allocation
(RE_ERR_NO_MEMORY), a negative barrier-poll limit makes the multi-workgroup
small SVD give up (RE_ERR_NO_CONVERGENCE), and a forced BF16 contraction whose
error floor phi_f = (u / sqrt 3) ||A||_F (1 / sqrt k + 1 / sqrt m) exceeds
eps sigma_1 / 4 is flagged (the acceptance test the AUTO precision applies).
After each error the same handle is reset and must give the reference
result."""
import numpy as np
import pytest
import torch

import paper_2105_07388_amd as re_
from paper_2105_07388_amd import _binding as B
from paper_2105_07388_amd import inputs

pytestmark = pytest.mark.gpu


def _matrix(m, n, seed, dtype=torch.float32):
    s = np.geomspace(1.0, 1e-6, min(m, n))
    return inputs.planted(m, n, s, seed, dtype, 0.0, "cuda")


def test_workspace_cap_reports_no_memory_and_the_handle_recovers():
    A = _matrix(2000, 1000, 11)
    ref = re_.rank_estimate(A, 1e-3, k=64, l=96, seed=5, handle=re_.Handle())
    h = re_.Handle()
    h.set_limits(max_workspace_bytes=4096)
    with pytest.raises(B.RankEstError) as ei:
        re_.rank_estimate(A, 1e-3, k=64, l=96, seed=5, handle=h)
    assert ei.value.status == B.RE_ERR_NO_MEMORY
    h.set_limits(max_workspace_bytes=0)
    r, s, info = re_.rank_estimate(A, 1e-3, k=64, l=96, seed=5, handle=h)
    assert r == ref[0] and np.array_equal(s, ref[1])


def test_workspace_cap_above_the_need_changes_nothing():
    A = _matrix(1500, 700, 12)
    ref = re_.rank_estimate(A, 1e-3, k=48, l=72, seed=2, handle=re_.Handle())
    h = re_.Handle()
    h.set_limits(max_workspace_bytes=1 << 30)
    r, s, _ = re_.rank_estimate(A, 1e-3, k=48, l=72, seed=2, handle=h)
    assert r == ref[0] and np.array_equal(s, ref[1])


def test_negative_cap_is_rejected():
    with pytest.raises(B.RankEstError) as ei:
        re_.Handle().set_limits(max_workspace_bytes=-1)
    assert ei.value.status == B.RE_ERR_INVALID_ARG


@pytest.mark.parametrize("l,k", [(576, 384), (300, 200)])
def test_forced_barrier_timeout_reports_no_convergence(l, k):
    """Sketches too large for one workgroup's LDS take the multi-workgroup
    bidiagonalisation; with barrier_polls < 0 its first grid barrier gives up."""
    g = torch.Generator().manual_seed(l + k)
    Cm = torch.randn(l, k, generator=g, dtype=torch.float64).cuda()
    ref = re_.singular_values(Cm, handle=re_.Handle()).cpu().numpy()
    h = re_.Handle()
    h.set_limits(barrier_polls=-1)
    with pytest.raises(B.RankEstError) as ei:
        re_.singular_values(Cm, handle=h)
        torch.cuda.synchronize()
    assert ei.value.status == B.RE_ERR_NO_CONVERGENCE
    h.set_limits(barrier_polls=0)
    s = re_.singular_values(Cm, handle=h).cpu().numpy()
    assert np.array_equal(s, ref)
    exact = np.linalg.svd(Cm.cpu().numpy(), compute_uv=False)
    assert np.max(np.abs(s - exact)) <= 1e-12 * exact[0]


def test_forced_barrier_timeout_through_the_estimate():
    A = _matrix(2000, 1000, 13)
    h = re_.Handle()
    h.set_limits(barrier_polls=-1)
    with pytest.raises(B.RankEstError) as ei:
        re_.rank_estimate(A, 1e-3, k=384, l=576, x="srht", y="srht", seed=3, handle=h)
    assert ei.value.status == B.RE_ERR_NO_CONVERGENCE
    h.set_limits(barrier_polls=0)
    r, s, _ = re_.rank_estimate(A, 1e-3, k=384, l=576, x="srht", y="srht", seed=3, handle=h)
    r0, s0, _ = re_.rank_estimate(A, 1e-3, k=384, l=576, x="srht", y="srht", seed=3, handle=re_.Handle())
    assert r == r0 and np.array_equal(s, s0)


def _phi(A, k, m, unit):
    return unit / np.sqrt(3.0) * float(A.double().norm()) * (1.0 / np.sqrt(k) + 1.0 / np.sqrt(m))


def test_forced_bf16_below_its_floor_is_flagged():
    m, n, k, l = 4096, 2048, 64, 96
    A = _matrix(m, n, 14)
    phi = _phi(A, k, m, 2.0**-8)
    # eps large enough for BF16's floor: no flag; small enough: flagged
    eps_ok, eps_low = 40.0 * phi, 0.4 * phi  # sigma_1 = 1 for the planted spectrum
    _, s, info = re_.rank_estimate(A, eps_ok, k=k, l=l, precision="bf16", seed=9)
    assert info["flags"] & re_.FLAG_USED_BF16
    assert phi <= eps_ok * s[0] / 4.0
    assert not info["flags"] & re_.FLAG_PREC_BELOW_FLOOR
    _, s, info = re_.rank_estimate(A, eps_low, k=k, l=l, precision="bf16", seed=9)
    assert info["flags"] & re_.FLAG_USED_BF16
    assert phi > eps_low * s[0] / 4.0
    assert info["flags"] & re_.FLAG_PREC_BELOW_FLOOR
    # the native form never sets it
    _, _, info = re_.rank_estimate(A, eps_low, k=k, l=l, seed=9)
    assert not info["flags"] & re_.FLAG_PREC_BELOW_FLOOR


def test_auto_below_every_floor_falls_back_without_the_forced_flag():
    m, n, k, l = 4096, 2048, 64, 96
    A = _matrix(m, n, 15)
    eps = 0.1 * _phi(A, k, m, 2.0**-11)  # below FP16's floor too: AUTO ends in FP32
    _, _, info = re_.rank_estimate(A, eps, k=k, l=l, precision="auto", seed=4)
    assert info["flags"] & re_.FLAG_PREC_FALLBACK
    assert not info["flags"] & (re_.FLAG_USED_BF16 | re_.FLAG_USED_FP16 | re_.FLAG_PREC_BELOW_FLOOR)


def test_small_svd_in_a_second_process_while_this_one_holds_the_device():
    """A process that has launched the multi-workgroup bidiagonalisation keeps
    the device's cooperative-launch resource while it lives; another process's
    call must still work (it falls back to a plain launch) and give the same
    values."""
    import json
    import os
    import subprocess
    import sys
    g = torch.Generator().manual_seed(7)
    Cm = torch.randn(576, 384, generator=g, dtype=torch.float64)
    s_here = re_.singular_values(Cm.cuda()).cpu().numpy()
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, json, torch; sys.path.insert(0, %r); import paper_2105_07388_amd as re_; "
            "g = torch.Generator().manual_seed(7); C = torch.randn(576, 384, generator=g, dtype=torch.float64); "
            "print(json.dumps(re_.singular_values(C.cuda()).cpu().tolist()))" % root)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    s_there = np.array(json.loads(r.stdout.strip().splitlines()[-1]))
    assert np.array_equal(s_there, s_here)


def test_estimates_in_flight_on_several_streams_match_one_at_a_time():
    """Handles on their own streams and host threads, their multi-workgroup
    small SVDs (576 x 384, pinned to the handles' XCDs, plain launches) running
    side by side: every estimate equals the same estimate run alone."""
    import threading
    A = _matrix(8192, 2048, 21)
    seeds = list(range(100, 112))
    ref = {}
    h0 = re_.Handle()
    for sd in seeds:
        ref[sd] = re_.rank_estimate(A, 1e-3, k=384, l=576, x="srht", y="srht", seed=sd, handle=h0)
    torch.cuda.synchronize()
    n = 4
    hs = [re_.Handle() for _ in range(n)]
    sts = [torch.cuda.Stream() for _ in range(n)]
    got = [dict() for _ in range(n)]
    errs = []

    def work(t):
        try:
            with torch.cuda.stream(sts[t]):
                for sd in seeds[t::n]:
                    got[t][sd] = re_.rank_estimate(A, 1e-3, k=384, l=576, x="srht", y="srht", seed=sd, handle=hs[t])
        except Exception as e:  # reported below, on the main thread
            errs.append(e)

    th = [threading.Thread(target=work, args=(t,)) for t in range(n)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    torch.cuda.synchronize()
    assert not errs, errs
    for t in range(n):
        for sd, (r, s, _) in got[t].items():
            assert r == ref[sd][0] and np.array_equal(s, ref[sd][1]), sd


def test_plain_svd_give_up_is_redone():
    """A plain-launched small SVD whose barrier gives up at its short poll limit
    (forced here: a limit below zero, set before the library loads, in a child
    process) is run again under the default limit: same estimate, and the flag
    says so."""
    import json
    import os
    import subprocess
    import sys
    A = _matrix(4096, 1024, 22)
    r0, s0, info0 = re_.rank_estimate(A, 1e-3, k=384, l=576, x="srht", y="srht", seed=8, handle=re_.Handle())
    assert not info0["flags"] & re_.FLAG_SVD_RELAUNCHED
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = ("import sys, json, numpy as np; sys.path.insert(0, %r); import paper_2105_07388_amd as re_; "
            "from paper_2105_07388_amd import inputs; "
            "s = np.geomspace(1.0, 1e-6, 1024); A = inputs.planted(4096, 1024, s, 22, __import__('torch').float32, 0.0, 'cuda'); "
            "r, sig, info = re_.rank_estimate(A, 1e-3, k=384, l=576, x='srht', y='srht', seed=8); "
            "print(json.dumps([r, sig.tolist(), info['flags']]))" % root)
    env = dict(os.environ, RANKEST_SVD_PLAIN_POLLS="-1")
    res = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0, res.stderr[-2000:]
    r1, s1, fl = json.loads(res.stdout.strip().splitlines()[-1])
    assert fl & re_.FLAG_SVD_RELAUNCHED
    assert r1 == r0 and np.array_equal(np.array(s1), s0)


def test_mixed_sketch_kinds_in_flight_match_one_at_a_time():
    """Four handles in flight, each running a different sketch pair (SRHT,
    BF16 Gaussian X with an SRHT Y, hashed DCT X with a subsampled DCT Y,
    subsampled DCT X), every multi-workgroup small SVD on a plain launch:
    each estimate equals the same estimate run alone, bit for bit."""
    import threading
    A = _matrix(8192, 4096, 23)
    kinds = [dict(x="srht", y="srht"), dict(x="gaussian", y="srht", precision="bf16"),
             dict(x="hrtt", y="srct"), dict(x="srct", y="srht")]
    eps = 1e-2
    ref = {}
    h0 = re_.Handle()
    for t, kw in enumerate(kinds):
        for sd in range(3):
            ref[(t, sd)] = re_.rank_estimate(A, eps, k=384, l=576, seed=50 + sd, handle=h0, **kw)
    torch.cuda.synchronize()
    hs = [re_.Handle() for _ in kinds]
    sts = [torch.cuda.Stream() for _ in kinds]
    got = {}
    errs = []

    def work(t):
        try:
            with torch.cuda.stream(sts[t]):
                for sd in range(3):
                    got[(t, sd)] = re_.rank_estimate(A, eps, k=384, l=576, seed=50 + sd, handle=hs[t], **kinds[t])
        except Exception as e:  # reported below, on the main thread
            errs.append(e)

    th = [threading.Thread(target=work, args=(t,)) for t in range(len(kinds))]
    for x in th:
        x.start()
    for x in th:
        x.join()
    torch.cuda.synchronize()
    assert not errs, errs
    for key, (r, s, info) in got.items():
        r0, s0, info0 = ref[key]
        assert r == r0 and np.array_equal(s, s0), key
        assert info["flags"] & ~re_.FLAG_SVD_RELAUNCHED == info0["flags"] & ~re_.FLAG_SVD_RELAUNCHED, key
