"""The library's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (GPU code built as usual), driven through the C ABI by
tests/host_sanitizer_driver.cpp.  On a machine without a GPU the driver runs
the argument checks and host-only entry points; on the GPU it also runs the
estimate in each form and the forced error paths.  The CPU test rebuilds the
executable when a source is newer; the GPU test runs the executable built
beforehand (paper_2105_07388_amd.build.build_host_sanitized, also run by
__graft_entry__.build())."""
import glob
import os
import subprocess

import pytest

from paper_2105_07388_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _stale() -> bool:
    if not os.path.exists(B.SAN_BIN):
        return True
    t = os.path.getmtime(B.SAN_BIN)
    srcs = glob.glob(os.path.join(B.CSRC, "*")) + [os.path.join(B.INCLUDE, "rankest.h"), B.SAN_DRIVER]
    return any(os.path.getmtime(s) > t for s in srcs)


def _run(env_extra):
    env = dict(os.environ)
    env.update(env_extra)
    return subprocess.run([B.SAN_BIN], capture_output=True, text=True, timeout=300, env=env, cwd=ROOT)


def test_host_code_under_sanitizers_cpu_paths():
    if _stale():
        B.build_host_sanitized()
    # hide any GPU: the host-only paths, with leak detection on
    r = _run({"HIP_VISIBLE_DEVICES": "-1", "ASAN_OPTIONS": "detect_leaks=1"})
    print(r.stdout, r.stderr)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "host sanitizer driver ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


@pytest.mark.gpu
def test_host_code_under_sanitizers_gpu_paths():
    if not os.path.exists(B.SAN_BIN):
        pytest.skip("the sanitizer build is missing: run paper_2105_07388_amd.build.build_host_sanitized() first")
    # the HIP runtime keeps allocations until exit, so leak detection stays off here
    r = _run({"ASAN_OPTIONS": "detect_leaks=0"})
    print(r.stdout, r.stderr[-4000:])
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "GPU paths run on device 0" in r.stdout
    assert "host sanitizer driver ok" in r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
