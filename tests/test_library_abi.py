"""The C-ABI library loads and exports every entry point that include/rankest.h
declares (no GPU needed: nothing is called that touches a device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rankest.h")
LIB = os.path.join(ROOT, "paper_2105_07388_amd", "librankest.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(re_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(LIB):
        from paper_2105_07388_amd import build as b
        b.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ["re_create", "re_destroy", "re_rank_estimate", "re_sketch_x", "re_sketch_y",
                 "re_singular_values", "re_rank_count", "re_srht_select", "re_srht_signs", "re_gauss_fill"]:
        assert must in names


def test_every_declared_symbol_is_exported(so):
    missing = [n for n in declared_functions() if not hasattr(so, n)]
    assert not missing, missing


def test_host_only_entry_points(so):
    so.re_r1_from_k.restype = ctypes.c_int32
    assert [so.re_r1_from_k(k) for k in (32, 40, 96, 384, 512)] == [29, 36, 87, 349, 465]
    so.re_status_string.restype = ctypes.c_char_p
    assert so.re_status_string(0) == b"ok"
    assert b"non-finite" in so.re_status_string(-5)
    so.re_sketch_y_rows.restype = ctypes.c_int64
    so.re_sketch_y_rows.argtypes = [ctypes.c_int64]
    assert so.re_sketch_y_rows(65536) == 65536
    assert so.re_sketch_y_rows(1000) == 1024
    assert so.re_sketch_y_rows(100) == 128
    # invalid handle / arguments are rejected before any device work
    assert so.re_destroy(None) == 0
    assert so.re_create(None, None) == -1


def test_noalloc_limits_on_the_host(so):
    """The allocation-free singular values reject what does not fit their fixed
    scratch before any device work."""
    so.re_singular_values_noalloc_fits.restype = ctypes.c_int32
    so.re_singular_values_noalloc_fits.argtypes = [ctypes.c_int64, ctypes.c_int64]
    fits = so.re_singular_values_noalloc_fits
    assert fits(576, 384) == 1 and fits(768, 512) == 1 and fits(144, 96) == 1 and fits(60, 40) == 1
    assert fits(4096, 1024) == 0 and fits(100, 200) == 0 and fits(10, 0) == 0
    f = so.re_singular_values_noalloc
    f.restype = ctypes.c_int32
    f.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                  ctypes.c_void_p]
    fake = ctypes.c_void_p(4096)  # never dereferenced: both calls are rejected on the host
    assert f(None, fake, 4096, 1024, 1.0, fake) == -7
    assert f(None, None, 576, 384, 1.0, fake) == -1
    so.re_status_string.restype = ctypes.c_char_p
    assert b"scratch" in so.re_status_string(-7)


def test_no_oracle_in_product():
    """The product library and package never reference the oracle."""
    pkg = os.path.join(ROOT, "paper_2105_07388_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "liboracle" not in txt, f
    with open(LIB, "rb") as fh:
        assert b"liboracle" not in fh.read()


def test_gap_rank_matches_oracle(so, orc):
    """re_gap_rank is host-only: checked against the oracle's definition here."""
    import math

    import numpy as np
    f = so.re_gap_rank
    f.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                  ctypes.POINTER(ctypes.c_double)]
    f.restype = ctypes.c_int32
    rng = np.random.default_rng(3)
    cases = [np.array([1.0] * 20 + [1e-8] * 20), np.array([3.0, 1.0, 0.5, 0.0, 0.0]), np.zeros(4), np.array([2.0]),
             np.sort(rng.random(50))[::-1].copy(), np.array([1.0, 1.0, 1.0])]
    for s in cases:
        for r1 in (0, 1, 2, 5, len(s), len(s) + 3):
            r = ctypes.c_int32(-1)
            q = ctypes.c_double(-1.0)
            assert f(s.ctypes.data_as(ctypes.c_void_p), len(s), r1, ctypes.byref(r), ctypes.byref(q)) == 0
            want_r, want_q = orc.gap.gap_rank(s, r1)
            assert r.value == want_r
            assert (math.isinf(q.value) and math.isinf(want_q)) or abs(q.value - want_q) <= 1e-15 * abs(want_q)
    r = ctypes.c_int32(0)
    assert f(None, 3, 2, ctypes.byref(r), None) == -1
