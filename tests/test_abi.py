"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and
validates arguments before touching the GPU (no device work is started)."""
import ctypes
import os
import re

import pytest

import paper_2002_06960_amd as pkg
from paper_2002_06960_amd import randutv as rb
from oracle import randutv_oracle as ro

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "randutv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(randutv_\w+)\s*\(", text)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = pkg.load()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n
    # the binding wraps exactly the declared entry points
    assert sorted(rb.SIGNATURES) == names


def test_strerror_codes():
    assert pkg.randutv_strerror(0) == "success"
    assert "converge" in pkg.randutv_strerror(4)
    assert "invalid" in pkg.randutv_strerror(-3)
    assert pkg.randutv_strerror(1).startswith("HIP")
    assert "rank deficient" in pkg.randutv_strerror(rb.ERR_RANK)
    for code in range(1, rb.ERR_RANK + 1):  # every positive code has its own message
        assert pkg.randutv_strerror(code) != "unknown error"


def test_argument_validation_without_device_work():
    lib = pkg.load()
    P = ctypes.c_void_p(0x1000)  # never dereferenced: every call below fails validation first
    f = lib.randutv_factor
    assert f(-1, 1, P, 1, 1, 0, 0, None, P, None) == -1
    assert f(3, 5, P, 3, 1, 0, 0, None, P, None) == -2       # n > m
    assert f(5, 3, None, 5, 1, 0, 0, None, P, None) == -3
    assert f(5, 3, P, 4, 1, 0, 0, None, P, None) == -4       # lda < m
    assert f(5, 3, P, 5, 0, 0, 0, None, P, None) == -5       # b < 1
    assert f(5, 3, P, 5, 2, -1, 0, None, P, None) == -6      # q < 0
    assert f(5, 3, P, 5, 2, 0, 0, None, None, None) == -9    # T NULL
    assert f(5, 3, P, 6, 2, 0, 0, None, P, None) == -9       # T aliases A with lda != m
    assert f(5, 3, P, 5, 2, 0, 0, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x2000), None) == -8
    assert f(0, 0, None, 1, 1, 0, 0, None, None, None) == 0  # empty: no-op
    assert f(5, 0, None, 5, 1, 0, 0, None, None, None) == 0
    t = lib.randutv_truncate
    assert t(4, 3, 4, P, P, P, P) == -3                       # k > n
    assert t(4, 3, 2, None, P, P, P) == -4
    g = lib.randutv_dgemm
    assert g(b"X", b"N", 1, 1, 1, 1.0, P, 1, P, 1, 0.0, P, 1) == -1
    assert g(b"N", b"N", 4, 4, 4, 1.0, P, 3, P, 4, 0.0, P, 4) == -8
    assert g(b"T", b"N", 4, 4, 6, 1.0, P, 5, P, 6, 0.0, P, 4) == -8   # lda < K for op T
    assert g(b"N", b"N", 4, 4, 4, 1.0, P, 4, P, 4, 0.0, P, 3) == -13
    assert lib.randutv_geqrf(3, 4, P, 3, P) == -2              # k > m
    assert lib.randutv_gesvj(-1, P, 1, P, P, P, None) == -1
    assert lib.randutv_gesvj(300, P, 300, P, P, P, None) == rb.ERR_TOO_LARGE
    assert lib.randutv_sketch(0, 0, -1, 3, P, 1) == -3
    assert lib.randutv_sketch(0, 0, 4, 3, P, 2) == -6
    assert lib.randutv_larft(5, 6, P, 5, P, P, 6) == -2
    fx = lib.randutv_factor_ex
    assert fx(5, 3, P, 5, 2, 0, 0, None, P, None, 8) == -11      # unknown sketch precision
    assert fx(5, 3, P, 4, 2, 0, 0, None, P, None, 32) == -4
    g32 = lib.randutv_gemm_f32
    assert g32(b"N", b"Q", 1, 1, 1, 1.0, P, 1, P, 1, 0.0, P, 1) == -2
    assert g32(b"N", b"N", 4, 4, 4, 1.0, P, 4, P, 4, 0.0, P, 3) == -13
    tg_ = lib.randutv_truncate_grad
    assert tg_(-1, 3, P, 5, 2, 0, 0, P, 5, P, 5) == -1
    assert tg_(4, 5, P, 4, 2, 0, 0, P, 4, P, 4) == -2                  # n > m
    assert tg_(5, 3, None, 5, 2, 0, 0, P, 5, P, 5) == -3
    assert tg_(5, 3, P, 4, 2, 0, 0, P, 5, P, 5) == -4
    assert tg_(5, 3, P, 5, 0, 0, 0, P, 5, P, 5) == -5
    assert tg_(5, 3, P, 5, 2, -1, 0, P, 5, P, 5) == -6
    assert tg_(5, 3, P, 5, 2, 65, 0, P, 5, P, 5) == -6                 # q above the kept products
    assert tg_(5, 3, P, 5, 2, 0, 0, None, 5, P, 5) == -8
    assert tg_(5, 3, P, 5, 2, 0, 0, P, 4, ctypes.c_void_p(0x2000), 5) == -9
    assert tg_(5, 3, P, 5, 2, 0, 0, ctypes.c_void_p(0x2000), 5, P, 5) == -10   # Abar aliases A
    assert tg_(5, 3, P, 5, 2, 0, 0, ctypes.c_void_p(0x2000), 5, ctypes.c_void_p(0x3000), 4) == -11
    assert tg_(600, 600, P, 600, 300, 0, 0, ctypes.c_void_p(0x2000), 600, ctypes.c_void_p(0x3000),
               600) == rb.ERR_TOO_LARGE
    assert tg_(0, 0, None, 1, 2, 0, 0, None, 1, None, 1) == 0
    fb = lib.randutv_truncate_first_block
    assert fb(-1, 3, P, 5, 2, 0, 0, P, 5) == -1
    assert fb(5, 3, P, 5, 2, 0, 0, P, 5) == -8                         # Ak aliases A
    assert fb(5, 3, P, 5, 2, 0, 0, ctypes.c_void_p(0x2000), 4) == -9
    assert fb(5, 3, P, 5, 2, -1, 0, ctypes.c_void_p(0x2000), 5) == -6
    hq = lib.randutv_hqrrp
    assert hq(-1, 3, P, 5, 2, 0, P, P) == -1
    assert hq(4, 5, P, 4, 2, 0, P, P) == -2
    assert hq(5, 3, None, 5, 2, 0, P, P) == -3
    assert hq(5, 3, P, 4, 2, 0, P, P) == -4
    assert hq(5, 3, P, 5, 0, 0, P, P) == -5
    assert hq(5, 3, P, 5, 2, 0, None, P) == -7
    assert hq(5, 3, P, 5, 2, 0, P, None) == -8
    assert hq(600, 600, P, 600, 300, 0, P, P) == rb.ERR_TOO_LARGE
    assert hq(40000, 40000, P, 40000, 64, 0, P, P) == rb.ERR_TOO_LARGE    # n > 32768
    assert lib.randutv_set_timing(3) == -1
    assert lib.randutv_set_timing(0) == 0
    g16 = lib.randutv_gemm_bf16
    assert g16(b"N", b"N", 4, 4, 4, 1.0, P, 4, P, 4, 0.0, P, 4, 2) == -14   # one or three terms
    assert g16(b"X", b"N", 4, 4, 4, 1.0, P, 4, P, 4, 0.0, P, 4, 3) == -1
    assert g16(b"N", b"N", 4, 4, 4, 1.0, P, 4, P, 4, 0.0, P, 3, 1) == -13


def test_b_above_kernel_limit_is_reported():
    lib = pkg.load()
    P = ctypes.c_void_p(0x1000)
    assert lib.randutv_factor(600, 600, P, 600, 300, 0, 0, None, P, None) == rb.ERR_TOO_LARGE


def test_no_device_is_a_hip_error_not_a_crash():
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a GPU is visible: this path is for hosts without one")
    lib = pkg.load()
    P = ctypes.c_void_p(0x1000)
    assert lib.randutv_factor(8, 8, P, 8, 4, 1, 0, None, P, None) == rb.ERR_HIP


def test_flop_count_matches_oracle_definition():
    for (m, n, q) in ((12000, 12000, 2), (16000, 8000, 2), (512, 512, 1)):
        for bu in (True, False):
            for bv in (True, False):
                assert abs(pkg.flops_std(m, n, q, bu, bv) / ro.flops_std(m, n, q, bu, bv) - 1) < 1e-14
