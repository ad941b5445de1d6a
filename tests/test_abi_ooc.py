"""CPU checks of the out-of-core entry point's argument validation (no device
work is started: every call below fails before the library touches the GPU)."""
import ctypes

import paper_2002_06960_amd as pkg
from paper_2002_06960_amd import randutv as rb

def test_ooc_argument_validation_without_device_work():
    lib = pkg.load()
    P, P2, P3 = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    o = lib.randutv_factor_ooc
    big = 1 << 30

    def call(m=5, n=3, A=P, lda=5, b=2, q=0, U=None, ldu=5, T=P2, ldt=5, V=None, ldv=3, budget=big,
             mode=2):
        return o(m, n, A, lda, b, q, 0, U, ldu, T, ldt, V, ldv, budget, mode, None)

    assert call(m=-1) == -1
    assert call(m=3, n=5) == -2                   # n > m
    assert call(A=None) == -3
    assert call(lda=4) == -4
    assert call(b=0) == -5
    assert call(q=-1) == -6
    assert call(U=P3, ldu=4) == -8
    assert call(U=P2) == -8                        # U aliases T
    assert call(T=None) == -9
    assert call(T=P, lda=6, ldt=5) == -9           # in place needs lda == ldt
    assert call(V=P3, ldv=2) == -10
    assert call(budget=8 * 5 * 2) == -11           # one tile only
    assert call(budget=-1) == -11
    assert call(mode=3) == -12
    assert call(m=40000, n=64, lda=40000, ldt=40000, b=64) == rb.ERR_TOO_LARGE
    assert call(m=600, n=600, lda=600, ldt=600, b=300) == rb.ERR_TOO_LARGE
    assert call(m=0, n=0) == 0

