"""randutv_factor_noalloc (the factorization with every temporary in the
library's fixed device scratch) against randutv_factor_ex on the same inputs,
called through the C ABI: two calls in a row, the second with a smaller
input, each compared with the allocating entry point (Section 3.1,
Figure 2).  Where both take the same K splits the outputs are bit-identical;
a problem large enough to shrink the split-K partial space changes only the
summation order, and is held to the FP64 gate (1e-11 |A| on T, residual and
orthogonality to the FP64 bar)."""
import ctypes

import numpy as np
import pytest

import paper_2002_06960_amd as pkg
from paper_2002_06960_amd import randutv as rb
from randutv_inputs import make_matrix
from gpu_util import invariants_dev, sign_align, to_dev, to_host

pytestmark = pytest.mark.gpu


def _call(entry, Ad, b, q, seed):
    import torch

    m, n = Ad.shape
    U = pkg.colmajor_empty(m, m, Ad.device)
    T = pkg.colmajor_empty(m, n, Ad.device)
    V = pkg.colmajor_empty(n, n, Ad.device)
    torch.cuda.synchronize()
    args = rb.make_args(m=m, n=n, A=Ad.data_ptr(), lda=Ad.stride(1), b=b, q=q, seed=seed,
                        U=U.data_ptr(), ldu=m, T=T.data_ptr(), ldt=m, V=V.data_ptr(), ldv=n)
    lib = pkg.load()
    print(f"noalloc: {entry} {m}x{n} b={b} q={q}", flush=True)
    rc = getattr(lib, entry)(ctypes.byref(args))
    assert rc == 0, (entry, rc, lib.randutv_strerror(rc))
    return U, T, V


@pytest.mark.parametrize("sizes", [((1500, 1200, 128, 2), (700, 500, 64, 1)),
                                   ((4096, 4096, 128, 2), (2048, 1500, 256, 1))])
def test_noalloc_matches_factor_ex_twice(sizes):
    for (m, n, b, q) in sizes:
        A = make_matrix("exp", m, n, seed=5)
        Ad = to_dev(A)
        U0, T0, V0 = _call("randutv_factor_ex", Ad, b, q, 0)
        U1, T1, V1 = _call("randutv_factor_noalloc", Ad, b, q, 0)
        same = bool((T0 == T1).all() and (U0 == U1).all() and (V0 == V1).all())
        nA = np.linalg.norm(A)
        Ts, flips = sign_align(to_host(T1), to_host(V1), to_host(V0))
        dT = np.linalg.norm(Ts - to_host(T0)) / nA
        res, eu, ev, lower = invariants_dev(Ad, U1, T1, V1)
        print(f"noalloc {m}x{n} b={b}: bit-identical {same}, |T - T_ex| / |A| = {dT:.2e}, "
              f"flips {flips}, residual {res:.2e}, orth {eu:.2e} {ev:.2e}", flush=True)
        assert dT <= 1e-11 and res <= 1e-11 and eu <= 1e-12 and ev <= 1e-12 and lower == 0.0
        if m * n <= 1500 * 1200:
            assert same  # the whole split-K space fits: the same launches


def test_noalloc_rejects_beyond_scratch():
    """A problem whose fixed temporaries exceed the scratch is refused before
    any device work, with its own status code."""
    import torch

    m = n = 12000
    Ad = pkg.colmajor_empty(m, n, "cuda")
    Ad.zero_()
    torch.cuda.synchronize()
    # factored in place (T == A): the size check comes before any device work
    args = rb.make_args(m=m, n=n, A=Ad.data_ptr(), lda=m, b=256, q=2, seed=0, T=Ad.data_ptr(), ldt=m)
    rc = pkg.load().randutv_factor_noalloc(ctypes.byref(args))
    assert rc == rb.ERR_SCRATCH, rc
    assert float(Ad.abs().max()) == 0.0
    args2 = rb.make_args(m=8, n=8, A=Ad.data_ptr(), lda=m, b=4, q=0, T=Ad.data_ptr(), ldt=m,
                         max_workspace_bytes=1)
    assert pkg.load().randutv_factor_noalloc(ctypes.byref(args2)) == -15
