"""The factorization without host synchronization (RANDUTV_FLAG_ASYNC;
Section 3.1, Figure 2: the same step loop, only enqueued differently).

* An asynchronous call on a side stream gives the synchronous call's U, T, V
  bit for bit, and randutv_factor_status reports its outcome afterwards (a
  non-finite input included: the call no longer stops before the kernels).
* Capture into a HIP graph (skipped): the allocation-free entry point
  captured once on a side stream, replayed three times on new contents of
  the same input, every replay against an eager factorization.  Its one run
  ended in a host-side segmentation fault inside the runtime's end of
  capture (no GPU fault, no kernel had run); the cause is not known, so
  capture is not supported and the test stays skipped.
"""
import numpy as np
import pytest
import torch

import paper_2002_06960_amd as pkg
from paper_2002_06960_amd import randutv as rb
from randutv_inputs import make_matrix
from gpu_util import to_dev

pytestmark = pytest.mark.gpu


def test_async_call_equals_synchronous():
    m, n, b, q = 1000, 800, 64, 2
    A = to_dev(make_matrix("exp", m, n, seed=1))
    U0, T0, V0 = pkg.randutv_factor(A, b, q, 0)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        U1, T1, V1 = pkg.randutv_factor(A, b, q, 0, asynchronous=True)
    assert pkg.randutv_factor_status() == 0
    torch.cuda.synchronize()
    assert torch.equal(T0, T1) and torch.equal(U0, U1) and torch.equal(V0, V1)


def test_async_call_reports_a_non_finite_input_afterwards():
    m, n, b, q = 600, 500, 64, 1
    X = make_matrix("iid", m, n, seed=2)
    X[17, 33] = np.nan
    A = to_dev(X)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        pkg.randutv_factor(A, b, q, 0, asynchronous=True)
    assert pkg.randutv_factor_status() == rb.ERR_NONFINITE
    # the library stays usable
    A2 = to_dev(make_matrix("iid", m, n, seed=3))
    pkg.randutv_factor(A2, b, q, 0)
    assert pkg.randutv_factor_status() == 0


@pytest.mark.skip(reason="ending the capture crashed in the HIP runtime (host SIGSEGV, no GPU fault); "
                         "cause unknown, capture not supported")
def test_graph_capture_replays_match_eager():
    m, n, b, q = 1500, 1300, 128, 2
    A = rb.colmajor_empty(m, n)
    A.copy_(to_dev(make_matrix("exp", m, n, seed=4)))
    U = rb.colmajor_empty(m, m)
    T = rb.colmajor_empty(m, n)
    V = rb.colmajor_empty(n, n)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # an eager call first: the library's streams and events exist
        pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V, asynchronous=True, noalloc=True)
    assert pkg.randutv_factor_status() == 0
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        pkg.randutv_factor(A, b, q, 0, U=U, T=T, V=V, asynchronous=True, noalloc=True)
    torch.cuda.synchronize()
    for seed, kind in ((5, "exp"), (6, "iid"), (7, "exp98")):
        X = make_matrix(kind, m, n, seed=seed)
        A.copy_(to_dev(X))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert pkg.randutv_factor_status() == 0, (seed, kind)
        Ue, Te, Ve = pkg.randutv_factor(to_dev(X), b, q, 0)
        torch.cuda.synchronize()
        print(f"replay {kind} seed {seed}: max|T - T_eager| = {(T - Te).abs().max().item():.3e}", flush=True)
        assert torch.equal(T, Te) and torch.equal(U, Ue) and torch.equal(V, Ve), (seed, kind)
