"""GPU HQRRP (randutv_hqrrp) against the FP64 CPU oracle."""
import numpy as np
import pytest
import scipy.linalg.lapack as lapack

import paper_2002_06960_amd as pkg
from oracle import hqrrp_oracle as ho
from oracle import randutv_oracle as ro
from randutv_inputs import make_matrix
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _q_of(F, tau):
    """Q's first n columns from the dgeqp3 layout via LAPACK dorgqr."""
    Q, _, info = lapack.dorgqr(np.asfortranarray(F), tau)
    assert info == 0
    return Q


@pytest.mark.parametrize("m,n,b,kind", [(500, 400, 64, "iid"), (777, 300, 50, "exp"), (300, 240, 256, "iid"),
                                        (256, 200, 1, "iid"), (1100, 1000, 128, "log8")])
def test_hqrrp_matches_oracle(m, n, b, kind):
    """Pivots bit-exact (integer decisions taken on the same sketch; the GEMM's
    rounding moves norms by ~1e-15 relative, far below the gaps between
    candidates here), then R to 1e-11 max|A| and each column's reflector and
    tau to 1e-11 max|A| / |R_jj|: both sides are backward stable, so the
    data a reflector is built from carries absolute errors of order
    u max|A|, relative u max|A| / |R_jj| (up to 1e-8 for the log8 spectrum)."""
    A = make_matrix(kind, m, n, seed=8)
    F, tau, jp = pkg.randutv_hqrrp(to_dev(A), b, 6)
    Fo, tauo, jpo = ho.hqrrp(A, b, 6)
    jp = to_host(jp)
    assert list(jp) == list(jpo)
    F, tau = to_host(F), to_host(tau)
    amax = np.abs(A).max()
    np.testing.assert_allclose(np.triu(F[:n, :]), np.triu(Fo[:n, :]), rtol=0, atol=1e-11 * amax)
    col_tol = 1e-11 * amax / np.maximum(np.abs(np.diag(Fo)), 1e-300)
    assert np.all(np.abs(tau - tauo) <= col_tol), np.max(np.abs(tau - tauo) / col_tol)
    low = np.tril(F, -1) - np.tril(Fo, -1)
    assert np.all(np.abs(low) <= col_tol[None, :]), np.max(np.abs(low) / col_tol[None, :])


@pytest.mark.parametrize("m,n,b", [(4000, 3000, 256), (3000, 3000, 200)])
def test_hqrrp_invariants_at_size(m, n, b):
    """A P = Q R with Q orthonormal and R upper trapezoidal; every pivot is a
    valid choice (checked against the oracle's pivots on the first step)."""
    A = make_matrix("exp", m, n, seed=1)
    F, tau, jp = pkg.randutv_hqrrp(to_dev(A), b, 3)
    F, tau, jp = to_host(F), to_host(tau), to_host(jp)
    assert sorted(jp) == list(range(n))
    Q = _q_of(F, tau)
    R = np.triu(F[:n, :])
    assert np.linalg.norm(A[:, jp] - Q @ R) <= 1e-13 * np.linalg.norm(A)
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-13
    G = ho.sketch_block(3, 0, m, b)
    J0 = ho.cpqr_pivots(G.T @ A, b)
    assert list(jp[:b]) == J0


def test_hqrrp_pivot_kernel_without_lds_slab():
    """n = 16640 with b = 256: the first step's 65 columns per workgroup do not
    fit in LDS, so the pivot kernel works on Y in global memory; its pivots
    equal the oracle's CPQR of the same sketch."""
    m = n = 16640
    b = 256
    A = np.random.default_rng(12).standard_normal((m, n))
    F, tau, jp = pkg.randutv_hqrrp(to_dev(A), b, 2)
    jp = to_host(jp)
    assert sorted(jp) == list(range(n))
    G = ho.sketch_block(2, 0, m, b)
    assert list(jp[:b]) == ho.cpqr_pivots(G.T @ A, b)
    del F, tau


def test_hqrrp_errors():
    A = np.ones((40, 30))
    A[2, 3] = np.inf
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_hqrrp(to_dev(A), 8, 0)
    assert e.value.code == 3


def test_hqrrp_padded_leading_dimension():
    """lda > m through the C ABI: the exchanges, the panel and the update all
    address A through lda; the padding rows stay untouched."""
    import ctypes
    import torch

    m, n, b, lda = 300, 220, 40, 311
    A = make_matrix("iid", m, n, seed=5)
    buf = torch.full((n, lda), 7.0, dtype=torch.float64, device="cuda")  # column-major with ld = lda
    buf.t()[:m, :] = to_dev(A)
    tau = torch.empty(n, dtype=torch.float64, device="cuda")
    jp = torch.empty(n, dtype=torch.int64, device="cuda")
    lib = pkg.load()
    torch.cuda.synchronize()
    rc = lib.randutv_hqrrp(m, n, ctypes.c_void_p(buf.data_ptr()), lda, b, 4,
                           ctypes.c_void_p(tau.data_ptr()), ctypes.c_void_p(jp.data_ptr()))
    assert rc == 0
    F = to_host(buf.t()[:m, :])
    assert np.all(to_host(buf.t()[m:, :]) == 7.0)
    Fo, tauo, jpo = ho.hqrrp(A, b, 4)
    assert list(to_host(jp)) == list(jpo)
    np.testing.assert_allclose(F, Fo, rtol=0, atol=1e-11 * np.abs(A).max())
    np.testing.assert_allclose(to_host(tau), tauo, rtol=0, atol=1e-12)


@pytest.mark.parametrize("m,n,b,kind", [(600, 400, 64, "iid"), (1000, 1000, 128, "exp"), (777, 300, 256, "iid"),
                                        (300, 240, 1000, "iid"), (513, 200, 48, "log8")])
def test_geqrf_blocked_matches_oracle(m, n, b, kind):
    """randutv_geqrf_blocked (HQRRP's step loop without the pivots) against the
    oracle's column-by-column Householder QR (itself pinned to LAPACK): R to
    1e-11 max|A|, each column's reflector and tau to 1e-11 max|A| / |R_jj| (the
    same backward-stability argument as for HQRRP above)."""
    A = make_matrix(kind, m, n, seed=9)
    F, tau = pkg.randutv_geqrf_blocked(to_dev(A), b)
    Wo, tauo, Ro = ro.householder_qr(A)
    F, tau = to_host(F), to_host(tau)
    amax = np.abs(A).max()
    np.testing.assert_allclose(np.triu(F[:n, :]), Ro, rtol=0, atol=1e-11 * amax)
    col_tol = 1e-11 * amax / np.maximum(np.abs(np.diag(Ro)), 1e-300)
    assert np.all(np.abs(tau - tauo) <= col_tol), np.max(np.abs(tau - tauo) / col_tol)
    low = np.tril(F, -1) - np.tril(Wo, -1)
    assert np.all(np.abs(low) <= col_tol[None, :]), np.max(np.abs(low) / col_tol[None, :])


def test_geqrf_blocked_reconstructs():
    """A = Q R to 1e-14 and Q orthonormal at 3000 x 2500, b = 256."""
    m, n, b = 3000, 2500, 256
    A = make_matrix("iid", m, n, seed=10)
    F, tau = pkg.randutv_geqrf_blocked(to_dev(A), b)
    F, tau = to_host(F), to_host(tau)
    Q = _q_of(F, tau)
    R = np.triu(F[:n, :])
    assert np.linalg.norm(A - Q @ R) <= 1e-14 * np.linalg.norm(A) * np.sqrt(n)
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= 1e-13
