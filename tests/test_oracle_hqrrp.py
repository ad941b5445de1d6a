"""Pins of the HQRRP oracle (CPU, FP64) against LAPACK and the factorization's invariants."""
import numpy as np
import pytest
import scipy.linalg as sl

from oracle import hqrrp_oracle as ho
from oracle import randutv_oracle as ro


@pytest.mark.parametrize("k,N,scaled", [(16, 200, False), (32, 33, False), (8, 8, False), (24, 500, True)])
def test_cpqr_pivots_and_exchanges_match_lapack(k, N, scaled):
    """k steps of CPQR on a k x N matrix choose LAPACK dgeqp3's pivots, and the
    exchange convention reproduces dgeqp3's whole permutation."""
    rng = np.random.default_rng(k * N)
    Y = rng.standard_normal((k, N))
    if scaled:
        Y *= np.logspace(0, -6, N)[rng.permutation(N)]
    perm = sl.qr(Y, pivoting=True, mode="r")[1]
    J = ho.cpqr_pivots(Y, k)
    assert J == list(perm[:k])
    assert list(ho.swap_permutation(J, N)) == list(perm)


def _check_factorization(A, F, tau, jpvt, tol=1e-13):
    m, n = A.shape
    assert sorted(jpvt) == list(range(n))
    Q = ho.explicit_q(F, tau)
    R = np.triu(F[:n, :])
    nA = np.linalg.norm(A)
    assert np.linalg.norm(A[:, jpvt] - Q @ R) <= tol * nA
    assert np.abs(Q.T @ Q - np.eye(n)).max() <= tol


@pytest.mark.parametrize("m,n,b", [(60, 45, 8), (50, 50, 50), (77, 30, 7), (40, 40, 1), (90, 64, 16)])
def test_hqrrp_is_a_pivoted_qr(m, n, b):
    A = np.random.default_rng(m + n + b).standard_normal((m, n))
    F, tau, jpvt = ho.hqrrp(A, b, seed=2)
    _check_factorization(A, F, tau, jpvt)


def test_single_block_is_cpqr_of_the_sketch_then_plain_qr():
    """b >= n: one step.  The pivots are those of CPQR on Y = G^T A, and R is
    LAPACK's unpivoted QR of the permuted A (same reflector sign convention)."""
    rng = np.random.default_rng(3)
    A = rng.standard_normal((70, 40))
    F, tau, jpvt = ho.hqrrp(A, 64, seed=5)
    G = ro.sketch_block(5, 0, 70, 40)
    perm = sl.qr(G.T @ A, pivoting=True, mode="r")[1]
    assert list(jpvt) == list(perm)
    R_lapack = sl.qr(A[:, jpvt], mode="r")[0][:40, :]
    np.testing.assert_allclose(np.triu(F[:40, :]), R_lapack, rtol=0, atol=1e-12 * np.abs(A).max())


def test_hqrrp_reveals_numerical_rank():
    """Rank 12 plus 1e-13 noise: after 12 pivots the trailing block of R is at
    the noise level, and the leading diagonal stays far above it."""
    rng = np.random.default_rng(4)
    A = rng.standard_normal((80, 12)) @ rng.standard_normal((12, 50)) + 1e-13 * rng.standard_normal((80, 50))
    F, tau, jpvt = ho.hqrrp(A, 4, seed=1)
    _check_factorization(A, F, tau, jpvt)
    R = np.triu(F[:50, :])
    assert np.abs(R[12:, 12:]).max() <= 1e-11 * np.abs(A).max()
    assert np.abs(np.diag(R)[:12]).min() >= 1e-3 * np.abs(A).max()
