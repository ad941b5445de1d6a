"""Pins of the first-block truncation derivative reference (CPU, FP64)."""
import numpy as np
import pytest

from oracle import randutv_oracle as ro
from oracle import truncation_grad as tg


def _matrix(m, n, seed, decay=0.9):
    rng = np.random.default_rng(seed)
    P = np.linalg.qr(rng.standard_normal((m, m)))[0]
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    s = decay ** np.arange(min(m, n))
    return (P[:, :n] * s) @ Q.T


def _algorithm_truncation(A, b, q, seed):
    U, T, V = ro.randutv(A, b, q, seed)
    return ro.truncate(U, T, V, min(b, A.shape[1]))


@pytest.mark.parametrize("m,n,b,q", [(60, 40, 8, 1), (50, 50, 10, 2), (45, 30, 6, 0), (30, 20, 25, 1)])
def test_closed_form_is_the_algorithms_first_block(m, n, b, q):
    """A_k of the step loop (U_k T_k V^T) equals Q Q^T A with Q = orth((A A^T)^(q+1) G(0))."""
    A = _matrix(m, n, seed=m + n)
    ref = _algorithm_truncation(A, b, q, 3)
    got = tg.first_block_truncation(A, b, q, 3)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(A).max()
    if b >= n:  # one step: the truncation at k = n is A itself
        assert np.abs(got - A).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("m,n,b,q", [(40, 30, 8, 1), (36, 36, 6, 2), (30, 24, 5, 0)])
def test_gradient_matches_finite_differences_of_the_algorithm(m, n, b, q):
    """<dL/dA, E> against central differences of L(A) = <Gbar, A_k(A)>, with
    A_k taken from the oracle's full randUTV step loop (not the closed form)."""
    A = _matrix(m, n, seed=7 * m + n, decay=0.8)
    rng = np.random.default_rng(11)
    Gbar = rng.standard_normal((m, n))
    grad = tg.first_block_truncation_grad(A, b, q, 5, Gbar)
    # central differences: error ~h^2 f''' (large here: the power iteration
    # amplifies curvature) plus ~eps |f| / h of rounding; h = 1e-6 keeps both
    # near 1e-8 relative
    h = 1e-6
    for t in range(3):
        E = rng.standard_normal((m, n))
        fp = np.sum(Gbar * _algorithm_truncation(A + h * E, b, q, 5))
        fm = np.sum(Gbar * _algorithm_truncation(A - h * E, b, q, 5))
        fd = (fp - fm) / (2 * h)
        an = np.sum(grad * E)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)


def test_gradient_has_the_subspace_term():
    """The derivative of the projector matters: dropping it (P Gbar alone) is
    far from the reference, so the pins above would catch that mistake."""
    A = _matrix(40, 30, seed=1, decay=0.8)
    rng = np.random.default_rng(2)
    Gbar = rng.standard_normal((40, 30))
    grad = tg.first_block_truncation_grad(A, 8, 1, 5, Gbar)
    Ak = tg.first_block_truncation(A, 8, 1, 5)
    Q = np.linalg.qr(Ak)[0][:, :8]
    naive = Q @ (Q.T @ Gbar)
    assert np.linalg.norm(grad - naive) > 0.1 * np.linalg.norm(grad)


def _algorithm_truncation_k(A, b, q, seed, k):
    U, T, V = ro.randutv(A, b, q, seed)
    return ro.truncate(U, T, V, k)


@pytest.mark.parametrize("m,n,b,q,k", [(60, 40, 8, 1, 3), (50, 50, 10, 2, 5), (45, 30, 6, 0, 1),
                                       (40, 40, 12, 1, 12), (30, 20, 25, 1, 7)])
def test_closed_form_k_is_the_algorithms_truncation(m, n, b, q, k):
    """For k <= b the step loop's A_k equals the projection onto the leading k
    left singular vectors of A orth(Y); at k = b it is Q Q^T A as before."""
    A = _matrix(m, n, seed=m + 3 * n)
    ref = _algorithm_truncation_k(A, b, q, 3, k)
    got = tg.first_block_truncation_k(A, b, q, 3, k)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(A).max()
    if k == min(b, n):
        assert np.abs(got - tg.first_block_truncation(A, b, q, 3)).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("m,n,b,q,k", [(40, 30, 8, 1, 4), (36, 36, 6, 2, 3), (30, 24, 10, 0, 9)])
def test_gradient_k_matches_finite_differences_of_the_algorithm(m, n, b, q, k):
    """k < b: the reference gradient (reverse mode through the QR of Y and the
    SVD of A orth(Y)) against central differences of the step loop's A_k."""
    A = _matrix(m, n, seed=5 * m + n, decay=0.8)
    rng = np.random.default_rng(13)
    Gbar = rng.standard_normal((m, n))
    grad = tg.first_block_truncation_k_grad(A, b, q, 5, k, Gbar)
    h = 1e-6
    for t in range(3):
        E = rng.standard_normal((m, n))
        fp = np.sum(Gbar * _algorithm_truncation_k(A + h * E, b, q, 5, k))
        fm = np.sum(Gbar * _algorithm_truncation_k(A - h * E, b, q, 5, k))
        fd = (fp - fm) / (2 * h)
        an = np.sum(grad * E)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (t, fd, an)


def test_gradient_k_has_the_in_block_term():
    """For k < b the singular-subspace rotation inside the first block
    contributes: the k = b formula's gradient (projector onto the whole block)
    misses the k < b one by far."""
    A = _matrix(40, 30, seed=2, decay=0.8)
    rng = np.random.default_rng(3)
    Gbar = rng.standard_normal((40, 30))
    gk = tg.first_block_truncation_k_grad(A, 8, 1, 5, 4, Gbar)
    gb = tg.first_block_truncation_grad(A, 8, 1, 5, Gbar)
    assert np.linalg.norm(gk - gb) > 0.1 * np.linalg.norm(gk)


@pytest.mark.parametrize("m,n,b,q,k", [(60, 40, 8, 1, 16), (50, 50, 10, 2, 15), (45, 30, 6, 0, 12),
                                       (40, 40, 12, 1, 13), (30, 20, 12, 1, 20)])
def test_two_block_closed_form_is_the_algorithms_truncation(m, n, b, q, k):
    """For b < k <= 2b the step loop's A_k equals the two-block closed form
    (U's second block from step 1 sketching in the coordinates of step 0's
    Householder complement columns)."""
    A = _matrix(m, n, seed=m + n, decay=0.85)
    ref = _algorithm_truncation_k(A, b, q, 3, k)
    got = tg.two_block_truncation(A, b, q, 3, k)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(A).max()


@pytest.mark.parametrize("m,n,b,q,k", [(40, 30, 8, 1, 16), (36, 36, 6, 2, 9), (30, 24, 5, 0, 10)])
def test_two_block_gradient_matches_finite_differences_of_the_algorithm(m, n, b, q, k):
    """b < k <= 2b: torch's reverse mode through the two-block closed form
    against central differences of the step loop (h = 1e-6; the curvature of
    the second block's sketch, which passes through the reflectors of step 0,
    makes the truncation error up to ~2e-6 relative here)."""
    A = _matrix(m, n, seed=7 * m + n, decay=0.8)
    rng = np.random.default_rng(11)
    Gbar = rng.standard_normal((m, n))
    grad = tg.two_block_truncation_grad(A, b, q, 5, k, Gbar)
    h = 1e-6
    for t in range(3):
        E = rng.standard_normal((m, n))
        fp = np.sum(Gbar * _algorithm_truncation_k(A + h * E, b, q, 5, k))
        fm = np.sum(Gbar * _algorithm_truncation_k(A - h * E, b, q, 5, k))
        fd = (fp - fm) / (2 * h)
        an = np.sum(grad * E)
        assert abs(fd - an) <= 1e-5 * max(1.0, abs(an)), (t, fd, an)


def test_two_block_gradient_depends_on_the_reflector_basis():
    """The sketch of step 1 lives in the coordinates of step 0's Householder
    complement: replacing that basis by another orthonormal complement (so
    that only subspaces enter) changes A_2b, so the reflectors must be
    differentiated, not only the projectors."""
    import torch

    A = _matrix(40, 30, seed=3, decay=0.8)
    At = torch.from_numpy(A)
    G0, G1 = (torch.from_numpy(g) for g in tg._two_block_sketches(A, 8, 5))
    ref = tg._closed_form_two_blocks(At, G0, G1, 1, 16).numpy()
    # the same formula with a different complement basis: Gamma from numpy's
    # complete QR instead of the reflector product
    Y0 = A.T @ G0.numpy()
    Y0 = A.T @ (A @ Y0)
    Qv = np.linalg.qr(Y0)[0]
    Qfull = np.linalg.qr(A @ Qv, mode="complete")[0]
    Uperp = Qfull[:, 8:] @ np.linalg.qr(np.random.default_rng(0).standard_normal((32, 32)))[0]
    Gam = Uperp @ G1.numpy()
    Qh = Qfull[:, :8]
    piu = lambda Z: Z - Qh @ (Qh.T @ Z)
    piv = lambda Z: Z - Qv @ (Qv.T @ Z)
    Yt = piv(A.T @ Gam)
    Yt = piv(A.T @ piu(A @ Yt))
    C1 = piu(A @ np.linalg.qr(Yt)[0])
    U2 = np.linalg.svd(C1, full_matrices=False)[0][:, :8]
    other = Qh @ (Qh.T @ A) + U2 @ (U2.T @ A)
    assert np.abs(other - ref).max() > 1e-6 * np.abs(A).max()
