"""GPU reverse pass of the first-block truncation (randutv_truncate_grad and
the torch.autograd binding) against the FP64 CPU reference gradient."""
import numpy as np
import pytest
import torch

import paper_2002_06960_amd as pkg
from oracle import truncation_grad as tg
from randutv_inputs import make_matrix
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("m,n,b,q,kind", [(512, 512, 64, 2, "exp"), (600, 400, 32, 1, "iid"),
                                          (700, 500, 128, 2, "exp98"), (257, 200, 48, 0, "exp")])
def test_grad_matches_reference(m, n, b, q, kind):
    """Same vector-Jacobian product as torch's reverse mode through the
    closed form on the CPU.  The two evaluate one formula in different
    orders; both go through M^+ = R^{-1} Q^T, so their difference is rounding
    amplified by the condition number of M = (A A^T)^(q+1) G(0), which the
    power iteration raises to the 2(q+1)-th power of the block's singular
    value spread (about 5e6 for s_i = 0.98^i with b = 128, q = 2).  Bound:
    100 u cond(M)."""
    A = make_matrix(kind, m, n, seed=4)
    rng = np.random.default_rng(m + n)
    Gbar = rng.standard_normal((m, n))
    ref = tg.first_block_truncation_grad(A, b, q, 9, Gbar)
    got = to_host(pkg.randutv_truncate_grad(to_dev(A), b, q, 9, to_dev(Gbar)))
    M = tg.first_block_sketch(A, b, 9)
    for _ in range(q + 1):
        M = A @ (A.T @ M)
    tol = max(1e-12, 100 * 2.0**-52 * np.linalg.cond(M))
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"truncation grad {m}x{n} b={b} q={q} {kind}: max rel err {err:.2e} (bound {tol:.1e})")
    assert err <= tol


def test_grad_is_gbar_when_one_block_covers_a():
    """k = n: A_k = A for every A near a full-rank A, so dL/dA = Gbar."""
    A = make_matrix("exp", 300, 200, seed=1)
    Gbar = np.random.default_rng(0).standard_normal((300, 200))
    got = to_host(pkg.randutv_truncate_grad(to_dev(A), 256, 1, 0, to_dev(Gbar)))
    assert np.abs(got - Gbar).max() <= 1e-9 * np.abs(Gbar).max()


def test_autograd_end_to_end():
    """L = ||A_k - B||_F^2 through first_block_truncation: forward equals the
    closed form, A.grad equals the reference with Gbar = 2 (A_k - B)."""
    m, n, b, q = 384, 320, 40, 2
    A = make_matrix("exp98", m, n, seed=2)
    B = np.random.default_rng(5).standard_normal((m, n))
    Ad = to_dev(A).requires_grad_(True)
    Ak = pkg.first_block_truncation(Ad, b, q, 7)
    loss = ((Ak - to_dev(B)) ** 2).sum()
    loss.backward()
    Ak_ref = tg.first_block_truncation(A, b, q, 7)
    assert np.abs(to_host(Ak.detach()) - Ak_ref).max() <= 1e-11 * np.abs(A).max()
    ref = tg.first_block_truncation_grad(A, b, q, 7, 2.0 * (Ak_ref - B))
    got = to_host(Ad.grad)
    assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max()


def test_grad_matches_finite_differences_of_the_gpu_forward():
    """Directional derivatives against central differences of the GPU's own
    forward pass (randutv_factor + randutv_truncate) in FP64 on 256 x 256."""
    m = n = 256
    b, q = 32, 2
    A = make_matrix("exp98", m, n, seed=3)
    rng = np.random.default_rng(1)
    Gbar = rng.standard_normal((m, n))
    Gd = to_dev(Gbar)
    grad = to_host(pkg.randutv_truncate_grad(to_dev(A), b, q, 4, Gd))

    def L(X):
        U, T, V = pkg.randutv_factor(to_dev(X), b, q, 4)
        return float((pkg.randutv_truncate(U, T, V, b) * Gd).sum())

    h = 1e-6
    for _ in range(3):
        E = rng.standard_normal((m, n))
        fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
        an = float(np.sum(grad * E))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_grad_errors():
    Z = np.zeros((64, 48))
    G = np.ones((64, 48))
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_truncate_grad(to_dev(Z), 16, 1, 0, to_dev(G))
    assert e.value.code == 7  # zero sketch: no derivative of the projector
    A = make_matrix("exp", 64, 48, seed=0)
    A[3, 5] = np.nan
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_truncate_grad(to_dev(A), 16, 1, 0, to_dev(G))
    assert e.value.code == 3


@pytest.mark.parametrize("m,n,b,q,kind", [(512, 512, 64, 2, "exp"), (700, 500, 128, 2, "exp98"),
                                          (300, 200, 256, 1, "iid")])
def test_first_step_forward(m, n, b, q, kind):
    """randutv_truncate_first_block against the closed form on the CPU and
    against the full factorization's truncation on the GPU; the subspaces
    agree to rounding amplified by cond(M) (as for the gradient)."""
    A = make_matrix(kind, m, n, seed=6)
    Ad = to_dev(A)
    got = to_host(pkg.randutv_truncate_first_block(Ad, b, q, 2))
    ref = tg.first_block_truncation(A, b, q, 2)
    U, T, V = pkg.randutv_factor(Ad, b, q, 2)
    full = to_host(pkg.randutv_truncate(U, T, V, min(b, n)))
    M = tg.first_block_sketch(A, b, 2)
    for _ in range(q + 1):
        M = A @ (A.T @ M)
    tol = max(1e-12, 100 * 2.0**-52 * np.linalg.cond(M)) * np.abs(A).max()
    assert np.abs(got - ref).max() <= tol
    assert np.abs(got - full).max() <= tol
    # the autograd binding's two forward forms give the same value
    Ak = pkg.first_block_truncation(Ad, b, q, 2, first_step_only=True)
    assert np.abs(to_host(Ak) - got).max() == 0.0


def test_autograd_batch():
    """A batch (3 x m x n) gives, matrix by matrix, the single-matrix values
    and gradients."""
    m, n, b, q = 256, 200, 32, 1
    As = np.stack([make_matrix("exp98", m, n, seed=20 + i) for i in range(3)])
    Bs = np.random.default_rng(9).standard_normal((3, m, n))
    X = torch.from_numpy(As).to("cuda").requires_grad_(True)
    Ak = pkg.first_block_truncation(X, b, q, 1)
    ((Ak - torch.from_numpy(Bs).to("cuda")) ** 2).sum().backward()
    for i in range(3):
        Y = to_dev(As[i]).requires_grad_(True)
        Aki = pkg.first_block_truncation(Y, b, q, 1)
        ((Aki - to_dev(Bs[i])) ** 2).sum().backward()
        assert np.array_equal(to_host(Ak[i].detach()), to_host(Aki.detach()))
        np.testing.assert_allclose(to_host(X.grad[i]), to_host(Y.grad), rtol=0, atol=1e-13 * np.abs(to_host(Y.grad)).max())


def test_grad_padded_leading_dimensions():
    """A and Gbar as column-major views with leading dimensions above m."""
    m, n, b, q = 300, 240, 32, 2
    A = make_matrix("exp", m, n, seed=11)
    Gbar = np.random.default_rng(3).standard_normal((m, n))
    Abuf = torch.zeros((n, m + 9), dtype=torch.float64, device="cuda")
    Gbuf = torch.zeros((n, m + 5), dtype=torch.float64, device="cuda")
    Av = Abuf.t()[:m, :]
    Gv = Gbuf.t()[:m, :]
    Av.copy_(to_dev(A))
    Gv.copy_(to_dev(Gbar))
    assert Av.stride() == (1, m + 9) and Gv.stride() == (1, m + 5)
    got = to_host(pkg.randutv_truncate_grad(Av, b, q, 2, Gv))
    ref = tg.first_block_truncation_grad(A, b, q, 2, Gbar)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
