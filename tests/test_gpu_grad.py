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


def _cond_y(A, b, q, seed):
    Y = A.T @ tg.first_block_sketch(A, b, seed)
    for _ in range(q):
        Y = A.T @ (A @ Y)
    return np.linalg.cond(Y)


@pytest.mark.parametrize("m,n,b,q,k,kind", [(512, 512, 64, 2, 32, "exp"), (600, 400, 32, 1, 7, "iid"),
                                            (700, 500, 128, 2, 100, "exp98"), (257, 200, 48, 0, 48, "exp"),
                                            (300, 300, 64, 1, 1, "exp")])
def test_grad_k_matches_reference(m, n, b, q, k, kind):
    """k <= b: the GPU reverse pass (randutv_truncate_grad_k) against torch's
    reverse mode through the QR of Y and the SVD of A orth(Y) on the CPU.  Both
    go through R_Y^{-1} and the eigenvalue gaps of the first block: bound
    100 u cond(Y) times the largest d_1^2 / (d_k^2 - d_{k+1}^2)."""
    A = make_matrix(kind, m, n, seed=6)
    rng = np.random.default_rng(m + n + k)
    Gbar = rng.standard_normal((m, n))
    ref = tg.first_block_truncation_k_grad(A, b, q, 9, k, Gbar)
    got = to_host(pkg.randutv_truncate_grad_k(to_dev(A), b, q, 9, k, to_dev(Gbar)))
    Y = A.T @ tg.first_block_sketch(A, b, 9)
    for _ in range(q):
        Y = A.T @ (A @ Y)
    Qy = np.linalg.qr(Y)[0]
    d = np.linalg.svd(A @ Qy, compute_uv=False)
    gap = d[0] ** 2 / (d[k - 1] ** 2 - d[k] ** 2) if k < min(b, n) else 1.0
    tol = max(1e-12, 100 * 2.0 ** -52 * np.linalg.cond(Y) * gap)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"truncation grad k={k} {m}x{n} b={b} q={q} {kind}: max rel err {err:.2e} (bound {tol:.1e})")
    assert err <= tol


def test_grad_k_at_b_equals_grad():
    A = make_matrix("exp", 400, 300, seed=8)
    Gbar = np.random.default_rng(2).standard_normal((400, 300))
    g1 = to_host(pkg.randutv_truncate_grad(to_dev(A), 64, 2, 3, to_dev(Gbar)))
    g2 = to_host(pkg.randutv_truncate_grad_k(to_dev(A), 64, 2, 3, 64, to_dev(Gbar)))
    tol = max(1e-12, 100 * 2.0 ** -52 * _cond_y(A, 64, 2, 3))
    assert np.abs(g1 - g2).max() <= tol * np.abs(g1).max()


@pytest.mark.parametrize("k", [16, 32])
def test_grad_k_matches_finite_differences_of_the_gpu_forward(k):
    """256 x 256, b = 32, q = 2: directional derivatives of <Gbar, A_k> with A_k
    from the GPU's full factorization (randutv_factor + randutv_truncate) at
    k = b/2 and k = b, against randutv_truncate_grad_k."""
    m = n = 256
    b, q = 32, 2
    A = make_matrix("exp98", m, n, seed=3)
    rng = np.random.default_rng(10 + k)
    Gbar = rng.standard_normal((m, n))
    Gd = to_dev(Gbar)
    grad = to_host(pkg.randutv_truncate_grad_k(to_dev(A), b, q, 4, k, Gd))

    def L(X):
        U, T, V = pkg.randutv_factor(to_dev(X), b, q, 4)
        return float((pkg.randutv_truncate(U, T, V, k) * Gd).sum())

    h = 1e-6
    for _ in range(3):
        E = rng.standard_normal((m, n))
        fd = (L(A + h * E) - L(A - h * E)) / (2 * h)
        an = float(np.sum(grad * E))
        print(f"fd k={k}: {fd:.10e} analytic {an:.10e}")
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_grad_k_errors():
    A = to_dev(make_matrix("exp", 64, 48, seed=1))
    G = to_dev(np.ones((64, 48)))
    lib = pkg.load()
    assert lib.randutv_truncate_grad_k(64, 48, A.data_ptr(), 64, 16, 1, 0, 0, G.data_ptr(), 64,
                                       G.data_ptr() + 8, 64) == -8          # k < 1
    assert lib.randutv_truncate_grad_k(64, 48, A.data_ptr(), 64, 16, 1, 0, 33, G.data_ptr(), 64,
                                       G.data_ptr() + 8, 64) == -8          # k > b_0 + b_1
    Z = to_dev(np.zeros((64, 48)))
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_truncate_grad_k(Z, 16, 1, 0, 8, G)
    assert e.value.code == 7  # RANDUTV_ERR_RANK: Y = 0 has no range to project on


def test_truncation_autograd_k_fp32_and_batch():
    """truncation(): k < b, float32 input (computed in FP64, returned in
    float32), a batch of two, forward from the first step against the full
    factorization's truncation, and A.grad against the CPU reference."""
    m, n, b, q, k = 320, 256, 64, 2, 24
    A = np.stack([make_matrix("exp98", m, n, seed=s) for s in (11, 12)])
    B = np.random.default_rng(4).standard_normal((2, m, n))
    Ad = torch.from_numpy(A).cuda().to(torch.float32).requires_grad_(True)
    Ak = pkg.truncation(Ad, b, q, 5, k)
    assert Ak.dtype == torch.float32 and Ak.shape == (2, m, n)
    loss = ((Ak - torch.from_numpy(B).cuda().to(torch.float32)) ** 2).sum()
    loss.backward()
    A32 = A.astype(np.float32).astype(np.float64)  # the values the library saw
    for t in range(2):
        ref_ak = tg.first_block_truncation_k(A32[t], b, q, 5, k)
        full = pkg.truncation(torch.from_numpy(A32[t]).cuda(), b, q, 5, k, full_factorization=True)
        assert np.abs(to_host(Ak.detach()[t]).astype(np.float64) - ref_ak).max() <= 1e-6 * np.abs(A32[t]).max()
        assert np.abs(to_host(full) - ref_ak).max() <= 1e-9 * np.abs(A32[t]).max()
        gbar = 2.0 * (to_host(Ak.detach()[t]).astype(np.float64) - B[t].astype(np.float32).astype(np.float64))
        ref = tg.first_block_truncation_k_grad(A32[t], b, q, 5, k, gbar)
        got = to_host(Ad.grad[t]).astype(np.float64)
        assert np.abs(got - ref).max() <= 1e-5 * np.abs(ref).max()


@pytest.mark.parametrize("k", [48, 20])
def test_truncate_batched_equals_single_calls(k):
    """randutv_truncate_batched (matrices spread over the library's streams)
    gives every matrix's forward value and reverse pass bit for bit as the
    single-matrix calls do, at k = b and k < b."""
    m, n, b, q = 300, 240, 48, 2
    A = np.stack([make_matrix("exp98", m, n, seed=s) for s in range(5)])
    G = np.random.default_rng(8).standard_normal((5, m, n))
    Ad = torch.from_numpy(A).cuda()
    Gd = torch.from_numpy(G).cuda()
    fwd = pkg.randutv_truncate_batched(Ad, b, q, 3, k)
    rev = pkg.randutv_truncate_batched(Ad, b, q, 3, k, Gd)
    for t in range(5):
        Xd = to_dev(A[t])
        f1 = (pkg.randutv_truncate_first_block(Xd, b, q, 3) if k == b
              else pkg.randutv_truncate_first_block_k(Xd, b, q, 3, k))
        r1 = (pkg.randutv_truncate_grad(Xd, b, q, 3, to_dev(G[t])) if k == b
              else pkg.randutv_truncate_grad_k(Xd, b, q, 3, k, to_dev(G[t])))
        assert torch.equal(fwd[t], f1) and torch.equal(rev[t], r1), t


@pytest.mark.parametrize("k", [128, 64])
def test_grad_at_the_benchmark_size(k):
    """The batched truncation workload's matrix size: 2048 x 2048, b = 128,
    q = 2, s_i = 0.98^i; k = b (the projector form) and k < b, against the
    oracle with the bounds of the smaller cases above."""
    m = n = 2048
    b, q = 128, 2
    A = make_matrix("exp98", m, n, seed=11)
    Gbar = np.random.default_rng(k).standard_normal((m, n))
    if k == b:
        ref = tg.first_block_truncation_grad(A, b, q, 5, Gbar)
        got = to_host(pkg.randutv_truncate_grad(to_dev(A), b, q, 5, to_dev(Gbar)))
        M = tg.first_block_sketch(A, b, 5)
        for _ in range(q + 1):
            M = A @ (A.T @ M)
        tol = max(1e-12, 100 * 2.0 ** -52 * np.linalg.cond(M))
    else:
        ref = tg.first_block_truncation_k_grad(A, b, q, 5, k, Gbar)
        got = to_host(pkg.randutv_truncate_grad_k(to_dev(A), b, q, 5, k, to_dev(Gbar)))
        Y = A.T @ tg.first_block_sketch(A, b, 5)
        for _ in range(q):
            Y = A.T @ (A @ Y)
        d = np.linalg.svd(A @ np.linalg.qr(Y)[0], compute_uv=False)
        gap = d[0] ** 2 / (d[k - 1] ** 2 - d[k] ** 2)
        tol = max(1e-12, 100 * 2.0 ** -52 * np.linalg.cond(Y) * gap)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    print(f"truncation grad 2048^2 b={b} q={q} k={k}: max rel err {err:.2e} (bound {tol:.1e})")
    assert err <= tol
