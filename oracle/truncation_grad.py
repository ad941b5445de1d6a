"""FP64 CPU reference for the derivative of randUTV's first-block truncation.
TEST INFRASTRUCTURE ONLY: only the tests may import this module; the GPU
library never calls it and shares no code with it.

For k = b_0 = min(b, n) the rank-k truncation of randUTV (Section 1.1,
A_k = U(:, 0:k) T(0:k, :) V^T) has a closed form.  T = U^T A V gives
T(0:k, :) V^T = U_k^T A, so A_k = U_k U_k^T A.  The first step of the method
(Section 3.1) takes V's first block from the QR of Y = (A^T A)^q A^T G(0), so
A V(:, 0:k) spans the range of M = A Y = (A A^T)^(q+1) G(0); the panel QR of
that block gives U_k with the same range, and the later steps (the b x b SVD
and every U update of steps >= 1) either rotate U_k within it or leave it
alone.  Hence A_k = Q Q^T A with Q an orthonormal basis of range(M), with
the sketch G(0) held fixed.

The reference gradient of L(A_k) with respect to A is torch's reverse-mode
differentiation of that closed form in FP64 on the CPU (torch.linalg.qr's own
derivative rule).  The tests pin it to the algorithm itself by central finite
differences of the oracle's randutv() truncation.
"""
import numpy as np
import torch

from .randutv_oracle import sketch_block


def first_block_sketch(A: np.ndarray, b: int, seed: int) -> np.ndarray:
    """G(0): the m x min(b, n) sketch that step 0 draws (reading R5/R6)."""
    m, n = A.shape
    return sketch_block(seed, 0, m, min(b, n))


def _closed_form(At, G, q: int):
    M = G
    for _ in range(q + 1):
        M = At @ (At.T @ M)  # (A A^T)^(q+1) G(0), no re-orthonormalisation (R9)
    Q, _ = torch.linalg.qr(M, mode="reduced")
    return Q @ (Q.T @ At)


def _closed_form_k(At, G, q: int, k: int):
    """A_k for k <= b_0: the projector onto the leading k left singular
    vectors of C = A orth(Y), Y = (A^T A)^q A^T G(0).  After step 0 the first
    b_0 columns of U are (panel Q of C) U_S with C = Q R, R = U_S D V_S^T the
    b x b SVD (Section 3.1), i.e. the left singular vectors of C in descending
    order; later steps leave them alone.  They do not depend on which
    orthonormal basis of range(Y) forms C, so any QR of Y gives the same A_k."""
    Y = At.T @ G
    for _ in range(q):
        Y = At.T @ (At @ Y)  # (A^T A)^q A^T G(0), no re-orthonormalisation (R9)
    Qv, _ = torch.linalg.qr(Y, mode="reduced")
    C = At @ Qv
    Uc, _, _ = torch.linalg.svd(C, full_matrices=False)
    Uk = Uc[:, :k]
    return Uk @ (Uk.T @ At)


def first_block_truncation_k(A: np.ndarray, b: int, q: int, seed: int, k: int) -> np.ndarray:
    """A_k for 0 < k <= min(b, n) from the closed form (leading left singular
    subspace of A orth(Y))."""
    At = torch.from_numpy(np.asarray(A, dtype=np.float64))
    G = torch.from_numpy(first_block_sketch(A, b, seed))
    return _closed_form_k(At, G, q, k).numpy()


def first_block_truncation_k_grad(A: np.ndarray, b: int, q: int, seed: int, k: int,
                                  Gbar: np.ndarray) -> np.ndarray:
    """d<Gbar, A_k>/dA for 0 < k <= min(b, n), G(0) fixed, by torch's reverse
    mode through the QR and the SVD (its rule needs distinct singular values
    of C around k, which holds for the test matrices here)."""
    At = torch.from_numpy(np.array(A, dtype=np.float64)).requires_grad_(True)
    G = torch.from_numpy(first_block_sketch(A, b, seed))
    Ak = _closed_form_k(At, G, q, k)
    (Ak * torch.from_numpy(np.asarray(Gbar, dtype=np.float64))).sum().backward()
    return At.grad.numpy()


def first_block_truncation(A: np.ndarray, b: int, q: int, seed: int = 0) -> np.ndarray:
    """A_k for k = min(b, n) from the closed form Q Q^T A."""
    At = torch.from_numpy(np.asarray(A, dtype=np.float64))
    G = torch.from_numpy(first_block_sketch(A, b, seed))
    return _closed_form(At, G, q).numpy()


def first_block_truncation_grad(A: np.ndarray, b: int, q: int, seed: int, Gbar: np.ndarray) -> np.ndarray:
    """d<Gbar, A_k>/dA for k = min(b, n), G(0) fixed: the vector-Jacobian
    product that a reverse pass receives Gbar = dL/dA_k for."""
    At = torch.from_numpy(np.array(A, dtype=np.float64)).requires_grad_(True)
    G = torch.from_numpy(first_block_sketch(A, b, seed))
    Ak = _closed_form(At, G, q)
    (Ak * torch.from_numpy(np.asarray(Gbar, dtype=np.float64))).sum().backward()
    return At.grad.numpy()


def _lu_unpivoted(M):
    """M = L U for an m x b matrix (m >= b) without pivoting: L unit lower
    trapezoidal (m x b), U upper triangular (b x b).  Column-by-column
    Doolittle in torch ops (differentiable)."""
    m, b = M.shape
    Lcols, Urows = [], []
    for j in range(b):
        # row j of U: M[j, j:] - L[j, :j] U[:j, j:]
        u = M[j, :]
        for t in range(j):
            u = u - Lcols[t][j] * Urows[t]
        u = torch.cat([torch.zeros(j, dtype=M.dtype), u[j:]])
        Urows.append(u)
        # column j of L: (M[:, j] - sum_t L[:, t] U[t, j]) / U[j, j], unit at row j, zero above
        l_ = M[:, j]
        for t in range(j):
            l_ = l_ - Lcols[t] * Urows[t][j]
        l_ = l_ / u[j]
        l_ = torch.cat([torch.zeros(j, dtype=M.dtype), torch.ones(1, dtype=M.dtype), l_[j + 1:]])
        Lcols.append(l_)
    return torch.stack(Lcols, dim=1), torch.stack(Urows, dim=0)


def _closed_form_two_blocks(At, G0, G1, q: int, k: int):
    """A_k for b_0 < k <= b_0 + b_1 (the first two blocks of U).

    Step 0 (Section 3.1): Q_V = Householder Q of Y_0 = (A^T A)^q A^T G(0), and
    U's first block spans C_0 = A Q_V, whose Householder QR gives the thin Q_H
    and the full reflector product H.  Step 1 sketches the trailing matrix
    B_1 = U_perp^T A V_perp in the coordinates of the complement columns
    U_perp = H(:, b_0:), V_perp of those Householder products; lifted back to A's
    space, its sketch is Gamma = U_perp G(1), its powered sketch spans
    Pi_V (A^T Pi_U A Pi_V)^q A^T Gamma (Pi_U = I - Q_H Q_H^T, Pi_V = I - Q_V Q_V^T),
    and U's second block holds the left singular vectors of
    C_1 = Pi_U A orth(that sketch).  Everything but U_perp depends on subspaces
    only; U_perp comes from the reflectors: with M = [I; 0] - Q_H = W (T W_1^T)
    (an LU factorization without pivoting: W unit lower trapezoidal, T W_1^T upper
    triangular), U_perp = [0; I] - M W_1^{-T} W_2^T.  So
    A_k = Q_H Q_H^T A + U_2 U_2^T A, U_2 the leading k - b_0 left singular
    vectors of C_1."""
    m, n = At.shape
    b0 = G0.shape[1]
    Y0 = At.T @ G0
    for _ in range(q):
        Y0 = At.T @ (At @ Y0)
    Qv, _ = torch.linalg.qr(Y0, mode="reduced")
    C0 = At @ Qv
    Qh, _ = torch.linalg.qr(C0, mode="reduced")
    I0 = torch.zeros((m, b0), dtype=At.dtype)
    I0[:b0, :b0] = torch.eye(b0, dtype=At.dtype)
    M = I0 - Qh
    W, _ = _lu_unpivoted(M)
    W1, W2 = W[:b0], W[b0:]
    # Gamma = [0; G(1)] - M W_1^{-T} (W_2^T G(1))
    X = torch.linalg.solve_triangular(W1.T, W2.T @ G1, upper=True, unitriangular=True)
    Gam = torch.cat([torch.zeros((b0, G1.shape[1]), dtype=At.dtype), G1], dim=0) - M @ X

    def pi_u(Z):
        return Z - Qh @ (Qh.T @ Z)

    def pi_v(Z):
        return Z - Qv @ (Qv.T @ Z)

    Yt = pi_v(At.T @ Gam)
    for _ in range(q):
        Yt = pi_v(At.T @ pi_u(At @ Yt))
    Qt, _ = torch.linalg.qr(Yt, mode="reduced")
    C1 = pi_u(At @ Qt)
    U1c, _, _ = torch.linalg.svd(C1, full_matrices=False)
    U2 = U1c[:, : k - b0]
    return Qh @ (Qh.T @ At) + U2 @ (U2.T @ At)


def _two_block_sketches(A: np.ndarray, b: int, seed: int):
    m, n = A.shape
    b0 = min(b, n)
    b1 = min(b, n - b0)
    return sketch_block(seed, 0, m, b0), sketch_block(seed, 1, m - b0, b1)


def two_block_truncation(A: np.ndarray, b: int, q: int, seed: int, k: int) -> np.ndarray:
    """A_k for b_0 < k <= b_0 + b_1 (b_0 = min(b, n), b_1 = min(b, n - b_0))."""
    At = torch.from_numpy(np.asarray(A, dtype=np.float64))
    G0, G1 = (torch.from_numpy(g) for g in _two_block_sketches(A, b, seed))
    return _closed_form_two_blocks(At, G0, G1, q, k).numpy()


def two_block_truncation_grad(A: np.ndarray, b: int, q: int, seed: int, k: int,
                              Gbar: np.ndarray) -> np.ndarray:
    """d<Gbar, A_k>/dA for b_0 < k <= b_0 + b_1, G(0) and G(1) fixed, by torch's
    reverse mode through the closed form (the QRs, the unpivoted LU of the
    reflector block and the SVD)."""
    At = torch.from_numpy(np.array(A, dtype=np.float64)).requires_grad_(True)
    G0, G1 = (torch.from_numpy(g) for g in _two_block_sketches(A, b, seed))
    Ak = _closed_form_two_blocks(At, G0, G1, q, k)
    (Ak * torch.from_numpy(np.asarray(Gbar, dtype=np.float64))).sum().backward()
    return At.grad.numpy()
