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
