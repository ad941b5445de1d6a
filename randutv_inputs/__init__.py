"""Seeded synthetic test matrices for randUTV experiments.

The paper's experiments use randomly generated real FP64 matrices (Section 4,
experimental setup).  This module builds such inputs with controlled spectra:

    A = P diag(s) Q^T,   P (m x n) and Q (n x n) with Haar-distributed
                          orthonormal columns (QR of a seeded Gaussian matrix,
                          columns scaled by sign(diag R), as in Mezzadri 2007),

or a plain i.i.d. N(0,1) matrix.  It holds none of randUTV's arithmetic: it is
input plumbing shared by the tests, the benchmark and the smoke check.  The
random sketch that randUTV itself draws is NOT produced here (each side of the
parity check generates it from the counter-based generator's definition).

Spectra (1-based index i, n singular values):
    "log8": s_i = 10^(-8 (i-1)/(n-1))            (eight decades, smooth decay)
    "exp":  s_i = 0.99^i                            (exponential decay)
    "exp98": s_i = 0.98^i                           (faster exponential decay)
    "step": s_i = 1 for i <= 400, 1e-6 otherwise, plus 1e-10 * N(0,1) noise on A
    "iid":  A itself has i.i.d. N(0,1) entries (no P, Q)
"""
from __future__ import annotations

import numpy as np

SPECTRA = ("log8", "exp", "exp98", "step", "iid")

# seed offsets for the independent random streams of one test matrix
_SEED_P, _SEED_Q, _SEED_NOISE, _SEED_IID = 1, 2, 3, 4


def spectrum(kind: str, n: int) -> np.ndarray:
    """Singular values (descending) of the named synthetic spectrum."""
    i = np.arange(1, n + 1, dtype=np.float64)
    if kind == "log8":
        if n == 1:
            return np.ones(1)
        return 10.0 ** (-8.0 * (i - 1.0) / (n - 1.0))
    if kind == "exp":
        return 0.99 ** i
    if kind == "exp98":
        return 0.98 ** i
    if kind == "step":
        s = np.full(n, 1e-6)
        s[: min(400, n)] = 1.0
        return s
    raise ValueError(f"spectrum {kind!r} has no closed form (or is unknown)")


def haar_orthonormal(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols matrix with Haar-distributed orthonormal columns (rows >= cols)."""
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((rows, cols))
    Qf, R = np.linalg.qr(Z, mode="reduced")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    return Qf * sgn[None, :]


def make_matrix(kind: str, m: int, n: int | None = None, seed: int = 0) -> np.ndarray:
    """Seeded m x n FP64 test matrix (column-major / Fortran order), m >= n."""
    n = m if n is None else n
    if kind == "iid":
        rng = np.random.default_rng(10 * seed + _SEED_IID)
        return np.asfortranarray(rng.standard_normal((m, n)))
    s = spectrum(kind, n)
    P = haar_orthonormal(m, n, 10 * seed + _SEED_P)
    Q = haar_orthonormal(n, n, 10 * seed + _SEED_Q)
    A = (P * s[None, :]) @ Q.T
    if kind == "step":
        rng = np.random.default_rng(10 * seed + _SEED_NOISE)
        A += 1e-10 * rng.standard_normal((m, n))
    return np.asfortranarray(A)


def make_matrix_device(kind: str, m: int, n: int | None = None, seed: int = 0,
                       device: str = "cuda"):
    """Same recipe built with torch on the GPU (for sizes where host LAPACK is slow).

    Returns a column-major (stride (1, m)) float64 tensor.  The random streams
    are torch's, so the matrix differs from make_matrix(...) for the same seed;
    it has the same spectrum and distribution.
    """
    import torch

    n = m if n is None else n
    g = torch.Generator(device=device)

    def gauss(r, c, sd):
        g.manual_seed(sd)
        return torch.randn((r, c), generator=g, device=device, dtype=torch.float64)

    if kind == "iid":
        A = gauss(m, n, 10 * seed + _SEED_IID)
    else:
        s = torch.as_tensor(spectrum(kind, n), device=device)

        def haar(r, c, sd):
            Qf, R = torch.linalg.qr(gauss(r, c, sd), mode="reduced")
            d = torch.sign(torch.diagonal(R))
            d[d == 0] = 1.0
            return Qf * d[None, :]

        P = haar(m, n, 10 * seed + _SEED_P)
        Q = haar(n, n, 10 * seed + _SEED_Q)
        A = (P * s[None, :]) @ Q.T
        del P, Q
        if kind == "step":
            A += 1e-10 * gauss(m, n, 10 * seed + _SEED_NOISE)
    # column-major storage: transpose of a contiguous n x m tensor
    return A.t().contiguous().t()
