"""Helpers shared by the GPU tests: host <-> device copies and the gated T
comparison.  Test infrastructure only."""
from __future__ import annotations

import numpy as np


def to_dev(a: np.ndarray):
    import torch

    a = np.asarray(a, dtype=np.float64)
    if a.ndim == 1:
        return torch.from_numpy(a.copy()).cuda()
    m, n = a.shape
    t = torch.empty((n, m), dtype=torch.float64, device="cuda").t()
    t.copy_(torch.from_numpy(np.ascontiguousarray(a)))
    return t


def to_host(t) -> np.ndarray:
    return t.detach().cpu().numpy()


def invariants_dev(A, U, T, V):
    """Residual and orthogonality of GPU factors, evaluated with torch FP64 products."""
    import torch

    nA = torch.linalg.norm(A)
    res = (torch.linalg.norm(A - U @ T @ V.T) / nA).item() if nA > 0 else torch.linalg.norm(U @ T @ V.T).item()
    eu = (U.T @ U - torch.eye(U.shape[0], dtype=U.dtype, device=U.device)).abs().max().item()
    ev = (V.T @ V - torch.eye(V.shape[0], dtype=V.dtype, device=V.device)).abs().max().item()
    lower = torch.tril(T, -1).abs().max().item() if T.shape[0] > 1 else 0.0
    return res, eu, ev, lower


def diag_blocks_ok(T: np.ndarray, b: int) -> bool:
    m, n = T.shape
    for s in range(0, n, b):
        e = min(n, s + b)
        D = T[s:e, s:e]
        if np.abs(D - np.diag(np.diag(D))).max() != 0.0:
            return False
        d = np.diag(D)
        if np.any(d < 0) or np.any(np.diff(d) > 0):
            return False
    return True


def sign_align(T_gpu: np.ndarray, V_gpu: np.ndarray, V_ora: np.ndarray) -> tuple[np.ndarray, int]:
    """Flip (u_j, v_j) pairs of the GPU result to the oracle's orientation:
    S T S with S_j = sign(<V_gpu(:, j), V_ora(:, j)>).  Returns (S T S, flips)."""
    dots = np.einsum("ij,ij->j", V_gpu, V_ora)
    s = np.where(dots < 0, -1.0, 1.0)
    m = T_gpu.shape[0]
    srow = np.ones(m)
    srow[: s.shape[0]] = s
    return (srow[:, None] * T_gpu) * s[None, :], int(np.sum(s < 0))


def stable_rows(T1: np.ndarray, T2: np.ndarray, nA: float, b: int, tol: float = 1e-12) -> int:
    """Number of leading rows (a multiple of b, or all) in which two oracle runs
    on ulp-perturbed input agree to tol * ||A||_F: the part of T that the
    input determines; beyond it several results are correct."""
    m, n = T1.shape
    r = 0
    while r < n:
        e = min(n, r + b)
        if np.linalg.norm(T1[r:e, :] - T2[r:e, :]) > tol * nA:
            break
        r = e
    return m if r >= n else r


def block_sensitivity(T1: np.ndarray, T2: np.ndarray, nA: float, b: int) -> np.ndarray:
    """Per b x b block of T, ||T1 - T2||_F / ||A||_F for two oracle runs on
    ulp-perturbed inputs: how far the input itself determines that block.
    Diagonal blocks (singular values of a projected block) are determined to
    ~u; off-diagonal blocks depend on the chosen bases of the sketched
    subspaces and move with cond(Y) * u, where Y is the powered sketch."""
    m, n = T1.shape
    nb_r, nb_c = -(-m // b), -(-n // b)
    out = np.zeros((nb_r, nb_c))
    for i in range(nb_r):
        for j in range(nb_c):
            d = T1[i * b:(i + 1) * b, j * b:(j + 1) * b] - T2[i * b:(i + 1) * b, j * b:(j + 1) * b]
            out[i, j] = np.linalg.norm(d) / nA
    return out
