"""Plain FP64 CPU oracle for HQRRP, the randomized blocked column-pivoted QR
A P = Q R of Section 2 (Sections 2.1 and 2.2: the step loop, the choice of
P^(i) from a sketch and of Q^(i) by unpivoted QR).  TEST INFRASTRUCTURE ONLY:
only the tests may import it; the GPU library never calls it and shares no
code with it.

Readings of Section 2 taken here (each also listed in the design notes):
  H1  Step i (0-based, s = i b, b_i = min(b, n - s)) draws G^(i) of size
      b_i x (m - s) as the transpose of the block that randUTV's step i
      draws, sketch_block(seed, i, m - s, b_i) (same Philox4x64-10 and
      Box-Muller stream); Y = G^(i) R22 is then b_i x (n - s).
  H2  "b steps of the traditional CPQR of Y": Householder QR with column
      pivoting; at step t the pivot is the not yet chosen column of largest
      residual norm over rows t.. (norms recomputed at every step; ties go
      to the lowest column index); its reflector (dlarfg conventions) is
      applied to every column not yet chosen.
  H3  P22 realises the chosen columns J[0..b_i) by successive exchanges:
      for t = 0, 1, ..., the column currently holding J[t] is exchanged with
      position t (the convention of LAPACK's dgeqp3).
  H4  P^(i) = diag(I, P22) multiplies R^(i-1) from the right, so the exchange
      moves whole columns (all m rows); Q22 comes from the unpivoted
      Householder QR of the first b_i permuted columns (rows s..m-1, reading
      R7 of the randUTV oracle), and Q22^T is applied to the remaining
      columns of those rows.
  H5  The last block is ragged (b_i = n - s).
Output in the dgeqp3 layout: R on and above the diagonal, the reflector
vectors (v(0) = 1 implied) below it, tau (n) and jpvt (n) with
A[:, jpvt] = Q R, Q = H_0 H_1 ... H_{n-1}.
"""
from __future__ import annotations

import numpy as np

from .randutv_oracle import householder_qr, householder_reflector, sketch_block  # noqa: F401


def cpqr_pivots(Y: np.ndarray, k: int) -> list:
    """Columns chosen by k steps of Householder CPQR of Y (reading H2)."""
    Y = np.array(Y, dtype=np.float64, copy=True)
    rows, cols = Y.shape
    used = np.zeros(cols, dtype=bool)
    J = []
    for t in range(min(k, rows, cols)):
        norms = np.full(cols, -1.0)
        live = ~used
        norms[live] = np.sum(Y[t:, live] ** 2, axis=0)
        p = int(np.argmax(norms))  # first (lowest index) maximum
        J.append(p)
        used[p] = True
        v, tau, _ = householder_reflector(Y[t:, p])
        if tau != 0.0:
            rest = np.nonzero(~used)[0]
            w = v @ Y[t:, rest]
            Y[t:, rest] -= tau * np.outer(v, w)
    return J


def swap_permutation(J, ncols: int) -> np.ndarray:
    """Local permutation idx (position -> original column) from exchanging the
    column holding J[t] with position t, t = 0, 1, ... (reading H3)."""
    idx = np.arange(ncols)
    where = np.arange(ncols)
    for t, c in enumerate(J):
        p = where[c]
        a = idx[t]
        idx[t], idx[p] = c, a
        where[c], where[a] = t, p
    return idx


def hqrrp(A: np.ndarray, b: int, seed: int = 0):
    """Returns (F, tau, jpvt): F holds R and the reflectors (dgeqp3 layout)."""
    F = np.array(A, dtype=np.float64, order="F", copy=True)
    m, n = F.shape
    if m < n:
        raise ValueError("hqrrp needs m >= n")
    tau = np.zeros(n)
    jpvt = np.arange(n)
    s = 0
    i = 0
    while s < n:
        bi = min(b, n - s)
        G = sketch_block(seed, i, m - s, bi)          # (m - s) x b_i; G^(i) is its transpose
        Y = G.T @ F[s:, s:]                           # b_i x (n - s)
        idx = swap_permutation(cpqr_pivots(Y, bi), n - s)
        F[:, s:] = F[:, s:][:, idx]
        jpvt[s:] = jpvt[s:][idx]
        W, t, R = householder_qr(F[s:, s:s + bi])
        tau[s:s + bi] = t
        C = F[s:, s + bi:]
        for j in range(bi):  # C <- H_{b_i-1} ... H_0 C = Q22^T C
            if t[j] != 0.0:
                C[j:, :] -= t[j] * np.outer(W[j:, j], W[j:, j] @ C[j:, :])
        F[s:, s + bi:] = C
        F[s:s + bi, s:s + bi] = R
        F[s + bi:, s:s + bi] = 0.0
        for j in range(bi):
            F[s + j + 1:, s + j] = W[j + 1:, j]
        s += bi
        i += 1
    return F, tau, jpvt


def explicit_q(F: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """The first n columns of Q = H_0 ... H_{n-1} from the dgeqp3 layout."""
    m, n = F.shape
    Q = np.eye(m)[:, :n]
    for j in reversed(range(n)):
        v = np.zeros(m)
        v[j] = 1.0
        v[j + 1:] = F[j + 1:, j]
        Q -= tau[j] * np.outer(v, v @ Q)
    return Q
