"""Plain FP64 CPU oracle for randUTV (A = U T V^T).  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  The GPU library never calls it and shares no code with it.

It follows the blocked randUTV of Heavner, Martinsson & Quintana-Orti,
"Computing rank-revealing factorizations of matrices stored out-of-core"
(arXiv 2002.06960): the method overview of Section 3.1 and the FLAME
formulation of Figure 2 ("randUTV adapted for algorithms-by-blocks"), with the
readings below where that figure is garbled or silent.  All arithmetic is real
FP64; matrix products use numpy's BLAS (a library primitive), everything else
(reflector generation, block-reflector factor, Jacobi SVD, the step loop) is
written out here.

Readings of the paper taken here (each also listed in the design notes):
  R1  The right transform of each step updates ALL m rows of the current
      column range, T(:, s:n) <- T(:, s:n) V^, as required by
      T^(i) = U^(i)* T^(i-1) V^(i) (Section 3.1) and by the per-step
      description "T <- T V^(0)" (Section 3.2.2); Figure 2 shows only the
      bottom-right 2x2 partition, which would not leave A = U T V^T.
  R2  The left update in Figure 2 is dimensionally garbled; it is read as
      C <- H_U^T C = C - W_U T_U^T W_U^T C with H_U = I - W_U T_U W_U^T.
  R3  "V_1 / U_1 has b rows" in Figure 2 means b columns.
  R4  The loop runs while n(A_TL) < n(A) with b_i = min(b, n - s) (Figure 2's
      guard on rows never ends when m > n).
  R5  Step i (0-based) draws G(i) of size (m - s) x b_i, s = i*b.
  R6  The sketch is i.i.d. N(0,1), drawn from Philox4x64-10 (Salmon et al.,
      SC'11) with key (seed, i) and counter (k, 0, 0, 0) for block k; each
      block's four 64-bit words give four normals by Box-Muller
      (z0 = r cos(2 pi u1), z1 = r sin(2 pi u1), r = sqrt(-2 ln u0),
      u0 = ((x0 >> 11) + 1) 2^-53 in (0, 1], u1 = (x1 >> 11) 2^-53 in [0, 1));
      normals fill G(i) in column-major order.
  R7  "unpivoted QR" is Householder QR with LAPACK dlarfg conventions and the
      forward column-wise compact-WY factor of dlarft.
  R8  The b x b SVD is one-sided Jacobi (round-robin ordering, rotate when
      |w_j.w_k| > b*u*|w_j||w_k|, at most 30 sweeps); d >= 0 descending (ties
      keep column order); u_j = w_j / d_j, completed by Gram-Schmidt over
      e_1, e_2, ... when d_j == 0; each pair (u_j, v_j) is negated if the
      largest-magnitude entry of v_j (lowest index on ties) is negative.
  R9  No re-orthonormalisation between power-iteration products
      (Section 3.1's formula is a plain product).
  R10 The last step is processed like every other (sketch included), as
      Figure 2 does.

Parity pins (tests/test_oracle.py): dgeqrf / dgeqrt (LAPACK) for the
reflectors and the WY factor, explicit reflector products, numpy.linalg.svd and
a tiny brute-force Jacobi for the SVD, Philox known-answer vectors and
distribution tests for the sketch, and randUTV's invariants and special cases
(single step = SVD, orthogonal input, zero input, rank-deficient input, the
step-0 range-finder closed form).  The rank-revealing quality of T (how close
|T_jj| is to sigma_j) is not fixed by the paper's surviving text: parity
unpinned, reported only.
"""
from __future__ import annotations

import math

import numpy as np

U_ROUNDOFF = 2.0 ** -53
JACOBI_MAX_SWEEPS = 30


# ----------------------------------------------------------------------------
# Random sketch G(i) (Section 3.1: "i.i.d. entries drawn from the standard
# normal distribution"; generator fixed by reading R6)
# ----------------------------------------------------------------------------
def philox_blocks(seed: int, step: int, nblocks: int) -> np.ndarray:
    """Raw Philox4x64-10 output, blocks k = 0..nblocks-1 -> (nblocks, 4) uint64.

    numpy's Philox bit generator is the published Philox4x64-10; it increments
    the counter before each block, so starting from all-ones wraps the first
    block to counter (0, 0, 0, 0).
    """
    if nblocks == 0:
        return np.zeros((0, 4), dtype=np.uint64)
    ones = np.array([2**64 - 1] * 4, dtype=np.uint64)
    key = np.array([seed & (2**64 - 1), step & (2**64 - 1)], dtype=np.uint64)
    bg = np.random.Philox(counter=ones, key=key)
    return bg.random_raw(4 * nblocks).reshape(nblocks, 4)


def sketch_block(seed: int, step: int, rows: int, cols: int) -> np.ndarray:
    """G(step), rows x cols, i.i.d. N(0,1) per reading R6 (column-major fill)."""
    count = rows * cols
    nblocks = (count + 3) // 4
    x = philox_blocks(seed, step, nblocks)
    two53 = 2.0 ** -53
    u0a = ((x[:, 0] >> np.uint64(11)).astype(np.float64) + 1.0) * two53
    u1a = (x[:, 1] >> np.uint64(11)).astype(np.float64) * two53
    u0b = ((x[:, 2] >> np.uint64(11)).astype(np.float64) + 1.0) * two53
    u1b = (x[:, 3] >> np.uint64(11)).astype(np.float64) * two53
    ra = np.sqrt(-2.0 * np.log(u0a))
    rb = np.sqrt(-2.0 * np.log(u0b))
    z = np.empty((nblocks, 4))
    z[:, 0] = ra * np.cos(2.0 * math.pi * u1a)
    z[:, 1] = ra * np.sin(2.0 * math.pi * u1a)
    z[:, 2] = rb * np.cos(2.0 * math.pi * u1b)
    z[:, 3] = rb * np.sin(2.0 * math.pi * u1b)
    return z.reshape(-1)[:count].reshape(cols, rows).T.copy(order="F")


# ----------------------------------------------------------------------------
# Householder QR (reading R7): reflector H = I - tau v v^T, v(0) = 1
# ----------------------------------------------------------------------------
def householder_reflector(x: np.ndarray):
    """dlarfg: returns (v, tau, beta) with H x = beta e_1, H = I - tau v v^T."""
    x = np.asarray(x, dtype=np.float64)
    alpha = float(x[0])
    v = np.zeros_like(x)
    v[0] = 1.0
    xnorm = float(np.linalg.norm(x[1:])) if x.shape[0] > 1 else 0.0
    if xnorm == 0.0:
        return v, 0.0, alpha
    beta = -math.copysign(math.hypot(alpha, xnorm), 1.0 if alpha >= 0.0 else -1.0)
    tau = (beta - alpha) / beta
    v[1:] = x[1:] / (alpha - beta)
    return v, tau, beta


def householder_qr(A: np.ndarray):
    """Unblocked Householder QR of an m x k matrix (m >= k), column by column.

    Returns W (m x k, explicit unit lower trapezoidal reflector vectors),
    tau (k,) and R (k x k upper triangular), with
    A = H_0 H_1 ... H_{k-1} [R; 0].
    """
    A = np.array(A, dtype=np.float64, order="F", copy=True)
    m, k = A.shape
    if m < k:
        raise ValueError("householder_qr needs m >= k")
    W = np.zeros((m, k))
    tau = np.zeros(k)
    for j in range(k):
        v, t, beta = householder_reflector(A[j:, j])
        W[j:, j] = v
        tau[j] = t
        if j + 1 < k and t != 0.0:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= t * np.outer(v, w)
        A[j, j] = beta
        A[j + 1:, j] = 0.0
    return W, tau, np.triu(A[:k, :])


def block_reflector_T(W: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Forward column-wise compact-WY factor (dlarft):
    H_0 H_1 ... H_{k-1} = I - W T W^T with T upper triangular."""
    k = tau.shape[0]
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = tau[j]
        if j > 0:
            T[:j, j] = -tau[j] * (T[:j, :j] @ (W[:, :j].T @ W[:, j]))
    return T


# ----------------------------------------------------------------------------
# b x b SVD by one-sided Jacobi (reading R8)
# ----------------------------------------------------------------------------
def round_robin_pairs(n: int):
    """Round-robin tournament: n-1 rounds (n even) of n/2 disjoint pairs (j<k)
    covering every pair once.  Odd n gets a dummy player n that sits out."""
    players = list(range(n + (n % 2)))
    p = len(players)
    rounds = []
    for _ in range(p - 1):
        pairs = []
        for t in range(p // 2):
            a, c = players[t], players[p - 1 - t]
            if a < n and c < n:
                pairs.append((min(a, c), max(a, c)))
        rounds.append(pairs)
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_svd(R: np.ndarray, max_sweeps: int = JACOBI_MAX_SWEEPS):
    """One-sided Jacobi SVD of a square matrix: R = Us diag(d) Vs^T.

    Returns (Us, d, Vs, sweeps, converged).
    """
    Wm = np.array(R, dtype=np.float64, copy=True)
    nb = Wm.shape[1]
    Vs = np.eye(nb)
    tol = nb * U_ROUNDOFF
    rounds = round_robin_pairs(nb)
    sweeps = 0
    converged = nb <= 1
    while not converged and sweeps < max_sweeps:
        sweeps += 1
        rotated = False
        for pairs in rounds:
            if not pairs:
                continue
            J = np.array([a for a, _ in pairs])
            K = np.array([c for _, c in pairs])
            wj, wk = Wm[:, J], Wm[:, K]
            alpha = np.einsum("ij,ij->j", wj, wj)
            beta = np.einsum("ij,ij->j", wk, wk)
            gamma = np.einsum("ij,ij->j", wj, wk)
            act = np.abs(gamma) > tol * np.sqrt(alpha) * np.sqrt(beta)
            if not act.any():
                continue
            rotated = True
            J, K = J[act], K[act]
            alpha, beta, gamma = alpha[act], beta[act], gamma[act]
            zeta = (beta - alpha) / (2.0 * gamma)
            t = np.sign(zeta) / (np.abs(zeta) + np.sqrt(1.0 + zeta * zeta))
            t[zeta == 0.0] = 1.0
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = c * t
            for M in (Wm, Vs):
                mj, mk = M[:, J].copy(), M[:, K].copy()
                M[:, J] = c * mj - s * mk
                M[:, K] = s * mj + c * mk
        if not rotated:
            converged = True
    d = np.sqrt(np.einsum("ij,ij->j", Wm, Wm))
    order = np.argsort(-d, kind="stable")
    d, Wm, Vs = d[order], Wm[:, order], Vs[:, order]
    Us = np.zeros_like(Wm)
    for j in range(nb):
        if d[j] > 0.0:
            Us[:, j] = Wm[:, j] / d[j]
    # complete U where d_j == 0: Gram-Schmidt over e_1, e_2, ... (twice, for
    # orthogonality), taking the first candidates with a non-negligible residual
    cand = 0
    for j in range(nb):
        if d[j] > 0.0:
            continue
        while cand < nb:
            e = np.zeros(nb)
            e[cand] = 1.0
            cand += 1
            for _ in range(2):
                e -= Us @ (Us.T @ e)
            ne = np.linalg.norm(e)
            if ne > 0.5:
                Us[:, j] = e / ne
                break
    # sign rule: largest-magnitude entry of v_j positive
    for j in range(nb):
        idx = int(np.argmax(np.abs(Vs[:, j])))
        if Vs[idx, j] < 0.0:
            Vs[:, j] = -Vs[:, j]
            Us[:, j] = -Us[:, j]
    return Us, d, Vs, sweeps, converged


# ----------------------------------------------------------------------------
# randUTV (Section 3.1; Figure 2 with readings R1-R10)
# ----------------------------------------------------------------------------
def randutv(A: np.ndarray, b: int, q: int, seed: int = 0, build_u: bool = True,
            build_v: bool = True, return_info: bool = False, max_steps: int | None = None):
    """Blocked randUTV: A = U T V^T with U, V orthogonal and T upper triangular.

    A: m x n FP64 with m >= n; b: block size (clamped to n); q: power steps.
    Returns (U, T, V) (U or V None when not built) and optionally an info dict
    with per-step Jacobi sweep counts.  max_steps stops after that many block
    steps (a partial factorization, still A = U T V^T; used to time a bounded
    sample of a large problem).
    """
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("randUTV needs m >= n")
    if b < 1 or q < 0:
        raise ValueError("need b >= 1 and q >= 0")
    T = np.array(A, order="F", copy=True)
    U = np.eye(m, order="F") if build_u else None
    V = np.eye(n, order="F") if build_v else None
    sweeps = []
    s, i = 0, 0
    while s < n and (max_steps is None or i < max_steps):
        bi = min(b, n - s)
        e = s + bi
        # --- right transform: V^ from the powered sketch (Section 3.1)
        B = T[s:, s:]
        G = sketch_block(seed, i, m - s, bi)
        Y = B.T @ G
        for _ in range(q):
            Y = B.T @ (B @ Y)
        WV, tauV, _ = householder_qr(Y)            # R_trash discarded
        TV = block_reflector_T(WV, tauV)
        T[:, s:] -= (T[:, s:] @ WV) @ TV @ WV.T     # all m rows (R1)
        if V is not None:
            V[:, s:] -= (V[:, s:] @ WV) @ TV @ WV.T
        # --- left transform: U^ from the QR of the current column block
        WU, tauU, R = householder_qr(T[s:, s:e])
        TU = block_reflector_T(WU, tauU)
        if e < n:
            T[s:, e:] -= WU @ (TU.T @ (WU.T @ T[s:, e:]))   # (R2)
        if U is not None:
            U[:, s:] -= (U[:, s:] @ WU) @ TU @ WU.T
        T[s:, s:e] = 0.0
        # --- small SVD of the b_i x b_i triangular block
        Us, d, Vs, nsw, ok = jacobi_svd(R)
        sweeps.append(nsw)
        if not ok:
            raise RuntimeError(f"Jacobi SVD did not converge at step {i}")
        T[s:e, s:e] = np.diag(d)
        if s > 0:
            T[:s, s:e] = T[:s, s:e] @ Vs
        if e < n:
            T[s:e, e:] = Us.T @ T[s:e, e:]
        if V is not None:
            V[:, s:e] = V[:, s:e] @ Vs
        if U is not None:
            U[:, s:e] = U[:, s:e] @ Us
        s, i = e, i + 1
    if return_info:
        return U, T, V, {"sweeps": sweeps, "steps": i}
    return U, T, V


def truncate(U: np.ndarray, T: np.ndarray, V: np.ndarray, k: int) -> np.ndarray:
    """Rank-k truncation A_k = U(:, 0:k) T(0:k, :) V^T (Section 1.1)."""
    return U[:, :k] @ (T[:k, :] @ V.T)


# ----------------------------------------------------------------------------
# Flop counts used to express throughput
# ----------------------------------------------------------------------------
def flops_std(m: int, n: int, q: int, build_u: bool = True, build_v: bool = True) -> float:
    """Leading-order randUTV flop count, summed term by term over the step list:
    sketch + q power steps (1+2q)(m n^2 - n^3/3); right update of all of T
    2 m n^2; left update 2 m n^2 - 2 n^3/3; V 2 n^3; U 4 m^2 n - 2 m n^2."""
    m, n = float(m), float(n)
    f = (1 + 2 * q) * (m * n * n - n ** 3 / 3.0) + 2 * m * n * n + (2 * m * n * n - 2 * n ** 3 / 3.0)
    if build_v:
        f += 2 * n ** 3
    if build_u:
        f += 4 * m * m * n - 2 * m * n * n
    return f


def flops_exact(m: int, n: int, b: int, q: int, build_u: bool = True, build_v: bool = True,
                max_steps: int | None = None) -> float:
    """Exact product count of the step list as computed here (GEMM-shaped work
    2*M*N*K per product, Householder QR 2 r c^2 - 2 c^3/3, T factor r c^2,
    small SVD applies).  Jacobi rotations are not counted."""
    f = 0.0
    s = 0
    steps = 0
    while s < n and (max_steps is None or steps < max_steps):
        steps += 1
        bi = min(b, n - s)
        mi, ni = m - s, n - s
        f += 2.0 * mi * ni * bi * (1 + 2 * q)          # sketch + power products
        f += 2.0 * ni * bi * bi - 2.0 * bi ** 3 / 3.0  # QR(Y)
        f += ni * bi * bi                              # T_V
        f += 2.0 * m * ni * bi * 2 + 2.0 * m * bi * bi  # right update of T
        if build_v:
            f += 2.0 * n * ni * bi * 2 + 2.0 * n * bi * bi
        f += 2.0 * mi * bi * bi - 2.0 * bi ** 3 / 3.0  # panel QR
        f += mi * bi * bi                              # T_U
        f += 2.0 * mi * (ni - bi) * bi * 2 + 2.0 * bi * bi * (ni - bi)  # left update
        if build_u:
            f += 2.0 * m * mi * bi * 2 + 2.0 * m * bi * bi
        f += 2.0 * bi * bi * (s + (ni - bi))           # A01 Vs, Us^T A12
        if build_v:
            f += 2.0 * n * bi * bi
        if build_u:
            f += 2.0 * m * bi * bi
        s += bi
    return f
