"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

Each check ties one part of the oracle to something other than itself:
LAPACK routines (dgeqrf, dgeqrt), numpy's SVD, explicit reflector products,
published Philox known-answer vectors, distribution tests, and the invariants /
special cases / closed forms of the rank-revealing UTV factorization
(Section 1.1 problem statement, Section 3.1 method).
"""
import math
import os

import numpy as np
import pytest
import scipy.linalg.lapack as lapack
import scipy.stats

import oracle
from oracle import randutv_oracle as ro
from randutv_inputs import spectrum, make_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _invariants(A, U, T, V, b):
    m, n = A.shape
    nA = np.linalg.norm(A)
    res = np.linalg.norm(A - U @ T @ V.T) / (nA if nA > 0 else 1.0)
    ou = np.abs(U.T @ U - np.eye(m)).max()
    ov = np.abs(V.T @ V - np.eye(n)).max()
    lower = np.abs(np.tril(T, -1)).max() if m > 1 else 0.0
    offdiag = 0.0
    descending = True
    for s in range(0, n, b):
        e = min(n, s + b)
        D = T[s:e, s:e]
        offdiag = max(offdiag, np.abs(D - np.diag(np.diag(D))).max())
        d = np.diag(D)
        descending &= bool(np.all(d >= 0) and np.all(np.diff(d) <= 0))
    return res, ou, ov, lower, offdiag, descending


# --------------------------------------------------------------------------- sketch
def test_philox_known_answer_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x64_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        ctr = [int(x, 16) for x in r[0:4]]
        key = [int(x, 16) for x in r[4:6]]
        want = [int(x, 16) for x in r[6:10]]
        # block k of the sketch stream uses counter (k, 0, 0, 0): compare the
        # oracle's stream where the KAT counter has that form, otherwise use the
        # generator directly with the counter pre-decremented
        v = sum(c << (64 * i) for i, c in enumerate(ctr))
        v = (v - 1) % (1 << 256)
        pre = np.array([(v >> (64 * i)) & (2**64 - 1) for i in range(4)], dtype=np.uint64)
        got = np.random.Philox(counter=pre, key=np.array(key, dtype=np.uint64)).random_raw(4)
        assert [int(x) for x in got] == want
    # the oracle's own stream: block 0 of (seed 0, step 0) is the all-zero KAT
    blk = ro.philox_blocks(0, 0, 1)[0]
    assert [int(x) for x in blk] == [int(x, 16) for x in rows[0][6:10]]
    # and seed/step all-ones with block index 2^64-1 is not reachable; check the
    # key order instead: key = (seed, step)
    b2 = ro.philox_blocks(0xFFFFFFFFFFFFFFFF, 0xFFFFFFFFFFFFFFFF, 2)
    ref = np.random.Philox(counter=np.array([2**64 - 1] * 4, dtype=np.uint64),
                           key=np.array([2**64 - 1] * 2, dtype=np.uint64)).random_raw(8)
    assert np.array_equal(b2.reshape(-1), ref)


def test_sketch_is_standard_normal():
    G = ro.sketch_block(7, 3, 1000, 1000)
    z = G.reshape(-1)
    assert abs(z.mean()) < 5.0 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5.0 * math.sqrt(2.0 / z.size)
    ks = scipy.stats.kstest(z, "norm")
    assert ks.pvalue > 1e-4
    # fourth moment of N(0,1) is 3
    assert abs((z**4).mean() - 3.0) < 0.05


def test_sketch_streams_independent_and_layout():
    a = ro.sketch_block(0, 0, 300, 40)
    b = ro.sketch_block(0, 1, 300, 40)
    c = ro.sketch_block(1, 0, 300, 40)
    for x, y in ((a, b), (a, c), (b, c)):
        r = np.corrcoef(x.reshape(-1), y.reshape(-1))[0, 1]
        assert abs(r) < 5.0 / math.sqrt(x.size)
    # column-major fill: a taller draw with the same (seed, step) starts with
    # the same numbers in the same linear order
    t = ro.sketch_block(0, 0, 12000, 1)
    assert np.array_equal(t[:300, 0], a[:, 0])
    assert np.array_equal(t[300:600, 0], a[:, 1])
    # columns uncorrelated
    C = np.corrcoef(ro.sketch_block(5, 2, 4000, 8).T)
    assert np.abs(C - np.eye(8)).max() < 0.08


# --------------------------------------------------------------------------- Householder
@pytest.mark.parametrize("shape", [(7, 3), (64, 64), (200, 37), (513, 64)])
def test_householder_qr_matches_dgeqrf(shape):
    rng = np.random.default_rng(shape[0] * 31 + shape[1])
    A = rng.standard_normal(shape)
    W, tau, R = ro.householder_qr(A)
    qr, tau_l, _, info = lapack.dgeqrf(np.asfortranarray(A))
    assert info == 0
    k = shape[1]
    Wl = np.tril(qr[:, :k], -1)
    Wl[np.arange(k), np.arange(k)] = 1.0
    np.testing.assert_allclose(tau, tau_l, rtol=0, atol=1e-14)
    np.testing.assert_allclose(W, Wl, rtol=0, atol=1e-12)
    np.testing.assert_allclose(R, np.triu(qr[:k, :k]), rtol=0, atol=1e-12 * np.abs(R).max())


def test_householder_special_cases():
    # zero column below the diagonal: tau = 0, beta = alpha (H = I)
    v, tau, beta = ro.householder_reflector(np.array([-3.0, 0.0, 0.0]))
    assert tau == 0.0 and beta == -3.0 and np.array_equal(v, [1.0, 0.0, 0.0])
    # alpha = 0 takes sign +1: beta = -|x|
    v, tau, beta = ro.householder_reflector(np.array([0.0, 3.0, 4.0]))
    assert beta == -5.0 and abs(tau - 1.0) < 1e-15
    # the reflector maps x to beta e_1
    x = np.array([1.0, -2.0, 0.5, 3.0])
    v, tau, beta = ro.householder_reflector(x)
    Hx = x - tau * v * (v @ x)
    np.testing.assert_allclose(Hx, [beta, 0, 0, 0], atol=1e-15)
    # QR of an exactly zero matrix: every tau = 0, R = 0
    W, tau, R = ro.householder_qr(np.zeros((6, 3)))
    assert np.all(tau == 0) and np.all(R == 0)


@pytest.mark.parametrize("shape", [(9, 4), (150, 32), (300, 64)])
def test_block_reflector_matches_dgeqrt_and_product(shape):
    rng = np.random.default_rng(shape[0])
    A = rng.standard_normal(shape)
    W, tau, _ = ro.householder_qr(A)
    Tf = ro.block_reflector_T(W, tau)
    m, k = shape
    # LAPACK dgeqrt with one block computes the same forward column-wise factor
    _, Tl, info = lapack.dgeqrt(k, np.asfortranarray(A))
    assert info == 0
    np.testing.assert_allclose(Tf, np.triu(Tl), rtol=0, atol=1e-12 * np.abs(Tl).max())
    # explicit product of the reflectors
    H = np.eye(m)
    for j in range(k):
        H = H @ (np.eye(m) - tau[j] * np.outer(W[:, j], W[:, j]))
    np.testing.assert_allclose(np.eye(m) - W @ Tf @ W.T, H, rtol=0, atol=1e-13)


# --------------------------------------------------------------------------- Jacobi SVD
def test_round_robin_covers_every_pair_once():
    for n in (1, 2, 5, 8, 64):
        seen = []
        for pairs in ro.round_robin_pairs(n):
            flat = [x for p in pairs for x in p]
            assert len(flat) == len(set(flat))  # disjoint within a round
            seen += pairs
        assert sorted(seen) == [(j, k) for j in range(n) for k in range(j + 1, n)]


@pytest.mark.parametrize("n,kind", [(16, "rand"), (64, "tri"), (128, "graded"), (33, "tri")])
def test_jacobi_svd_matches_numpy(n, kind):
    rng = np.random.default_rng(n)
    R = rng.standard_normal((n, n))
    if kind in ("tri", "graded"):
        # triangular factors of the kind randUTV produces: well conditioned up
        # to a column scaling (a random triangular matrix is exponentially
        # ill-conditioned and needs many more sweeps)
        R = np.triu(R) / math.sqrt(n) + np.eye(n)
    if kind == "graded":
        R = R * (10.0 ** -np.linspace(0, 10, n))[None, :]
    Us, d, Vs, sweeps, ok = ro.jacobi_svd(R)
    assert ok and sweeps <= ro.JACOBI_MAX_SWEEPS
    sv = np.linalg.svd(R, compute_uv=False)
    np.testing.assert_allclose(d, sv, rtol=0, atol=4e-15 * n * sv[0])
    assert np.all(np.diff(d) <= 0) and np.all(d >= 0)
    np.testing.assert_allclose(Us.T @ Us, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(Vs.T @ Vs, np.eye(n), atol=1e-13)
    np.testing.assert_allclose(Us @ np.diag(d) @ Vs.T, R, atol=1e-13 * sv[0])
    # sign rule: the largest-magnitude entry of each v_j is positive
    idx = np.argmax(np.abs(Vs), axis=0)
    assert np.all(Vs[idx, np.arange(n)] > 0)


def test_jacobi_svd_two_by_two_closed_form():
    # [[a, b], [0, c]]: singular values from the 2x2 closed form
    a, b, c = 3.0, 4.0, 1.0
    Us, d, Vs, _, _ = ro.jacobi_svd(np.array([[a, b], [0.0, c]]))
    fro2 = a * a + b * b + c * c
    det = abs(a * c)
    s1 = math.sqrt((fro2 + math.sqrt(fro2 * fro2 - 4 * det * det)) / 2)
    s2 = det / s1
    np.testing.assert_allclose(d, [s1, s2], rtol=1e-15)


def test_jacobi_svd_degenerate_inputs():
    # zero matrix: no rotation, identity vectors (Gram-Schmidt completion)
    Us, d, Vs, sweeps, ok = ro.jacobi_svd(np.zeros((5, 5)))
    assert ok and np.all(d == 0) and np.array_equal(Us, np.eye(5)) and np.array_equal(Vs, np.eye(5))
    # identity: already orthogonal, ties keep column order
    Us, d, Vs, _, _ = ro.jacobi_svd(np.eye(6))
    assert np.array_equal(Us, np.eye(6)) and np.array_equal(Vs, np.eye(6)) and np.all(d == 1)
    # exact rank deficiency (zero column): U completed to an orthogonal matrix
    rng = np.random.default_rng(0)
    R = np.triu(rng.standard_normal((8, 8)))
    R[:, 3] = 0.0
    Us, d, Vs, _, ok = ro.jacobi_svd(R)
    assert ok and d[-1] == 0.0
    np.testing.assert_allclose(Us.T @ Us, np.eye(8), atol=1e-14)
    np.testing.assert_allclose(Us @ np.diag(d) @ Vs.T, R, atol=1e-13)


# --------------------------------------------------------------------------- randUTV
@pytest.mark.parametrize("m,n,b,q,kind", [
    (96, 96, 16, 1, "log8"),
    (100, 70, 16, 2, "exp"),      # tall, ragged last block (70 = 4*16 + 6)
    (128, 128, 32, 0, "iid"),
    (64, 64, 64, 1, "exp"),       # single step
    (40, 40, 7, 2, "log8"),       # odd block size
])
def test_randutv_invariants(m, n, b, q, kind):
    A = make_matrix(kind, m, n, seed=3)
    U, T, V = ro.randutv(A, b, q, seed=11)
    res, ou, ov, lower, offdiag, desc = _invariants(A, U, T, V, b)
    assert res <= 1e-13 and ou <= 1e-13 and ov <= 1e-13
    assert lower == 0.0 and offdiag == 0.0 and desc


def test_randutv_config1_invariants():
    """512 x 512, s_i = 10^(-8(i-1)/511), b = 64, q = 1, sketch seed 0."""
    A = make_matrix("log8", 512, seed=0)
    U, T, V = ro.randutv(A, 64, 1, seed=0)
    res, ou, ov, lower, offdiag, desc = _invariants(A, U, T, V, 64)
    assert res <= 1e-13 and ou <= 1e-13 and ov <= 1e-13
    assert lower == 0.0 and offdiag == 0.0 and desc
    sv = spectrum("log8", 512)
    # interlacing of the first block (d_j <= sigma_j) and Eckart-Young tails
    d0 = np.diag(T)[:64]
    assert np.all(d0 <= sv[:64] * (1 + 1e-12))
    nA = np.linalg.norm(A)
    for k in (64, 128, 256, 448):
        tail = np.linalg.norm(T[k:, k:])
        assert tail >= math.sqrt(np.sum(sv[k:] ** 2)) - 1e-13 * nA
    # T and U, V built or not: T is the same
    _, T2, _ = ro.randutv(A, 64, 1, seed=0, build_u=False, build_v=False)
    assert np.array_equal(T, T2)


def test_single_step_is_the_svd():
    """b >= n: one step, T = [diag(sigma(A)); 0] (checked against numpy's SVD)."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 20))
    U, T, V = ro.randutv(A, 64, 1, seed=0)
    sv = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(np.diag(T), sv, rtol=0, atol=1e-14 * sv[0] * 20)
    Tz = T.copy()
    Tz[np.arange(20), np.arange(20)] = 0.0
    assert np.abs(Tz).max() == 0.0


def test_orthogonal_input_gives_identity_T():
    Q = np.linalg.qr(np.random.default_rng(2).standard_normal((48, 48)))[0]
    U, T, V = ro.randutv(Q, 16, 1, seed=0)
    np.testing.assert_allclose(T, np.eye(48), atol=1e-13)


def test_zero_input_is_exact():
    U, T, V = ro.randutv(np.zeros((20, 12)), 5, 2, seed=4)
    assert np.array_equal(T, np.zeros((20, 12)))
    assert np.array_equal(U, np.eye(20)) and np.array_equal(V, np.eye(12))


def test_rank_deficient_tail():
    rng = np.random.default_rng(5)
    r = 10
    A = rng.standard_normal((60, r)) @ rng.standard_normal((r, 60))
    U, T, V = ro.randutv(A, 16, 2, seed=0)
    nA = np.linalg.norm(A)
    assert np.linalg.norm(T[r:, r:]) <= 1e-13 * nA
    res, ou, ov, *_ = _invariants(A, U, T, V, 16)
    assert res <= 1e-13 and ou <= 1e-13 and ov <= 1e-13


@pytest.mark.parametrize("q", [0, 1, 2])
def test_step0_range_finder_closed_form(q):
    """After step 0: d(0:b) = sigma(A orth(Y0)) with Y0 = (A^T A)^q A^T G(0), and
    the rank-b truncation is the range-finder projection Q Q^T A with
    Q = orth((A A^T)^(q+1) G(0)) (Section 3.1).  Computed with numpy's QR/SVD,
    not with the oracle's Householder or Jacobi code."""
    A = make_matrix("exp", 150, 120, seed=1)
    b = 24
    U, T, V = ro.randutv(A, b, q, seed=9)
    G0 = ro.sketch_block(9, 0, 150, b)
    Y0 = A.T @ G0
    for _ in range(q):
        Y0 = A.T @ (A @ Y0)
    Qy = np.linalg.qr(Y0)[0]
    d_ref = np.linalg.svd(A @ Qy, compute_uv=False)
    np.testing.assert_allclose(np.diag(T)[:b], d_ref, rtol=0, atol=1e-13)
    Qa = np.linalg.qr(A @ Qy)[0]
    Ab = ro.truncate(U, T, V, b)
    np.testing.assert_allclose(Ab, Qa @ (Qa.T @ A), rtol=0, atol=1e-13)


def test_flop_counts():
    n, q = 1200, 2
    assert math.isclose(ro.flops_std(n, n, q), (24 + 4 * q) / 3.0 * n**3, rel_tol=1e-12)
    assert math.isclose(ro.flops_std(n, n, q, False, False), (12 + 4 * q) / 3.0 * n**3, rel_tol=1e-12)
    # the exact step sum exceeds the leading-order count by O(b/n)
    ex = ro.flops_exact(n, n, 64, q)
    assert 1.0 < ex / ro.flops_std(n, n, q) < 1.0 + 8 * 64 / n


# --------------------------------------------------------------------------- planted mistakes
def test_pins_catch_planted_mistakes(monkeypatch):
    """Plant plausible mistakes in the oracle (on the CPU) and check that the
    invariants reject each of them."""
    A = make_matrix("exp", 64, 64, seed=2)

    def res_of():
        U, T, V = ro.randutv(A, 16, 1, seed=0)
        return _invariants(A, U, T, V, 16)

    good = res_of()
    assert good[0] < 1e-13
    # 1) transposed compact-WY factor
    orig_T = ro.block_reflector_T
    monkeypatch.setattr(ro, "block_reflector_T", lambda W, t: orig_T(W, t).T)
    assert res_of()[0] > 1e-6 or res_of()[1] > 1e-6
    monkeypatch.setattr(ro, "block_reflector_T", orig_T)
    # 2) wrong sign of the reflector scalar
    orig_r = ro.householder_reflector

    def bad_reflector(x):
        v, tau, beta = orig_r(x)
        return v, -tau, beta

    monkeypatch.setattr(ro, "householder_reflector", bad_reflector)
    r = res_of()
    assert r[0] > 1e-6 or r[1] > 1e-6 or r[2] > 1e-6 or r[3] > 1e-6
    monkeypatch.setattr(ro, "householder_reflector", orig_r)
    # 3) SVD vectors swapped
    orig_j = ro.jacobi_svd
    monkeypatch.setattr(ro, "jacobi_svd", lambda R, **k: (lambda u, d, v, s, c: (v, d, u, s, c))(*orig_j(R)))
    assert res_of()[0] > 1e-6
    monkeypatch.setattr(ro, "jacobi_svd", orig_j)


# ----------------------------------------------------------------------------
# brute-force pin of the b x b SVD and of the single-step factorization
# ----------------------------------------------------------------------------
def _brute_force_singular_values(A):
    """Singular values of a tiny matrix as the n largest eigenvalues of the
    symmetric matrix [[0, A], [A^T, 0]] (its eigenvalues are +-sigma_i and
    zeros), found by the classical cyclic two-sided Jacobi eigenvalue method
    (symmetric 2 x 2 Schur rotations; Golub & Van Loan, Matrix Computations,
    Section 8.5) in plain Python loops.  Shares nothing with the oracle's
    one-sided Jacobi and does not square A."""
    m, n = A.shape
    N = m + n
    S = [[0.0] * N for _ in range(N)]
    for i in range(m):
        for j in range(n):
            S[i][m + j] = S[m + j][i] = float(A[i, j])
    total = sum(S[i][j] ** 2 for i in range(N) for j in range(N))
    for _ in range(60):
        off = sum(S[i][j] ** 2 for i in range(N) for j in range(N) if i != j)
        if off <= 1e-30 * total:
            break
        for p in range(N - 1):
            for q in range(p + 1, N):
                apq = S[p][q]
                if apq == 0.0:
                    continue
                th = (S[q][q] - S[p][p]) / (2.0 * apq)
                t = (1.0 if th >= 0.0 else -1.0) / (abs(th) + math.sqrt(1.0 + th * th))
                c = 1.0 / math.sqrt(1.0 + t * t)
                s = t * c
                for k in range(N):
                    a, b = S[k][p], S[k][q]
                    S[k][p], S[k][q] = c * a - s * b, s * a + c * b
                for k in range(N):
                    a, b = S[p][k], S[q][k]
                    S[p][k], S[q][k] = c * a - s * b, s * a + c * b
    return np.array(sorted((S[i][i] for i in range(N)), reverse=True)[:n])


@pytest.mark.parametrize("n,kind", [(1, "iid"), (2, "iid"), (5, "iid"), (9, "graded"), (16, "iid"),
                                    (16, "graded")])
def test_jacobi_svd_against_brute_force(n, kind):
    """The oracle's one-sided Jacobi singular values equal the brute-force
    two-sided Jacobi ones on tiny triangular blocks (as the b x b step sees them)."""
    rng = np.random.default_rng(40 + n)
    R = np.triu(rng.standard_normal((n, n)))
    if kind == "graded":
        R = R * np.logspace(0, -6, n)[None, :]
    _, d, _, _, ok = ro.jacobi_svd(R)
    assert ok
    sv = _brute_force_singular_values(R)
    np.testing.assert_allclose(d, sv, rtol=0, atol=1e-13 * sv[0])


@pytest.mark.parametrize("m,n,kind", [(12, 9, "iid"), (16, 16, "log8"), (7, 5, "exp"), (16, 13, "iid")])
def test_single_step_diag_T_against_brute_force(m, n, kind):
    """b >= n: one step, and |diag T| is the singular values of A; on tiny
    inputs they equal the brute-force ones.  With b < n the first block's
    |T_jj| interlace below sigma_j."""
    A = make_matrix(kind, m, n, seed=2)
    sv = _brute_force_singular_values(A)
    _, T, _ = ro.randutv(A, n + 3, 2, 0)
    np.testing.assert_allclose(np.abs(np.diag(T)), sv, rtol=0, atol=1e-13 * sv[0])
    b = max(1, n // 3)
    _, T2, _ = ro.randutv(A, b, 1, 0)
    d0 = np.abs(np.diag(T2))[:b]
    assert np.all(d0 <= sv[:b] * (1 + 1e-12) + 1e-15 * sv[0])
