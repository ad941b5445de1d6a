"""GPU checks of the individual kernels against the CPU oracle / numpy (FP64)."""
import itertools
import math

import numpy as np
import pytest

import paper_2002_06960_amd as pkg
from oracle import randutv_oracle as ro
from gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,step,rows,cols", [
    (0, 0, 512, 64), (7, 3, 777, 13), (2**63 + 5, 46, 12000, 256), (1, 1, 1, 1), (3, 2, 5, 3)])
def test_sketch_matches_oracle(seed, step, rows, cols):
    G = to_host(pkg.randutv_sketch(seed, step, rows, cols))
    R = ro.sketch_block(seed, step, rows, cols)
    # the Philox words are integers (bit-exact); log/cos/sin may differ in the last ulps
    assert np.abs(G - R).max() <= 1e-13 * max(1.0, np.abs(R).max())


GEMM_SHAPES = [(1, 1, 1), (37, 53, 29), (300, 257, 1000), (129, 65, 17), (2500, 256, 3000),
               (256, 2000, 2400), (700, 700, 256), (64, 64, 0)]


@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("M,N,K", GEMM_SHAPES)
def test_dgemm_matches_numpy(ta, tb, M, N, K):
    rng = np.random.default_rng(M * 7 + N * 3 + K)
    A = rng.standard_normal((K, M) if ta == "T" else (M, K))
    B = rng.standard_normal((N, K) if tb == "T" else (K, N))
    C0 = rng.standard_normal((M, N))
    opA = A.T if ta == "T" else A
    opB = B.T if tb == "T" else B
    for alpha, beta in ((1.0, 0.0), (-1.0, 1.0), (0.5, -2.0)):
        C = pkg.randutv_dgemm(ta, tb, alpha, to_dev(A), to_dev(B), beta, to_dev(C0))
        ref = alpha * (opA @ opB) + beta * C0
        bound = (abs(alpha) * (np.abs(opA) @ np.abs(opB)) + abs(beta) * np.abs(C0)) * (K + 2) * 2.0**-52
        err = np.abs(to_host(C) - ref)
        assert np.all(err <= bound + 1e-300), (alpha, beta, err.max())


def test_dgemm_large_skinny_split_k():
    """The sketch shape of the 12000 x 12000, b = 256 workload (split over K)."""
    rng = np.random.default_rng(0)
    A = rng.standard_normal((12000, 12000))
    G = rng.standard_normal((12000, 256))
    Y = to_host(pkg.randutv_dgemm("T", "N", 1.0, to_dev(A), to_dev(G)))
    ref = A.T @ G
    assert np.abs(Y - ref).max() <= 12000 * 2.0**-52 * (np.abs(A).T @ np.abs(G)).max()


def _reflectors(F):
    k = F.shape[1]
    W = np.tril(F[:, :k], -1)
    W[np.arange(k), np.arange(k)] = 1.0
    return W, np.triu(F[:k, :k])


# (333, 33), (4001, 200) and (97, 40): the last workgroup's slab has an odd
# number of rows (slabs are whole 16-row units), so its last row pair of the
# trailing sweep is shifted down by one row
@pytest.mark.parametrize("m,k", [(50, 7), (1000, 64), (4000, 128), (12000, 256), (256, 256),
                                 (16000, 64), (333, 33), (17, 1), (4001, 200), (97, 40)])
def test_geqrf_matches_oracle(m, k):
    rng = np.random.default_rng(m + k)
    A = rng.standard_normal((m, k))
    F, tau = pkg.randutv_geqrf(to_dev(A))
    Wg, Rg = _reflectors(to_host(F))
    Wo, tauo, Ro = ro.householder_qr(A)
    np.testing.assert_allclose(to_host(tau), tauo, rtol=0, atol=1e-13)
    np.testing.assert_allclose(Wg, Wo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(Rg, Ro, rtol=0, atol=1e-12 * np.abs(Ro).max())


def test_geqrf_degenerate_columns():
    # exactly zero sub-diagonal parts (tau = 0) and a zero column
    A = np.zeros((300, 20))
    A[:20, :20] = np.triu(np.arange(1.0, 401.0).reshape(20, 20))
    A[:, 5] = 0.0
    F, tau = pkg.randutv_geqrf(to_dev(A))
    Wo, tauo, Ro = ro.householder_qr(A)
    assert np.array_equal(to_host(tau), tauo)
    np.testing.assert_allclose(_reflectors(to_host(F))[1], Ro, atol=0)


def _restart_case(kind):
    rng = np.random.default_rng(7)
    m, k = 2000, 256
    if kind == "rank100":
        return rng.standard_normal((m, 100)) @ rng.standard_normal((100, k))
    if kind == "near_parallel":
        A = rng.standard_normal((m, k))
        for j in range(1, k, 2):
            A[:, j] = A[:, j - 1] + 1e-6 * rng.standard_normal(m)
        return A
    return rng.standard_normal((m, k)) * np.logspace(0, -12, k)  # graded column scales


@pytest.mark.parametrize("kind,rtol_r", [("rank100", 1e-12), ("near_parallel", 1e-8), ("graded", 1e-12)])
def test_geqrf_cancelling_columns(kind, rtol_r):
    """Panels whose columns cancel against the earlier reflectors: the leaf
    passes must stop at such columns and restart from a fresh Gram matrix.
    The factorization must stay exact (A = QR, Q orthogonal); R is compared
    with the oracle where it is well determined by the data."""
    A = _restart_case(kind)
    m, k = A.shape
    F, tau = pkg.randutv_geqrf(to_dev(A))
    Wg, Rg = _reflectors(to_host(F))
    taug = to_host(tau)
    T = ro.block_reflector_T(Wg, taug)
    Q = np.eye(m)[:, :k] - Wg @ (T @ Wg[:k, :].T)
    assert np.linalg.norm(A - Q @ Rg) <= 1e-13 * np.linalg.norm(A)
    assert np.abs(Q.T @ Q - np.eye(k)).max() <= 1e-13
    Wo, tauo, Ro = ro.householder_qr(A)
    np.testing.assert_allclose(Rg, Ro, rtol=0, atol=rtol_r * np.abs(Ro).max())


@pytest.mark.parametrize("m,k", [(500, 64), (12000, 256), (4000, 100), (40, 33)])
def test_larft_matches_oracle(m, k):
    rng = np.random.default_rng(k)
    A = rng.standard_normal((m, k))
    Wo, tauo, _ = ro.householder_qr(A)
    To = ro.block_reflector_T(Wo, tauo)
    F = Wo.copy()
    F[np.arange(k), np.arange(k)] = 123.0  # diagonal and upper part are ignored
    F[:k, :k] += np.triu(np.ones((k, k)), 1) * 7.0
    Tg = to_host(pkg.randutv_larft(to_dev(F), to_dev(tauo)))
    np.testing.assert_allclose(Tg, To, rtol=0, atol=1e-12 * np.abs(To).max())


def _svd_case(k, kind):
    rng = np.random.default_rng(k)
    if kind == "sep":  # well separated singular values, triangular like randUTV's R
        Q1 = np.linalg.qr(rng.standard_normal((k, k)))[0]
        Q2 = np.linalg.qr(rng.standard_normal((k, k)))[0]
        s = 1.0 - np.arange(k) / (2.0 * k)
        return np.linalg.qr(Q1 @ np.diag(s) @ Q2.T)[1]
    if kind == "graded":
        return (np.triu(rng.standard_normal((k, k))) / math.sqrt(k) + np.eye(k)) * (10.0 ** -np.linspace(0, 6, k))
    raise ValueError(kind)


@pytest.mark.parametrize("k,kind", [(256, "sep"), (64, "sep"), (33, "sep"), (128, "graded"), (224, "sep")])
def test_gesvj_matches_oracle(k, kind):
    R = _svd_case(k, kind)
    Us, d, Vs, sweeps = pkg.randutv_gesvj(to_dev(R))
    Uo, do, Vo, so, ok = ro.jacobi_svd(R)
    assert ok
    d = to_host(d)
    np.testing.assert_allclose(d, do, rtol=0, atol=4e-15 * k * do[0])
    if kind == "sep":
        np.testing.assert_allclose(to_host(Vs), Vo, rtol=0, atol=1e-11)
        np.testing.assert_allclose(to_host(Us), Uo, rtol=0, atol=1e-11)
    Ug, Vg = to_host(Us), to_host(Vs)
    assert np.abs(Ug.T @ Ug - np.eye(k)).max() < 1e-13
    assert np.abs(Vg.T @ Vg - np.eye(k)).max() < 1e-13
    assert np.abs(Ug @ np.diag(d) @ Vg.T - R).max() < 1e-13 * do[0]
    assert abs(sweeps - so) <= 2


def test_gesvj_degenerate():
    for R, expect in ((np.zeros((7, 7)), np.zeros(7)), (np.eye(9), np.ones(9))):
        Us, d, Vs, sweeps = pkg.randutv_gesvj(to_dev(R))
        k = R.shape[0]
        assert np.array_equal(to_host(d), expect)
        assert np.array_equal(to_host(Us), np.eye(k)) and np.array_equal(to_host(Vs), np.eye(k))
    rng = np.random.default_rng(0)
    R = np.triu(rng.standard_normal((8, 8)))
    R[:, 3] = 0.0
    Us, d, Vs, _ = pkg.randutv_gesvj(to_dev(R))
    Uo, do, Vo, _, _ = ro.jacobi_svd(R)
    assert to_host(d)[-1] == 0.0
    np.testing.assert_allclose(to_host(Us), Uo, atol=1e-12)


def test_gesvj_rejects_nonfinite():
    R = np.triu(np.ones((40, 40)))
    R[3, 7] = np.nan
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_gesvj(to_dev(R))
    assert e.value.code == 3


@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("M,N,K", [(37, 53, 29), (300, 257, 1000), (2500, 256, 3000), (700, 700, 256)])
def test_gemm_f32_matches_numpy(ta, tb, M, N, K):
    """FP64 operands rounded to FP32 and multiplied on the FP32 matrix cores:
    each product carries two roundings of the operands and at most K + 1 of the
    accumulation (2^-24 each), the FP64 epilogue adds beta C exactly enough."""
    rng = np.random.default_rng(M * 5 + N * 7 + K)
    A = rng.standard_normal((K, M) if ta == "T" else (M, K))
    B = rng.standard_normal((N, K) if tb == "T" else (K, N))
    C0 = rng.standard_normal((M, N))
    opA = A.T if ta == "T" else A
    opB = B.T if tb == "T" else B
    for alpha, beta in ((1.0, 0.0), (-1.0, 1.0)):
        C = pkg.randutv_dgemm(ta, tb, alpha, to_dev(A), to_dev(B), beta, to_dev(C0), f32=True)
        ref = alpha * (opA @ opB) + beta * C0
        bound = abs(alpha) * (np.abs(opA) @ np.abs(opB)) * (K + 4) * 2.0**-24 + abs(beta) * np.abs(C0) * 2.0**-50
        err = np.abs(to_host(C) - ref)
        assert np.all(err <= bound), (alpha, beta, (err / bound).max())
        # and it is not the FP64 result: the operands really are rounded
        if K >= 256:
            C64 = to_host(pkg.randutv_dgemm(ta, tb, alpha, to_dev(A), to_dev(B), beta, to_dev(C0)))
            assert np.abs(to_host(C) - C64).max() > 1e3 * 2.0**-52 * np.abs(ref).max()


@pytest.mark.parametrize("terms", [1, 3])
@pytest.mark.parametrize("ta,tb", list(itertools.product("NT", "NT")))
@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (37, 53, 29), (300, 257, 1000), (129, 65, 17),
                                   (2500, 256, 3000), (700, 700, 256), (64, 64, 0)])
def test_gemm_bf16_matches_numpy(terms, ta, tb, M, N, K):
    """FP64 operands on the BF16 matrix cores.  An operand x goes to FP32 (f,
    relative error 2^-24) and to BF16 (hi, 2^-8); with three terms the
    remainder f - hi (exact in FP32) is rounded to BF16 too (lo), and
    hi*hi + hi*lo + lo*hi misses r_a f_b + f_a r_b + lo_a lo_b with
    |r| <= 2^-16 |f|.  BF16 x BF16 products are exact in FP32; each MFMA adds
    into an FP32 accumulator, at most terms*K + 4 roundings of 2^-24."""
    rng = np.random.default_rng(M * 11 + N * 5 + K + terms)
    A = rng.standard_normal((K, M) if ta == "T" else (M, K))
    B = rng.standard_normal((N, K) if tb == "T" else (K, N))
    C0 = rng.standard_normal((M, N))
    opA = A.T if ta == "T" else A
    opB = B.T if tb == "T" else B
    absAB = np.abs(opA) @ np.abs(opB)
    rel = (2 * (2.0**-8 + 2.0**-24) + 2.0**-16) if terms == 1 else (3.1 * 2.0**-16 + 3 * 2.0**-24)
    for alpha, beta in ((1.0, 0.0), (-1.0, 1.0), (0.5, -2.0)):
        C = pkg.randutv_dgemm(ta, tb, alpha, to_dev(A), to_dev(B), beta, to_dev(C0), bf16_terms=terms)
        ref = alpha * (opA @ opB) + beta * C0
        bound = abs(alpha) * absAB * (rel + (terms * K + 4) * 2.0**-24) + abs(beta) * np.abs(C0) * 2.0**-50
        err = np.abs(to_host(C) - ref)
        assert np.all(err <= bound), (alpha, beta, (err / np.maximum(bound, 1e-300)).max())
        if K >= 256 and alpha == 1.0:
            rms = np.sqrt(np.mean(err**2)) / np.sqrt(np.mean(absAB**2))
            # the operands really are rounded: far from FP64, and the split form
            # is far closer than one BF16 product (about 2^-8 / sqrt(K) vs 2^-16)
            assert rms > 1e-9
            if terms == 1:
                assert rms > 1e-5
            else:
                assert rms < 1e-5
