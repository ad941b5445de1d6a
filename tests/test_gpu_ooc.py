"""Out-of-core factorization (randutv_factor_ooc, Section 3.2): A, U, T and V in
page-locked host memory, an HBM tile cache smaller than the matrices, and the
three dispatch variants of Section 3.2.4 (traditional, cached, overlapped).

The tiles are block columns and every operation of a step (Section 3.1,
Figure 2) is a sum over tiles, so the result is the in-core factorization's up
to the summation order: T within 1e-11 ||A||_F of randutv_factor's (after
aligning the signs of the (u_j, v_j) pairs), the residual and orthogonality to
the FP64 bar, and, at 4000 x 4000 (b = 128, q = 2) with a cache of 15 of the
96 tiles, T against the FP64 CPU oracle on the rows that the input determines
(as for the in-core path).
"""
import numpy as np
import pytest

import paper_2002_06960_amd as pkg
from oracle import randutv_oracle as ro
from randutv_inputs import make_matrix
from gpu_util import diag_blocks_ok, invariants_dev, sign_align, stable_rows, to_dev, to_host

pytestmark = pytest.mark.gpu


def _perturbed(A, seed=123):
    rng = np.random.default_rng(seed)
    return A * (1.0 + 2.0 ** -52 * rng.standard_normal(A.shape))


def _host(A):
    import torch

    m, n = A.shape
    H = pkg.host_colmajor_empty(m, n)
    H.copy_(torch.from_numpy(np.asarray(A)))
    return H


def _tile_bytes(m, n, b):
    return 8 * max(m, n) * min(b, n)


def _check_vs_incore(A, b, q, U, T, V, build_u=True, build_v=True, tag=""):
    import torch

    m, n = A.shape
    Ad = to_dev(A)
    Ui, Ti, Vi = pkg.randutv_factor(Ad, b, q, 0, build_u=build_u, build_v=build_v)
    nA = np.linalg.norm(A)
    Th = T.numpy()
    assert np.abs(np.tril(Th, -1)).max() == 0.0 and diag_blocks_ok(Th, min(b, n))
    if build_v:
        Ts, flips = sign_align(Th, V.numpy(), to_host(Vi))
    else:
        Ts, flips = Th, 0
    d = np.linalg.norm(Ts - to_host(Ti)) / nA
    msg = f"ooc {tag} {m}x{n} b={b} q={q}: |T_ooc - T_incore| / |A| = {d:.2e}, flips {flips}"
    if build_u and build_v:
        res, eu, ev, lower = invariants_dev(Ad, U.cuda(), T.cuda(), V.cuda())
        msg += f", residual {res:.2e}, orth {eu:.2e} {ev:.2e}"
        assert res <= 1e-11 and eu <= 1e-12 and ev <= 1e-12 and lower == 0.0, (res, eu, ev)
    print(msg, flush=True)
    assert d <= 1e-11, d
    del Ui, Ti, Vi, Ad
    torch.cuda.empty_cache()
    return Ts


@pytest.mark.parametrize("mode", ["traditional", "cached", "overlapped"])
@pytest.mark.parametrize("m,n,b,q,kind,slots", [
    (1000, 800, 64, 1, "exp", 2),      # tall, the smallest cache
    (600, 600, 96, 2, "exp", 3),       # ragged last tile (600 = 6 * 96 + 24)
    (900, 457, 128, 0, "iid", 5),      # ragged, no power iteration
])
def test_ooc_matches_incore(m, n, b, q, kind, slots, mode):
    A = make_matrix(kind, m, n, seed=3)
    U, T, V, st = pkg.randutv_factor_ooc(_host(A), b, q, 0, slots * _tile_bytes(m, n, b), mode)
    print(f"ooc {mode}: {st}", flush=True)
    assert st["slots"] == slots
    _check_vs_incore(A, b, q, U, T, V, tag=mode)
    assert st["tile_loads"] >= -(-n // b)          # every tile of A arrives at least once
    if mode == "traditional":
        assert st["tile_hits"] == 0


def test_ooc_in_place_and_without_u_v():
    m, n, b, q = 700, 500, 64, 1
    A = make_matrix("exp", m, n, seed=4)
    H = _host(A)
    U, T, V, st = pkg.randutv_factor_ooc(H, b, q, 0, 3 * _tile_bytes(m, n, b), "overlapped",
                                         build_u=False, build_v=False, in_place=True)
    assert U is None and V is None and T.data_ptr() == H.data_ptr()
    _check_vs_incore(A, b, q, U, T, V, build_u=False, build_v=False, tag="in place")


def test_ooc_4000_forced_eviction_against_oracle_and_incore():
    """4000 x 4000, b = 128, q = 2 (the 4000^2 workload), exp spectrum, a cache
    of 15 tiles for the 96 tiles of T, U and V: T against the in-core T and
    the oracle's (rows that the input determines)."""
    m = n = 4000
    b, q = 128, 2
    A = make_matrix("exp", m, n, seed=0)
    res = {}
    for mode in ("overlapped", "cached", "traditional"):
        U, T, V, st = pkg.randutv_factor_ooc(_host(A), b, q, 0, 15 * _tile_bytes(m, n, b), mode)
        print(f"ooc 4000^2 {mode}: real {st['real_ms']:.1f} ms, compute {st['compute_ms']:.1f} ms, "
              f"io {st['io_ms']:.1f} ms, h2d {st['h2d_bytes'] / 1e9:.2f} GB, "
              f"d2h {st['d2h_bytes'] / 1e9:.2f} GB, loads {st['tile_loads']}, hits {st['tile_hits']}",
              flush=True)
        res[mode] = st
        Ts = _check_vs_incore(A, b, q, U, T, V, tag=mode)
        if mode == "overlapped":
            Uo, To, Vo = ro.randutv(A, b, q, 0, build_u=False)
            _, To2, _ = ro.randutv(_perturbed(A), b, q, 0, build_u=False, build_v=False)
            nA = np.linalg.norm(A)
            rows = stable_rows(To, To2, nA, b)
            Ts, flips = sign_align(T.numpy(), V.numpy(), Vo)
            diff = np.linalg.norm(Ts[:rows] - To[:rows]) / nA
            print(f"ooc 4000^2 vs oracle: stable rows {rows}, |S T S - T_ora| / |A| = {diff:.2e}", flush=True)
            assert rows == m and diff <= 1e-11
        del U, T, V
    # the cache saves copies: every variant moves at least the matrices once,
    # the traditional one the most
    assert res["traditional"]["h2d_bytes"] > res["cached"]["h2d_bytes"]
    assert res["cached"]["tile_hits"] > 0 and res["overlapped"]["tile_hits"] > 0
