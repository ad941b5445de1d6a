"""The C ABI's factorization options through randutv_factor_ex (Section 3.1,
Figure 2): caller-provided sketches on the device and on the host, explicit
leading dimensions, ordering on the caller's stream, the sketch stream's raw
generator words against an independent implementation of the published
generator, and the run-time error paths forced from the host."""
import ctypes

import numpy as np
import pytest

import paper_2002_06960_amd as pkg
from paper_2002_06960_amd import randutv as rb
from oracle import randutv_oracle as ro
from randutv_inputs import make_matrix
from gpu_util import invariants_dev, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("seed,step,first,nblocks", [
    (0, 0, 0, 4096), (7, 3, 1000, 513), (2**63 + 5, 46, 719_000, 4096), (2**64 - 1, 2**40, 2**50, 7)])
def test_sketch_words_bit_exact(seed, step, first, nblocks):
    """The GPU's Philox4x64-10 words equal numpy's implementation of the
    published generator (itself pinned to the known-answer vectors) bit for bit."""
    got = pkg.randutv_sketch_words(seed, step, first, nblocks)
    ref = ro.philox_blocks(seed, step, first + nblocks)[first:] if first < 10**6 else None
    if ref is None:
        # far counters: numpy's generator advanced to the first block
        ones = np.array([2**64 - 1] * 4, dtype=np.uint64)
        bg = np.random.Philox(counter=ones, key=np.array([seed, step], dtype=np.uint64))
        bg.advance(first)
        ref = bg.random_raw(4 * nblocks).reshape(nblocks, 4)
    assert got.dtype == np.uint64
    assert np.array_equal(got, ref)


def test_sketch_host_equals_device_sketches():
    m, n, b = 700, 530, 128
    Gh = pkg.randutv_sketch_host(3, m, n, b)
    offs = pkg.sketch_offsets(m, n, b)
    assert Gh.shape == (offs[-1],)
    for i, s in enumerate(range(0, n, b)):
        mi, bi = m - s, min(b, n - s)
        Gd = to_host(pkg.randutv_sketch(3, i, mi, bi))
        blk = Gh[offs[i]:offs[i + 1]].reshape(bi, mi).T
        assert np.array_equal(blk, Gd)


@pytest.mark.parametrize("where", ["device", "host"])
def test_caller_sketch_gives_identical_factorization(where):
    import torch

    m, n, b, q, seed = 900, 700, 128, 2, 11
    A = to_dev(make_matrix("exp", m, n, seed=3))
    U0, T0, V0 = pkg.randutv_factor(A, b, q, seed)
    Gh = pkg.randutv_sketch_host(seed, m, n, b)
    G = torch.from_numpy(Gh).cuda() if where == "device" else Gh
    U1, T1, V1 = pkg.randutv_factor(A, b, q, seed + 1, G=G)  # the seed is unused with a caller G
    for x, y in ((U0, U1), (T0, T1), (V0, V1)):
        assert torch.equal(x, y)


def test_caller_sketch_is_used():
    """A different caller G gives a different (but valid) factorization."""
    import torch

    m, n, b, q = 300, 300, 64, 1
    A = to_dev(make_matrix("exp", m, n, seed=4))
    _, T0, _ = pkg.randutv_factor(A, b, q, 0)
    G = torch.from_numpy(pkg.randutv_sketch_host(1, m, n, b)).cuda()
    U1, T1, V1 = pkg.randutv_factor(A, b, q, 0, G=G)
    assert not torch.equal(T0, T1)
    res, eu, ev, lower = invariants_dev(A, U1, T1, V1)
    assert res <= 1e-11 and eu <= 1e-12 and ev <= 1e-12 and lower == 0.0


def _colmajor_view(buf, rows, cols, ld):
    """rows x cols column-major view with leading dimension ld into buf (cols x ld)."""
    return buf.reshape(-1)[: ld * cols].reshape(cols, ld).t()[:rows, :]


def test_explicit_leading_dimensions():
    """U, T, V with leading dimensions above their row counts (views into larger
    buffers) give the same bits as the compact layout, and the padding rows are
    not written."""
    import torch

    m, n, b, q = 400, 260, 64, 1
    A = to_dev(make_matrix("iid", m, n, seed=5))
    U0, T0, V0 = pkg.randutv_factor(A, b, q, 2)
    lib = pkg.load()
    lu, lt, lv = m + 40, m + 24, n + 8
    Ubuf = torch.full((m, lu), 7.0, dtype=torch.float64, device="cuda")
    Tbuf = torch.full((n, lt), 7.0, dtype=torch.float64, device="cuda")
    Vbuf = torch.full((n, lv), 7.0, dtype=torch.float64, device="cuda")
    a = rb.make_args(m=m, n=n, A=A.data_ptr(), lda=m, b=b, q=q, seed=2,
                     U=Ubuf.data_ptr(), ldu=lu, T=Tbuf.data_ptr(), ldt=lt,
                     V=Vbuf.data_ptr(), ldv=lv, flags=rb.FLAG_STREAM,
                     stream=torch.cuda.current_stream().cuda_stream)
    assert lib.randutv_factor_ex(ctypes.byref(a)) == 0
    assert torch.equal(_colmajor_view(Ubuf, m, m, lu), U0)
    assert torch.equal(_colmajor_view(Tbuf, m, n, lt), T0)
    assert torch.equal(_colmajor_view(Vbuf, n, n, lv), V0)
    assert torch.all(Ubuf[:, m:] == 7.0) and torch.all(Tbuf[:, m:] == 7.0) and torch.all(Vbuf[:, n:] == 7.0)


def test_factor_on_a_side_stream_waits_for_prior_work():
    """The call is ordered on torch's current stream: work queued there before
    the call (a delay, then the copy that produces A) finishes before the
    library reads A, and the result matches the default-stream call."""
    import torch

    m, n, b, q = 1500, 1200, 128, 2
    Ah = make_matrix("exp", m, n, seed=6)
    A0 = to_dev(Ah)
    U0, T0, V0 = pkg.randutv_factor(A0, b, q, 4)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    A1 = torch.zeros_like(A0)  # column-major like A0
    src = A0.clone()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        torch.cuda._sleep(20_000_000)
        A1.copy_(src)
        U1, T1, V1 = pkg.randutv_factor(A1, b, q, 4)
        Tsum = T1.sum()  # queued on the side stream after the call
    side.synchronize()
    assert torch.equal(T0, T1) and torch.equal(U0, U1) and torch.equal(V0, V1)
    assert Tsum.item() == T0.sum().item()


def test_forced_error_paths_leave_the_library_usable():
    """ERR_NOCONV (a one-sweep cap), ERR_SYNC (waits that give up after a couple
    of polls: every kernel still ends) and ERR_NOMEM (a workspace cap) returned
    from whole factorizations; afterwards an ordinary call gives the same bits
    as before."""
    import torch

    m, n, b, q = 600, 600, 128, 1
    A = to_dev(make_matrix("iid", m, n, seed=7))
    U0, T0, V0 = pkg.randutv_factor(A, b, q, 0)
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_factor(A, b, q, 0, jacobi_max_sweeps=1)
    assert e.value.code == rb.ERR_NOCONV
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_factor(A, b, q, 0, spin_limit=1)
    assert e.value.code == rb.ERR_SYNC
    with pytest.raises(pkg.RandUTVError) as e:
        pkg.randutv_factor(A, b, q, 0, max_workspace_bytes=4096)
    assert e.value.code == rb.ERR_NOMEM
    U1, T1, V1 = pkg.randutv_factor(A, b, q, 0)
    assert torch.equal(T0, T1) and torch.equal(U0, U1) and torch.equal(V0, V1)


def test_no_finite_check_flag_same_result():
    import torch

    A = to_dev(make_matrix("log8", 300, 250, seed=8))
    _, T0, _ = pkg.randutv_factor(A, 64, 1, 0)
    _, T1, _ = pkg.randutv_factor(A, 64, 1, 0, finite_check=False)
    assert torch.equal(T0, T1)


def test_kernel_trace_matches_the_class_totals():
    """randutv_kernel_trace: one record per timed launch of the last call, on
    the library's four streams, whose durations add up to the per-class
    totals of randutv_kernel_stats; the critical stream (T) runs the sketch
    and the sketch's panel QR, stream P the column-block panels, stream S the
    SVD batches."""
    m = n = 2000
    b, q = 128, 2
    A = to_dev(make_matrix("exp", m, n, seed=2))
    try:
        pkg.randutv_set_timing(True)
        pkg.randutv_factor(A, b, q, 0)
        tr = pkg.randutv_kernel_trace()
        stats = pkg.randutv_kernel_stats()
    finally:
        pkg.randutv_set_timing(False)
    steps = -(-n // b)
    assert len(tr) == sum(v[0] for v in stats.values())
    assert {s for _, s, _, _ in tr} <= {"T", "P", "UV", "S"}
    for cls, (launches, ms, _) in stats.items():
        recs = [d for c, _, _, d in tr if c == cls]
        assert len(recs) == launches, cls
        assert abs(sum(recs) - ms) <= 1e-3 * max(ms, 1e-3), (cls, sum(recs), ms)
    assert all(t0 >= -1e-3 and d >= 0.0 for _, _, t0, d in tr)
    by = lambda cls: {s for c, s, _, _ in tr if c == cls}
    assert by("sketch") == {"T"} and by("jacobi_svd") == {"S"}
    panels = [s for c, s, _, _ in tr if c == "panel_qr"]
    assert panels.count("T") == steps and panels.count("P") == steps
    end = max(t0 + d for _, _, t0, d in tr)
    assert 0.0 < end < 5e3
