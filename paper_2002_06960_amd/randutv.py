"""Python binding of the gfx950 randUTV library (ctypes over include/randutv.h).

Argument marshalling only: every step of the factorization runs in the HIP
kernels of librandutv.so.  Torch is used for device memory and streams:
matrices are float64 CUDA (HIP) tensors in column-major layout (stride
(1, ld)); inputs in another layout are copied to column-major first.  The
factorization is ordered on torch's current stream (randutv_factor_ex with
RANDUTV_FLAG_STREAM): it starts after the work already queued there and the
work queued there afterwards sees its outputs; the other entry points
synchronise the current stream first.  Every call returns when its device work
has finished.  A missing or unloadable library raises RuntimeError.
"""
from __future__ import annotations

import atexit
import ctypes
import os
from typing import Optional, Tuple

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librandutv.so")

RANDUTV_OK = 0
ERR_HIP, ERR_NOMEM, ERR_NONFINITE, ERR_NOCONV, ERR_SYNC, ERR_TOO_LARGE, ERR_RANK = 1, 2, 3, 4, 5, 6, 7
ERR_SCRATCH = 8
NOALLOC_SCRATCH_BYTES = 128 << 20
FLAG_G_HOST, FLAG_NO_FINITE_CHECK, FLAG_STREAM, FLAG_ASYNC = 1, 2, 4, 8
PRECISION_BITS = (64, 32, 16, 48)


class RandutvArgs(ctypes.Structure):
    """struct randutv_args of include/randutv.h (field for field)."""
    _fields_ = [("struct_size", ctypes.c_int64), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("lda", ctypes.c_int64), ("b", ctypes.c_int64),
                ("q", ctypes.c_int32), ("sketch_bits", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("U", ctypes.c_void_p), ("ldu", ctypes.c_int64), ("T", ctypes.c_void_p),
                ("ldt", ctypes.c_int64), ("V", ctypes.c_void_p), ("ldv", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("G", ctypes.c_void_p), ("update_bits", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("jacobi_max_sweeps", ctypes.c_int32),
                ("spin_limit", ctypes.c_uint32), ("max_workspace_bytes", ctypes.c_int64)]


class RandutvOocStats(ctypes.Structure):
    """struct randutv_ooc_stats of include/randutv.h (field for field)."""
    _fields_ = [("struct_size", ctypes.c_int64), ("real_ms", ctypes.c_double),
                ("compute_ms", ctypes.c_double), ("io_ms", ctypes.c_double),
                ("h2d_ms", ctypes.c_double), ("d2h_ms", ctypes.c_double),
                ("h2d_bytes", ctypes.c_int64), ("d2h_bytes", ctypes.c_int64),
                ("tile_loads", ctypes.c_int64), ("tile_writebacks", ctypes.c_int64),
                ("tile_hits", ctypes.c_int64), ("slots", ctypes.c_int64),
                ("slot_bytes", ctypes.c_int64), ("fixed_bytes", ctypes.c_int64)]


OOC_MODES = {"traditional": 0, "cached": 1, "overlapped": 2}


def make_args(**kw) -> RandutvArgs:
    a = RandutvArgs()
    ctypes.memset(ctypes.byref(a), 0, ctypes.sizeof(a))
    a.struct_size = ctypes.sizeof(a)
    for k, v in kw.items():
        setattr(a, k, v)
    return a

# name -> (restype, argtypes)
_I64, _I32, _U64, _D, _P, _C = (ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double,
                                ctypes.c_void_p, ctypes.c_char)
SIGNATURES = {
    "randutv_factor": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _I32, _U64, _P, _P, _P]),
    "randutv_factor_ex": (ctypes.c_int, [ctypes.POINTER(RandutvArgs)]),
    "randutv_factor_noalloc": (ctypes.c_int, [ctypes.POINTER(RandutvArgs)]),
    "randutv_factor_status": (ctypes.c_int, []),
    "randutv_factor_ooc": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _I32, _U64, _P, _I64, _P, _I64,
                                          _P, _I64, _I64, _I32, ctypes.c_void_p]),
    "randutv_sketch_host": (ctypes.c_int, [_U64, _I64, _I64, _I64, _P]),
    "randutv_sketch_words": (ctypes.c_int, [_U64, _U64, _U64, _I64, _P]),
    "randutv_finalize": (ctypes.c_int, []),
    "randutv_truncate": (ctypes.c_int, [_I64, _I64, _I64, _P, _P, _P, _P]),
    "randutv_truncate_grad": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _I32, _U64, _P, _I64, _P, _I64]),
    "randutv_truncate_first_block": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _I32, _U64, _P, _I64]),
    "randutv_truncate_grad_k": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _I32, _U64, _I64, _P, _I64,
                                               _P, _I64]),
    "randutv_truncate_first_block_k": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _I32, _U64, _I64, _P,
                                                      _I64]),
    "randutv_truncate_batched": (ctypes.c_int, [_I64, _I32, _I64, _I64, _P, _I64, _I64, _I64, _I32, _U64,
                                                _I64, _P, _I64, _I64, _P, _I64, _I64]),
    "randutv_hqrrp": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _U64, _P, _P]),
    "randutv_geqrf_blocked": (ctypes.c_int, [_I64, _I64, _P, _I64, _I64, _P]),
    "randutv_sketch": (ctypes.c_int, [_U64, _U64, _I64, _I64, _P, _I64]),
    "randutv_dgemm": (ctypes.c_int, [_C, _C, _I64, _I64, _I64, _D, _P, _I64, _P, _I64, _D, _P, _I64]),
    "randutv_gemm_f32": (ctypes.c_int, [_C, _C, _I64, _I64, _I64, _D, _P, _I64, _P, _I64, _D, _P, _I64]),
    "randutv_gemm_bf16": (ctypes.c_int, [_C, _C, _I64, _I64, _I64, _D, _P, _I64, _P, _I64, _D, _P, _I64,
                                         _I32]),
    "randutv_geqrf": (ctypes.c_int, [_I64, _I64, _P, _I64, _P]),
    "randutv_larft": (ctypes.c_int, [_I64, _I64, _P, _I64, _P, _P, _I64]),
    "randutv_gesvj": (ctypes.c_int, [_I64, _P, _I64, _P, _P, _P, ctypes.POINTER(_I32)]),
    "randutv_set_timing": (ctypes.c_int, [_I32]),
    "randutv_kernel_stats": (ctypes.c_int, [_I32, ctypes.POINTER(ctypes.c_char_p),
                                            ctypes.POINTER(_I64), ctypes.POINTER(_D),
                                            ctypes.POINTER(_D)]),
    "randutv_kernel_bytes": (ctypes.c_int, [_I32, ctypes.POINTER(_D)]),
    "randutv_kernel_trace": (ctypes.c_int, [_I32, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                            ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "randutv_last_sweeps": (ctypes.c_int, [_I32, ctypes.POINTER(_I32)]),
    "randutv_last_hip_error": (ctypes.c_char_p, []),
    "randutv_strerror": (ctypes.c_char_p, [ctypes.c_int]),
}

_lib = None


class RandUTVError(RuntimeError):
    def __init__(self, fn: str, code: int):
        self.code = code
        lib = load()
        msg = lib.randutv_strerror(code).decode() if code > 0 else f"argument {-code} is invalid"
        if code in (ERR_HIP, ERR_NOMEM):
            msg += f" [{lib.randutv_last_hip_error().decode()}]"
        super().__init__(f"{fn} returned {code}: {msg}")


def load(path: Optional[str] = None):
    """Load librandutv.so (built in-tree by paper_2002_06960_amd/build.py)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    # Bind the library to the HIP runtime that torch has already loaded (same
    # SONAME): loading it first would bring in a second HIP runtime, and two
    # runtimes in one process do not share devices or memory.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with paper_2002_06960_amd/build.py "
                           "(or __graft_entry__.build())")
    lib = ctypes.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
        # release the library's streams and workspace before the HIP runtime
        # is torn down at exit
        atexit.register(lib.randutv_finalize)
    return lib


def _check(fn: str, code: int):
    if code != RANDUTV_OK:
        raise RandUTVError(fn, code)


# --------------------------------------------------------------------------- tensors
def _torch():
    import torch
    return torch


def colmajor_empty(rows: int, cols: int, device=None):
    torch = _torch()
    return torch.empty((cols, rows), dtype=torch.float64, device=device or "cuda").t()


def as_colmajor(x):
    """Return (tensor, ld): x as a float64 CUDA tensor with stride (1, ld)."""
    torch = _torch()
    if x.dtype != torch.float64 or not x.is_cuda:
        raise TypeError("expected a float64 CUDA tensor")
    if x.dim() == 1:
        x = x.reshape(-1, 1)
    m, n = x.shape
    if x.stride(0) == 1 and (n <= 1 or x.stride(1) >= max(1, m)):
        return x, max(1, x.stride(1) if n > 1 else m)
    y = x.t().contiguous().t()
    return y, max(1, m)


def _ptr(x) -> int:
    return 0 if x is None else x.data_ptr()


def _sync():
    torch = _torch()
    torch.cuda.current_stream().synchronize()


# --------------------------------------------------------------------------- API
def _check_f64(x, name: str, shape):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or not x.is_cuda:
        raise TypeError(f"{name} must be a float64 CUDA tensor")
    if tuple(x.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(x.shape)}")


def _out(x, rows, cols, device, name="output"):
    if x is None:
        return colmajor_empty(rows, cols, device)
    _check_f64(x, name, (rows, cols))
    if x.stride(0) != 1 or (cols > 1 and x.stride(1) != rows):
        raise ValueError(f"{name} must be column-major with leading dimension {rows}")
    return x


def _stream_handle() -> int:
    """HIP handle of torch's current stream on the current device (0 = null stream)."""
    torch = _torch()
    return int(torch.cuda.current_stream().cuda_stream)


def sketch_offsets(m: int, n: int, b: int):
    """Element offsets of G(0), G(1), ... in the concatenated sketch layout
    (G(i) of (m - i b) x min(b, n - i b), ld m - i b); the last entry is the total."""
    b = min(b, n)
    offs, off, s = [], 0, 0
    while s < n:
        offs.append(off)
        off += (m - s) * min(b, n - s)
        s += b
    offs.append(off)
    return offs


def randutv_factor(A, b: int, q: int, seed: int = 0, build_u: bool = True,
                   build_v: bool = True, in_place: bool = False, U=None, T=None, V=None,
                   sketch_bits: int = 64, update_bits: int = 64, G=None,
                   jacobi_max_sweeps: int = 0, spin_limit: int = 0,
                   max_workspace_bytes: int = 0, finite_check: bool = True,
                   asynchronous: bool = False, noalloc: bool = False) -> Tuple:
    """A = U T V^T.  Returns (U, T, V) column-major tensors (U/V None if not built).

    U, T, V may be given as preallocated column-major outputs.  sketch_bits
    selects the arithmetic of the sketch and power-iteration products, and
    update_bits that of the compact-WY updates of T, U and V: 64 the FP64
    matrix cores, 32 the FP32 matrix cores, 16 the BF16 matrix cores, 48
    three BF16 products of split operands.  G, if given, holds the caller's
    sketches in the layout of sketch_offsets: a float64 CUDA tensor, or a
    numpy float64 array / CPU tensor (host memory).  The call is ordered on
    torch's current stream.  asynchronous: return once the work is enqueued
    (no host synchronization); randutv_factor_status() gives its outcome
    later.  noalloc: the
    allocation-free entry point (every temporary in the library's fixed
    device scratch)."""
    torch = _torch()
    lib = load()
    A, lda = as_colmajor(A)
    m, n = A.shape
    if in_place and lda == m:
        T = A
    else:
        T = _out(T, m, n, A.device, "T")
    U = _out(U, m, m, A.device, "U") if build_u else None
    V = _out(V, n, n, A.device, "V") if build_v else None
    flags = FLAG_STREAM | (0 if finite_check else FLAG_NO_FINITE_CHECK) | (FLAG_ASYNC if asynchronous else 0)
    gptr, keep = 0, None
    if G is not None:
        total = sketch_offsets(m, n, b)[-1]
        if isinstance(G, torch.Tensor) and G.is_cuda:
            if G.dtype != torch.float64 or G.numel() != total or not G.is_contiguous():
                raise ValueError(f"G must be a contiguous float64 tensor of {total} elements")
            gptr = G.data_ptr()
        else:
            import numpy as np
            keep = np.ascontiguousarray(G.numpy() if isinstance(G, torch.Tensor) else G,
                                        dtype=np.float64).reshape(-1)
            if keep.size != total:
                raise ValueError(f"G must hold {total} elements")
            gptr = keep.ctypes.data
            flags |= FLAG_G_HOST
    args = make_args(m=m, n=n, A=_ptr(A), lda=lda, b=b, q=q, seed=seed & (2**64 - 1),
                     U=_ptr(U), ldu=m, T=_ptr(T), ldt=m, V=_ptr(V), ldv=n,
                     stream=_stream_handle() if m and n else 0, G=gptr,
                     sketch_bits=sketch_bits, update_bits=update_bits, flags=flags,
                     jacobi_max_sweeps=jacobi_max_sweeps, spin_limit=spin_limit,
                     max_workspace_bytes=max_workspace_bytes)
    if noalloc:
        _check("randutv_factor_noalloc", lib.randutv_factor_noalloc(ctypes.byref(args)))
    else:
        _check("randutv_factor_ex", lib.randutv_factor_ex(ctypes.byref(args)))
    del keep
    return U, T, V


def randutv_factor_status() -> int:
    """Outcome of the last factorization (e.g. an asynchronous call): waits
    for the device, returns 0 or a RANDUTV_ERR_* code."""
    return load().randutv_factor_status()


def host_colmajor_empty(rows: int, cols: int, pinned: bool = True):
    """Column-major float64 host tensor (page-locked unless pinned=False)."""
    torch = _torch()
    return torch.empty((cols, rows), dtype=torch.float64, pin_memory=pinned).t()


def _host_colmajor(x, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or x.is_cuda:
        raise TypeError(f"{name} must be a float64 host (CPU) tensor")
    if x.dim() != 2 or x.stride(0) != 1 or (x.shape[1] > 1 and x.stride(1) < x.shape[0]):
        raise ValueError(f"{name} must be column-major (stride (1, ld), ld >= rows)")
    return x, max(1, x.stride(1) if x.shape[1] > 1 else x.shape[0])


def randutv_factor_ooc(A, b: int, q: int, seed: int = 0, hbm_budget_bytes: int = 1 << 30,
                       mode: str = "overlapped", build_u: bool = True, build_v: bool = True,
                       in_place: bool = False, U=None, T=None, V=None):
    """Out-of-core A = U T V^T with A, U, T, V in host memory and at most
    hbm_budget_bytes of HBM for the tile cache (mode: traditional, cached or
    overlapped).  A is a column-major float64 CPU tensor (page-locked for
    overlapped copies).  Returns (U, T, V, stats) with page-locked
    column-major CPU tensors (U/V None if not built) and the call's
    statistics as a dict."""
    lib = load()
    A, lda = _host_colmajor(A, "A")
    m, n = A.shape
    if mode not in OOC_MODES:
        raise ValueError(f"mode must be one of {sorted(OOC_MODES)}")
    if in_place:
        T, ldt = A, lda
    else:
        T = host_colmajor_empty(m, n) if T is None else T
        T, ldt = _host_colmajor(T, "T")
    if build_u:
        U = host_colmajor_empty(m, m) if U is None else U
        U, ldu = _host_colmajor(U, "U")
    else:
        U, ldu = None, m
    if build_v:
        V = host_colmajor_empty(n, n) if V is None else V
        V, ldv = _host_colmajor(V, "V")
    else:
        V, ldv = None, n
    for x, name, shape in ((T, "T", (m, n)), (U, "U", (m, m)), (V, "V", (n, n))):
        if x is not None and tuple(x.shape) != shape:
            raise ValueError(f"{name} must have shape {shape}")
    st = RandutvOocStats()
    st.struct_size = ctypes.sizeof(st)
    _check("randutv_factor_ooc",
           lib.randutv_factor_ooc(m, n, A.data_ptr(), lda, b, q, seed, _ptr(U), ldu, T.data_ptr(), ldt,
                                  _ptr(V), ldv, int(hbm_budget_bytes), OOC_MODES[mode],
                                  ctypes.byref(st)))
    stats = {f: getattr(st, f) for f, _ in RandutvOocStats._fields_ if f != "struct_size"}
    return U, T, V, stats


def randutv_truncate(U, T, V, k: int):
    """A_k = U(:, :k) T(:k, :) V^T."""
    lib = load()
    if T.dim() != 2:
        raise ValueError("T must be a matrix")
    m, n = T.shape
    _check_f64(U, "U", (m, m))
    _check_f64(T, "T", (m, n))
    _check_f64(V, "V", (n, n))
    for x, ld in ((U, m), (T, m), (V, n)):
        if x.stride(0) != 1 or (x.shape[1] > 1 and x.stride(1) != ld):
            raise ValueError("randutv_truncate expects the column-major outputs of randutv_factor")
    if not 0 <= k <= n:
        raise ValueError(f"k must lie in [0, {n}]")
    Ak = colmajor_empty(m, n, T.device)
    _sync()
    _check("randutv_truncate", lib.randutv_truncate(m, n, k, _ptr(U), _ptr(T), _ptr(V), _ptr(Ak)))
    return Ak


def randutv_hqrrp(A, b: int, seed: int = 0):
    """Randomized blocked column-pivoted QR A P = Q R.  Returns (F, tau, jpvt):
    F (column-major copy of A) in the dgeqp3 layout, tau (n), jpvt (n, int64)."""
    torch = _torch()
    lib = load()
    A, _ = as_colmajor(A)
    m, n = A.shape
    F = colmajor_empty(m, n, A.device)
    F.copy_(A)
    tau = torch.empty(n, dtype=torch.float64, device=F.device)
    jpvt = torch.empty(n, dtype=torch.int64, device=F.device)
    _sync()
    _check("randutv_hqrrp", lib.randutv_hqrrp(m, n, _ptr(F), max(1, m), b, seed & (2**64 - 1),
                                              _ptr(tau), _ptr(jpvt)))
    return F, tau, jpvt


def randutv_geqrf_blocked(A, b: int):
    """Unpivoted blocked Householder QR A = Q R (HQRRP's step loop without the
    pivots).  Returns (F, tau): F (column-major copy of A) in the dgeqrf layout."""
    torch = _torch()
    lib = load()
    A, _ = as_colmajor(A)
    m, n = A.shape
    F = colmajor_empty(m, n, A.device)
    F.copy_(A)
    tau = torch.empty(n, dtype=torch.float64, device=F.device)
    _sync()
    _check("randutv_geqrf_blocked", lib.randutv_geqrf_blocked(m, n, _ptr(F), max(1, m), b, _ptr(tau)))
    return F, tau


def randutv_truncate_first_block(A, b: int, q: int, seed: int = 0):
    """A_k, k = min(b, n), of randutv_factor(A, b, q, seed) from the first
    step alone (Q Q^T A with Q spanning (A A^T)^(q+1) G(0))."""
    lib = load()
    A, lda = as_colmajor(A)
    m, n = A.shape
    Ak = colmajor_empty(m, n, A.device)
    _sync()
    _check("randutv_truncate_first_block",
           lib.randutv_truncate_first_block(m, n, _ptr(A), lda, b, q, seed & (2**64 - 1), _ptr(Ak),
                                            max(1, m)))
    return Ak


def randutv_truncate_grad(A, b: int, q: int, seed: int, Gbar):
    """dL/dA for the first-block truncation A_k (k = min(b, n)) of
    randutv_factor(A, b, q, seed), given Gbar = dL/dA_k (sketch held fixed)."""
    lib = load()
    A, lda = as_colmajor(A)
    Gbar, ldg = as_colmajor(Gbar)
    m, n = A.shape
    if tuple(Gbar.shape) != (m, n):
        raise ValueError("Gbar must have the shape of A")
    Abar = colmajor_empty(m, n, A.device)
    _sync()
    _check("randutv_truncate_grad", lib.randutv_truncate_grad(m, n, _ptr(A), lda, b, q,
                                                              seed & (2**64 - 1), _ptr(Gbar), ldg,
                                                              _ptr(Abar), max(1, m)))
    return Abar


def randutv_truncate_grad_k(A, b: int, q: int, seed: int, k: int, Gbar):
    """dL/dA for the truncation A_k (0 < k <= b_0 + b_1, b_0 = min(b, n),
    b_1 = min(b, n - b_0): the first two blocks of U) of
    randutv_factor(A, b, q, seed), given Gbar = dL/dA_k (sketches held fixed)."""
    lib = load()
    A, lda = as_colmajor(A)
    Gbar, ldg = as_colmajor(Gbar)
    m, n = A.shape
    if tuple(Gbar.shape) != (m, n):
        raise ValueError("Gbar must have the shape of A")
    Abar = colmajor_empty(m, n, A.device)
    _sync()
    _check("randutv_truncate_grad_k",
           lib.randutv_truncate_grad_k(m, n, _ptr(A), lda, b, q, seed & (2**64 - 1), k, _ptr(Gbar), ldg,
                                       _ptr(Abar), max(1, m)))
    return Abar


def randutv_truncate_first_block_k(A, b: int, q: int, seed: int, k: int):
    """A_k (0 < k <= b_0 + b_1) of randutv_factor(A, b, q, seed) from its first
    step (k <= b_0: the projection of A onto the leading k left singular
    vectors of A orth((A^T A)^q A^T G(0))) or first two steps alone."""
    lib = load()
    A, lda = as_colmajor(A)
    m, n = A.shape
    Ak = colmajor_empty(m, n, A.device)
    _sync()
    _check("randutv_truncate_first_block_k",
           lib.randutv_truncate_first_block_k(m, n, _ptr(A), lda, b, q, seed & (2**64 - 1), k, _ptr(Ak),
                                              max(1, m)))
    return Ak


def randutv_truncate_batched(A, b: int, q: int, seed: int, k: int, Gbar=None):
    """For a batch A (batch x m x n, float64 CUDA): A_k of every matrix
    (Gbar None) or dL/dA given Gbar = dL/dA_k (same shape), in one call that
    spreads the matrices over the library's streams."""
    torch = _torch()
    lib = load()
    if A.dim() != 3 or A.dtype != torch.float64 or not A.is_cuda:
        raise TypeError("A must be a float64 CUDA tensor of shape (batch, m, n)")
    B_, m, n = A.shape
    # column-major matrices, one after the other: (batch, n, m) contiguous, transposed
    Ac = A.transpose(1, 2).contiguous().transpose(1, 2)
    out = torch.empty((B_, n, m), dtype=torch.float64, device=A.device).transpose(1, 2)
    gptr, stride_g = 0, m * n
    if Gbar is not None:
        if tuple(Gbar.shape) != (B_, m, n) or Gbar.dtype != torch.float64 or not Gbar.is_cuda:
            raise ValueError("Gbar must be a float64 CUDA tensor shaped like A")
        Gc = Gbar.transpose(1, 2).contiguous().transpose(1, 2)
        gptr = Gc.data_ptr()
    _sync()
    _check("randutv_truncate_batched",
           lib.randutv_truncate_batched(B_, 1 if Gbar is not None else 0, m, n, Ac.data_ptr(), max(1, m),
                                        m * n, b, q, seed & (2**64 - 1), k, gptr, max(1, m), stride_g,
                                        out.data_ptr(), max(1, m), m * n))
    return out


def _autograd_function():
    torch = _torch()

    class Truncation(torch.autograd.Function):
        """A -> A_k (0 < k <= b_0 + b_1), the sketches held fixed.  Forward:
        randutv_truncate_first_block(_k) (the first one or two steps fix A_k), or with
        full_factorization randutv_factor then randutv_truncate; reverse:
        randutv_truncate_grad(_k) (the _k forms for k < min(b, n)); a batch goes
        through randutv_truncate_batched (one call, the matrices spread over
        the library's streams).  The library computes in FP64; a float32
        input is promoted and the results are returned as float32."""

        @staticmethod
        def forward(ctx, A, b, q, seed, k, full_factorization):
            dtype = A.dtype
            X64 = A.to(torch.float64)

            def one(X):
                if full_factorization:
                    U, T, V = randutv_factor(X, b, q, seed, build_u=True, build_v=True)
                    return randutv_truncate(U, T, V, k)
                if k == min(b, X.shape[1]):  # the whole first block: Q Q^T A
                    return randutv_truncate_first_block(X, b, q, seed)
                return randutv_truncate_first_block_k(X, b, q, seed, k)

            if A.dim() == 3 and not full_factorization:
                Ak = randutv_truncate_batched(X64, b, q, seed, k)
            else:
                Ak = torch.stack([one(X) for X in X64]) if A.dim() == 3 else one(X64)
            ctx.save_for_backward(X64)
            ctx.b, ctx.q, ctx.seed, ctx.k, ctx.dtype = b, q, seed, k, dtype
            return Ak.to(dtype)

        @staticmethod
        def backward(ctx, gout):
            (A,) = ctx.saved_tensors
            g64 = gout.to(torch.float64)
            def one(X, G):
                if ctx.k == min(ctx.b, X.shape[1]):
                    return randutv_truncate_grad(X, ctx.b, ctx.q, ctx.seed, G)
                return randutv_truncate_grad_k(X, ctx.b, ctx.q, ctx.seed, ctx.k, G)

            if A.dim() == 3:
                g = randutv_truncate_batched(A, ctx.b, ctx.q, ctx.seed, ctx.k, g64)
            else:
                g = one(A, g64)
            return g.to(ctx.dtype), None, None, None, None, None

    return Truncation


_truncation_fn = None


def truncation(A, b: int, q: int, seed: int = 0, k: Optional[int] = None,
               full_factorization: bool = False):
    """Differentiable rank-k truncation A_k = U_k T_k V^T of randutv_factor(A,
    b, q, seed) for 0 < k <= b_0 + b_1 (b_0 = min(b, n), b_1 = min(b, n - b_0);
    default k = b_0), the sketches G(0) and G(1) held fixed.  The forward value
    comes from the first step (k <= b_0) or the first two steps alone by
    default: they already fix U's first b_0 or b_0 + b_1 columns, so the
    later steps do not change A_k (full_factorization=True runs them anyway;
    both agree to rounding amplified by the conditioning of the sketch).
    A may be a batch (batch x m x n), float64 or float32 (computed in FP64)."""
    global _truncation_fn
    if _truncation_fn is None:
        _truncation_fn = _autograd_function()
    n = A.shape[-1]
    b0 = min(b, n)
    kmax = b0 + min(b, n - b0)
    kk = b0 if k is None else int(k)
    if not 0 < kk <= kmax:
        raise ValueError(f"k must lie in 1..b_0 + b_1 = {kmax}")
    return _truncation_fn.apply(A, b, q, seed, kk, full_factorization)


def first_block_truncation(A, b: int, q: int, seed: int = 0, first_step_only: bool = False):
    """truncation() at k = min(b, n); first_step_only=False runs the whole
    factorization for the forward value."""
    return truncation(A, b, q, seed, None, full_factorization=not first_step_only)


def randutv_sketch(seed: int, step: int, rows: int, cols: int, device=None):
    lib = load()
    G = colmajor_empty(rows, cols, device)
    _sync()
    _check("randutv_sketch", lib.randutv_sketch(seed & (2**64 - 1), step, rows, cols, _ptr(G),
                                                max(1, rows)))
    return G


def randutv_sketch_host(seed: int, m: int, n: int, b: int):
    """Every sketch G(0), ..., G(p-1) of a factorization with these sizes, as a
    host numpy float64 array in the concatenated layout (sketch_offsets)."""
    import numpy as np
    lib = load()
    G = np.empty(max(1, sketch_offsets(m, n, b)[-1]) if m and n else 1, dtype=np.float64)
    _check("randutv_sketch_host", lib.randutv_sketch_host(seed & (2**64 - 1), m, n, b,
                                                          G.ctypes.data))
    return G[: sketch_offsets(m, n, b)[-1]] if m and n else G[:0]


def randutv_sketch_words(seed: int, step: int, first_block: int, nblocks: int, device=None):
    """Raw Philox4x64-10 words of blocks first_block .. first_block + nblocks - 1
    of the (seed, step) stream, as a host numpy uint64 array (nblocks, 4)."""
    import numpy as np
    torch = _torch()
    lib = load()
    out = torch.empty(4 * max(nblocks, 1), dtype=torch.int64, device=device or "cuda")
    _sync()
    _check("randutv_sketch_words", lib.randutv_sketch_words(seed & (2**64 - 1), step, first_block,
                                                            nblocks, _ptr(out)))
    return out.cpu().numpy().view(np.uint64)[: 4 * nblocks].reshape(nblocks, 4)


def randutv_dgemm(transa: str, transb: str, alpha: float, A, B, beta: float = 0.0, C=None,
                  f32: bool = False, bf16_terms: int = 0):
    """C = alpha op(A) op(B) + beta C (FP64 MFMA kernels; f32: FP64 operands and
    result, FP32 matrix-core arithmetic; bf16_terms 1 or 3: BF16 matrix-core
    arithmetic with one product of rounded operands or three of split ones).
    Returns C."""
    lib = load()
    A, lda = as_colmajor(A)
    B, ldb = as_colmajor(B)
    M = A.shape[1] if transa in "Tt" else A.shape[0]
    K = A.shape[0] if transa in "Tt" else A.shape[1]
    N = B.shape[0] if transb in "Tt" else B.shape[1]
    if (B.shape[1] if transb in "Tt" else B.shape[0]) != K:
        raise ValueError("inner dimensions of op(A) and op(B) differ")
    if C is None:
        C = colmajor_empty(M, N, A.device)
        ldc = max(1, M)
    else:
        _check_f64(C, "C", (M, N))
        if C.stride(0) != 1 or (N > 1 and C.stride(1) < M):
            raise ValueError("C must be column-major")
        ldc = max(1, C.stride(1) if N > 1 else M)
    _sync()
    args = (transa.encode(), transb.encode(), M, N, K, alpha, _ptr(A), lda, _ptr(B), ldb, beta,
            _ptr(C), ldc)
    if bf16_terms:
        _check("randutv_gemm_bf16", lib.randutv_gemm_bf16(*args, bf16_terms))
    else:
        fn = "randutv_gemm_f32" if f32 else "randutv_dgemm"
        _check(fn, getattr(lib, fn)(*args))
    return C


def randutv_geqrf(A):
    """Householder QR in place (dgeqr2 conventions).  Returns (A_factored, tau)."""
    torch = _torch()
    lib = load()
    A, lda = as_colmajor(A.clone())
    m, k = A.shape
    tau = torch.empty(k, dtype=torch.float64, device=A.device)
    _sync()
    _check("randutv_geqrf", lib.randutv_geqrf(m, k, _ptr(A), lda, _ptr(tau)))
    return A, tau


def randutv_larft(W, tau):
    """Forward column-wise compact-WY factor of the reflectors below the diagonal of W."""
    lib = load()
    W, ldw = as_colmajor(W)
    m, k = W.shape
    Tf = colmajor_empty(k, k, W.device)
    _sync()
    _check("randutv_larft", lib.randutv_larft(m, k, _ptr(W), ldw, _ptr(tau), _ptr(Tf), max(1, k)))
    return Tf


def randutv_gesvj(R):
    """One-sided Jacobi SVD of a square matrix: returns (Us, d, Vs, sweeps)."""
    torch = _torch()
    lib = load()
    R, ldr = as_colmajor(R)
    k = R.shape[0]
    d = torch.empty(k, dtype=torch.float64, device=R.device)
    Us = colmajor_empty(k, k, R.device)
    Vs = colmajor_empty(k, k, R.device)
    sw = _I32(0)
    _sync()
    _check("randutv_gesvj", lib.randutv_gesvj(k, _ptr(R), ldr, _ptr(d), _ptr(Us), _ptr(Vs),
                                              ctypes.byref(sw)))
    return Us, d, Vs, sw.value


def randutv_set_timing(enable, gemm_only: bool = False, serialize_gemm: bool = False):
    """Per-launch HIP-event timing of later randutv_factor calls (all kernel
    classes, or the GEMM launches only; serialize_gemm: the GEMM launches only,
    each run alone on the chip)."""
    mode = (3 if serialize_gemm else 2 if gemm_only else 1) if enable else 0
    _check("randutv_set_timing", load().randutv_set_timing(mode))


def randutv_kernel_stats():
    """{kernel class: (launches, ms, flops)} for the last timed randutv_factor call."""
    lib = load()
    cap = 32
    names = (ctypes.c_char_p * cap)()
    la = (_I64 * cap)()
    ms = (_D * cap)()
    fl = (_D * cap)()
    n = lib.randutv_kernel_stats(cap, names, la, ms, fl)
    return {names[i].decode(): (la[i], ms[i], fl[i]) for i in range(n)}


STREAM_NAMES = ("T", "P", "UV", "S")


def randutv_kernel_trace():
    """Per-launch record of the last timed randutv_factor call: a list of
    (kernel class, stream name, start ms, duration ms) in enqueue order."""
    lib = load()
    n = lib.randutv_kernel_trace(0, None, None, None, None)
    if n <= 0:
        return []
    cls = (_I32 * n)()
    st = (_I32 * n)()
    t0 = (_D * n)()
    dt = (_D * n)()
    n = min(n, lib.randutv_kernel_trace(n, cls, st, t0, dt))
    cap = 32
    names = (ctypes.c_char_p * cap)()
    k = lib.randutv_kernel_stats(cap, names, None, None, None)
    cname = [names[i].decode() for i in range(k)]
    return [(cname[cls[i]] if 0 <= cls[i] < k else "?", STREAM_NAMES[st[i]] if 0 <= st[i] < 4 else "?",
             t0[i], dt[i]) for i in range(n)]


def randutv_kernel_bytes():
    """{kernel class: algorithmic bytes} over the same launches as randutv_kernel_stats."""
    lib = load()
    cap = 32
    names = (ctypes.c_char_p * cap)()
    by = (_D * cap)()
    n = lib.randutv_kernel_stats(cap, names, None, None, None)
    lib.randutv_kernel_bytes(cap, by)
    return {names[i].decode(): by[i] for i in range(n)}


def randutv_last_sweeps():
    lib = load()
    cap = 4096
    buf = (_I32 * cap)()
    n = lib.randutv_last_sweeps(cap, buf)
    return [buf[i] for i in range(min(n, cap))]


def randutv_strerror(code: int) -> str:
    return load().randutv_strerror(code).decode()
