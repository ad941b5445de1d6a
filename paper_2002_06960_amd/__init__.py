"""randUTV (A = U T V^T) for one AMD Instinct MI355X (gfx950).

The factorization runs in hand-written HIP kernels behind a C ABI
(include/randutv.h, librandutv.so); this package is the thin Python binding.
"""
from .randutv import (  # noqa: F401
    RandUTVError,
    RandutvArgs,
    make_args,
    sketch_offsets,
    randutv_sketch_host,
    randutv_sketch_words,
    as_colmajor,
    colmajor_empty,
    first_block_truncation,
    truncation,
    load,
    randutv_dgemm,
    randutv_factor,
    randutv_factor_ooc,
    host_colmajor_empty,
    randutv_geqrf,
    randutv_gesvj,
    randutv_hqrrp,
    randutv_geqrf_blocked,
    randutv_kernel_stats,
    randutv_kernel_bytes,
    randutv_kernel_trace,
    randutv_factor_status,
    randutv_larft,
    randutv_last_sweeps,
    randutv_set_timing,
    randutv_sketch,
    randutv_strerror,
    randutv_truncate,
    randutv_truncate_first_block,
    randutv_truncate_first_block_k,
    randutv_truncate_batched,
    randutv_truncate_grad,
    randutv_truncate_grad_k,
)


def flops_std(m: int, n: int, q: int, build_u: bool = True, build_v: bool = True) -> float:
    """Leading-order flop count of randUTV used to express throughput:
    (1+2q)(m n^2 - n^3/3) + 2 m n^2 + (2 m n^2 - 2n^3/3) [+ 2 n^3 for V]
    [+ 4 m^2 n - 2 m n^2 for U]."""
    m, n = float(m), float(n)
    f = (1 + 2 * q) * (m * n * n - n ** 3 / 3.0) + 4 * m * n * n - 2 * n ** 3 / 3.0
    if build_v:
        f += 2 * n ** 3
    if build_u:
        f += 4 * m * m * n - 2 * m * n * n
    return f
