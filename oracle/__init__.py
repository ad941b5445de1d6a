"""FP64 CPU oracle for randUTV.  TEST INFRASTRUCTURE ONLY: imported by tests/,
__graft_entry__.smoke() and bench.py's CPU-baseline leg, never by the library."""
from .randutv_oracle import (  # noqa: F401
    JACOBI_MAX_SWEEPS,
    block_reflector_T,
    flops_exact,
    flops_std,
    householder_qr,
    householder_reflector,
    jacobi_svd,
    philox_blocks,
    randutv,
    round_robin_pairs,
    sketch_block,
    truncate,
)
