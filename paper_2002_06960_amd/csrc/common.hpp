// Shared definitions of the gfx950 randUTV library (device and host side).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/randutv.h"

namespace rutv {

using i64 = int64_t;

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// wave / block reductions (fixed order, hence deterministic)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

// ---------------------------------------------------------------------------
// grid-wide barrier for kernels whose workgroups are all resident (grids no
// larger than a fraction of the chip).  The counter must be zero at launch;
// the n-th barrier waits for n * gridDim.x arrivals.  The wait is bounded: on
// expiry it records RANDUTV_ERR_SYNC in *err and returns, so every wave exits.
//
// Arrival is a release increment (one L2 write-back); the wait polls with
// relaxed loads and ends with a single acquire fence.  An acquire load per
// poll would invalidate the L2 of the XCD on every iteration, which starves
// whatever else runs there (the GEMMs of the other streams).  Every increment
// is a read-modify-write, so the value that ends the wait lies in the release
// sequence of every arrival and the fence synchronizes with all of them.
// ---------------------------------------------------------------------------
constexpr unsigned kSpinLimit = 1u << 26;

__device__ __forceinline__ void grid_barrier(unsigned* counter, unsigned target, int* err,
                                             unsigned limit = kSpinLimit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    unsigned spins = 0;
    while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > limit) {
        __hip_atomic_store(err, RANDUTV_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// host-side helpers
// ---------------------------------------------------------------------------
// remembers the last HIP error seen by the library (for randutv_last_hip_error)
void note_hip_error(hipError_t e);

inline int hip_code(hipError_t e) {
  if (e == hipSuccess) return RANDUTV_OK;
  note_hip_error(e);
  if (e == hipErrorOutOfMemory) return RANDUTV_ERR_NOMEM;
  return RANDUTV_ERR_HIP;
}

#define RUTV_TRY(expr)                             \
  do {                                             \
    hipError_t _e = (expr);                        \
    if (_e != hipSuccess) return ::rutv::hip_code(_e); \
  } while (0)

#define RUTV_CHECK(expr)           \
  do {                             \
    int _c = (expr);               \
    if (_c != RANDUTV_OK) return _c; \
  } while (0)

inline i64 cdiv(i64 a, i64 b) { return (a + b - 1) / b; }

}  // namespace rutv
