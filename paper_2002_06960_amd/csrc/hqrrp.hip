// HQRRP, the randomized blocked column-pivoted QR A P = Q R (Section 2): the
// pivot choice of one step (b steps of Householder CPQR on the sketch
// Y = G R22, Section 2.2) and the column exchanges that realise it.  The
// sketch product, the panel QR and the trailing update are the library's GEMM,
// panel and compact-WY kernels (randutv.hip drives the step loop).
#include <climits>

#include "kernels.hpp"

namespace rutv {

constexpr int kCpThreads = 256;
constexpr int kCpWaves = kCpThreads / WAVE;
constexpr int kCpMaxWG = 256;
constexpr int kCpMaxCols = 1024;  // columns owned by one workgroup
constexpr int kCpMinCols = 32;

static int cpqr_grid(i64 N) { return (int)std::min<i64>(kCpMaxWG, std::max<i64>(1, cdiv(N, kCpMinCols))); }

// (value, column) order of the pivot search: larger residual norm first, the
// lower column index on equal norms
__device__ __forceinline__ bool better(double v, int i, double bv, int bi) {
  return v > bv || (v == bv && i < bi);
}

// k steps of Householder CPQR on Y (k x N, ld ldy, k <= 256), Y overwritten.
// Workgroup w owns a contiguous range of columns; a step is: residual norms
// of the owned unused columns (rows t..k-1) -> per-workgroup best ->
// grid barrier -> every workgroup takes the global best p and forms the
// reflector of column p (same code and data everywhere, so the same bits)
// -> each applies it to its owned unused columns.  Column p is never written
// after it is chosen, so reading it across workgroups needs no second barrier.
// The slots alternate by step parity: a slot is rewritten two steps later,
// after a barrier that every reader of it has passed.
__global__ __launch_bounds__(kCpThreads) void cpqr_pivots_kernel(
    int k, int N, double* __restrict__ Y, i64 ldy, int* __restrict__ J,
    double* __restrict__ sval, int* __restrict__ sidx, unsigned* __restrict__ counter,
    int* __restrict__ err) {
  const int P = gridDim.x, w = blockIdx.x, tid = threadIdx.x, lane = tid & (WAVE - 1),
            wave = tid / WAVE;
  const int chunk = (N + P - 1) / P;
  const int c0 = min(N, w * chunk), c1 = min(N, c0 + chunk), nc = c1 - c0;
  __shared__ unsigned char used[kCpMaxCols];
  __shared__ double v[kPanelMaxCols];
  __shared__ double bestv[kCpWaves];
  __shared__ int besti[kCpWaves];
  __shared__ double tau_s;
  __shared__ int piv_s, stop_s;
  for (int e = tid; e < nc; e += kCpThreads) used[e] = 0;
  __syncthreads();
  unsigned nbar = 0;
  for (int t = 0; t < k; ++t) {
    // residual norms of the owned unused columns
    double bv = -1.0;
    int bi = INT_MAX;
    for (int e = wave; e < nc; e += kCpWaves) {
      if (used[e]) continue;
      const double* y = Y + (i64)(c0 + e) * ldy;
      double s = 0.0;
      for (int r = t + lane; r < k; r += WAVE) s += y[r] * y[r];
      s = wave_sum(s);
      if (!(s >= 0.0)) s = -0.5;  // NaN: still a candidate, below every real norm
      if (better(s, c0 + e, bv, bi)) bv = s, bi = c0 + e;
    }
    if (lane == 0) bestv[wave] = bv, besti[wave] = bi;
    __syncthreads();
    if (tid == 0) {
      double v0 = bestv[0];
      int i0 = besti[0];
      for (int q = 1; q < kCpWaves; ++q)
        if (better(bestv[q], besti[q], v0, i0)) v0 = bestv[q], i0 = besti[q];
      sval[(t & 1) * P + w] = v0;
      sidx[(t & 1) * P + w] = i0;
    }
    grid_barrier(counter, (++nbar) * (unsigned)P, err);
    if (tid == 0) stop_s = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    __syncthreads();
    if (stop_s) return;
    // the global pivot
    if (wave == 0) {
      double v0 = -2.0;
      int i0 = INT_MAX;
      for (int q = lane; q < P; q += WAVE)
        if (better(sval[(t & 1) * P + q], sidx[(t & 1) * P + q], v0, i0))
          v0 = sval[(t & 1) * P + q], i0 = sidx[(t & 1) * P + q];
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v0, off, WAVE);
        const int oi = __shfl_xor(i0, off, WAVE);
        if (better(ov, oi, v0, i0)) v0 = ov, i0 = oi;
      }
      if (lane == 0) piv_s = i0;
    }
    __syncthreads();
    const int p = piv_s;
    if (w == 0 && tid == 0) J[t] = p;
    if (tid == 0 && p >= c0 && p < c1) used[p - c0] = 1;
    // reflector of column p, rows t..k-1 (dlarfg): H x = beta e_1
    if (wave == 0) {
      const double* x = Y + (i64)p * ldy;
      const double alpha = x[t];
      double s = 0.0;
      for (int r = t + 1 + lane; r < k; r += WAVE) s += x[r] * x[r];
      s = wave_sum(s);
      const double xnorm = sqrt(s);
      double tau = 0.0, den = 1.0;
      if (xnorm != 0.0) {
        const double beta = alpha >= 0.0 ? -hypot(alpha, xnorm) : hypot(alpha, xnorm);
        tau = (beta - alpha) / beta;
        den = alpha - beta;
      }
      for (int r = t + lane; r < k; r += WAVE) v[r] = r == t ? 1.0 : (tau != 0.0 ? x[r] / den : 0.0);
      if (lane == 0) tau_s = tau;
    }
    __syncthreads();
    const double tau = tau_s;
    if (tau != 0.0) {
      for (int e = wave; e < nc; e += kCpWaves) {
        if (used[e]) continue;
        double* y = Y + (i64)(c0 + e) * ldy;
        double s = 0.0;
        for (int r = t + lane; r < k; r += WAVE) s += v[r] * y[r];
        s = wave_sum(s) * tau;
        for (int r = t + lane; r < k; r += WAVE) y[r] -= s * v[r];
      }
    }
    __syncthreads();
  }
}

// The same steps with the workgroup's columns held in LDS (when they fit):
// Y is read once; every workgroup also publishes its best column (rows t..)
// beside its norm, and after the barrier all take the winner's copy.
constexpr int kCpSlab = 16384;  // doubles of LDS for the owned columns (128 KiB)

__global__ __launch_bounds__(kCpThreads) void cpqr_pivots_lds_kernel(
    int k, int N, const double* __restrict__ Y, i64 ldy, int* __restrict__ J,
    double* __restrict__ sval, int* __restrict__ sidx, double* __restrict__ scol,
    unsigned* __restrict__ counter, int* __restrict__ err) {
  const int P = gridDim.x, w = blockIdx.x, tid = threadIdx.x, lane = tid & (WAVE - 1),
            wave = tid / WAVE;
  const int chunk = (N + P - 1) / P;
  const int c0 = min(N, w * chunk), c1 = min(N, c0 + chunk), nc = c1 - c0;
  __shared__ double slab[kCpSlab];  // owned column e, row r at e * k + r
  __shared__ unsigned char used[kCpMaxCols];
  __shared__ double v[kPanelMaxCols];
  __shared__ double bestv[kCpWaves];
  __shared__ int besti[kCpWaves];
  __shared__ double tau_s;
  __shared__ int piv_s, win_s, stop_s, mybest_s;
  for (int e = tid; e < nc; e += kCpThreads) used[e] = 0;
  for (int q = tid; q < nc * k; q += kCpThreads) {
    const int e = q / k, r = q - e * k;
    slab[q] = Y[r + (i64)(c0 + e) * ldy];
  }
  __syncthreads();
  unsigned nbar = 0;
  for (int t = 0; t < k; ++t) {
    double bv = -1.0;
    int bi = INT_MAX;
    for (int e = wave; e < nc; e += kCpWaves) {
      if (used[e]) continue;
      const double* y = slab + e * k;
      double s = 0.0;
      for (int r = t + lane; r < k; r += WAVE) s += y[r] * y[r];
      s = wave_sum(s);
      if (!(s >= 0.0)) s = -0.5;
      if (better(s, c0 + e, bv, bi)) bv = s, bi = c0 + e;
    }
    if (lane == 0) bestv[wave] = bv, besti[wave] = bi;
    __syncthreads();
    if (tid == 0) {
      double v0 = bestv[0];
      int i0 = besti[0];
      for (int q = 1; q < kCpWaves; ++q)
        if (better(bestv[q], besti[q], v0, i0)) v0 = bestv[q], i0 = besti[q];
      sval[(t & 1) * P + w] = v0;
      sidx[(t & 1) * P + w] = i0;
      mybest_s = i0;
    }
    __syncthreads();
    // publish the candidate column (rows t..k-1)
    if (mybest_s != INT_MAX) {
      const double* y = slab + (mybest_s - c0) * k;
      double* dst = scol + ((i64)(t & 1) * P + w) * kPanelMaxCols;
      for (int r = t + tid; r < k; r += kCpThreads) dst[r] = y[r];
    }
    grid_barrier(counter, (++nbar) * (unsigned)P, err);
    if (tid == 0) stop_s = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
    __syncthreads();
    if (stop_s) return;
    if (wave == 0) {
      double v0 = -2.0;
      int i0 = INT_MAX, q0 = 0;
      for (int q = lane; q < P; q += WAVE)
        if (better(sval[(t & 1) * P + q], sidx[(t & 1) * P + q], v0, i0))
          v0 = sval[(t & 1) * P + q], i0 = sidx[(t & 1) * P + q], q0 = q;
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(v0, off, WAVE);
        const int oi = __shfl_xor(i0, off, WAVE), oq = __shfl_xor(q0, off, WAVE);
        if (better(ov, oi, v0, i0)) v0 = ov, i0 = oi, q0 = oq;
      }
      if (lane == 0) piv_s = i0, win_s = q0;
    }
    __syncthreads();
    const int p = piv_s;
    if (w == 0 && tid == 0) J[t] = p;
    if (tid == 0 && p >= c0 && p < c1) used[p - c0] = 1;
    if (wave == 0) {
      const double* x = scol + ((i64)(t & 1) * P + win_s) * kPanelMaxCols;
      const double alpha = x[t];
      double s = 0.0;
      for (int r = t + 1 + lane; r < k; r += WAVE) s += x[r] * x[r];
      s = wave_sum(s);
      const double xnorm = sqrt(s);
      double tau = 0.0, den = 1.0;
      if (xnorm != 0.0) {
        const double beta = alpha >= 0.0 ? -hypot(alpha, xnorm) : hypot(alpha, xnorm);
        tau = (beta - alpha) / beta;
        den = alpha - beta;
      }
      for (int r = t + lane; r < k; r += WAVE) v[r] = r == t ? 1.0 : (tau != 0.0 ? x[r] / den : 0.0);
      if (lane == 0) tau_s = tau;
    }
    __syncthreads();
    const double tau = tau_s;
    if (tau != 0.0) {
      for (int e = wave; e < nc; e += kCpWaves) {
        if (used[e]) continue;
        double* y = slab + e * k;
        double s = 0.0;
        for (int r = t + lane; r < k; r += WAVE) s += v[r] * y[r];
        s = wave_sum(s) * tau;
        for (int r = t + lane; r < k; r += WAVE) y[r] -= s * v[r];
      }
    }
    __syncthreads();
  }
}

int cpqr_pivots(hipStream_t st, i64 k, i64 N, double* Y, i64 ldy, int* J, CpqrWork& w) {
  if (k <= 0 || N <= 0) return RANDUTV_OK;
  if (k > kPanelMaxCols || k > N) return RANDUTV_ERR_TOO_LARGE;
  const int P = cpqr_grid(N);
  if (cdiv(N, P) > kCpMaxCols || N > INT32_MAX) return RANDUTV_ERR_TOO_LARGE;
  RUTV_CHECK(fill_zero_u32(st, w.counter, 1));
  if (cdiv(N, P) * k <= kCpSlab)
    cpqr_pivots_lds_kernel<<<P, kCpThreads, 0, st>>>((int)k, (int)N, Y, ldy, J, w.sval, w.sidx,
                                                     w.scol, w.counter, w.err);
  else
    cpqr_pivots_kernel<<<P, kCpThreads, 0, st>>>((int)k, (int)N, Y, ldy, J, w.sval, w.sidx,
                                                 w.counter, w.err);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// tmp(:, u) := A(:, idx[chg[u]]), jtmp[u] := jp[idx[chg[u]]] for u < *cnt
__global__ __launch_bounds__(256) void gather_cols_kernel(i64 m, int maxc, const int* __restrict__ chg,
                                                          const int* __restrict__ cnt,
                                                          const int* __restrict__ idx,
                                                          const double* __restrict__ A, i64 lda,
                                                          double* __restrict__ tmp,
                                                          const int64_t* __restrict__ jp,
                                                          int64_t* __restrict__ jtmp) {
  const int c = *cnt;
  const i64 total = m * (i64)maxc;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const int u = (int)(e / m);
    const i64 r = e - (i64)u * m;
    if (u >= c) continue;
    const int src = idx[chg[u]];
    tmp[r + (i64)u * m] = A[r + (i64)src * lda];
    if (r == 0) jtmp[u] = jp[src];
  }
}

// A(:, chg[u]) := tmp(:, u), jp[chg[u]] := jtmp[u] for u < *cnt
__global__ __launch_bounds__(256) void scatter_cols_kernel(i64 m, int maxc, const int* __restrict__ chg,
                                                           const int* __restrict__ cnt,
                                                           const double* __restrict__ tmp,
                                                           double* __restrict__ A, i64 lda,
                                                           const int64_t* __restrict__ jtmp,
                                                           int64_t* __restrict__ jp) {
  const int c = *cnt;
  const i64 total = m * (i64)maxc;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const int u = (int)(e / m);
    const i64 r = e - (i64)u * m;
    if (u >= c) continue;
    const int dst = chg[u];
    A[r + (i64)dst * lda] = tmp[r + (i64)u * m];
    if (r == 0) jp[dst] = jtmp[u];
  }
}

// idx (position -> original column, N <= 32768 entries) from exchanging the
// column holding J[t] with position t, t = 0..k-1, walked in LDS; chg lists
// the positions whose column changed (at most 2k; their order does not matter
// to the gather and scatter), *cnt their number
constexpr int kExMaxLds = 32768;
__global__ __launch_bounds__(256) void exchange_plan_lds_kernel(int k, int N, const int* __restrict__ J,
                                                                int* __restrict__ idx,
                                                                int* __restrict__ chg,
                                                                int* __restrict__ cnt) {
  __shared__ unsigned short ix[kExMaxLds], wh[kExMaxLds];
  __shared__ int n_s;
  for (int q = threadIdx.x; q < N; q += 256) ix[q] = (unsigned short)q, wh[q] = (unsigned short)q;
  if (threadIdx.x == 0) n_s = 0;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int t = 0; t < k; ++t) {
      const int c = J[t];
      if (c < 0 || c >= N) continue;  // cannot happen (every step has a candidate); keeps accesses in bounds
      const int p = wh[c], a = ix[t];
      ix[t] = (unsigned short)c;
      ix[p] = (unsigned short)a;
      wh[c] = (unsigned short)t;
      wh[a] = (unsigned short)p;
    }
  }
  __syncthreads();
  for (int q = threadIdx.x; q < N; q += 256) {
    idx[q] = ix[q];
    if (ix[q] != q) {
      const int u = atomicAdd(&n_s, 1);
      if (u < 2 * k) chg[u] = q;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *cnt = min(n_s, 2 * k);
}

int exchange_columns(hipStream_t st, i64 m, i64 k, i64 N, const int* J, double* A, i64 lda,
                     int64_t* jp, ExchangeWork& w) {
  if (k <= 0 || N <= 0 || m <= 0) return RANDUTV_OK;
  if (N > kExMaxLds || k > N) return RANDUTV_ERR_TOO_LARGE;
  exchange_plan_lds_kernel<<<1, 256, 0, st>>>((int)k, (int)N, J, w.idx, w.chg, w.cnt);
  RUTV_TRY(hipGetLastError());
  const int maxc = (int)(2 * k);
  const int blocks = (int)std::min<i64>(cdiv(m * maxc, 256), 8192);
  gather_cols_kernel<<<blocks, 256, 0, st>>>(m, maxc, w.chg, w.cnt, w.idx, A, lda, w.tmp, jp, w.jtmp);
  RUTV_TRY(hipGetLastError());
  scatter_cols_kernel<<<blocks, 256, 0, st>>>(m, maxc, w.chg, w.cnt, w.tmp, A, lda, w.jtmp, jp);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

__global__ __launch_bounds__(256) void iota_kernel(i64 n, int64_t* __restrict__ x) {
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < n; e += (i64)gridDim.x * 256) x[e] = e;
}

int set_iota(hipStream_t st, i64 n, int64_t* x) {
  if (n <= 0) return RANDUTV_OK;
  iota_kernel<<<(int)std::min<i64>(cdiv(n, 256), 4096), 256, 0, st>>>(n, x);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

}  // namespace rutv
