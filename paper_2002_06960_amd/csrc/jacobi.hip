// SVD of the b x b diagonal block (Figure 2, "[A11, U_SVD, V_SVD] := SVD(A11)")
// by one-sided Jacobi in a single workgroup.
//
// W := R, V := I; sweeps of the round-robin tournament ordering (b-1 rounds of
// b/2 disjoint column pairs, one wave per pair); pair (j, k) is rotated when
// |w_j.w_k| > b u |w_j| |w_k| (u = 2^-53) with the Rutishauser rotation
// zeta = (|w_k|^2 - |w_j|^2) / (2 w_j.w_k), t = sign(zeta)/(|zeta| + sqrt(1+zeta^2)).
// A sweep without rotation ends the iteration (cap: 30 sweeps).  Then
// d_j = |w_j|, columns sorted by descending d (ties keep order),
// u_j = w_j / d_j (Gram-Schmidt completion over e_1, e_2, ... where d_j = 0),
// and (u_j, v_j) negated when the largest-magnitude entry of v_j (lowest
// index on ties) is negative.
#include "kernels.hpp"

namespace rutv {

constexpr int kJThreads = 1024;
constexpr int kJWaves = kJThreads / WAVE;
constexpr int kJRows = kJacobiMaxN / WAVE;  // rows per lane

i64 jacobi_work_elems(i64 k) { return 2 * k * k; }

__device__ __forceinline__ int rr_player(int x, int round, int p) {
  if (x == 0) return 0;
  int v = (x - 1 - round) % (p - 1);
  if (v < 0) v += p - 1;
  return 1 + v;
}

__global__ __launch_bounds__(kJThreads) void jacobi_kernel(int k, const double* __restrict__ R,
                                                           i64 ldr, double* __restrict__ d,
                                                           double* __restrict__ Us,
                                                           double* __restrict__ Vs,
                                                           double* __restrict__ work,
                                                           int* __restrict__ status) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double* W = work;          // k x k, ld k
  double* V = work + (i64)k * k;
  __shared__ int rotated;
  __shared__ double dn[kJacobiMaxN];
  __shared__ int perm[kJacobiMaxN];
  __shared__ double sgn[kJacobiMaxN];

  for (int e = tid; e < k * k; e += kJThreads) {
    const int r = e % k, c = e / k;
    W[e] = R[r + (i64)c * ldr];
    V[e] = r == c ? 1.0 : 0.0;
  }
  __syncthreads();

  const double tol = (double)k * 0x1p-53;
  const int p = k + (k & 1);
  int sweeps = 0;
  bool converged = k <= 1;
  while (!converged && sweeps < kJacobiMaxSweeps) {
    ++sweeps;
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < p - 1; ++round) {
      for (int t = wave; t < p / 2; t += kJWaves) {
        int a = rr_player(t, round, p), c = rr_player(p - 1 - t, round, p);
        if (a >= k || c >= k) continue;
        const int j = min(a, c), q = max(a, c);
        double* wj = W + (i64)j * k;
        double* wq = W + (i64)q * k;
        double xj[kJRows], xq[kJRows];
        double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
        for (int e = 0; e < kJRows; ++e) {
          const int r = lane + WAVE * e;
          xj[e] = r < k ? wj[r] : 0.0;
          xq[e] = r < k ? wq[r] : 0.0;
          al += xj[e] * xj[e];
          be += xq[e] * xq[e];
          ga += xj[e] * xq[e];
        }
        al = wave_sum(al);
        be = wave_sum(be);
        ga = wave_sum(ga);
        if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) continue;
        const double zeta = (be - al) / (2.0 * ga);
        double tn = 1.0;
        if (zeta != 0.0) tn = (zeta > 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double cs = 1.0 / sqrt(1.0 + tn * tn);
        const double sn = cs * tn;
        double* vj = V + (i64)j * k;
        double* vq = V + (i64)q * k;
#pragma unroll
        for (int e = 0; e < kJRows; ++e) {
          const int r = lane + WAVE * e;
          if (r < k) {
            wj[r] = cs * xj[e] - sn * xq[e];
            wq[r] = sn * xj[e] + cs * xq[e];
            const double yj = vj[r], yq = vq[r];
            vj[r] = cs * yj - sn * yq;
            vq[r] = sn * yj + cs * yq;
          }
        }
        if (lane == 0) rotated = 1;
      }
      __syncthreads();
    }
    converged = rotated == 0;
    __syncthreads();
  }
  if (tid == 0) {
    status[0] = sweeps;
    status[1] = converged ? 1 : 0;
  }

  // column norms
  for (int c = wave; c < k; c += kJWaves) {
    const double* wc = W + (i64)c * k;
    double s = 0.0;
#pragma unroll
    for (int e = 0; e < kJRows; ++e) {
      const int r = lane + WAVE * e;
      if (r < k) s += wc[r] * wc[r];
    }
    s = wave_sum(s);
    if (lane == 0) dn[c] = sqrt(s);
  }
  __syncthreads();
  // stable descending order
  if (tid < k) {
    const double dj = dn[tid];
    int rank = 0;
    for (int i = 0; i < k; ++i) {
      const double di = dn[i];
      rank += (di > dj || (di == dj && i < tid)) ? 1 : 0;
    }
    perm[rank] = tid;
  }
  __syncthreads();
  // sign of each output column from its v: largest |entry|, lowest index on ties
  for (int qo = wave; qo < k; qo += kJWaves) {
    const double* vc = V + (i64)perm[qo] * k;
    double mx = 0.0;
    int idx = k;
#pragma unroll
    for (int e = 0; e < kJRows; ++e) {
      const int r = lane + WAVE * e;
      if (r < k) {
        const double a = fabs(vc[r]);
        if (a > mx || idx == k) { mx = a; idx = r; }
      }
    }
    // reduce (max |v|, then min index)
    double gmx = wave_max(mx);
    int cand = (mx == gmx && idx < k) ? idx : k;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cand = min(cand, __shfl_xor(cand, off, WAVE));
    if (lane == 0) sgn[qo] = vc[cand] < 0.0 ? -1.0 : 1.0;
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += kJThreads) {
    const int r = e % k, qo = e / k;
    const int src = perm[qo];
    const double s = sgn[qo];
    Vs[r + (i64)qo * k] = s * V[r + (i64)src * k];
    const double dv = dn[src];
    Us[r + (i64)qo * k] = dv > 0.0 ? s * (W[r + (i64)src * k] / dv) : 0.0;
  }
  if (tid < k) d[tid] = dn[perm[tid]];
  __syncthreads();
  // completion of u_j where d_j == 0 (they sit at the end of the order)
  if (wave == 0) {
    int cand = 0;
    for (int qo = 0; qo < k; ++qo) {
      if (dn[perm[qo]] > 0.0) continue;
      while (cand < k) {
        double x[kJRows];
#pragma unroll
        for (int e = 0; e < kJRows; ++e) x[e] = (lane + WAVE * e) == cand ? 1.0 : 0.0;
        ++cand;
        for (int pass = 0; pass < 2; ++pass) {
          // x -= Us (Us^T x), columns of Us in order
          double y[kJRows];
#pragma unroll
          for (int e = 0; e < kJRows; ++e) y[e] = x[e];
          for (int c = 0; c < k; ++c) {
            const double* uc = Us + (i64)c * k;
            double s = 0.0;
#pragma unroll
            for (int e = 0; e < kJRows; ++e) {
              const int r = lane + WAVE * e;
              if (r < k) s += uc[r] * x[e];
            }
            s = wave_sum(s);
#pragma unroll
            for (int e = 0; e < kJRows; ++e) {
              const int r = lane + WAVE * e;
              if (r < k) y[e] -= uc[r] * s;
            }
          }
#pragma unroll
          for (int e = 0; e < kJRows; ++e) x[e] = y[e];
        }
        double nr = 0.0;
#pragma unroll
        for (int e = 0; e < kJRows; ++e) nr += x[e] * x[e];
        nr = sqrt(wave_sum(nr));
        if (nr > 0.5) {
          const double s = sgn[qo] / nr;
#pragma unroll
          for (int e = 0; e < kJRows; ++e) {
            const int r = lane + WAVE * e;
            if (r < k) Us[r + (i64)qo * k] = s * x[e];
          }
          break;
        }
      }
    }
  }
}

int jacobi_svd(hipStream_t st, i64 k, const double* R, i64 ldr, double* d, double* Us, double* Vs,
               double* work, int* status) {
  if (k <= 0) return RANDUTV_OK;
  if (k > kJacobiMaxN) return RANDUTV_ERR_TOO_LARGE;
  LaunchTimer* tm = launch_timer();
  if (tm) tm->begin(st, K_JACOBI);
  jacobi_kernel<<<1, kJThreads, 0, st>>>((int)k, R, ldr, d, Us, Vs, work, status);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->end(st, K_JACOBI, 0.0);
  return RANDUTV_OK;
}

}  // namespace rutv
