// SVD of the b x b diagonal block that each step of Figure 2 diagonalizes,
// by one-sided Jacobi, spread over P <= 8 workgroups.
//
// W := R, V := I.  The k columns are split into 2P blocks of up to 16
// columns.  A sweep is a round-robin tournament over the blocks (2P-1
// rounds): in each round every workgroup takes one pair of blocks into LDS
// (W and V columns), rotates every column pair across the two blocks (and,
// in the first round, the pairs inside each block), and writes the blocks
// back; a grid barrier separates rounds.  Every column pair is visited once
// per sweep.  Pair (j, q), j < q, is rotated when |w_j.w_q| > k u |w_j||w_q|
// (u = 2^-53) with the Rutishauser rotation
//   zeta = (|w_q|^2 - |w_j|^2) / (2 w_j.w_q),
//   t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),  c = 1/sqrt(1+t^2), s = c t,
//   w_j <- c w_j - s w_q,  w_q <- s w_j + c w_q  (same on V).
// A sweep without rotation ends the iteration (cap: 30 sweeps).  Then
// d_j = |w_j|, columns sorted by descending d (ties keep order),
// u_j = w_j / d_j (Gram-Schmidt completion over e_1, e_2, ... where d_j = 0),
// and (u_j, v_j) negated when the largest-magnitude entry of v_j (lowest
// index on ties) is negative.
//
// Inside a workgroup (4 waves) the 16 disjoint pairs of a step are handled by
// 16-lane groups, each lane holding 16 rows; the dot products are summed
// across the group by DPP butterflies, which leave the bit-identical total in
// all 16 lanes (every lane of a group takes the same rotation decision).
#include <algorithm>

#include "kernels.hpp"

namespace rutv {

constexpr int kJThreads = 256;
constexpr int kJWaves = kJThreads / WAVE;
constexpr int kJRows = kJacobiMaxN / WAVE;  // rows per lane (a wave per column)
constexpr int kJG = 16;                     // lanes per column pair
constexpr int kJRowsG = kJacobiMaxN / kJG;  // rows per lane (a 16-lane group per pair)
constexpr int kJU = 8;                      // block loads in flight per thread
constexpr int kJBW = 16;                    // columns per block
constexpr int kJMaxWG = kJacobiMaxN / (2 * kJBW);

i64 jacobi_work_elems(i64 k) { return 2 * k * k + 64; }

__device__ __forceinline__ int rr_player(int x, int round, int p) {
  if (x == 0) return 0;
  int v = (x - 1 - round) % (p - 1);
  if (v < 0) v += p - 1;
  return 1 + v;
}

__device__ __forceinline__ void wave_sum3(double& a, double& b, double& c) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, WAVE);
    b += __shfl_xor(b, off, WAVE);
    c += __shfl_xor(c, off, WAVE);
  }
}

// rotate columns x (global index gj) and y (global index gq) held in LDS
// (W at wx/wy, V at vx/vy, k rows); returns 1 if rotated
__device__ __forceinline__ int jacobi_pair(int k, int lane, double tol, double* wx, double* wy,
                                           double* vx, double* vy) {
  double xj[kJRows], xq[kJRows];
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int e = 0; e < kJRows; ++e) {
    const int r = lane + WAVE * e;
    xj[e] = r < k ? wx[r] : 0.0;
    xq[e] = r < k ? wy[r] : 0.0;
    al += xj[e] * xj[e];
    be += xq[e] * xq[e];
    ga += xj[e] * xq[e];
  }
  wave_sum3(al, be, ga);
  if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) return 0;
  const double zeta = (be - al) / (2.0 * ga);
  double tn = 1.0;
  if (zeta != 0.0) tn = (zeta > 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + tn * tn);
  const double sn = cs * tn;
#pragma unroll
  for (int e = 0; e < kJRows; ++e) {
    const int r = lane + WAVE * e;
    if (r < k) {
      wx[r] = cs * xj[e] - sn * xq[e];
      wy[r] = sn * xj[e] + cs * xq[e];
      const double yj = vx[r], yq = vy[r];
      vx[r] = cs * yj - sn * yq;
      vy[r] = sn * yj + cs * yq;
    }
  }
  return 1;
}

// one butterfly step across lanes l and l ^ mask inside a 16-lane row (DPP):
// both lanes form the same sum, so the row total is bit-identical in all 16
template <int kCtrl>
__device__ __forceinline__ double dpp_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), kCtrl, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_swap<0xB1>(v);   // quad_perm [1, 0, 3, 2]: lane ^ 1
  v += dpp_swap<0x4E>(v);   // quad_perm [2, 3, 0, 1]: lane ^ 2
  v += dpp_swap<0x141>(v);  // row_half_mirror: lane ^ 7 within 8
  v += dpp_swap<0x140>(v);  // row_mirror: lane ^ 15 within 16
  return v;
}

// the same rotation for a pair handled by a 16-lane group: lane l16 holds
// rows l16 + 16 e (e = 0..15); returns 1 if rotated
__device__ __forceinline__ int jacobi_pair16(int k, int l16, double tol, double* wx, double* wy,
                                             double* vx, double* vy) {
  double xj[kJRowsG], xq[kJRowsG];
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int e = 0; e < kJRowsG; ++e) {
    const int r = l16 + kJG * e;
    xj[e] = r < k ? wx[r] : 0.0;
    xq[e] = r < k ? wy[r] : 0.0;
    al += xj[e] * xj[e];
    be += xq[e] * xq[e];
    ga += xj[e] * xq[e];
  }
  al = row16_sum(al);
  be = row16_sum(be);
  ga = row16_sum(ga);
  if (!(fabs(ga) > tol * sqrt(al) * sqrt(be))) return 0;
  const double zeta = (be - al) / (2.0 * ga);
  double tn = 1.0;
  if (zeta != 0.0) tn = (zeta > 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  const double cs = 1.0 / sqrt(1.0 + tn * tn);
  const double sn = cs * tn;
#pragma unroll
  for (int e = 0; e < kJRowsG; ++e) {
    const int r = l16 + kJG * e;
    if (r < k) {
      wx[r] = cs * xj[e] - sn * xq[e];
      wy[r] = sn * xj[e] + cs * xq[e];
      const double yj = vx[r], yq = vy[r];
      vx[r] = cs * yj - sn * yq;
      vy[r] = sn * yj + cs * yq;
    }
  }
  return 1;
}

// Batched: problem p = blockIdx.x / P uses R + p rs, d + p ds, Us/Vs + p us,
// work + p ws, status + 3 p; every problem is k x k except the last (k_last).
// Per-problem work layout: W (k x k, ld k), V (k x k, ld k), then counters:
// ctr[0] barrier, ctr[1] cumulative rotation count
__global__ __launch_bounds__(kJThreads) void jacobi_block_kernel(int kfull, int k_last, int P,
                                                                 const double* __restrict__ Rall,
                                                                 i64 ldr, i64 rs,
                                                                 double* __restrict__ dall, i64 ds,
                                                                 double* __restrict__ Usall,
                                                                 double* __restrict__ Vsall, i64 us,
                                                                 double* __restrict__ wall, i64 ws,
                                                                 int* __restrict__ stall,
                                                                 int max_sweeps, unsigned spin_limit) {
  const int prob = blockIdx.x / P, wg = blockIdx.x % P;
  const int count = gridDim.x / P;
  const int k = prob == count - 1 ? k_last : kfull;
  const double* R = Rall + prob * rs;
  double* d = dall + prob * ds;
  double* Us = Usall + prob * us;
  double* Vs = Vsall + prob * us;
  double* work = wall + prob * ws;
  int* status = stall + 3 * prob;
  unsigned* ctr = reinterpret_cast<unsigned*>(work + 2 * (i64)kfull * kfull);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nblk = 2 * P;
  double* W = work;
  double* V = work + (i64)k * k;
  __shared__ double Wl[2][kJBW][kJacobiMaxN];
  __shared__ double Vl[2][kJBW][kJacobiMaxN];
  __shared__ int lrot;
  __shared__ double dn[kJacobiMaxN];
  __shared__ int perm[kJacobiMaxN];
  __shared__ int s_done;
  unsigned nbar = 0;
  int* err = status + 2;

  // W := R, V := I (each workgroup its share of the columns)
  for (i64 e = (i64)wg * kJThreads + tid; e < (i64)k * k; e += (i64)P * kJThreads) {
    const int r = (int)(e % k), c = (int)(e / k);
    W[e] = R[r + (i64)c * ldr];
    V[e] = r == c ? 1.0 : 0.0;
  }
  grid_barrier(ctr, (++nbar) * (unsigned)P, err, spin_limit);

  const double tol = (double)k * 0x1p-53;
  int sweeps = 0;
  bool converged = k <= 1;
  unsigned prev_total = 0;
  while (!converged && sweeps < max_sweeps) {
    ++sweeps;
    if (tid == 0) lrot = 0;
    for (int round = 0; round < nblk - 1 || (nblk == 2 && round == 0); ++round) {
      const int pa = rr_player(wg, round, nblk), pb = rr_player(nblk - 1 - wg, round, nblk);
      const int ba = min(pa, pb), bb = max(pa, pb);
      const int blk[2] = {ba, bb};
      // load both blocks (column c of block x is global column x*16 + c),
      // kJU elements per thread in flight at a time
      {
        const int ne = 2 * kJBW * k;
        for (int e0 = tid; e0 < ne; e0 += kJThreads * kJU) {
          double wv[kJU], vv[kJU];
#pragma unroll
          for (int u = 0; u < kJU; ++u) {
            const int e = min(e0 + kJThreads * u, ne - 1);
            const int r = e % k, cc = e / k, x = cc / kJBW, c = cc % kJBW;
            const int gc = min(blk[x] * kJBW + c, k - 1);
            wv[u] = W[r + (i64)gc * k];
            vv[u] = V[r + (i64)gc * k];
          }
#pragma unroll
          for (int u = 0; u < kJU; ++u) {
            const int e = e0 + kJThreads * u;
            if (e < ne) {
              const int r = e % k, cc = e / k, x = cc / kJBW, c = cc % kJBW;
              const bool in = blk[x] * kJBW + c < k;
              Wl[x][c][r] = in ? wv[u] : 0.0;
              Vl[x][c][r] = in ? vv[u] : 0.0;
            }
          }
        }
      }
      __syncthreads();
      int myrot = 0;
      // 16 disjoint pairs at a time, one per 16-lane group (pg = 0..15)
      const int pg = wave * (WAVE / kJG) + (lane >> 4), l16 = lane & (kJG - 1);
      if (round == 0) {
        // pairs inside each block: 15 inner rounds of 8 pairs per block
        const int x = pg / 8, p = pg % 8;
        for (int ir = 0; ir < kJBW - 1; ++ir) {
          const int c1 = rr_player(p, ir, kJBW), c2 = rr_player(kJBW - 1 - p, ir, kJBW);
          const int cj = min(c1, c2), cq = max(c1, c2);
          if (blk[x] * kJBW + cq < k)
            myrot += jacobi_pair16(k, l16, tol, Wl[x][cj], Wl[x][cq], Vl[x][cj], Vl[x][cq]);
          __syncthreads();
        }
      }
      // pairs across the two blocks: 16 inner steps of 16 disjoint pairs
      for (int t = 0; t < kJBW; ++t) {
        const int i = pg, j2 = (pg + t) % kJBW;
        if (ba != bb && ba * kJBW + i < k && bb * kJBW + j2 < k)
          myrot += jacobi_pair16(k, l16, tol, Wl[0][i], Wl[1][j2], Vl[0][i], Vl[1][j2]);
        __syncthreads();
      }
      if (l16 == 0 && myrot) atomicAdd(&lrot, myrot);  // one count per pair group
      // blocks back to global memory
      {
        const int ne = 2 * kJBW * k;
#pragma unroll 4
        for (int e = tid; e < ne; e += kJThreads) {
          const int r = e % k, cc = e / k, x = cc / kJBW, c = cc % kJBW;
          const int gc = blk[x] * kJBW + c;
          if (gc < k) {
            W[r + (i64)gc * k] = Wl[x][c][r];
            V[r + (i64)gc * k] = Vl[x][c][r];
          }
        }
      }
      const bool last = (round == nblk - 2) || nblk == 2;
      if (last) {
        __syncthreads();
        if (tid == 0)
          __hip_atomic_fetch_add(&ctr[1], (unsigned)lrot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      grid_barrier(ctr, (++nbar) * (unsigned)P, err, spin_limit);
      if (last) {
        if (tid == 0) {
          const unsigned tot = __hip_atomic_load(&ctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          s_done = tot == prev_total ? 1 : 0;
          lrot = (int)tot;  // reuse as broadcast of the total
        }
        __syncthreads();
        converged = s_done != 0;
        prev_total = (unsigned)lrot;
        __syncthreads();
        break;
      }
    }
  }
  if (wg == 0 && tid == 0) {
    status[0] = sweeps;
    status[1] = converged ? 1 : 0;
  }

  // ---- outputs: norms, stable descending order, signs (every workgroup
  // derives the same order; each writes its share of the columns)
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
  // rank with a total order (a non-finite norm ranks last), so perm is a
  // permutation of 0..k-1 whatever the values
  if (tid < k) {
    const double dj = isfinite(dn[tid]) ? dn[tid] : -1.0;
    int rank = 0;
    for (int i = 0; i < k; ++i) {
      const double di = isfinite(dn[i]) ? dn[i] : -1.0;
      rank += (di > dj || (di == dj && i < tid)) ? 1 : 0;
    }
    perm[rank] = tid;
  }
  __syncthreads();
  bool any_zero = false;
  for (int qo = wave; qo < k; qo += kJWaves) {
    const int src = perm[qo];
    const double* vc = V + (i64)src * k;
    double mx = 0.0;
    int idx = k;
#pragma unroll
    for (int e = 0; e < kJRows; ++e) {
      const int r = lane + WAVE * e;
      if (r < k) {
        const double a = fabs(vc[r]);
        if (a > mx || idx == k) {
          mx = a;
          idx = r;
        }
      }
    }
    const double gmx = wave_max(mx);
    int cand = (mx == gmx && idx < k) ? idx : k;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) cand = min(cand, __shfl_xor(cand, off, WAVE));
    if (cand >= k) cand = 0;  // only when v holds NaN
    const double sg = vc[cand] < 0.0 ? -1.0 : 1.0;
    if (qo % P != wg) continue;
    const double dv = dn[src];
    const double* wc = W + (i64)src * k;
#pragma unroll
    for (int e = 0; e < kJRows; ++e) {
      const int r = lane + WAVE * e;
      if (r < k) {
        Vs[r + (i64)qo * k] = sg * vc[r];
        Us[r + (i64)qo * k] = dv > 0.0 ? sg * (wc[r] / dv) : 0.0;
      }
    }
    if (lane == 0) d[qo] = dv;
  }
  any_zero = dn[perm[k - 1]] == 0.0;
  if (!any_zero) return;
  // rare: exact zero singular values -> complete U (workgroup 0, wave 0)
  grid_barrier(ctr, (++nbar) * (unsigned)P, err, spin_limit);
  if (wg != 0 || wave != 0) return;
  int cand = 0;
  for (int qo = 0; qo < k; ++qo) {
    const int src = perm[qo];
    if (dn[src] > 0.0) continue;
    // sign of v for this column
    const double* vc = V + (i64)src * k;
    double mx = 0.0;
    int idx = k;
    for (int e = 0; e < kJRows; ++e) {
      const int r = lane + WAVE * e;
      if (r < k && (fabs(vc[r]) > mx || idx == k)) {
        mx = fabs(vc[r]);
        idx = r;
      }
    }
    const double gmx = wave_max(mx);
    int ci = (mx == gmx && idx < k) ? idx : k;
    for (int off = 32; off > 0; off >>= 1) ci = min(ci, __shfl_xor(ci, off, WAVE));
    if (ci >= k) ci = 0;
    const double sg = vc[ci] < 0.0 ? -1.0 : 1.0;
    while (cand < k) {
      double x[kJRows];
#pragma unroll
      for (int e = 0; e < kJRows; ++e) x[e] = (lane + WAVE * e) == cand ? 1.0 : 0.0;
      ++cand;
      for (int pass = 0; pass < 2; ++pass) {
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
        const double s = sg / nr;
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

__global__ void jacobi_zero_kernel(int count, int kfull, double* __restrict__ wall, i64 ws,
                                   int* __restrict__ stall) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  unsigned* ctr = reinterpret_cast<unsigned*>(wall + p * ws + 2 * (i64)kfull * kfull);
  ctr[0] = 0u;
  ctr[1] = 0u;
  stall[3 * p] = stall[3 * p + 1] = stall[3 * p + 2] = 0;
}

int jacobi_svd_batched(hipStream_t st, int count, i64 k, i64 k_last, const double* R, i64 ldr,
                       i64 rs, double* d, i64 ds, double* Us, double* Vs, i64 us, double* work,
                       int* status, int max_sweeps, unsigned spin_limit) {
  if (count <= 0 || k <= 0) return RANDUTV_OK;
  if (k > kJacobiMaxN || k_last > k || k_last <= 0) return RANDUTV_ERR_TOO_LARGE;
  const int P = (int)std::max<i64>(1, std::min<i64>(kJMaxWG, cdiv(k, 2 * kJBW)));
  const i64 ws = jacobi_work_elems(k);
  LaunchTimer* tm = launch_timer();
  jacobi_zero_kernel<<<(count + 63) / 64, 64, 0, st>>>(count, (int)k, work, ws, status);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->begin(st, K_JACOBI);
  jacobi_block_kernel<<<P * count, kJThreads, 0, st>>>(
      (int)k, (int)k_last, P, R, ldr, rs, d, ds, Us, Vs, us, work, ws, status,
      max_sweeps > 0 ? max_sweeps : kJacobiMaxSweeps, spin_limit ? spin_limit : kSpinLimit);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->end(st, K_JACOBI, 0.0, 0.0);
  return RANDUTV_OK;
}

int jacobi_svd(hipStream_t st, i64 k, const double* R, i64 ldr, double* d, double* Us, double* Vs,
               double* work, int* status, int max_sweeps, unsigned spin_limit) {
  return jacobi_svd_batched(st, 1, k, k, R, ldr, 0, d, 0, Us, Vs, 0, work, status, max_sweeps,
                            spin_limit);
}

}  // namespace rutv
