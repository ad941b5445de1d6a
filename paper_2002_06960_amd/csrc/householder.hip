// Householder QR of a tall panel (m x k, k <= 256) and the compact-WY factor.
//
// "unpivoted_QR" of Figure 2 (used for the sketch Y and for the current
// column block of T) with LAPACK dgeqr2 conventions: reflector H_j =
// I - tau_j v_j v_j^T, v_j(j) = 1, beta_j = -sign(alpha_j) ||x_j||,
// tau_j = (beta_j - alpha_j)/beta_j, sign(0) = +1, tau_j = 0 when the part
// below the diagonal is exactly zero.
//
// Panel kernel layout: P workgroups each own a contiguous slab of rows.  The
// panel is processed in leaves of 16 columns.  Within a leaf each column
// needs one grid-wide reduction (sum of squares below the diagonal plus the
// dot products with the leaf's remaining columns, combined with the pivot
// row): every workgroup publishes its partial sums, passes a grid barrier and
// sums all partials in the same order, so every workgroup derives the
// bit-identical reflector and updates its own rows.  After a leaf, the rest
// of the panel receives the leaf's block reflector C <- (I - W Tl W^T)^T C
// (Gram of the leaf vectors and W^T C reduced across workgroups).
#include <algorithm>

#include "kernels.hpp"

namespace rutv {

constexpr int kPQThreads = 256;
constexpr int kPQNB = 16;          // leaf width
constexpr int kPQMaxRows = 320;    // rows of one workgroup's slab
constexpr int kPQColPart = kPQNB + 1;
constexpr int kPQTrail = kPQNB * kPQNB + kPQNB * kPanelMaxCols;

static int panel_grid(i64 m) {
  i64 P = std::max<i64>(cdiv(m, kPQMaxRows), std::min<i64>(128, cdiv(m, 64)));
  return (int)std::max<i64>(P, 1);
}

i64 panel_work_elems(i64 m) {
  const i64 P = panel_grid(m);
  return 2 * P * kPQColPart + 2 * kPQNB + P * kPQTrail + kPQTrail;
}

__global__ __launch_bounds__(kPQThreads) void panel_qr_kernel(int m, int k, double* __restrict__ A,
                                                              i64 lda, double* __restrict__ tau,
                                                              double* __restrict__ work,
                                                              unsigned* __restrict__ bar,
                                                              int* __restrict__ err) {
  const int P = gridDim.x, wg = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = (int)((i64)m * wg / P), r1 = (int)((i64)m * (wg + 1) / P), R = r1 - r0;
  double* colpart = work;                          // [2][P][kPQColPart]
  double* piv = colpart + 2 * P * kPQColPart;      // [2][kPQNB]
  double* tpart = piv + 2 * kPQNB;                 // [P][kPQTrail]
  double* ttot = tpart + (i64)P * kPQTrail;        // [kPQTrail]

  __shared__ double L[kPQNB * kPQMaxRows];
  __shared__ double red[4 * kPQColPart];
  __shared__ double tot[kPQColPart];
  __shared__ double bc[kPQNB + 4];
  __shared__ double Gs[kPQNB * kPQNB];
  __shared__ double Tl[kPQNB * kPQNB];
  __shared__ double Yt[kPQNB * kPanelMaxCols];
  __shared__ double taul[kPQNB];
  unsigned nbar = 0;

  for (int c0 = 0; c0 < k; c0 += kPQNB) {
    const int nbl = min(kPQNB, k - c0);
    for (int e = tid; e < R * nbl; e += kPQThreads) {
      const int r = e % R, c = e / R;
      L[c * kPQMaxRows + r] = A[(i64)(r0 + r) + (i64)(c0 + c) * lda];
    }
    __syncthreads();

    for (int jj = 0; jj < nbl; ++jj) {
      const int j = c0 + jj;
      // ---- partial sums over own rows strictly below the diagonal
      double acc[kPQColPart];
#pragma unroll
      for (int c = 0; c < kPQColPart; ++c) acc[c] = 0.0;
      for (int r = tid; r < R; r += kPQThreads) {
        if (r0 + r > j) {
          const double x = L[jj * kPQMaxRows + r];
          acc[0] += x * x;
#pragma unroll
          for (int c = 0; c < kPQNB; ++c)
            if (c > jj && c < nbl) acc[1 + c] += x * L[c * kPQMaxRows + r];
        }
      }
#pragma unroll
      for (int c = 0; c < kPQColPart; ++c) {
        const double v = wave_sum(acc[c]);
        if (lane == 0) red[wave * kPQColPart + c] = v;
      }
      __syncthreads();
      double* cp = colpart + ((j & 1) * P + wg) * kPQColPart;
      if (tid < kPQColPart)
        cp[tid] = ((red[tid] + red[kPQColPart + tid]) + red[2 * kPQColPart + tid]) +
                  red[3 * kPQColPart + tid];
      if (j >= r0 && j < r1 && tid >= jj && tid < nbl)
        piv[(j & 1) * kPQNB + tid] = L[tid * kPQMaxRows + (j - r0)];
      grid_barrier(bar, (++nbar) * (unsigned)P, err);

      // ---- totals, summed in the same order in every workgroup
      {
        double v[kPQColPart];
#pragma unroll
        for (int c = 0; c < kPQColPart; ++c) v[c] = 0.0;
        const double* cpb = colpart + (j & 1) * P * kPQColPart;
        if (tid < P) {
#pragma unroll
          for (int c = 0; c < kPQColPart; ++c) v[c] = cpb[tid * kPQColPart + c];
        }
#pragma unroll
        for (int c = 0; c < kPQColPart; ++c) {
          const double s = wave_sum(v[c]);
          if (lane == 0) red[wave * kPQColPart + c] = s;
        }
        __syncthreads();
        if (tid < kPQColPart)
          tot[tid] = ((red[tid] + red[kPQColPart + tid]) + red[2 * kPQColPart + tid]) +
                     red[3 * kPQColPart + tid];
        __syncthreads();
      }
      if (tid == 0) {
        const double s = tot[0];
        const double alpha = piv[(j & 1) * kPQNB + jj];
        double t = 0.0, scale = 0.0, beta = alpha;
        if (s != 0.0) {
          const double nrm = sqrt(alpha * alpha + s);
          beta = alpha >= 0.0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        bc[0] = t;
        bc[1] = scale;
        bc[2] = beta;
        for (int c = jj + 1; c < nbl; ++c) bc[4 + c] = piv[(j & 1) * kPQNB + c] + scale * tot[1 + c];
        taul[jj] = t;
        if (wg == 0) tau[j] = t;
      }
      __syncthreads();
      const double t = bc[0], scale = bc[1];
      for (int r = tid; r < R; r += kPQThreads) {
        const int gr = r0 + r;
        if (gr > j) {
          const double vr = L[jj * kPQMaxRows + r] * scale;
          L[jj * kPQMaxRows + r] = vr;
          for (int c = jj + 1; c < nbl; ++c) L[c * kPQMaxRows + r] -= t * vr * bc[4 + c];
        } else if (gr == j) {
          L[jj * kPQMaxRows + r] = bc[2];
          for (int c = jj + 1; c < nbl; ++c) L[c * kPQMaxRows + r] -= t * bc[4 + c];
        }
      }
      __syncthreads();
    }

    // leaf back to memory
    for (int e = tid; e < R * nbl; e += kPQThreads) {
      const int r = e % R, c = e / R;
      A[(i64)(r0 + r) + (i64)(c0 + c) * lda] = L[c * kPQMaxRows + r];
    }

    const int ncr = k - c0 - nbl;
    if (ncr <= 0) break;

    // ---- trailing columns of the panel: C <- C - W (Tl^T (W^T C))
    // W(r, a) = 0 above the diagonal row c0+a, 1 on it, L below it.
    double* tp = tpart + (i64)wg * kPQTrail;
    if (tid < ncr) {
      double xa[kPQNB];
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) xa[a] = 0.0;
      const double* Ac = A + (i64)(c0 + nbl + tid) * lda;
      for (int r = 0; r < R; ++r) {
        const int gr = r0 + r;
        const double av = Ac[gr];
#pragma unroll
        for (int a = 0; a < kPQNB; ++a) {
          const int dr = c0 + a;
          if (a < nbl && gr >= dr) xa[a] += (gr > dr ? L[a * kPQMaxRows + r] : 1.0) * av;
        }
      }
#pragma unroll
      for (int a = 0; a < kPQNB; ++a)
        if (a < nbl) tp[kPQNB * kPQNB + a * kPanelMaxCols + tid] = xa[a];
    }
    {
      const int a = tid % kPQNB, c = tid / kPQNB;  // 256 threads = 16 x 16 pairs
      double g = 0.0;
      if (a < c && c < nbl) {
        for (int r = 0; r < R; ++r) {
          const int gr = r0 + r, da = c0 + a, dc = c0 + c;
          if (gr < dc) continue;
          const double wc = gr > dc ? L[c * kPQMaxRows + r] : 1.0;
          const double wa = gr > da ? L[a * kPQMaxRows + r] : 1.0;  // gr >= dc > da
          g += wa * wc;
        }
      }
      tp[tid] = g;
    }
    grid_barrier(bar, (++nbar) * (unsigned)P, err);
    // two-phase reduction: entry e summed over workgroups in order by one thread
    for (int e = wg * kPQThreads + tid; e < kPQTrail; e += P * kPQThreads) {
      const int a = e < kPQNB * kPQNB ? -1 : (e - kPQNB * kPQNB) / kPanelMaxCols;
      const int col = e < kPQNB * kPQNB ? 0 : (e - kPQNB * kPQNB) % kPanelMaxCols;
      double s = 0.0;
      if (e < kPQNB * kPQNB || (a < nbl && col < ncr))
        for (int w = 0; w < P; ++w) s += tpart[(i64)w * kPQTrail + e];
      ttot[e] = s;
    }
    grid_barrier(bar, (++nbar) * (unsigned)P, err);
    Gs[tid] = ttot[tid];
    for (int e = tid; e < nbl * kPanelMaxCols; e += kPQThreads) Yt[e] = ttot[kPQNB * kPQNB + e];
    for (int e = tid; e < kPQNB * kPQNB; e += kPQThreads) Tl[e] = 0.0;
    __syncthreads();
    // leaf T factor, column by column: T(i, c) = -tau_c sum_{l=i}^{c-1} T(i, l) G(l, c)
    for (int c = 0; c < nbl; ++c) {
      if (tid < c) {
        double s = 0.0;
        for (int l = tid; l < c; ++l) s += Tl[tid + l * kPQNB] * Gs[l + c * kPQNB];
        Tl[tid + c * kPQNB] = -taul[c] * s;
      }
      if (tid == c) Tl[c + c * kPQNB] = taul[c];
      __syncthreads();
    }
    // Yt <- Tl^T X (each thread its own column)
    if (tid < ncr) {
      double x[kPQNB];
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) x[a] = a < nbl ? Yt[a * kPanelMaxCols + tid] : 0.0;
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l <= a; ++l) s += Tl[l + a * kPQNB] * x[l];
        if (a < nbl) Yt[a * kPanelMaxCols + tid] = s;
      }
    }
    __syncthreads();
    if (tid < ncr) {
      double y[kPQNB];
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) y[a] = a < nbl ? Yt[a * kPanelMaxCols + tid] : 0.0;
      double* Ac = A + (i64)(c0 + nbl + tid) * lda;
      for (int r = 0; r < R; ++r) {
        const int gr = r0 + r;
        double s = 0.0;
#pragma unroll
        for (int a = 0; a < kPQNB; ++a) {
          const int dr = c0 + a;
          if (a < nbl && gr >= dr) s += (gr > dr ? L[a * kPQMaxRows + r] : 1.0) * y[a];
        }
        Ac[gr] -= s;
      }
    }
    __syncthreads();
  }
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int panel_qr(hipStream_t st, i64 m, i64 k, double* A, i64 lda, double* tau, const PanelWork& w) {
  if (k <= 0 || m <= 0) return RANDUTV_OK;
  if (k > kPanelMaxCols || m < k) return RANDUTV_ERR_TOO_LARGE;
  const int P = panel_grid(m);
  if (P > 256 || cdiv(m, P) > kPQMaxRows) return RANDUTV_ERR_TOO_LARGE;
  LaunchTimer* tm = launch_timer();
  zero_u32_kernel<<<1, 64, 0, st>>>(w.bar, 1);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->begin(st, K_PANEL);
  panel_qr_kernel<<<P, kPQThreads, 0, st>>>((int)m, (int)k, A, lda, tau, w.part, w.bar, w.err);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->end(st, K_PANEL, 2.0 * m * k * k - 2.0 * k * k * k / 3.0);
  return RANDUTV_OK;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void extract_kernel(int m, int k, double* __restrict__ Pn, i64 ldp,
                                                      double* __restrict__ W, i64 ldw,
                                                      double* __restrict__ R, i64 ldr,
                                                      int zero_panel) {
  const i64 total = (i64)m * k;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const int r = (int)(e % m), c = (int)(e / m);
    double* p = Pn + r + (i64)c * ldp;
    const double a = *p;
    W[r + (i64)c * ldw] = r > c ? a : (r == c ? 1.0 : 0.0);
    if (R && r < k) R[r + (i64)c * ldr] = r <= c ? a : 0.0;
    if (zero_panel) *p = 0.0;
  }
}

int extract_reflectors(hipStream_t st, i64 m, i64 k, double* P, i64 ldp, double* W, i64 ldw,
                       double* R, i64 ldr, bool zero_panel) {
  if (m <= 0 || k <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(m * k, 256), 8192);
  LaunchTimer* tm = launch_timer();
  if (tm) tm->begin(st, K_EXTRACT);
  extract_kernel<<<blocks, 256, 0, st>>>((int)m, (int)k, P, ldp, W, ldw, R, ldr, zero_panel ? 1 : 0);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->end(st, K_EXTRACT, 0.0);
  return RANDUTV_OK;
}

// ---------------------------------------------------------------------------
// Compact-WY factor from the Gram matrix G = W^T W (dlarft, forward,
// column-wise): T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j).
// Blocked in 32 x 32 blocks: diagonal blocks by the column recurrence, then
// T(I, K) = -(sum_{L=I}^{K-1} T(I, L) G(L, K)) T(K, K), block rows in parallel.
// ---------------------------------------------------------------------------
constexpr int kTB = 32;

__global__ __launch_bounds__(256) void larft_diag_kernel(int k, const double* __restrict__ G, i64 ldg,
                                                         const double* __restrict__ tau,
                                                         double* __restrict__ Tf, i64 ldt) {
  const int I = blockIdx.x, tid = threadIdx.x;
  const int o = I * kTB, nb = min(kTB, k - o);
  __shared__ double Gd[kTB * kTB];
  __shared__ double Td[kTB * kTB];
  __shared__ double ta[kTB];
  for (int e = tid; e < kTB * kTB; e += 256) {
    const int r = e % kTB, c = e / kTB;
    Gd[e] = (r < nb && c < nb) ? G[(o + r) + (i64)(o + c) * ldg] : 0.0;
    Td[e] = 0.0;
  }
  if (tid < kTB) ta[tid] = tid < nb ? tau[o + tid] : 0.0;
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    if (tid < c) {
      double s = 0.0;
      for (int l = tid; l < c; ++l) s += Td[tid + l * kTB] * Gd[l + c * kTB];
      Td[tid + c * kTB] = -ta[c] * s;
    }
    if (tid == c) Td[c + c * kTB] = ta[c];
    __syncthreads();
  }
  // diagonal block and the zero blocks below it
  for (int e = tid; e < (k - o) * nb; e += 256) {
    const int r = e % (k - o), c = e / (k - o);
    Tf[(o + r) + (i64)(o + c) * ldt] = r < nb ? Td[r + c * kTB] : 0.0;
  }
}

__global__ __launch_bounds__(256) void larft_offdiag_kernel(int k, const double* __restrict__ G,
                                                            i64 ldg, double* __restrict__ Tf,
                                                            i64 ldt) {
  const int I = blockIdx.x, tid = threadIdx.x;
  const int nblk = (k + kTB - 1) / kTB;
  const int oi = I * kTB, ni = min(kTB, k - oi);
  __shared__ double Ta[kTB * (kTB + 1)];
  __shared__ double Gb[kTB * (kTB + 1)];
  __shared__ double S[kTB * (kTB + 1)];
  const int r = tid % kTB, c0 = (tid / kTB) * 4;  // each thread: row r, columns c0..c0+3
  for (int K = I + 1; K < nblk; ++K) {
    const int ok = K * kTB, nk = min(kTB, k - ok);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int Lb = I; Lb < K; ++Lb) {
      const int ol = Lb * kTB, nl = min(kTB, k - ol);
      __syncthreads();
      for (int e = tid; e < kTB * kTB; e += 256) {
        const int rr = e % kTB, cc = e / kTB;
        Ta[rr + cc * (kTB + 1)] = (rr < ni && cc < nl) ? Tf[(oi + rr) + (i64)(ol + cc) * ldt] : 0.0;
        Gb[rr + cc * (kTB + 1)] = (rr < nl && cc < nk) ? G[(ol + rr) + (i64)(ok + cc) * ldg] : 0.0;
      }
      __syncthreads();
      for (int l = 0; l < kTB; ++l) {
        const double a = Ta[r + l * (kTB + 1)];
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] += a * Gb[l + (c0 + q) * (kTB + 1)];
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) S[r + (c0 + q) * (kTB + 1)] = s[q];
    for (int e = tid; e < kTB * kTB; e += 256) {
      const int rr = e % kTB, cc = e / kTB;
      Gb[rr + cc * (kTB + 1)] = (rr < nk && cc < nk) ? Tf[(ok + rr) + (i64)(ok + cc) * ldt] : 0.0;
    }
    __syncthreads();
    double o4[4] = {0.0, 0.0, 0.0, 0.0};
    for (int l = 0; l < kTB; ++l) {
      const double a = S[r + l * (kTB + 1)];
#pragma unroll
      for (int q = 0; q < 4; ++q) o4[q] += a * Gb[l + (c0 + q) * (kTB + 1)];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (r < ni && c0 + q < nk) Tf[(oi + r) + (i64)(ok + c0 + q) * ldt] = -o4[q];
    __syncthreads();
  }
}

int larft_from_gram(hipStream_t st, i64 k, const double* G, i64 ldg, const double* tau, double* Tf,
                    i64 ldt) {
  if (k <= 0) return RANDUTV_OK;
  const int nblk = (int)cdiv(k, kTB);
  LaunchTimer* tm = launch_timer();
  if (tm) tm->begin(st, K_LARFT);
  larft_diag_kernel<<<nblk, 256, 0, st>>>((int)k, G, ldg, tau, Tf, ldt);
  RUTV_TRY(hipGetLastError());
  if (nblk > 1) {
    larft_offdiag_kernel<<<nblk - 1, 256, 0, st>>>((int)k, G, ldg, Tf, ldt);
    RUTV_TRY(hipGetLastError());
  }
  if (tm) tm->end(st, K_LARFT, (double)k * k * k / 3.0);
  return RANDUTV_OK;
}

}  // namespace rutv
