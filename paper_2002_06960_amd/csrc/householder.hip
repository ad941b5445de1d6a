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

constexpr int kPQMaxRows = 384;           // rows of one workgroup's slab
constexpr int kPQThreads = 512;           // 8 waves
constexpr int kPQWaves = kPQThreads / WAVE;
constexpr int kPQRowsPerLane = kPQMaxRows / WAVE;  // leaf rows per lane of wave 0
constexpr int kPQNB = 16;                 // leaf width
constexpr int kPQLd = kPQMaxRows + 1;     // padded leading dimension of the leaf in LDS
constexpr int kPQColPart = kPQNB + 1;
constexpr int kPQTrail = kPQNB * kPQNB + kPQNB * kPanelMaxCols;
constexpr int kPQMaxWG = 64;

typedef double dbl4 __attribute__((ext_vector_type(4)));

static int panel_grid(i64 m) {
  i64 P = std::max<i64>(cdiv(m, kPQMaxRows), std::min<i64>(32, cdiv(m, 128)));
  return (int)std::max<i64>(P, 1);
}

i64 panel_work_elems(i64 m) {
  const i64 P = panel_grid(m);
  return 2 * P * kPQColPart + 2 * kPQNB + P * kPQTrail + kPQTrail;
}

// arrival + wait of one workgroup at the panel's grid barrier, executed by a
// single lane: release on arrival, relaxed polling, one acquire fence
__device__ __forceinline__ void panel_arrive_wait(unsigned* counter, unsigned target, int* err) {
  __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  unsigned spins = 0;
  while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    __builtin_amdgcn_s_sleep(1);
    if (++spins > kSpinLimit) {
      __hip_atomic_store(err, RANDUTV_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

__device__ __forceinline__ void panel_barrier(unsigned* counter, unsigned target, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) panel_arrive_wait(counter, target, err);
  __syncthreads();
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

  // L: the leaf's slab (column a at L[a * kPQLd + r]); after the leaf, the explicit W
  __shared__ double L[kPQNB * kPQLd];
  // S: lane partials / gathered partials (leaf phase); reduced X, then Tl^T X
  __shared__ double S[kPQNB * kPanelMaxCols];
  __shared__ double tot[kPQColPart];
  __shared__ double pv[kPQNB];
  __shared__ double Gs[kPQNB * kPQNB];
  __shared__ double Tl[kPQNB * kPQNB];
  __shared__ double taul[kPQNB];
  static_assert(kPQMaxWG * kPQColPart <= kPQNB * kPanelMaxCols, "S holds the gathered partials");
  static_assert(WAVE * kPQColPart <= kPQNB * kPanelMaxCols, "S holds the lane partials");
  unsigned nbar = 0;

  for (int c0 = 0; c0 < k; c0 += kPQNB) {
    const int nbl = min(kPQNB, k - c0);
    for (int e = tid; e < kPQNB * kPQMaxRows; e += kPQThreads) {
      const int r = e % kPQMaxRows, c = e / kPQMaxRows;
      L[c * kPQLd + r] = (r < R && c < nbl) ? A[(i64)(r0 + r) + (i64)(c0 + c) * lda] : 0.0;
    }
    __syncthreads();

    // ---- the leaf's columns, one at a time, by wave 0 alone (lane l owns
    // rows l, l + 64, ... of the slab); waves 1-3 wait at the next barrier
    if (wave == 0) {
      for (int jj = 0; jj < nbl; ++jj) {
        const int j = c0 + jj;
        // column masks (branch-free loops; L is zero outside the slab and leaf)
        double msk[kPQNB];
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) msk[c] = (c > jj && c < nbl) ? 1.0 : 0.0;
        double acc[kPQColPart];
#pragma unroll
        for (int c = 0; c < kPQColPart; ++c) acc[c] = 0.0;
#pragma unroll 2
        for (int i = 0; i < kPQRowsPerLane; ++i) {
          const int r = lane + WAVE * i;
          const double x = (r0 + r > j) ? L[jj * kPQLd + r] : 0.0;
          acc[0] += x * x;
#pragma unroll
          for (int c = 0; c < kPQNB; ++c) acc[1 + c] += x * L[c * kPQLd + r];
        }
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) acc[1 + c] *= msk[c];
        // lane partials -> LDS, then lane c < 17 sums the 64 lanes in order
#pragma unroll
        for (int c = 0; c < kPQColPart; ++c) S[lane * kPQColPart + c] = acc[c];
        __builtin_amdgcn_wave_barrier();
        double* cp = colpart + ((j & 1) * P + wg) * kPQColPart;
        {
          // lane (c, h), h < 3: lanes 22h .. 22h+21 (in order), then the 3 in order
          const int c = lane % kPQColPart, h = lane / kPQColPart;
          double sv = 0.0;
          if (h < 3) {
            double v[22];
#pragma unroll
            for (int i = 0; i < 22; ++i) {
              const int w = 22 * h + i;
              v[i] = w < WAVE ? S[w * kPQColPart + c] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 22; ++i) sv += v[i];
          }
          const double s1 = __shfl(sv, c + kPQColPart, WAVE), s2 = __shfl(sv, c + 2 * kPQColPart, WAVE);
          if (lane < kPQColPart) cp[lane] = (sv + s1) + s2;
        }
        if (j >= r0 && j < r1 && lane >= jj && lane < nbl)
          piv[(j & 1) * kPQNB + lane] = L[lane * kPQLd + (j - r0)];
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) panel_arrive_wait(bar, (++nbar) * (unsigned)P, err);
        else ++nbar;
        __builtin_amdgcn_wave_barrier();
        // gather all partials and the pivot row in one batch of loads
        const double* cpb = colpart + (j & 1) * P * kPQColPart;
        {
          constexpr int NG = (kPQMaxWG * kPQColPart + WAVE - 1) / WAVE;
          double g[NG];
#pragma unroll
          for (int i = 0; i < NG; ++i) {
            const int e = lane + WAVE * i;
            g[i] = e < P * kPQColPart ? cpb[e] : 0.0;
          }
          const double pvv = (lane >= jj && lane < nbl) ? piv[(j & 1) * kPQNB + lane] : 0.0;
#pragma unroll
          for (int i = 0; i < NG; ++i) {
            const int e = lane + WAVE * i;
            if (e < kPQMaxWG * kPQColPart) S[e] = g[i];
          }
          if (lane < kPQNB) pv[lane] = pvv;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < kPQColPart) {
          // S past P * 17 holds zeros (set by the gather above)
          double v[kPQMaxWG];
#pragma unroll
          for (int w = 0; w < kPQMaxWG; ++w) v[w] = S[w * kPQColPart + lane];
          double sv = 0.0;
#pragma unroll
          for (int w = 0; w < kPQMaxWG; ++w) sv += v[w];
          tot[lane] = sv;
        }
        __builtin_amdgcn_wave_barrier();
        // every lane derives the reflector (identical arithmetic everywhere)
        const double sq = tot[0];
        const double alpha = pv[jj];
        double t = 0.0, scale = 0.0, beta = alpha;
        if (sq != 0.0) {
          const double nrm = sqrt(alpha * alpha + sq);
          beta = alpha >= 0.0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        if (lane == 0) {
          taul[jj] = t;
          if (wg == 0) tau[j] = t;
        }
        double wc[kPQNB];
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) wc[c] = msk[c] * (pv[c] + scale * tot[1 + c]);
#pragma unroll 1
        for (int i = 0; i < kPQRowsPerLane; ++i) {
          const int r = lane + WAVE * i;
          const int gr = r0 + r;
          const bool live = r < R && gr >= j;
          double row[kPQNB];
#pragma unroll
          for (int c = 0; c < kPQNB; ++c) row[c] = L[c * kPQLd + r];
          const double lj = L[jj * kPQLd + r];
          const double vr = gr > j ? lj * scale : 1.0;
          const double tv = live ? t * vr : 0.0;
#pragma unroll
          for (int c = 0; c < kPQNB; ++c) row[c] -= tv * wc[c];
#pragma unroll
          for (int c = 0; c < kPQNB; ++c) L[c * kPQLd + r] = row[c];
          if (live) L[jj * kPQLd + r] = gr > j ? vr : beta;
        }
        __builtin_amdgcn_wave_barrier();
      }
    } else {
      nbar += nbl;
    }
    __syncthreads();

    // leaf back to memory, then L := explicit W of the leaf (1 on the
    // diagonal row, 0 above it, the reflector below it; zero past nbl)
    for (int e = tid; e < kPQNB * kPQMaxRows; e += kPQThreads) {
      const int r = e % kPQMaxRows, c = e / kPQMaxRows;
      const int gr = r0 + r, dr = c0 + c;
      const double lv = L[c * kPQLd + r];
      if (r < R && c < nbl) A[(i64)gr + (i64)dr * lda] = lv;
      L[c * kPQLd + r] = (r < R && c < nbl) ? (gr > dr ? lv : (gr == dr ? 1.0 : 0.0)) : 0.0;
    }
    __syncthreads();

    const int ncr = k - c0 - nbl;
    if (ncr <= 0) break;

    // ---- trailing columns of the panel: C <- C - W (Tl^T (W^T C))
    // partials on the matrix cores: wave w forms X(:, 16q:16q+16) =
    // W_slab^T C_slab(:, 16q:16q+16) for the chunks q = w, w + 4, w + 8,
    // w + 12; the Gram W^T W goes to wave 3 (it has at most 3 chunks)
    double* tp = tpart + (i64)wg * kPQTrail;
    const int nchunk = (ncr + 15) / 16;
    const int lr = lane >> 4, lc = lane & 15;
    {
      // wave w forms X(:, 16q:16q+16) = W_slab^T C_slab(:, 16q:16q+16) for
      // the chunks q = w, w + 8 (ncr <= 240: at most 15 chunks); the last
      // wave (one chunk at most) also forms the Gram W^T W.  Rows are taken 4
      // per MFMA; the C values of the next kPF row groups are in flight.
      constexpr int kPF = 8, NQ = 2;
      const bool gram = wave == kPQWaves - 1;
      const double* Ac[NQ];
      bool cok[NQ], live[NQ];
      dbl4 acc[NQ], accg = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int qd = 0; qd < NQ; ++qd) {
        const int tcol = 16 * (wave + kPQWaves * qd) + lc;
        live[qd] = wave + kPQWaves * qd < nchunk;
        cok[qd] = tcol < ncr;
        Ac[qd] = A + (i64)(c0 + nbl + min(tcol, ncr - 1)) * lda + r0;
        acc[qd] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
      const int nst = (R + 3) / 4;
      double pf[NQ][kPF];
#pragma unroll
      for (int i = 0; i < kPF; ++i)
#pragma unroll
        for (int qd = 0; qd < NQ; ++qd) {
          const int r = 4 * i + lr;
          pf[qd][i] = (cok[qd] && r < R) ? Ac[qd][r] : 0.0;
        }
      for (int st0 = 0; st0 < nst; st0 += kPF) {
        double cv[NQ][kPF];
#pragma unroll
        for (int i = 0; i < kPF; ++i)
#pragma unroll
          for (int qd = 0; qd < NQ; ++qd) {
            cv[qd][i] = pf[qd][i];
            const int r = 4 * (st0 + kPF + i) + lr;
            pf[qd][i] = (cok[qd] && r < R) ? Ac[qd][r] : 0.0;
          }
#pragma unroll
        for (int i = 0; i < kPF; ++i) {
          const int r = 4 * (st0 + i) + lr;
          const double wa = r < kPQMaxRows ? L[lc * kPQLd + r] : 0.0;  // W(r, a = lc)
#pragma unroll
          for (int qd = 0; qd < NQ; ++qd)
            if (live[qd]) acc[qd] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, cv[qd][i], acc[qd], 0, 0, 0);
          if (gram) accg = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, wa, accg, 0, 0, 0);
        }
      }
      // D(4q + lr, lc): X[a = 4q + lr][t], Gram[a][c = lc]
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int a = 4 * qq + lr;
#pragma unroll
        for (int qd = 0; qd < NQ; ++qd) {
          const int tcol = 16 * (wave + kPQWaves * qd) + lc;
          if (live[qd] && tcol < ncr) tp[kPQNB * kPQNB + a * kPanelMaxCols + tcol] = acc[qd][qq];
        }
        if (gram) tp[a + lc * kPQNB] = accg[qq];
      }
    }
    panel_barrier(bar, (++nbar) * (unsigned)P, err);
    // two-phase reduction: workgroup wg sums entries e = wg * 256 + ..., over
    // the workgroups in order
    for (int e = wg * kPQThreads + tid; e < kPQTrail; e += P * kPQThreads) {
      const bool g = e < kPQNB * kPQNB;
      const int a = g ? 0 : (e - kPQNB * kPQNB) / kPanelMaxCols;
      const int col = g ? 0 : (e - kPQNB * kPQNB) % kPanelMaxCols;
      double sv = 0.0;
      if (g || (a < nbl && col < ncr)) {
        double v[kPQMaxWG];
#pragma unroll
        for (int w = 0; w < kPQMaxWG; ++w) v[w] = w < P ? tpart[(i64)w * kPQTrail + e] : 0.0;
#pragma unroll
        for (int w = 0; w < kPQMaxWG; ++w) sv += v[w];
      }
      ttot[e] = sv;
    }
    panel_barrier(bar, (++nbar) * (unsigned)P, err);
    if (tid < kPQNB * kPQNB) {
      Gs[tid] = ttot[tid];
      Tl[tid] = 0.0;
    }
    for (int e = tid; e < nbl * kPanelMaxCols; e += kPQThreads) S[e] = ttot[kPQNB * kPQNB + e];
    __syncthreads();
    // leaf T factor, column by column (wave 0 alone, lanes = rows):
    // T(i, c) = -tau_c sum_{l=i}^{c-1} T(i, l) G(l, c)
    if (wave == 0 && lane < kPQNB) {
      double trow[kPQNB];
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) trow[c] = 0.0;
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) {
        if (c >= nbl) break;
        double sdot = 0.0;
#pragma unroll
        for (int l = 0; l < kPQNB; ++l)
          if (l >= lane && l < c) sdot += trow[l] * Gs[l + c * kPQNB];
        trow[c] = lane < c ? -taul[c] * sdot : (lane == c ? taul[c] : 0.0);
      }
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) Tl[lane + c * kPQNB] = trow[c];
    }
    __syncthreads();
    // S <- Tl^T X (thread t owns column t; ncr <= 240 < threads)
    if (tid < ncr) {
      double x[kPQNB];
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) x[a] = a < nbl ? S[a * kPanelMaxCols + tid] : 0.0;
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) {
        double sv = 0.0;
#pragma unroll
        for (int l = 0; l <= a; ++l) sv += Tl[l + a * kPQNB] * x[l];
        S[a * kPanelMaxCols + tid] = a < nbl ? sv : 0.0;
      }
    }
    __syncthreads();
    // update on the matrix cores: 16-row x 16-column blocks of C -= W Y with
    // Y = S (16 x ncr); the MFMA forms the block transposed, so a lane holds
    // 4 columns of one row: C[rb + lc][t0 + 4q + lr] (16 rows per column per
    // store).  Blocks are dealt to the waves; the next block's C is fetched
    // while the current one is computed.
    {
      const int nrb = (R + 15) / 16;
      const int nblocks = nrb * nchunk;
      constexpr int kRing = 4;
      double ring[kRing][4];
      auto fetch = [&](int bi, double (&dst)[4]) {
        const int rb = 16 * (bi % nrb), t0 = 16 * (bi / nrb);
        const int r = rb + lc;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int t = t0 + 4 * q + lr;
          dst[q] = (bi < nblocks && r < R && t < ncr) ? A[(i64)(r0 + r) + (i64)(c0 + nbl + t) * lda] : 0.0;
        }
      };
#pragma unroll
      for (int u = 0; u < kRing; ++u) fetch(wave + kPQWaves * u, ring[u]);
      for (int bidx = wave, it = 0; bidx < nblocks; bidx += kPQWaves, ++it) {
        double cc[4];
        const int slot = it % kRing;
#pragma unroll
        for (int u = 0; u < kRing; ++u)
          if (u == slot)
#pragma unroll
            for (int q = 0; q < 4; ++q) cc[q] = ring[u][q];
        double nx[4];
        fetch(bidx + kPQWaves * kRing, nx);
#pragma unroll
        for (int u = 0; u < kRing; ++u)
          if (u == slot)
#pragma unroll
            for (int q = 0; q < 4; ++q) ring[u][q] = nx[q];
        const int rb = 16 * (bidx % nrb), t0 = 16 * (bidx / nrb);
        dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < kPQNB; kk += 4) {
          const double yv = S[(kk + lr) * kPanelMaxCols + t0 + lc];   // Y^T(t0 + lc, kk + lr)
          const double wv = L[(kk + lr) * kPQLd + rb + lc];           // W^T(kk + lr, rb + lc)
          d = __builtin_amdgcn_mfma_f64_16x16x4f64(yv, wv, d, 0, 0, 0);
        }
        const int r = rb + lc;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int t = t0 + 4 * q + lr;
          if (r < R && t < ncr) A[(i64)(r0 + r) + (i64)(c0 + nbl + t) * lda] = cc[q] - d[q];
        }
      }
    }
    __syncthreads();
  }
}

int panel_qr(hipStream_t st, i64 m, i64 k, double* A, i64 lda, double* tau, const PanelWork& w) {
  if (k <= 0 || m <= 0) return RANDUTV_OK;
  if (k > kPanelMaxCols || m < k) return RANDUTV_ERR_TOO_LARGE;
  const int P = panel_grid(m);
  if (P > kPQMaxWG || cdiv(m, P) > kPQMaxRows) return RANDUTV_ERR_TOO_LARGE;
  LaunchTimer* tm = launch_timer();
  RUTV_CHECK(fill_zero_u32(st, w.bar, 1));
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
