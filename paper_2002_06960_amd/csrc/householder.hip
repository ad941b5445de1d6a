// Householder QR of a tall panel (m x k, k <= 256) and the compact-WY factor.
//
// "unpivoted_QR" of Figure 2 (used for the sketch Y and for the current
// column block of T) with LAPACK dgeqr2 conventions: reflector H_j =
// I - tau_j v_j v_j^T, v_j(j) = 1, beta_j = -sign(alpha_j) ||x_j||,
// tau_j = (beta_j - alpha_j)/beta_j, sign(0) = +1, tau_j = 0 when the part
// below the diagonal is exactly zero.
//
// Panel kernel layout: P workgroups of 8 waves each own a contiguous slab of
// at most 512 rows.  The panel is processed in leaves of 16 columns whose rows
// stay in the registers of waves 0-3 (two rows per thread); all 8 waves share
// the matrix-core work of the trailing updates.  Within a leaf each column needs one sum over
// all rows (squares below the diagonal plus the dot products with the leaf's
// remaining columns, combined with the pivot row): every workgroup publishes
// its partial sums, reads everybody's and adds them in the same order, so all
// workgroups derive the bit-identical reflector and update their own rows.
// After a leaf, the rest of the panel receives the leaf's block reflector
// C <- (I - W Tl W^T)^T C, with the Gram matrix of the leaf vectors and W^T C
// summed over the workgroups in two rounds (each workgroup reduces a share of
// the entries, then everybody reads the totals).
//
// Workgroups exchange values without grid barriers or memory fences: a double
// travels as two 64-bit words, each holding one 32-bit half of it and the
// 32-bit number of the exchange round, written and read with relaxed
// device-scope atomics.  A reader polls until every word it needs carries the
// current round number; since each word validates itself, only per-location
// coherence is needed.  Round numbers start at 1 in every launch, whose
// exchange area is cleared before the launch.  Column rounds alternate
// between two buffers: a workgroup can only be one round ahead of the
// slowest reader.
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace rutv {

typedef unsigned long long u64;
typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int kPQThreads = 512;  // 8 waves (two per SIMD keep the FP64 matrix cores busy)
constexpr int kPQWaves = kPQThreads / WAVE;
constexpr int kPQLeafThreads = 256;  // waves 0-3 hold the leaf rows
constexpr int kPQLeafWaves = kPQLeafThreads / WAVE;
constexpr int kPQRpt = 2;            // leaf rows per thread
constexpr int kPQMaxRows = kPQLeafThreads * kPQRpt;
constexpr int kPQNB = 16;                  // leaf width
constexpr int kPQLdW = kPQMaxRows + 1;     // padded leading dimension of the leaf's W in LDS
constexpr int kPQMaxWG = 64;
constexpr int kPQTrail = kPQNB * kPQNB + kPQNB * (kPanelMaxCols - kPQNB);  // Gram + W^T C entries
constexpr unsigned kPQSpinLimit = 1u << 22;

// exchange area (64-bit words; a double is a pair of words)
constexpr i64 kXCol = 0;                                 // [2][kPQMaxWG][kPQNB][2] column partials
constexpr i64 kXPiv = kXCol + 2 * kPQMaxWG * kPQNB * 2;  // [2][kPQNB][2] pivot row
constexpr i64 kXTot = kXPiv + 2 * kPQNB * 2;             // [kPQTrail][2] reduced trailing sums
constexpr i64 kXPart = kXTot + kPQTrail * 2;             // [P][kPQTrail][2] trailing partials

static int panel_grid(i64 m) {
  i64 P = std::max<i64>(cdiv(m, kPQMaxRows), std::min<i64>(32, cdiv(m, 128)));
  return (int)std::max<i64>(P, 1);
}

static i64 panel_words(int P) { return kXPart + (i64)P * kPQTrail * 2; }

i64 panel_work_elems(i64 m) { return panel_words(panel_grid(m)); }

__device__ __forceinline__ void xput(u64* p, double v, unsigned tag) {
  const u64 b = (u64)__double_as_longlong(v), t = (u64)tag << 32;
  __hip_atomic_store(p, (b & 0xffffffffull) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(p + 1, (b >> 32) | t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ u64 xget(u64* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ bool xhas(u64 w, unsigned tag) { return (unsigned)(w >> 32) == tag; }
__device__ __forceinline__ double xval(u64 lo, u64 hi) {
  return __longlong_as_double((long long)((lo & 0xffffffffull) | (hi << 32)));
}

// one halving step of a wave reduce-scatter of kPQNB values: lanes with bit
// OFF set keep values N..2N-1, the others 0..N-1, each adding its partner's
template <int N, int OFF>
__device__ __forceinline__ void reduce_scatter_step(double (&v)[kPQNB], int lane) {
  const bool up = (lane & OFF) != 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double send = up ? v[i] : v[i + N];
    const double keep = up ? v[i + N] : v[i];
    v[i] = keep + __shfl_xor(send, OFF, WAVE);
  }
}

// calls f(integral_constant<int, J>) for J = J0, J0 + 1, ... while J < n
template <int J0>
struct ForColumns {
  template <class F>
  __device__ __forceinline__ static void run(int n, F& f) {
    if (J0 < n) {
      f(std::integral_constant<int, J0>{});
      ForColumns<J0 + 1>::run(n, f);
    }
  }
};
template <>
struct ForColumns<kPQNB> {
  template <class F>
  __device__ __forceinline__ static void run(int, F&) {}
};

__global__ __launch_bounds__(kPQThreads) void panel_qr_kernel(int m, int k, double* __restrict__ A,
                                                              i64 lda, double* __restrict__ tau,
                                                              u64* __restrict__ xch,
                                                              int* __restrict__ err) {
  const int P = gridDim.x, wg = blockIdx.x;
  const int r0 = (int)((i64)m * wg / P), r1 = (int)((i64)m * (wg + 1) / P), R = r1 - r0;

  __shared__ double Wl[kPQNB * kPQLdW];        // explicit W of the finished leaf
  __shared__ double S[kPQNB * kPanelMaxCols];  // X = W^T C, then Tl^T X
  __shared__ double red[kPQLeafWaves * kPQNB]; // per-wave column sums
  __shared__ double pivl[kPQNB];               // pivot row (its owner only)
  __shared__ double tsum[kPQNB];               // column totals
  __shared__ double pivs[kPQNB];               // the pivot row as read back
  __shared__ double Gs[kPQNB * kPQNB];
  __shared__ double Tl[kPQNB * kPQNB];
  __shared__ double taul[kPQNB];
  __shared__ int dead;
  if (threadIdx.x == 0) dead = 0;
  __syncthreads();
  unsigned rnd = 0;

  // a bounded wait: on expiry record the error and stop waiting for good
  auto give_up = [&](unsigned& spins) -> bool {
    if (*(volatile int*)&dead) return true;
    if (++spins > kPQSpinLimit) {
      dead = 1;
      __hip_atomic_store(err, RANDUTV_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
    return false;
  };

  for (int c0 = 0; c0 < k; c0 += kPQNB) {
    const int nbl = min(kPQNB, k - c0);
    // opaque zero and thread index: every address below is recomputed per leaf
    // instead of being hoisted out of this loop (they would not fit in registers)
    int z = 0, tid = threadIdx.x;
    asm volatile("" : "+s"(z), "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double* const Ab = A + z;
    u64* const xcol = xch + z + kXCol;
    u64* const xpiv = xch + z + kXPiv;
    u64* const xtot = xch + z + kXTot;
    u64* const xpart = xch + z + kXPart;
    double row[kPQRpt][kPQNB];
    int gr[kPQRpt];
    bool own[kPQRpt];
#pragma unroll
    for (int i = 0; i < kPQRpt; ++i) {
      const int r = tid + kPQLeafThreads * i;
      own[i] = tid < kPQLeafThreads && r < R;
      gr[i] = r0 + r;
#pragma unroll
      for (int c = 0; c < kPQNB; ++c)
        row[i][c] = (own[i] && c < nbl) ? Ab[(i64)gr[i] + (i64)(c0 + c) * lda] : 0.0;
    }

    // one column of the leaf; jj is a compile-time constant in each instance
    auto column = [&](auto jc) {
      constexpr int jj = decltype(jc)::value;
      const int j = c0 + jj;
      const unsigned tag = ++rnd;
      int zc = 0;
      asm volatile("" : "+s"(zc));
      // column masks (constants: the loop is unrolled, so the leaf stays in registers)
      double msk[kPQNB];
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) msk[c] = c > jj ? 1.0 : 0.0;
      double x[kPQRpt];
#pragma unroll
      for (int i = 0; i < kPQRpt; ++i) {
        double xj = 0.0;
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) xj = c == jj ? row[i][c] : xj;
        x[i] = (own[i] && gr[i] > j) ? xj : 0.0;
      }
      // slot 0: squares below the diagonal; slot c > jj: dot with column c
      if (wave < kPQLeafWaves) {
      double v[kPQNB];
      v[0] = 0.0;
#pragma unroll
      for (int i = 0; i < kPQRpt; ++i) v[0] += x[i] * x[i];
#pragma unroll
      for (int c = 1; c < kPQNB; ++c) {
        v[c] = 0.0;
#pragma unroll
        for (int i = 0; i < kPQRpt; ++i) v[c] += x[i] * row[i][c];
        v[c] *= msk[c];
      }
      // wave reduce-scatter: afterwards lane l holds slot l / 4
      reduce_scatter_step<8, 32>(v, lane);
      reduce_scatter_step<4, 16>(v, lane);
      reduce_scatter_step<2, 8>(v, lane);
      reduce_scatter_step<1, 4>(v, lane);
      v[0] += __shfl_xor(v[0], 2, WAVE);
      v[0] += __shfl_xor(v[0], 1, WAVE);
      if ((lane & 3) == 0) red[wave * kPQNB + (lane >> 2)] = v[0];
      }
#pragma unroll
      for (int i = 0; i < kPQRpt; ++i)
        if (own[i] && gr[i] == j)
#pragma unroll
          for (int c = 0; c < kPQNB; ++c) pivl[c] = row[i][c];
      __syncthreads();

      {
        const int s = lane & 15, g = lane >> 4;
        u64* const xc = xcol + zc + (i64)(tag & 1) * kPQMaxWG * kPQNB * 2;
        u64* const xp = xpiv + zc + (i64)(tag & 1) * kPQNB * 2;
        if (wave == 0) {
          if (g == 0) {
            double ts = red[s];
#pragma unroll
            for (int w = 1; w < kPQLeafWaves; ++w) ts += red[w * kPQNB + s];
            xput(xc + ((i64)wg * kPQNB + s) * 2, ts, tag);
          } else if (g == 1 && j >= r0 && j < r1) {
            xput(xp + s * 2, pivl[s], tag);
          }
        }
        // wave w < 4 gathers slots 4 w .. 4 w + 3: lane (s4, g) reads slot
        // 4 w + s4 of workgroups g, g + 16, ...; lanes g = 0 also the pivot row
        if (wave < kPQLeafWaves) {
          constexpr int NG = kPQMaxWG / 16;
          const int s4 = lane & 3, gq = lane >> 2, slot = 4 * wave + s4;
          u64 lo[NG], hi[NG], plo, phi;
          unsigned spins = 0;
          while (true) {
            // branch-free: every lane loads valid words (clamped indices), the
            // masks decide what counts
#pragma unroll
            for (int i = 0; i < NG; ++i) {
              const int w = min(gq + 16 * i, P - 1);
              lo[i] = xget(xc + ((i64)w * kPQNB + slot) * 2);
              hi[i] = xget(xc + ((i64)w * kPQNB + slot) * 2 + 1);
            }
            plo = xget(xp + slot * 2);
            phi = xget(xp + slot * 2 + 1);
            int have = (gq != 0) | (xhas(plo, tag) & xhas(phi, tag));
#pragma unroll
            for (int i = 0; i < NG; ++i)
              have &= (gq + 16 * i >= P) | (xhas(lo[i], tag) & xhas(hi[i], tag));
            if (__all(have)) break;
            if (give_up(spins)) break;
          }
          double acc = 0.0;
#pragma unroll
          for (int i = 0; i < NG; ++i) acc += gq + 16 * i < P ? xval(lo[i], hi[i]) : 0.0;
          acc += __shfl_xor(acc, 4, WAVE);
          acc += __shfl_xor(acc, 8, WAVE);
          acc += __shfl_xor(acc, 16, WAVE);
          acc += __shfl_xor(acc, 32, WAVE);
          if (gq == 0) {
            tsum[slot] = acc;
            pivs[slot] = xval(plo, phi);
          }
        }
      }
      __syncthreads();

      // every thread derives the reflector from the same totals
      double t = 0.0, scale = 0.0, beta, wc[kPQNB];
      {
        double tot[kPQNB];
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) tot[c] = tsum[c];
        double alpha = 0.0;
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) alpha = c == jj ? pivs[c] : alpha;
        const double sq = tot[0];
        beta = alpha;
        if (sq != 0.0) {
          const double nrm = sqrt(alpha * alpha + sq);
          beta = alpha >= 0.0 ? -nrm : nrm;
          t = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) wc[c] = (c < nbl) ? msk[c] * (pivs[c] + scale * tot[c]) : 0.0;
        if (tid == 0) {
          taul[jj] = t;
          if (wg == 0) tau[j] = t;
        }
      }
#pragma unroll
      for (int i = 0; i < kPQRpt; ++i) {
        if (wave >= kPQLeafWaves) break;
        const bool live = own[i] && gr[i] >= j, below = gr[i] > j;
        const double vr = below ? x[i] * scale : 1.0;
        const double tv = live ? t * vr : 0.0;
        const double nj = below ? vr : beta;
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) {
          row[i][c] -= tv * wc[c];
          if (c == jj && live) row[i][c] = nj;
        }
      }
    };
    ForColumns<0>::run(nbl, column);

    // leaf back to memory; Wl := explicit W of the leaf (1 on the diagonal
    // row, 0 above it, the reflector below it; zero past nbl and past the slab)
#pragma unroll
    for (int i = 0; i < kPQRpt; ++i) {
      if (tid >= kPQLeafThreads) break;
      const int r = tid + kPQLeafThreads * i;
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) {
        const bool live = own[i] && c < nbl;
        if (live) Ab[(i64)gr[i] + (i64)(c0 + c) * lda] = row[i][c];
        const int dr = c0 + c;
        Wl[c * kPQLdW + r] = live ? (gr[i] > dr ? row[i][c] : (gr[i] == dr ? 1.0 : 0.0)) : 0.0;
      }
    }
    __syncthreads();

    const int ncr = k - c0 - nbl;
    if (ncr <= 0) break;

    // ---- trailing columns of the panel: C <- C - W (Tl^T (W^T C))
    const int nchunk = (ncr + 15) / 16;
    const int lr = lane >> 4, lc = lane & 15;
    const int E = kPQNB * kPQNB + kPQNB * ncr;  // Gram entries, then X(a, t) at 256 + a ncr + t
    const unsigned tag1 = ++rnd, tag2 = ++rnd;
    {
      // wave w forms X(:, 16q:16q+16) = W_slab^T C_slab(:, 16q:16q+16) for the
      // chunks q = w, w + W, ... (W waves; ncr <= 240: at most 15 chunks); the
      // last wave also forms the Gram W^T W.  Rows are taken 4 per MFMA; the
      // C values of the next kPF row groups are in flight.
      constexpr int kPF = 8, NQ = (kPanelMaxCols / 16 - 1 + kPQWaves - 1) / kPQWaves;
      const bool gram = wave == kPQWaves - 1;
      // live chunks of this wave (uniform); loads are unconditional at clamped
      // addresses: rows past the slab meet zero rows of Wl, columns past ncr
      // are never stored
      const int nq = min(NQ, max(0, (nchunk - wave + kPQWaves - 1) / kPQWaves));
      const double* Ac[NQ];
      dbl4 acc[NQ], accg = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int qd = 0; qd < NQ; ++qd) {
        const int tcol = min(16 * (wave + kPQWaves * qd) + lc, ncr - 1);
        Ac[qd] = Ab + (i64)(c0 + nbl + tcol) * lda + r0;
        acc[qd] = dbl4{0.0, 0.0, 0.0, 0.0};
      }
      const int nst = (R + 3) / 4;
      double pf[NQ][kPF];
#pragma unroll
      for (int i = 0; i < kPF; ++i)
#pragma unroll
        for (int qd = 0; qd < NQ; ++qd) pf[qd][i] = Ac[qd][min(4 * i + lr, R - 1)];
      for (int st0 = 0; st0 < nst; st0 += kPF) {
        double cv[NQ][kPF];
#pragma unroll
        for (int i = 0; i < kPF; ++i)
#pragma unroll
          for (int qd = 0; qd < NQ; ++qd) {
            cv[qd][i] = pf[qd][i];
            pf[qd][i] = Ac[qd][min(4 * (st0 + kPF + i) + lr, R - 1)];
          }
#pragma unroll
        for (int i = 0; i < kPF; ++i) {
          const int r = 4 * (st0 + i) + lr;
          const double wa = r < kPQMaxRows ? Wl[lc * kPQLdW + min(r, kPQMaxRows - 1)] : 0.0;  // W(r, a = lc)
#pragma unroll
          for (int qd = 0; qd < NQ; ++qd)
            if (qd < nq) acc[qd] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, cv[qd][i], acc[qd], 0, 0, 0);
          if (gram) accg = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, wa, accg, 0, 0, 0);
        }
      }
      // D(4qq + lr, lc): X[a = 4qq + lr][t], Gram[a][c = lc]
      u64* const mine = xpart + (i64)wg * kPQTrail * 2;
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) {
        const int a = 4 * qq + lr;
#pragma unroll
        for (int qd = 0; qd < NQ; ++qd) {
          const int tcol = 16 * (wave + kPQWaves * qd) + lc;
          if (qd < nq && tcol < ncr)
            xput(mine + (i64)(kPQNB * kPQNB + a * ncr + tcol) * 2, acc[qd][qq], tag1);
        }
        if (gram) xput(mine + (i64)(a + lc * kPQNB) * 2, accg[qq], tag1);
      }
    }
    // round 1: workgroup wg sums entries [e0, e1) over all workgroups, in order
    {
      const int e0 = (int)((i64)E * wg / P), e1 = (int)((i64)E * (wg + 1) / P);
      constexpr int NB = 16;
      for (int e = e0 + tid; e < e1; e += kPQThreads) {
        double sv = 0.0;
        for (int w0 = 0; w0 < P; w0 += NB) {
          u64 lo[NB], hi[NB];
          unsigned spins = 0;
          while (true) {
#pragma unroll
            for (int i = 0; i < NB; ++i) {
              u64* p = xpart + ((i64)min(w0 + i, P - 1) * kPQTrail + e) * 2;
              lo[i] = xget(p);
              hi[i] = xget(p + 1);
            }
            int have = 1;
#pragma unroll
            for (int i = 0; i < NB; ++i) have &= (w0 + i >= P) | (xhas(lo[i], tag1) & xhas(hi[i], tag1));
            if (have || give_up(spins)) break;
          }
#pragma unroll
          for (int i = 0; i < NB; ++i) sv += w0 + i < P ? xval(lo[i], hi[i]) : 0.0;
        }
        xput(xtot + (i64)e * 2, sv, tag2);
      }
    }
    // round 2: every workgroup reads all totals
    {
      constexpr int NE = kPQTrail / kPQThreads;
      u64 lo[NE], hi[NE];
      unsigned spins = 0;
      while (true) {
#pragma unroll
        for (int i = 0; i < NE; ++i) {
          const int e = min(tid + kPQThreads * i, E - 1);
          lo[i] = xget(xtot + (i64)e * 2);
          hi[i] = xget(xtot + (i64)e * 2 + 1);
        }
        int have = 1;
#pragma unroll
        for (int i = 0; i < NE; ++i) have &= (xhas(lo[i], tag2) & xhas(hi[i], tag2));
        if (have || give_up(spins)) break;
      }
#pragma unroll
      for (int i = 0; i < NE; ++i) {
        const int e = tid + kPQThreads * i;
        if (e < E) {
          const double val = xval(lo[i], hi[i]);
          if (e < kPQNB * kPQNB) {
            Gs[e] = val;
          } else {
            const int a = (e - kPQNB * kPQNB) / ncr, tc = (e - kPQNB * kPQNB) % ncr;
            S[a * kPanelMaxCols + tc] = val;
          }
        }
      }
      if (tid < kPQNB * kPQNB) Tl[tid] = 0.0;
    }
    __syncthreads();
    // leaf T factor, column by column (wave 0 alone, lanes = rows):
    // T(i, c) = -tau_c sum_{l=i}^{c-1} T(i, l) G(l, c)
    if (wave == 0 && lane < kPQNB) {
      double trow[kPQNB];
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) trow[c] = 0.0;
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) {
        double sdot = 0.0;
#pragma unroll
        for (int l = 0; l < c; ++l) sdot += l >= lane ? trow[l] * Gs[l + c * kPQNB] : 0.0;
        const double tc = lane < c ? -taul[c] * sdot : (lane == c ? taul[c] : 0.0);
        trow[c] = c < nbl ? tc : 0.0;
      }
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) Tl[lane + c * kPQNB] = trow[c];
    }
    __syncthreads();
    // S <- Tl^T X (thread t owns column t; ncr <= 240 < threads)
    if (tid < ncr) {
      double xv[kPQNB];
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) xv[a] = a < nbl ? S[a * kPanelMaxCols + tid] : 0.0;
#pragma unroll
      for (int a = 0; a < kPQNB; ++a) {
        double sv = 0.0;
#pragma unroll
        for (int l = 0; l <= a; ++l) sv += Tl[l + a * kPQNB] * xv[l];
        S[a * kPanelMaxCols + tid] = a < nbl ? sv : 0.0;
      }
    }
    __syncthreads();
    // update on the matrix cores: 16-row x 16-column blocks of C -= W Y with
    // Y = S (16 x ncr); the MFMA forms the block transposed, so a lane holds
    // 4 columns of one row: C[rb + lc][t0 + 4q + lr] (16 rows per column per
    // store).  Blocks are dealt to the waves; the next blocks' C values are
    // fetched while the current one is computed.
    {
      const int nrb = (R + 15) / 16;
      const int nblocks = nrb * nchunk;
      constexpr int kRing = 4;
      double ring[kRing][4];
      // unconditional loads at clamped addresses (the stores are guarded)
      auto fetch = [&](int bi, double (&dst)[4]) {
        const int bc = min(bi, nblocks - 1);
        const int rb = 16 * (bc % nrb), t0 = 16 * (bc / nrb);
        const int r = min(rb + lc, R - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int tc = min(t0 + 4 * q + lr, ncr - 1);
          dst[q] = Ab[(i64)(r0 + r) + (i64)(c0 + nbl + tc) * lda];
        }
      };
#pragma unroll
      for (int u = 0; u < kRing; ++u) fetch(wave + kPQWaves * u, ring[u]);
      for (int b0 = wave; b0 < nblocks; b0 += kPQWaves * kRing) {
#pragma unroll
        for (int u = 0; u < kRing; ++u) {
          const int bidx = b0 + kPQWaves * u;
          double cc[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) cc[q] = ring[u][q];
          fetch(bidx + kPQWaves * kRing, ring[u]);
          if (bidx < nblocks) {
            const int rb = 16 * (bidx % nrb), t0 = 16 * (bidx / nrb);
            dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < kPQNB; kk += 4) {
              const double yv = S[(kk + lr) * kPanelMaxCols + t0 + lc];  // Y^T(t0 + lc, kk + lr)
              const double wv = Wl[(kk + lr) * kPQLdW + rb + lc];        // W^T(kk + lr, rb + lc)
              d = __builtin_amdgcn_mfma_f64_16x16x4f64(yv, wv, d, 0, 0, 0);
            }
            const int r = rb + lc;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int tc = t0 + 4 * q + lr;
              if (r < R && tc < ncr) Ab[(i64)(r0 + r) + (i64)(c0 + nbl + tc) * lda] = cc[q] - d[q];
            }
          }
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
  RUTV_CHECK(fill_zero_u32(st, reinterpret_cast<unsigned*>(w.xch), 2 * panel_words(P)));
  if (tm) tm->begin(st, K_PANEL);
  panel_qr_kernel<<<P, kPQThreads, 0, st>>>((int)m, (int)k, A, lda, tau, w.xch, w.err);
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
