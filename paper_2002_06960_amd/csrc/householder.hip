// Householder QR of a tall panel (m x k, k <= 256) and the compact-WY factor.
//
// The unpivoted Householder QR of Figure 2 (of the sketch Y and of the
// current column block of T) with LAPACK dgeqr2 conventions: reflector H_j =
// I - tau_j v_j v_j^T, v_j(j) = 1, beta_j = -sign(alpha_j) ||x_j||,
// tau_j = (beta_j - alpha_j)/beta_j, sign(0) = +1, tau_j = 0 when the part
// below the diagonal is exactly zero.
//
// Panel kernel layout: P workgroups (8 waves, or 4 in the variant that shares
// its CU with a GEMM workgroup) each own a contiguous slab of at most 256 rows,
// made of whole 16-row units.  The panel is processed in leaves of 16 columns
// whose rows stay in the registers of waves 0-3 (one row per thread); all
// waves share the matrix-core work.
//
// A leaf's reflectors need sums over all rows.  Rather than one exchange
// between the workgroups per column, a leaf takes one exchange per pass: the
// workgroups publish the Gram matrix G = B^T B of their rows below the leaf's
// 16 x 16 diagonal block (B), the owners publish that block (the top block),
// and every workgroup then runs the column recurrence of the leaf on 16 x 16
// data alone.  The bottom part of every current column stays B m_c for a
// 16-vector m_c (M = I at the start of a pass), so its squared norm is
// m_c^T G m_c and its dot products m_c^T G m_d; the top block is updated
// explicitly.  A pass ends with the coefficient matrix K that maps the
// pass-start rows of B to their new values (v_j = scale_j B m_j for a
// finished column j, B m_c for a column still open), applied by every
// workgroup to its own rows.  The Gram form loses accuracy when a column's
// bottom part has cancelled against the earlier reflectors; the pass stops
// at a column whose bound (sum_a |m_a| sqrt(G_aa))^2 exceeds kGramCap times
// its squared norm, and the next pass starts there from a fresh Gram matrix
// of the current rows (the first column of a pass always has M = I, so
// every pass finishes at least one column).  In exact arithmetic the result
// is the column-by-column factorization.
//
// After a leaf, the rest of the panel receives the leaf's block reflector
// C <- (I - W Tl W^T)^T C, with the Gram matrix of the leaf vectors and W^T C
// summed over the workgroups in two rounds (each workgroup reduces a share of
// the entries, then everybody reads the totals).  Every sum over the
// workgroups is split into parts of at most 16 workgroups, each read by one
// thread in one batch of loads, and the parts are added in order.
//
// Workgroups exchange values without grid barriers or memory fences: a double
// travels as two 64-bit words, each holding one 32-bit half of it and the
// 32-bit number of the exchange round, written and read with relaxed
// device-scope atomics.  A reader polls until every word it needs carries the
// current round number; since each word validates itself, only per-location
// coherence is needed.  Round numbers start at 1 in every launch, whose
// exchange area is cleared before the launch.  Leaf passes alternate between
// two buffers: a workgroup can only be one pass ahead of the slowest reader.
// Every workgroup sums the exchanged values in the same order, so all of them
// take the same decisions and derive bit-identical reflectors.  Readers first
// wait on a per-exchange arrival counter (one word, bumped by each workgroup
// after it has published) and only then read the data: polling the data words
// themselves would flood the memory system with atomic loads while the slower
// workgroups are still computing.  The counter is a hint only; the round
// numbers in the data words still decide.
#include <algorithm>
#include <type_traits>

#include "kernels.hpp"

namespace rutv {

typedef unsigned long long u64;
typedef double dbl4 __attribute__((ext_vector_type(4)));
// two consecutive doubles of a column, 8-byte aligned (one 16-byte load)
typedef double dbl2u __attribute__((ext_vector_type(2), aligned(8)));

constexpr int kPQLeafThreads = 256;  // waves 0-3 hold the leaf rows
constexpr int kPQRpt = 1;            // leaf rows per thread
constexpr int kPQMaxRows = kPQLeafThreads * kPQRpt;
constexpr int kPQNB = 16;                  // leaf width
constexpr int kPQLdW = kPQMaxRows + 1;     // padded leading dimension of the leaf in LDS
constexpr int kPQMaxWG = 128;
constexpr int kPQTrail = kPQNB * kPQNB + kPQNB * (kPanelMaxCols - kPQNB);  // Gram + W^T C entries
constexpr int kPQGramE = kPQNB * (kPQNB + 1) / 2;  // packed upper triangle of a leaf Gram matrix
constexpr double kGramCap = 16.0;  // tolerated cancellation of a Gram-derived squared norm
constexpr unsigned kPQSpinLimit = 1u << 22;

// exchange area (64-bit words; a double is a pair of words)
constexpr i64 kXCnt = 0;                                      // arrival counters, one per 128-byte line
constexpr i64 kXGram = kXCnt + 3 * 16;                        // [2][kPQMaxWG][kPQGramE][2] leaf Gram partials
constexpr i64 kXTop = kXGram + 2 * kPQMaxWG * kPQGramE * 2;   // [2][kPQNB][kPQNB][2] leaf top block
constexpr i64 kXTot = kXTop + 2 * kPQNB * kPQNB * 2;          // [kPQTrail][2] reduced trailing sums
constexpr i64 kXPart = kXTot + kPQTrail * 2;                  // [P][kPQTrail][2] trailing partials

static int panel_grid(i64 m) {
  i64 P = std::max<i64>(cdiv(m, kPQMaxRows), std::min<i64>(32, cdiv(m, 64)));
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

// value of lane l (a wave-uniform index) in every lane
__device__ __forceinline__ double lane_value(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// calls f(integral_constant<int, J>) for J = J0, J0 + 1, ..., kPQNB - 1
template <int J0>
struct ForColumns {
  template <class F>
  __device__ __forceinline__ static void run(F& f) {
    f(std::integral_constant<int, J0>{});
    ForColumns<J0 + 1>::run(f);
  }
};
template <>
struct ForColumns<kPQNB> {
  template <class F>
  __device__ __forceinline__ static void run(F&) {}
};

// kPQThreads = 512: 8 waves, two per SIMD (256 registers each), a CU to itself;
// 256: 4 waves, one per SIMD, which fit beside one GEMM workgroup (2 waves of
// 128 registers per SIMD), so the workgroup is placed while GEMMs keep the chip
// busy.  Waves 0-3 hold the leaf rows in both; the matrix-core work is shared
// by all waves.
template <int kPQThreads>
__global__ __launch_bounds__(kPQThreads, 2) void panel_qr_kernel(
    int m, int k, double* __restrict__ A, i64 lda, double* __restrict__ tau, u64* __restrict__ xch,
    int* __restrict__ err, unsigned spin_limit) {
  constexpr int kPQWaves = kPQThreads / WAVE;
  const int P = gridDim.x, wg = blockIdx.x;
  // slabs are whole 16-row units (the last one ends at m), so that a column
  // segment of 16 rows is one 128-byte line when the column is line-aligned
  const int m16 = (m + 15) / 16;
  const int r0 = min(m, 16 * (int)((i64)m16 * wg / P)), r1 = min(m, 16 * (int)((i64)m16 * (wg + 1) / P));
  const int R = r1 - r0;

  __shared__ double Wl[kPQNB * kPQLdW];        // leaf rows during a pass, then the leaf's explicit W
  __shared__ double S[kPQNB * kPanelMaxCols];  // per-wave Gram partials; X = W^T C, then Tl^T X
  __shared__ double Gs[kPQNB * kPQNB];         // Gram matrix (pass: bottom rows; trailing: W^T W)
  __shared__ double Tl[kPQNB * kPQNB];
  __shared__ double Tops[kPQNB * kPQNB];       // top block, row-major
  __shared__ double Kl[kPQNB * kPQNB];         // pass coefficients K(a, c) at a * 16 + c
  __shared__ double taul[kPQNB];
  __shared__ double dgs[kPQNB];                // sqrt of the Gram diagonal
  __shared__ int jstop;
  __shared__ int dead;
  if (threadIdx.x == 0) dead = 0;
  __syncthreads();
  unsigned rnd = 0;

  // a bounded wait: on expiry record the error and stop waiting for good
  auto give_up = [&](unsigned& spins) -> bool {
    if (*(volatile int*)&dead) return true;
    if (++spins > spin_limit) {
      dead = 1;
      __hip_atomic_store(err, RANDUTV_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return true;
    }
    __builtin_amdgcn_s_sleep(1);
    return false;
  };

  // publish-then-wait on counter ctr (every workgroup adds 1 per exchange;
  // n-th exchange of that kind waits for n * P arrivals)
  unsigned narr[3] = {0, 0, 0};
  auto arrive_and_wait = [&](int ctr) {
    __syncthreads();
    ++narr[ctr];
    if (threadIdx.x == 0) {
      unsigned* cw = reinterpret_cast<unsigned*>(xch + kXCnt + 16 * ctr);
      __hip_atomic_fetch_add(cw, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned target = narr[ctr] * (unsigned)P;
      unsigned spins = 0;
      while (__hip_atomic_load(cw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target)
        if (give_up(spins)) break;
    }
    __syncthreads();
  };

  // the sum, in order, of the doubles published by workgroups [wb, we) (at
  // most 16) at base + w * stride pairs of words: one batch of loads,
  // repeated until every word carries the round's tag.  Sums over more
  // workgroups are split into such parts over several threads (one round
  // trip each instead of one per 16 workgroups), and the parts added in order.
  auto sum16 = [&](u64* base, i64 stride, int wb, int we, unsigned tg) -> double {
    constexpr int NB = 16;
    u64 lo[NB], hi[NB];
    unsigned spins = 0;
    while (true) {
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        u64* p = base + (i64)min(wb + i, we - 1) * stride * 2;
        lo[i] = xget(p);
        hi[i] = xget(p + 1);
      }
      int have = 1;
#pragma unroll
      for (int i = 0; i < NB; ++i) have &= (int)(wb + i >= we) | ((int)xhas(lo[i], tg) & (int)xhas(hi[i], tg));
      if (have || give_up(spins)) break;
    }
    double sv = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) sv += wb + i < we ? xval(lo[i], hi[i]) : 0.0;
    return sv;
  };
  const int nparts = (P + 15) / 16;

  for (int c0 = 0; c0 < k; c0 += kPQNB) {
    const int nbl = min(kPQNB, k - c0);
    // opaque zero and thread index: every address below is recomputed per leaf
    // instead of being hoisted out of this loop (they would not fit in registers)
    int z = 0, tid = threadIdx.x;
    asm volatile("" : "+s"(z), "+v"(tid));
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    double* const Ab = A + z;
    u64* const xgram = xch + z + kXGram;
    u64* const xtop = xch + z + kXTop;
    u64* const xtot = xch + z + kXTot;
    u64* const xpart = xch + z + kXPart;
    // the leaf's rows live in LDS (X(r, c) at Wl[c * kPQLdW + r]) through its
    // passes; loads are unconditional at clamped addresses, so all 16 are in
    // flight together
    int gr[kPQRpt];
    bool own[kPQRpt];
#pragma unroll
    for (int i = 0; i < kPQRpt; ++i) {
      const int r = tid + kPQLeafThreads * i;
      own[i] = tid < kPQLeafThreads && r < R;
      gr[i] = r0 + r;
      if (tid < kPQLeafThreads)
#pragma unroll
        for (int c = 0; c < kPQNB; ++c) {
          const double v = Ab[(i64)min(gr[i], m - 1) + (i64)(c0 + min(c, nbl - 1)) * lda];
          Wl[c * kPQLdW + r] = (own[i] && c < nbl) ? v : 0.0;
        }
    }

    for (int j0 = 0; j0 < nbl;) {
      const unsigned tag = ++rnd;
      const int par = (int)(tag & 1);
      u64* const xg = xgram + (i64)par * kPQMaxWG * kPQGramE * 2;
      u64* const xt = xtop + (i64)par * kPQNB * kPQNB * 2;
      // the owners of top-block rows publish them
      if (tid < kPQLeafThreads) {
#pragma unroll
        for (int i = 0; i < kPQRpt; ++i) {
          const int r = tid + kPQLeafThreads * i;
          const int t = gr[i] - c0;
          if (own[i] && t >= 0 && t < nbl)
#pragma unroll
            for (int c = 0; c < kPQNB; ++c) xput(xt + (i64)(t * kPQNB + c) * 2, Wl[c * kPQLdW + r], tag);
        }
      }
      __syncthreads();
      // Gram matrix of the rows below the top block on the matrix cores: wave
      // w takes local rows kRowsPerWave w .. kRowsPerWave (w + 1) - 1, four
      // per step; lane l supplies X(r, l % 16) as both operands,
      // D(a, b) = sum_r X(r, a) X(r, b)
      {
        dbl4 g = {0.0, 0.0, 0.0, 0.0};
        const int c = lane & 15;
        constexpr int kRowsPerWave = kPQMaxRows / kPQWaves;
#pragma unroll
        for (int s4 = 0; s4 < kRowsPerWave / 4; ++s4) {
          const int r = kRowsPerWave * wave + 4 * s4 + (lane >> 4);
          const double x = Wl[c * kPQLdW + r];
          g = __builtin_amdgcn_mfma_f64_16x16x4f64((r < R && r0 + r >= c0 + nbl) ? x : 0.0,
                                                   (r < R && r0 + r >= c0 + nbl) ? x : 0.0, g, 0, 0, 0);
        }
        // register q of lane l holds D(4 q + l / 16, l % 16)
#pragma unroll
        for (int q = 0; q < 4; ++q) S[wave * 256 + (4 * q + (lane >> 4)) * kPQNB + c] = g[q];
      }
      __syncthreads();
      // this workgroup's Gram entries (waves summed in order), packed upper
      // triangle e = b (b + 1) / 2 + a for a <= b
      if (tid < kPQNB * kPQNB) {
        const int a = tid & 15, b = tid >> 4;
        if (a <= b) {
          double sv = S[tid];
#pragma unroll
          for (int w = 1; w < kPQWaves; ++w) sv += S[w * 256 + tid];
          xput(xg + ((i64)wg * kPQGramE + b * (b + 1) / 2 + a) * 2, sv, tag);
        }
      }
      arrive_and_wait(0);
      // gather: items 0 .. nparts * 136 - 1 sum one part of one Gram entry
      // (into S), the next 64 read four entries of the top block each (one
      // batch); then the parts of each Gram entry are added in order
      {
        const int ng = kPQGramE * nparts;
        for (int it = tid; it < ng + kPQNB * kPQNB / 4; it += kPQThreads) {
          if (it < ng) {
            const int e = it % kPQGramE, part = it / kPQGramE;
            S[it] = sum16(xg + (i64)e * 2, kPQGramE, 16 * part, min(16 * part + 16, P), tag);
          } else {
            const int e = 4 * (it - ng), t = e >> 4;
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            if (t < nbl) {
              unsigned spins = 0;
              u64 lo[4], hi[4];
              while (true) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                  lo[i] = xget(xt + (i64)(e + i) * 2);
                  hi[i] = xget(xt + (i64)(e + i) * 2 + 1);
                }
                int have = 1;
#pragma unroll
                for (int i = 0; i < 4; ++i) have &= (int)xhas(lo[i], tag) & (int)xhas(hi[i], tag);
                if (have || give_up(spins)) break;
              }
#pragma unroll
              for (int i = 0; i < 4; ++i) v[i] = xval(lo[i], hi[i]);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) Tops[e + i] = v[i];
          }
        }
        __syncthreads();
        if (tid < kPQGramE) {
          double sv = S[tid];
          for (int part = 1; part < nparts; ++part) sv += S[part * kPQGramE + tid];
          int b = 0;
          while ((b + 1) * (b + 2) / 2 <= tid) ++b;
          const int a = tid - b * (b + 1) / 2;
          Gs[a * kPQNB + b] = sv;
          Gs[b * kPQNB + a] = sv;
        }
      }
      __syncthreads();
      if (tid < kPQNB) dgs[tid] = sqrt(fmax(Gs[tid * (kPQNB + 1)], 0.0));

      // the leaf's column recurrence from column j0 (wave 0; lane c % 16
      // follows column c: its top-block column Tc, its bottom coefficients Mc)
      if (wave == 0) {
        const int c = lane & 15;
        double Tc[kPQNB], Mc[kPQNB];
#pragma unroll
        for (int a = 0; a < kPQNB; ++a) {
          Tc[a] = Tops[a * kPQNB + c];
          Mc[a] = a == c ? 1.0 : 0.0;
        }
        int jf = nbl;
        auto step = [&](auto jc) {
          constexpr int jj = decltype(jc)::value;
          if (jj < j0 || jj >= jf) return;
          double mj[kPQNB], tj[kPQNB];
#pragma unroll
          for (int a = 0; a < kPQNB; ++a) mj[a] = a <= jj ? lane_value(Mc[a], jj) : 0.0;
#pragma unroll
          for (int t = jj; t < kPQNB; ++t) tj[t] = lane_value(Tc[t], jj);
          // g = G m_j (lane c: g_c), then d_c = (top and bottom) column j . column c
          double gcv = 0.0;
#pragma unroll
          for (int a = 0; a <= jj; ++a) gcv += Gs[c * kPQNB + a] * mj[a];
          double dc = 0.0;
#pragma unroll
          for (int t = jj + 1; t < kPQNB; ++t) dc += tj[t] * Tc[t];
#pragma unroll
          for (int a = 0; a < kPQNB; ++a) dc += lane_value(gcv, a) * Mc[a];
          const double sig2 = lane_value(dc, jj);  // squared norm below the diagonal
          double eb = 0.0;
#pragma unroll
          for (int a = 0; a <= jj; ++a) eb += fabs(mj[a]) * dgs[a];
          if (jj > j0 && eb * eb > kGramCap * sig2) {
            jf = jj;
            return;
          }
          const double alpha = tj[jj];
          double t = 0.0, scale = 0.0, beta = alpha;
          if (sig2 != 0.0) {
            const double nrm = sqrt(alpha * alpha + sig2);
            beta = alpha >= 0.0 ? -nrm : nrm;
            t = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
          }
          if (c > jj) {
            const double w = Tc[jj] + scale * dc;
            const double f = t * scale * w;
            Tc[jj] -= t * w;
#pragma unroll
            for (int r = jj + 1; r < kPQNB; ++r) Tc[r] -= f * tj[r];
#pragma unroll
            for (int a = 0; a <= jj; ++a) Mc[a] -= f * mj[a];
          } else if (c == jj) {
#pragma unroll
            for (int a = 0; a < kPQNB; ++a) Mc[a] = scale * mj[a];
            Tc[jj] = beta;
#pragma unroll
            for (int r = jj + 1; r < kPQNB; ++r) Tc[r] = scale * tj[r];
          }
          if (lane == 0) {
            taul[jj] = t;
            if (wg == 0) tau[c0 + jj] = t;
          }
        };
        ForColumns<0>::run(step);
        // K(:, c): identity before j0, scale_c m_c for finished columns, m_c
        // for the open ones
        if (lane < kPQNB) {
#pragma unroll
          for (int a = 0; a < kPQNB; ++a) {
            Kl[a * kPQNB + c] = c < j0 ? (a == c ? 1.0 : 0.0) : Mc[a];
            Tops[a * kPQNB + c] = Tc[a];
          }
        }
        if (lane == 0) jstop = jf;
      }
      __syncthreads();
      // apply the pass to this workgroup's rows, in place in Wl: top-block
      // rows from the recurrence, rows below through K (X K on the matrix
      // cores, a 16-row block per wave at a time: lane l supplies X(rb + l % 16,
      // k) and K(k, l % 16) for k = 4s + l / 16, and register q of the result
      // is row rb + 4q + l / 16, column l % 16), rows above unchanged.  A block
      // is read and written by its wave only.
      {
        const int lr = lane >> 4, lc = lane & 15;
        for (int rb = 16 * wave; rb < kPQMaxRows; rb += 16 * kPQWaves) {
          dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4) {
            const int kr = 4 * s4 + lr;
            d = __builtin_amdgcn_mfma_f64_16x16x4f64(Wl[kr * kPQLdW + rb + lc], Kl[kr * kPQNB + lc], d, 0, 0, 0);
          }
#pragma unroll
          for (int qq = 0; qq < 4; ++qq) {
            const int r = rb + 4 * qq + lr, t = r0 + r - c0;
            if (r < R) {
              if (t >= nbl) Wl[lc * kPQLdW + r] = d[qq];
              else if (t >= 0) Wl[lc * kPQLdW + r] = Tops[t * kPQNB + lc];
            }
          }
        }
      }
      j0 = jstop;
      __syncthreads();
    }

    // leaf back to memory; Wl := explicit W of the leaf (1 on the diagonal
    // row, 0 above it, the reflector below it; zero past nbl and past the slab)
#pragma unroll
    for (int i = 0; i < kPQRpt; ++i) {
      if (tid >= kPQLeafThreads) break;
      const int r = tid + kPQLeafThreads * i;
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) {
        const bool live = own[i] && c < nbl;
        const double v = Wl[c * kPQLdW + r];
        if (live) Ab[(i64)gr[i] + (i64)(c0 + c) * lda] = v;
        const int dr = c0 + c;
        Wl[c * kPQLdW + r] = live ? (gr[i] > dr ? v : (gr[i] == dr ? 1.0 : 0.0)) : 0.0;
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
      // last wave also forms the Gram W^T W.  The sum over rows is taken in
      // steps of 8 rows: lane (lr, lc) loads rows 8s + 2lr and 8s + 2lr + 1 of
      // column lc with one 16-byte load (a load instruction then touches 16
      // cache lines for 64 bytes each, not 32) and feeds them to two MFMAs,
      // against the same two rows of W.  Steps are taken in groups of kPF
      // whose C values are loaded one group ahead into alternating register
      // sets (a single set would have to wait for every load in flight before
      // it is refilled).
      constexpr int kPF = 4, NQ = (kPanelMaxCols / 16 - 1 + kPQWaves - 1) / kPQWaves;
      static_assert(NQ <= 4, "chunk dispatch below handles up to four chunks per wave");
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
      // a row pair starts at most at R - 2, so that both rows lie in the slab
      // (R >= 17 whenever trailing columns exist); a pair moved down that way
      // holds the wanted row R - 1 in its second element, and rows past the
      // slab meet zero rows of Wl
      const int nst = (R + 7) / 8;
      // one sweep over the slab for NQC live chunks (and the Gram when G)
      auto sweep = [&](auto nqc, auto gc) {
        constexpr int NQC = decltype(nqc)::value;
        constexpr bool G = decltype(gc)::value;
        constexpr int NS = NQC > 0 ? NQC : 1;
        dbl2u ca[NS][kPF], cb[NS][kPF];
        auto fetch = [&](dbl2u (&dst)[NS][kPF], int st0) {
#pragma unroll
          for (int i = 0; i < kPF; ++i) {
            const int p = min(8 * (st0 + i) + 2 * lr, R - 2);
#pragma unroll
            for (int qd = 0; qd < NQC; ++qd) dst[qd][i] = *reinterpret_cast<const dbl2u*>(Ac[qd] + p);
          }
        };
        auto work = [&](dbl2u (&src)[NS][kPF], int st0) {
#pragma unroll
          for (int i = 0; i < kPF; ++i) {
            const int ra = 8 * (st0 + i) + 2 * lr;
            const bool first_in_place = ra <= R - 2;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
              const int r = ra + j;
              const double wa = r < kPQMaxRows ? Wl[lc * kPQLdW + min(r, kPQMaxRows - 1)] : 0.0;  // W(r, a = lc)
#pragma unroll
              for (int qd = 0; qd < NQC; ++qd) {
                const double cv = (j == 0 && first_in_place) ? src[qd][i].x : src[qd][i].y;
                acc[qd] = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, cv, acc[qd], 0, 0, 0);
              }
              if (G) accg = __builtin_amdgcn_mfma_f64_16x16x4f64(wa, wa, accg, 0, 0, 0);
            }
          }
        };
        fetch(ca, 0);
        for (int st0 = 0; st0 < nst; st0 += 2 * kPF) {
          fetch(cb, st0 + kPF);
          work(ca, st0);
          fetch(ca, st0 + 2 * kPF);
          work(cb, st0 + kPF);
        }
      };
      using I0 = std::integral_constant<int, 0>;
      using I1 = std::integral_constant<int, 1>;
      using I2 = std::integral_constant<int, 2>;
      using I3 = std::integral_constant<int, NQ >= 3 ? 3 : NQ>;
      using I4 = std::integral_constant<int, NQ >= 4 ? 4 : NQ>;
      auto dispatch = [&](auto gc) {
        if (nq >= 4) sweep(I4{}, gc);
        else if (nq == 3) sweep(I3{}, gc);
        else if (nq == 2) sweep(I2{}, gc);
        else if (nq == 1) sweep(I1{}, gc);
        else if (decltype(gc)::value) sweep(I0{}, gc);
      };
      if (gram) dispatch(std::true_type{});
      else dispatch(std::false_type{});
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
    arrive_and_wait(1);
    // first exchange: workgroup wg sums entries [e0, e1) over all workgroups
    // (parts of at most 16 workgroups on separate threads, then the parts in
    // order)
    {
      const int e0 = (int)((i64)E * wg / P), e1 = (int)((i64)E * (wg + 1) / P), ne = e1 - e0;
      for (int it = tid; it < ne * nparts; it += kPQThreads) {
        const int e = e0 + it % ne, part = it / ne;
        S[it] = sum16(xpart + (i64)e * 2, kPQTrail, 16 * part, min(16 * part + 16, P), tag1);
      }
      __syncthreads();
      for (int e = e0 + tid; e < e1; e += kPQThreads) {
        double sv = S[e - e0];
        for (int part = 1; part < nparts; ++part) sv += S[part * ne + e - e0];
        xput(xtot + (i64)e * 2, sv, tag2);
      }
    }
    arrive_and_wait(2);
    // second exchange: every workgroup reads all totals
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
        for (int i = 0; i < NE; ++i) have &= ((int)xhas(lo[i], tag2) & (int)xhas(hi[i], tag2));
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
        // the Gram column is read unconditionally (a masked product per term
        // would put an LDS round trip on the chain of every term)
        double g[kPQNB];
#pragma unroll
        for (int l = 0; l < c; ++l) g[l] = Gs[l + c * kPQNB];
        const double tauc = taul[c];
        double sdot = 0.0;
#pragma unroll
        for (int l = 0; l < c; ++l) sdot += (l >= lane ? trow[l] : 0.0) * g[l];
        const double tc = lane < c ? -tauc * sdot : (lane == c ? tauc : 0.0);
        trow[c] = c < nbl ? tc : 0.0;
      }
#pragma unroll
      for (int c = 0; c < kPQNB; ++c) Tl[lane + c * kPQNB] = trow[c];
    }
    __syncthreads();
    // S <- Tl^T X on the matrix cores, a 16-column chunk per wave: lane l
    // supplies Tl^T(l % 16, k) and X(k, t0 + l % 16) for k = 4s + l / 16, and
    // register q of the result is S(4q + l / 16, t0 + l % 16).  A chunk is read
    // and written by its wave only.  Rows a >= nbl of X and columns a >= nbl of
    // Tl are zero (for a partial last leaf), so those rows of S come out zero.
    for (int q = wave; q < nchunk; q += kPQWaves) {
      const int t0 = 16 * q;
      dbl4 d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int kr = 4 * s4 + lr;
        const double tv = Tl[kr + lc * kPQNB];                                  // Tl^T(lc, kr)
        const double xv = kr < nbl ? S[kr * kPanelMaxCols + t0 + lc] : 0.0;  // X(kr, t0 + lc)
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(tv, xv, d, 0, 0, 0);
      }
#pragma unroll
      for (int qq = 0; qq < 4; ++qq) S[(4 * qq + lr) * kPanelMaxCols + t0 + lc] = d[qq];
    }
    __syncthreads();
    // update on the matrix cores: 16-row x 16-column blocks of C -= W Y with
    // Y = S (16 x ncr); the MFMA forms the block transposed, so a lane holds
    // 4 columns of one row: C[rb + lc][t0 + 4q + lr] (16 rows per column per
    // store).  A wave keeps the W fragment of its 16-row block in registers
    // and walks the chunks of 16 columns, kU at a time (independent MFMA
    // chains); the C values of the next kU chunks are loaded into the other
    // register set before the current ones are computed and stored (the wait
    // for a load then never includes the stores issued after it).  With fewer
    // row blocks than waves, the waves of one row block take every G-th chunk.
    {
      const int nrb = (R + 15) / 16;
      const int G = nrb >= kPQWaves ? 1 : kPQWaves / nrb;
      constexpr int kU = 4;
      const int t_first = wave % G;
      const int nmine = t_first < nchunk ? (nchunk - t_first + G - 1) / G : 0;  // chunks of this wave
      const int nsteps = (nmine + kU - 1) / kU;
      for (int rbi = wave / G; rbi < nrb; rbi += kPQWaves / G) {
        const int rb = 16 * rbi;
        const bool row_ok = rb + lc < R;
        // row rb + lc (clamped into the slab; rows past it load but never store)
        // of the trailing columns
        double* const Cr = Ab + (i64)(r0 + min(rb + lc, R - 1)) + (i64)(c0 + nbl) * lda;
        double wv[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) wv[kk] = Wl[(4 * kk + lr) * kPQLdW + rb + lc];  // W^T(4kk + lr, rb + lc)
        // chunk index of slot u of step st
        auto chunk = [&](int st, int u) { return t_first + G * (kU * st + u); };
        // unconditional loads at clamped addresses (the stores are guarded)
        auto fetch = [&](int st, double (&dst)[kU][4]) {
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int t0 = 16 * chunk(st, u);
#pragma unroll
            for (int q = 0; q < 4; ++q) dst[u][q] = Cr[(i64)min(t0 + 4 * q + lr, ncr - 1) * lda];
          }
        };
        auto finish = [&](int st, double (&src)[kU][4]) {
          dbl4 d[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int t0 = 16 * min(chunk(st, u), nchunk - 1);
            d[u] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) {
              const double yv = S[(4 * kk + lr) * kPanelMaxCols + t0 + lc];  // Y^T(t0 + lc, 4kk + lr)
              d[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv, wv[kk], d[u], 0, 0, 0);
            }
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const int t0 = 16 * chunk(st, u);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const int tc = t0 + 4 * q + lr;
              if (row_ok && tc < ncr) Cr[(i64)tc * lda] = src[u][q] - d[u][q];
            }
          }
        };
        double ga[kU][4], gb[kU][4];
        if (nsteps > 0) fetch(0, ga);
        for (int st = 0; st < nsteps; st += 2) {
          fetch(st + 1, gb);
          finish(st, ga);
          fetch(st + 2, ga);
          finish(st + 1, gb);
        }
      }
    }
    __syncthreads();
  }
}

int panel_qr(hipStream_t st, i64 m, i64 k, double* A, i64 lda, double* tau, const PanelWork& w,
             bool shared_cus) {
  if (k <= 0 || m <= 0) return RANDUTV_OK;
  if (k > kPanelMaxCols || m < k) return RANDUTV_ERR_TOO_LARGE;
  const int P = panel_grid(m);
  if (P > kPQMaxWG || 16 * cdiv(cdiv(m, 16), P) > kPQMaxRows) return RANDUTV_ERR_TOO_LARGE;
  LaunchTimer* tm = launch_timer();
  RUTV_CHECK(fill_zero_u32(st, reinterpret_cast<unsigned*>(w.xch), 2 * panel_words(P)));
  if (tm) tm->begin(st, K_PANEL);
  const unsigned lim = w.spin_limit ? w.spin_limit : kPQSpinLimit;
  if (shared_cus)
    panel_qr_kernel<256><<<P, 256, 0, st>>>((int)m, (int)k, A, lda, tau, w.xch, w.err, lim);
  else
    panel_qr_kernel<512><<<P, 512, 0, st>>>((int)m, (int)k, A, lda, tau, w.xch, w.err, lim);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->end(st, K_PANEL, 2.0 * m * k * k - 2.0 * k * k * k / 3.0, 0.0);
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
  if (tm) tm->end(st, K_EXTRACT, 0.0, 0.0);
  return RANDUTV_OK;
}

// ---------------------------------------------------------------------------
// Compact-WY factor from the Gram matrix G = W^T W (dlarft, forward,
// column-wise): T(j, j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j).
// Row i of T depends only on row i itself: T(i, j) = -tau_j sum_{l=i}^{j-1}
// T(i, l) G(l, j).  One workgroup owns a block of 32 rows and keeps them in
// LDS; it walks the 32-column blocks K of its rows: the part of the sum over
// the earlier column blocks is one product P = T(rows, o:oK) G(o:oK, K) on
// the matrix cores, the rest is the recurrence inside block K, one row per
// lane.  The workgroups do not depend on each other.
// ---------------------------------------------------------------------------
constexpr int kTB = 32;
constexpr int kTLd = kPanelMaxCols + 1;  // padded row length of the block row in LDS

__global__ __launch_bounds__(256) void larft_rows_kernel(int k, const double* __restrict__ G,
                                                         i64 ldg, const double* __restrict__ tau,
                                                         double* __restrict__ Tf, i64 ldt) {
  const int I = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int o = I * kTB, nblk = (k + kTB - 1) / kTB;
  __shared__ double Tr[kTB * kTLd];        // T(o + i, c) at i * kTLd + c
  __shared__ double Pb[kTB * (kTB + 1)];   // P(i, jj) at i * (kTB + 1) + jj
  __shared__ double Gd[kTB * (kTB + 1)];   // G(oK + l, oK + jj) at l * (kTB + 1) + jj
  __shared__ double tk[kTB];
  for (int e = tid; e < kTB * kTLd; e += 256) Tr[e] = 0.0;
  for (int K = I; K < nblk; ++K) {
    const int ok = K * kTB, nk = min(kTB, k - ok);
    // P = T(o:o+32, o:ok) G(o:ok, ok:ok+32): wave w forms the 16 x 16 tile
    // (rows 16 (w & 1), columns 16 (w >> 1)); lane l supplies
    // T(row l % 16, col 4 s + l / 16) and G(row 4 s + l / 16, col l % 16)
    {
      const int ti = 16 * (wave & 1), tj = 16 * (wave >> 1);
      dbl4 d = {0.0, 0.0, 0.0, 0.0};
      const int gc = min(ok + tj + (lane & 15), k - 1);
      for (int s4 = 0; s4 < (ok - o) / 4; ++s4) {
        const int l = o + 4 * s4 + (lane >> 4);
        const double a = Tr[(ti + (lane & 15)) * kTLd + l];
        const double g = G[l + (i64)gc * ldg];
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, g, d, 0, 0, 0);
      }
      // register r of lane l holds D(4 r + l / 16, l % 16)
#pragma unroll
      for (int r = 0; r < 4; ++r) Pb[(ti + 4 * r + (lane >> 4)) * (kTB + 1) + tj + (lane & 15)] = d[r];
    }
    for (int e = tid; e < kTB * kTB; e += 256) {
      const int l = e % kTB, jj = e / kTB;
      Gd[l * (kTB + 1) + jj] = (l < nk && jj < nk) ? G[(ok + l) + (i64)(ok + jj) * ldg] : 0.0;
    }
    if (tid < kTB) tk[tid] = tid < nk ? tau[ok + tid] : 0.0;
    __syncthreads();
    // recurrence inside block K, lane i = row o + i (rows past k stay zero)
    if (wave == 0 && lane < kTB && o + lane < k) {
      const int i = lane;
      double row[kTB];
#pragma unroll
      for (int jj = 0; jj < kTB; ++jj) row[jj] = 0.0;
#pragma unroll
      for (int jj = 0; jj < kTB; ++jj) {
        if (jj < nk) {
          double sv = Pb[i * (kTB + 1) + jj];
#pragma unroll
          for (int l = 0; l < jj; ++l) sv += row[l] * Gd[l * (kTB + 1) + jj];
          const int j = ok + jj;
          row[jj] = j < o + i ? 0.0 : (j == o + i ? tk[jj] : -tk[jj] * sv);
        }
      }
#pragma unroll
      for (int jj = 0; jj < kTB; ++jj)
        if (jj < nk) Tr[i * kTLd + ok + jj] = row[jj];
    }
    __syncthreads();
  }
  // the block row to memory (zeros left of the diagonal block)
  for (int e = tid; e < kTB * k; e += 256) {
    const int i = e % kTB, c = e / kTB;
    if (o + i < k) Tf[(o + i) + (i64)c * ldt] = Tr[i * kTLd + c];
  }
}

int larft_from_gram(hipStream_t st, i64 k, const double* G, i64 ldg, const double* tau, double* Tf,
                    i64 ldt) {
  if (k <= 0) return RANDUTV_OK;
  if (k > kPanelMaxCols) return RANDUTV_ERR_TOO_LARGE;
  const int nblk = (int)cdiv(k, kTB);
  LaunchTimer* tm = launch_timer();
  if (tm) tm->begin(st, K_LARFT);
  larft_rows_kernel<<<nblk, 256, 0, st>>>((int)k, G, ldg, tau, Tf, ldt);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->end(st, K_LARFT, (double)k * k * k / 3.0, 0.0);
  return RANDUTV_OK;
}

}  // namespace rutv
