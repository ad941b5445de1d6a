// FP64 GEMM on the CDNA4 matrix cores: C = alpha op(A) op(B) + beta C.
//
// Every product of the randUTV step loop (sketch, power iteration, the X = A W
// products of the compact-WY updates and the rank-b updates A -= X Z^T) goes
// through this kernel.  Tiles of BM x BN are staged through LDS in BK-deep
// slices, double buffered: global loads run two slices ahead of the matrix
// cores and the LDS stores one slice ahead, at the top of each iteration.
// Tiles wholly inside C with a K range of whole slices (nearly all of them)
// take a loop without clamps or masks whose load addresses are a scalar base
// plus a per-thread offset.  Eight waves per workgroup, a 2 x 4 grid,
// each own a (BM/2) x (BN/4) sub-tile built from 16x16 blocks of
// v_mfma_f64_16x16x4; with two workgroups per CU every SIMD interleaves four
// waves, which hides the LDS and barrier latency of the matrix-core work.
//
// The MFMA is issued with the operands swapped (op(B)^T block as the 16x4
// operand, op(A)^T block as the 4x16 operand) so that the 16 lanes of a lane
// group hold 16 consecutive rows of one C column; a store instruction then
// covers 4 columns x 16 consecutive rows, i.e. full 128-byte segments of
// column-major C.
//
// Skinny products (an n x b output with K in the thousands) split K; each
// split writes alpha * partial to a buffer and a second kernel sums the splits
// in a fixed order (deterministic).
#include <type_traits>

#include "kernels.hpp"

namespace rutv {

typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// matrix-core step of one compute type: D(16 x 16) += A(16 x 4) B(4 x 16), lane
// l supplying A[l % 16][l / 16] and B[l / 16][l % 16]; kRow(r, lane) is the
// row of D that register r of the lane holds (its column is lane % 16)
template <class CT>
struct Mfma;
template <>
struct Mfma<double> {
  using V4 = dbl4;
  // NEG = 1: D += (-A) B, the matrix core's negate modifier on the first
  // operand (exact, so the result equals that of negated inputs bit for bit)
  template <int NEG = 0>
  __device__ __forceinline__ static V4 mma(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, NEG);
  }
  __device__ __forceinline__ static int row(int r, int lane) { return 4 * r + (lane >> 4); }
};
template <>
struct Mfma<float> {
  using V4 = flt4;
  template <int NEG = 0>
  __device__ __forceinline__ static V4 mma(float a, float b, V4 c) {
    static_assert(NEG == 0, "no negate modifier on the FP32 matrix-core step");
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static int row(int r, int lane) { return 4 * (lane >> 4) + r; }
};

constexpr int kWavesM = 2, kWavesN = 4;  // wave grid of a workgroup
#ifndef RUTV_GEMM_PIPE
#define RUTV_GEMM_PIPE 1
#endif
constexpr bool kGemmPipe2 = RUTV_GEMM_PIPE != 0;
#ifndef RUTV_GEMM_FAST
#define RUTV_GEMM_FAST 1
#endif
constexpr bool kGemmFast = RUTV_GEMM_FAST != 0;
constexpr int kGemmThreads = 64 * kWavesM * kWavesN;

// Global -> register loads of one operand slice.  An operand is either
// contiguous along the tile edge ("edge-major": op(A) = A, op(B) = B^T) or
// contiguous along K ("k-major": op(A) = A^T, op(B) = B).  Every thread keeps
// its own base offsets; indices are clamped into the matrix and out-of-range
// values replaced by zero, so the loads are unconditional (no branches around
// them, so the wait counters can pipeline them).
// x if keep else +0.0, as a bit mask (a select would let the compiler move
// the load into a branch)
__device__ __forceinline__ double keep_or_zero(double x, bool keep) {
  const long long m = -(long long)keep;
  return __longlong_as_double(__double_as_longlong(x) & m);
}

template <bool KMAJOR, int BE_, int BX, int BK, int NT>
struct SliceLoader {
  static constexpr int kStride = NT / (KMAJOR ? BK : BX);  // tile-edge (or k) step per r
  const double* base;  // matrix pointer
  i64 ld;
  int e0;              // this thread's first edge index (edge-major: fixed; k-major: + kStride r)
  int k_off;           // this thread's first k offset (edge-major: + kStride r; k-major: fixed)
  int tile0, edge_total;

  __device__ __forceinline__ void init(const double* p, i64 ldp, int tid, int t0, int et) {
    base = p;
    ld = ldp;
    tile0 = t0;
    edge_total = et;
    e0 = KMAJOR ? tid / BK : tid % BX;
    k_off = KMAJOR ? tid % BK : tid / BX;
  }
  // raw values of slice [k0, k0 + BK) (clamped addresses) and which of them
  // lie inside the matrix; the mask is applied when the values are written to
  // LDS, after the matrix-core work that hides the loads
  __device__ __forceinline__ void load(double (&v)[BE_], bool (&keep)[BE_], int k0, int kend) const {
    if (KMAJOR) {
      const int k = k0 + k_off;
      const bool kok = k < kend;
      const double* p = base + min(k, kend - 1);
#pragma unroll
      for (int r = 0; r < BE_; ++r) {
        const int e = tile0 + e0 + kStride * r;
        v[r] = p[(i64)min(e, edge_total - 1) * ld];
        keep[r] = kok && e < edge_total;
      }
    } else {
      const int e = tile0 + e0;
      const bool eok = e < edge_total;
      const double* p = base + min(e, edge_total - 1);
#pragma unroll
      for (int r = 0; r < BE_; ++r) {
        const int k = k0 + k_off + kStride * r;
        v[r] = p[(i64)min(k, kend - 1) * ld];
        keep[r] = eok && k < kend;
      }
    }
  }
  // slice [k0, k0 + BK) of a tile wholly inside the matrix with k0 + BK <=
  // kend: no clamps and no masks; the address of value r is a base that is
  // the same for every lane plus this thread's byte offset (below 2^32: at
  // most NT / BK edge steps or NT / BX k steps of ld), so the loads take the
  // scalar-base form and need no per-slice vector arithmetic
  __device__ __forceinline__ unsigned fast_offset() const {
    return (unsigned)(8 * (KMAJOR ? (i64)k_off + (i64)e0 * ld : (i64)e0 + (i64)k_off * ld));
  }
  __device__ __forceinline__ void load_fast(double (&v)[BE_], int k0, unsigned voff) const {
#pragma unroll
    for (int r = 0; r < BE_; ++r) {
      const double* sb = KMAJOR ? base + k0 + (i64)(tile0 + kStride * r) * ld
                                : base + tile0 + (i64)(k0 + kStride * r) * ld;
      v[r] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(sb) + voff);
    }
  }
  // LDS position (k, edge) of value r
  __device__ __forceinline__ int lds_k(int r) const { return KMAJOR ? k_off : k_off + kStride * r; }
  __device__ __forceinline__ int lds_e(int r) const { return KMAJOR ? e0 + kStride * r : e0; }
};

// Work item of workgroup L.  Workgroups are dealt to the 8 XCDs round-robin
// (L mod 8), so XCD x receives the x-th contiguous range of an ordering in
// which K splits are slowest and, within a split, the tile grid is walked in
// groups of kGroupM tile rows (all tile columns of a group, rows fastest):
// the concurrent workgroups of one XCD then share op(A) row panels and op(B)
// column panels in its L2.
constexpr int kGroupM = 8;

__device__ __forceinline__ void tile_of(int L, int tilesM, int tilesN, int splits, int& mt,
                                        int& nt, int& kz) {
  const int per = tilesM * tilesN, total = per * splits;
  const int q = total >> 3, r = total & 7, x = L & 7;
  const int idx = x * q + min(x, r) + (L >> 3);
  kz = idx / per;
  const int t = idx - kz * per;
  const int g = t / (kGroupM * tilesN);
  const int mb = g * kGroupM, gm = min(kGroupM, tilesM - mb);
  const int t2 = t - g * kGroupM * tilesN;
  mt = mb + t2 % gm;
  nt = t2 / gm;
}

// MINB: workgroups that must fit on a CU at once (the launch bound counts
// waves per SIMD, four SIMDs per CU)
template <class CT, bool TA, bool TB, int BM, int BN, int BK, int MINB = 2, int WGM = 2, int WGN = 2,
          int CINIT = 0>
__global__ __launch_bounds__(64 * WGM * WGN, MINB * WGM * WGN / 4) void dgemm_mfma_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, i64 lda,
    const double* __restrict__ B, i64 ldb, double beta, double* __restrict__ C, i64 ldc,
    int kchunk, double* __restrict__ part, int tilesM, int tilesN, int splits) {
  constexpr int NT = 64 * WGM * WGN;  // threads: a WGM x WGN grid of waves
  constexpr int cinit = CINIT;
  constexpr int WM = BM / WGM, WN = BN / WGN;
  constexpr int MI = WM / 16, NJ = WN / 16;
  constexpr int LDAS = BM + 1, LDBS = BN + 1;  // +1 double: conflict-free transposing stores
  constexpr int AE = BM * BK / NT, BE = BN * BK / NT;
  static_assert(AE * NT == BM * BK && BE * NT == BN * BK, "tile/threads");
  using MT = Mfma<CT>;
  using V4 = typename MT::V4;
  __shared__ CT As[2][BK * LDAS];
  __shared__ CT Bs[2][BK * LDBS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % WGM) * WM, wn0 = (wave / WGM) * WN;

  int mt, nt, kz;
  tile_of(blockIdx.x, tilesM, tilesN, splits, mt, nt, kz);
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = kz * kchunk;
  const int kend = min(K, kbeg + kchunk);

  SliceLoader<TA, AE, BM, BK, NT> la;
  SliceLoader<!TB, BE, BN, BK, NT> lb;
  la.init(A, lda, tid, m0, M);
  lb.init(B, ldb, tid, n0, N);
  double ra[AE], rb[BE];
  bool ka[AE], kb[BE];
  // cinit (FP64 only, one K split, beta = 1, alpha = +-1): the accumulators
  // start from C and the products enter with the sign of alpha (the negate
  // modifier of the matrix-core step for alpha = -1), so the result
  // C + alpha op(A) op(B) needs no read of C after the K loop
  constexpr int kNegB = cinit == 1 ? 1 : 0;
  auto sstore = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < AE; ++r)
      As[buf][la.lds_k(r) * LDAS + la.lds_e(r)] = static_cast<CT>(keep_or_zero(ra[r], ka[r]));
#pragma unroll
    for (int r = 0; r < BE; ++r)
      Bs[buf][lb.lds_k(r) * LDBS + lb.lds_e(r)] = static_cast<CT>(keep_or_zero(rb[r], kb[r]));
  };
  auto sstore_fast = [&](int buf) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < AE; ++r)
      As[buf][la.lds_k(r) * LDAS + la.lds_e(r)] = static_cast<CT>(ra[r]);
#pragma unroll
    for (int r = 0; r < BE; ++r) Bs[buf][lb.lds_k(r) * LDBS + lb.lds_e(r)] = static_cast<CT>(rb[r]);
  };
  V4 acc[MI][NJ];
  // interior: C addresses need no clamps (a different instruction sequence
  // per kind also keeps the loads inside their branch)
  auto init_acc = [&](auto interiorc) __attribute__((always_inline)) {
    constexpr bool I = decltype(interiorc)::value;
    if constexpr (cinit != 0) {
      const int cm = lane & 15;
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int gm = m0 + wm0 + 16 * i + cm;
        const int gmc = I ? gm : min(gm, M - 1);
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int gn = n0 + wn0 + 16 * j + MT::row(r, lane);
            const int gnc = I ? gn : min(gn, N - 1);
            acc[i][j][r] = static_cast<CT>(C[gmc + (i64)gnc * ldc]);
          }
      }
    } else {
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j) acc[i][j] = V4{0, 0, 0, 0};
    }
  };

  // tiles wholly inside C whose K range is whole slices take unmasked loads
  // with scalar bases (a uniform branch: the loop is compiled once per kind)
  // (the per-thread byte offsets stay below 2^32 for ld < 2^24)
  const bool fast = kGemmFast && m0 + BM <= M && n0 + BN <= N && (kend - kbeg) % BK == 0 &&
                    lda < (i64(1) << 24) && ldb < (i64(1) << 24);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  auto compute = [&](int cur) __attribute__((always_inline)) {
    const CT* as = As[cur];
    const CT* bs = Bs[cur];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4), cl = lane & 15;
      CT af[MI], bf[NJ];
#pragma unroll
      for (int i = 0; i < MI; ++i) af[i] = as[kr * LDAS + wm0 + 16 * i + cl];
#pragma unroll
      for (int j = 0; j < NJ; ++j) bf[j] = bs[kr * LDBS + wn0 + 16 * j + cl];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
          acc[i][j] = MT::template mma<kNegB>(bf[j], af[i], acc[i][j]);
    }
  };
  auto kloop = [&](auto fastc) __attribute__((always_inline)) {
    constexpr bool F = decltype(fastc)::value;
    unsigned voa = 0, vob = 0;
    if constexpr (F) {
      voa = la.fast_offset();
      vob = lb.fast_offset();
    }
    auto load_slice = [&](int t) __attribute__((always_inline)) {
      if constexpr (F) {
        la.load_fast(ra, kbeg + t * BK, voa);
        lb.load_fast(rb, kbeg + t * BK, vob);
      } else {
        la.load(ra, ka, kbeg + t * BK, kend);
        lb.load(rb, kb, kbeg + t * BK, kend);
      }
    };
    auto store_slice = [&](int buf) __attribute__((always_inline)) {
      if constexpr (F)
        sstore_fast(buf);
      else
        sstore(buf);
    };
    init_acc(fastc);
    if (nk == 0) return;
    load_slice(0);
    store_slice(0);
    if constexpr (kGemmPipe2) {
      // loads run two slices ahead of the matrix cores and LDS stores one:
      // slice t + 1 goes to the free buffer at the top of iteration t (its
      // previous contents were read before the barrier that ended t - 1), so
      // a load has a whole iteration to arrive and the stores overlap the
      // other waves' matrix-core work instead of preceding the barrier
      if (nk > 1) load_slice(1);
      __syncthreads();
      for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        if (t + 1 < nk) {
          store_slice(cur ^ 1);
          if (t + 2 < nk) load_slice(t + 2);
        }
        compute(cur);
        __syncthreads();
      }
    } else {
      __syncthreads();
      for (int t = 0; t < nk; ++t) {
        const int cur = t & 1;
        if (t + 1 < nk) load_slice(t + 1);
        compute(cur);
        if (t + 1 < nk) store_slice(cur ^ 1);
        __syncthreads();
      }
    }
  };
  if (fast)
    kloop(std::true_type{});
  else
    kloop(std::false_type{});

  // register r of a lane holds D(MT::row(r, lane), lane % 16); with the swapped
  // operands D is the transposed C block, so the lane holds
  // C[m0+wm0+16i+(lane&15)][n0+wn0+16j+MT::row(r, lane)], r = 0..3.  The C
  // values of row block i + 1 are loaded (clamped addresses) before the
  // results of row block i are stored, into alternating register sets, so
  // that the wait for a load never includes the stores issued after it.
  const int cm = lane & 15;
  const bool read_c = !part && beta != 0.0 && !cinit;
  double cva[NJ][4], cvb[NJ][4];
  auto load_c = [&](int i, double (&cv)[NJ][4]) {
    const int gmc = min(m0 + wm0 + 16 * i + cm, M - 1);
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gnc = min(n0 + wn0 + 16 * j + MT::row(r, lane), N - 1);
        cv[j][r] = C[gmc + (i64)gnc * ldc];
      }
  };
  auto store_c = [&](int i, const double (&cv)[NJ][4]) {
    const int gm = m0 + wm0 + 16 * i + cm;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gn = n0 + wn0 + 16 * j + MT::row(r, lane);
        double v = cinit ? static_cast<double>(acc[i][j][r]) : alpha * static_cast<double>(acc[i][j][r]);
        if (read_c) v += beta * cv[j][r];
        if (gm < M && gn < N) {
          if (part)
            part[(i64)kz * M * N + gm + (i64)gn * M] = v;
          else
            C[gm + (i64)gn * ldc] = v;
        }
      }
  };
  if (read_c) load_c(0, cva);
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    if (i % 2 == 0) {
      if (read_c && i + 1 < MI) load_c(i + 1, cvb);
      store_c(i, cva);
    } else {
      if (read_c && i + 1 < MI) load_c(i + 1, cva);
      store_c(i, cvb);
    }
  }
}

__global__ __launch_bounds__(256) void splitk_reduce_kernel(int M, int N, int S,
                                                            const double* __restrict__ part,
                                                            double beta, double* __restrict__ C,
                                                            i64 ldc) {
  const i64 MN = (i64)M * N;
  for (i64 idx = (i64)blockIdx.x * 256 + threadIdx.x; idx < MN; idx += (i64)gridDim.x * 256) {
    const int m = (int)(idx % M);
    const i64 n = idx / M;
    double s = 0.0;
    for (int z = 0; z < S; ++z) s += part[(i64)z * MN + idx];
    double* c = C + m + n * ldc;
    if (beta != 0.0) s += beta * *c;
    *c = s;
  }
}

// ---- BF16 products --------------------------------------------------------
// The sketch and power-iteration products only choose a subspace, so they may
// run on the BF16 matrix cores.  An FP64 operand value x is rounded to FP32
// (f) and then to BF16 (hi); with kTerms = 3 the remainder f - hi, exact in
// FP32, is rounded to BF16 as well (lo), and the product is formed as
// hi*hi + hi*lo + lo*hi (about 16 significant bits per operand instead of 8;
// lo*lo is below that).  Each 16x16x32 MFMA accumulates in FP32.
//
// Tiles are 128 x 128 with 32-deep slices, eight waves in a 2 x 4 grid as in
// the FP64 kernel.  LDS holds each slice k-contiguous ([edge][k], 40 values a
// row): a lane's 8 consecutive k of one row or column are one 16-byte read,
// and the 80-byte row pitch spreads the 16 rows of a lane group over
// distinct banks.  The conversion to BF16 happens once per element, when the
// slice is written to LDS.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBfBK = 32;         // k per slice: one 16x16x32 MFMA step
constexpr int kBfLd = kBfBK + 8;  // LDS row pitch (BF16 values)
constexpr int kBfThreads = 512;

// Global loads of one 128 x 32 slice of an operand, 8 values per thread.
// edge-major (contiguous along the tile edge): edge tid % 128, k 8*(tid/128)+r;
// k-major (contiguous along k): k tid % 32, edge tid/32 + 16 r.  Addresses are
// clamped into the matrix, out-of-range values masked to zero at the LDS
// store (as in SliceLoader).
template <bool KMAJOR>
struct BfLoader {
  const double* base;
  i64 ld;
  int tile0, edge_total;
  __device__ __forceinline__ int e_of(int tid, int r) const {
    return KMAJOR ? tid / kBfBK + 16 * r : tid % 128;
  }
  __device__ __forceinline__ int k_of(int tid, int r) const {
    return KMAJOR ? tid % kBfBK : 8 * (tid / 128) + r;
  }
  __device__ __forceinline__ void load(double (&v)[8], bool (&keep)[8], int tid, int k0,
                                       int kend) const {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int e = tile0 + e_of(tid, r), k = k0 + k_of(tid, r);
      const i64 ec = min(e, edge_total - 1), kc = min(k, kend - 1);
      v[r] = KMAJOR ? base[kc + ec * ld] : base[ec + kc * ld];
      keep[r] = e < edge_total && k < kend;
    }
  }
};

struct BfPair {
  __bf16 hi, lo;
};
__device__ __forceinline__ BfPair bf_split(double x) {
  const float f = static_cast<float>(x);
  const __bf16 hi = static_cast<__bf16>(f);
  return {hi, static_cast<__bf16>(f - static_cast<float>(hi))};
}

template <bool TA, bool TB, int kTerms>
__global__ __launch_bounds__(kBfThreads, 4) void gemm_bf16_kernel(
    int M, int N, int K, double alpha, const double* __restrict__ A, i64 lda,
    const double* __restrict__ B, i64 ldb, double beta, double* __restrict__ C, i64 ldc,
    int kchunk, double* __restrict__ part, int tilesM, int tilesN, int splits) {
  static_assert(kTerms == 1 || kTerms == 3, "one or three BF16 products");
  constexpr int kPlanes = kTerms == 3 ? 2 : 1;  // hi (and lo) parts
  constexpr int BM = 128, BN = 128, WM = BM / kWavesM, WN = BN / kWavesN;
  constexpr int MI = WM / 16, NJ = WN / 16;
  __shared__ __attribute__((aligned(16))) __bf16 As[2][kPlanes][BM * kBfLd];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][kPlanes][BN * kBfLd];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % kWavesM) * WM, wn0 = (wave / kWavesM) * WN;
  int mt, nt, kz;
  tile_of(blockIdx.x, tilesM, tilesN, splits, mt, nt, kz);
  const int m0 = mt * BM, n0 = nt * BN;
  const int kbeg = kz * kchunk;
  const int kend = min(K, kbeg + kchunk);

  const BfLoader<TA> la{A, lda, m0, M};
  const BfLoader<!TB> lb{B, ldb, n0, N};
  double ra[8], rb[8];
  bool ka[8], kb[8];
  auto sstore = [&](int buf) {
    if (TA) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const BfPair p = bf_split(keep_or_zero(ra[r], ka[r]));
        const int o = la.e_of(tid, r) * kBfLd + la.k_of(tid, r);
        As[buf][0][o] = p.hi;
        if (kTerms == 3) As[buf][kPlanes - 1][o] = p.lo;
      }
    } else {
      bf16x8 h, l;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const BfPair p = bf_split(keep_or_zero(ra[r], ka[r]));
        h[r] = p.hi;
        l[r] = p.lo;
      }
      const int o = la.e_of(tid, 0) * kBfLd + la.k_of(tid, 0);
      *reinterpret_cast<bf16x8*>(&As[buf][0][o]) = h;
      if (kTerms == 3) *reinterpret_cast<bf16x8*>(&As[buf][kPlanes - 1][o]) = l;
    }
    if (!TB) {
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const BfPair p = bf_split(keep_or_zero(rb[r], kb[r]));
        const int o = lb.e_of(tid, r) * kBfLd + lb.k_of(tid, r);
        Bs[buf][0][o] = p.hi;
        if (kTerms == 3) Bs[buf][kPlanes - 1][o] = p.lo;
      }
    } else {
      bf16x8 h, l;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const BfPair p = bf_split(keep_or_zero(rb[r], kb[r]));
        h[r] = p.hi;
        l[r] = p.lo;
      }
      const int o = lb.e_of(tid, 0) * kBfLd + lb.k_of(tid, 0);
      *reinterpret_cast<bf16x8*>(&Bs[buf][0][o]) = h;
      if (kTerms == 3) *reinterpret_cast<bf16x8*>(&Bs[buf][kPlanes - 1][o]) = l;
    }
  };

  flt4 acc[MI][NJ];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = flt4{0, 0, 0, 0};

  const int nk = kend > kbeg ? (kend - kbeg + kBfBK - 1) / kBfBK : 0;
  if (nk > 0) {
    la.load(ra, ka, tid, kbeg, kend);
    lb.load(rb, kb, tid, kbeg, kend);
    sstore(0);
    __syncthreads();
    // lane group g = lane / 16 supplies k = 8g .. 8g+7 of both operands (the
    // same k for the same operand slot, so the pairing is consistent)
    const int kq = 8 * (lane >> 4), cl = lane & 15;
    for (int t = 0; t < nk; ++t) {
      const int cur = t & 1;
      if (t + 1 < nk) {
        la.load(ra, ka, tid, kbeg + (t + 1) * kBfBK, kend);
        lb.load(rb, kb, tid, kbeg + (t + 1) * kBfBK, kend);
      }
      bf16x8 bh[NJ], bl[NJ];
#pragma unroll
      for (int j = 0; j < NJ; ++j) {
        const int o = (wn0 + 16 * j + cl) * kBfLd + kq;
        bh[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][0][o]);
        if (kTerms == 3) bl[j] = *reinterpret_cast<const bf16x8*>(&Bs[cur][kPlanes - 1][o]);
      }
#pragma unroll
      for (int i = 0; i < MI; ++i) {
        const int o = (wm0 + 16 * i + cl) * kBfLd + kq;
        const bf16x8 ah = *reinterpret_cast<const bf16x8*>(&As[cur][0][o]);
        bf16x8 al;
        if (kTerms == 3) al = *reinterpret_cast<const bf16x8*>(&As[cur][kPlanes - 1][o]);
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
          // swapped operands, as in the FP64 kernel: D is the transposed C block
          if (kTerms == 3) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bl[j], ah, acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], al, acc[i][j], 0, 0, 0);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bh[j], ah, acc[i][j], 0, 0, 0);
        }
      }
      if (t + 1 < nk) sstore(cur ^ 1);
      __syncthreads();
    }
  }

  // register r of a lane holds C[m0+wm0+16i+(lane&15)][n0+wn0+16j+4(lane>>4)+r]
  const int gm0 = m0 + wm0 + (lane & 15);
  const bool read_c = !part && beta != 0.0;
#pragma unroll
  for (int i = 0; i < MI; ++i) {
    const int gm = gm0 + 16 * i;
    if (gm >= M) continue;
#pragma unroll
    for (int j = 0; j < NJ; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gn = n0 + wn0 + 16 * j + 4 * (lane >> 4) + r;
        if (gn >= N) continue;
        double v = alpha * static_cast<double>(acc[i][j][r]);
        if (part) {
          part[(i64)kz * M * N + gm + (i64)gn * M] = v;
        } else {
          if (read_c) v += beta * C[gm + (i64)gn * ldc];
          C[gm + (i64)gn * ldc] = v;
        }
      }
  }
}

namespace {

struct Plan {
  int bm;      // square tile edge: 64 or 128
  int splits;  // K splits
  int kchunk;  // K per split (multiple of 16)
};

constexpr int kBK = 16;
#ifndef RUTV_GEMM_CINIT
#define RUTV_GEMM_CINIT 1
#endif
constexpr bool kCInit = RUTV_GEMM_CINIT != 0;
#ifndef RUTV_SPLITK_RESIDENT
#define RUTV_SPLITK_RESIDENT 768
#endif
constexpr i64 kResident = RUTV_SPLITK_RESIDENT;  // workgroups resident at once (two per CU)

Plan choose_plan(i64 M, i64 N, i64 K) {
  const i64 t128 = cdiv(M, 128) * cdiv(N, 128);
  Plan p{128, 1, (int)std::max<i64>(K, 1)};
  if (K <= 512) {  // rank-b updates and small products: no split
    if (t128 < kResident) p.bm = 64;
    return p;
  }
  if (t128 >= 2 * kResident) return p;
  // skinny output with long K: split K.  Cost model: rounds
  // of resident workgroups times (K per split + a fixed per-tile overhead of
  // about 256 of K); at least 128 of K per split.
  i64 best_s = 1;
  double best = 1e300;
  for (i64 s = 1; s <= 32; ++s) {
    const i64 chunk = cdiv(cdiv(K, s), kBK) * kBK;
    const i64 ns = cdiv(K, chunk);
    if (ns != s || (s > 1 && chunk < 128)) continue;
    const double cost = (double)cdiv(t128 * s, kResident) * (double)(chunk + 256);
    if (cost < best * 0.999) {
      best = cost;
      best_s = s;
    }
  }
  const i64 chunk = cdiv(cdiv(K, best_s), kBK) * kBK;
  p.splits = (int)cdiv(K, chunk);
  p.kchunk = (int)chunk;
  return p;
}

template <class CT, bool TA, bool TB>
void launch_tile(hipStream_t st, int bm, int M, int N, int K, double alpha, const double* A,
                 i64 lda, const double* B, i64 ldb, double beta, double* C, i64 ldc, int kchunk,
                 int splits, double* part) {
  const int tilesM = (int)cdiv(M, bm), tilesN = (int)cdiv(N, bm);
  const dim3 grid(tilesM * tilesN * splits);
  // accumulate onto C (no read of C after the K loop) for C += +-op(A) op(B)
  // in FP64 without a K split
  int cinit = 0;
  if (std::is_same<CT, double>::value && !part && beta == 1.0 && K > 0 &&
      (alpha == 1.0 || alpha == -1.0) && kCInit)
    cinit = alpha == -1.0 ? 1 : 2;
  auto go = [&](auto ci) {
    constexpr int CI = decltype(ci)::value;
    if (bm == 128)
      dgemm_mfma_kernel<CT, TA, TB, 128, 128, kBK, 2, kWavesM, kWavesN, CI>
          <<<grid, kGemmThreads, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part,
                                          tilesM, tilesN, splits);
    else
      dgemm_mfma_kernel<CT, TA, TB, 64, 64, kBK, 2, kWavesM, kWavesN, CI>
          <<<grid, kGemmThreads, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, kchunk, part,
                                          tilesM, tilesN, splits);
  };
  if (cinit == 1)
    go(std::integral_constant<int, std::is_same<CT, double>::value ? 1 : 0>{});
  else if (cinit == 2)
    go(std::integral_constant<int, std::is_same<CT, double>::value ? 2 : 0>{});
  else
    go(std::integral_constant<int, 0>{});
}

template <bool TA, bool TB>
void launch_bf16(hipStream_t st, int terms, int M, int N, int K, double alpha, const double* A,
                 i64 lda, const double* B, i64 ldb, double beta, double* C, i64 ldc, int kchunk,
                 int splits, double* part) {
  const int tilesM = (int)cdiv(M, 128), tilesN = (int)cdiv(N, 128);
  const dim3 grid(tilesM * tilesN * splits);
  if (terms == 3)
    gemm_bf16_kernel<TA, TB, 3><<<grid, kBfThreads, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta,
                                                              C, ldc, kchunk, part, tilesM, tilesN,
                                                              splits);
  else
    gemm_bf16_kernel<TA, TB, 1><<<grid, kBfThreads, 0, st>>>(M, N, K, alpha, A, lda, B, ldb, beta,
                                                              C, ldc, kchunk, part, tilesM, tilesN,
                                                              splits);
}

}  // namespace

i64 dgemm_work_elems(i64 M, i64 N, i64 K) {
  const Plan p = choose_plan(M, N, K);
  return p.splits > 1 ? (i64)p.splits * M * N : 0;
}

int dgemm(hipStream_t st, bool ta, bool tb, i64 M, i64 N, i64 K, double alpha, const double* A,
          i64 lda, const double* B, i64 ldb, double beta, double* C, i64 ldc, double* work,
          i64 work_elems, int prec) {
  if (M <= 0 || N <= 0) return RANDUTV_OK;
  if (M > INT32_MAX || N > INT32_MAX || K > INT32_MAX) return RANDUTV_ERR_TOO_LARGE;
  Plan p = choose_plan(M, N, K);
  if (p.splits > 1 && (work == nullptr || (i64)p.splits * M * N > work_elems)) {
    // not enough partial space: fall back to as many splits as fit
    i64 s = work ? work_elems / (M * N) : 0;
    if (s <= 1) {
      p.splits = 1;
      p.kchunk = (int)std::max<i64>(K, 1);
    } else {
      i64 chunk = cdiv(cdiv(K, s), kBK) * kBK;
      p.splits = (int)cdiv(K, chunk);
      p.kchunk = (int)chunk;
    }
  }
  const bool bf16 = prec == PREC_BF16 || prec == PREC_BF16X3;
  if (bf16) p.bm = 128;  // one tile shape for the BF16 kernel
  if (cdiv(M, p.bm) * cdiv(N, p.bm) * p.splits > INT32_MAX) return RANDUTV_ERR_TOO_LARGE;
  double* part = p.splits > 1 ? work : nullptr;
  const int cls = ta ? (tb ? K_GEMM_TT : K_GEMM_TN) : (tb ? K_GEMM_NT : K_GEMM_NN);
  LaunchTimer* tm = launch_timer();
  if (tm) tm->begin(st, cls);
  auto go = [&](auto ct) {
    using CT = decltype(ct);
    if (!ta && !tb)
      launch_tile<CT, false, false>(st, p.bm, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta,
                                    C, ldc, p.kchunk, p.splits, part);
    else if (ta && !tb)
      launch_tile<CT, true, false>(st, p.bm, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta,
                                   C, ldc, p.kchunk, p.splits, part);
    else if (!ta && tb)
      launch_tile<CT, false, true>(st, p.bm, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta,
                                   C, ldc, p.kchunk, p.splits, part);
    else
      launch_tile<CT, true, true>(st, p.bm, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta,
                                  C, ldc, p.kchunk, p.splits, part);
  };
  if (bf16) {
    const int terms = prec == PREC_BF16X3 ? 3 : 1;
    auto go16 = [&](auto ta_, auto tb_) {
      launch_bf16<decltype(ta_)::value, decltype(tb_)::value>(
          st, terms, (int)M, (int)N, (int)K, alpha, A, lda, B, ldb, beta, C, ldc, p.kchunk,
          p.splits, part);
    };
    using F = std::false_type;
    using T = std::true_type;
    if (!ta && !tb)
      go16(F{}, F{});
    else if (ta && !tb)
      go16(T{}, F{});
    else if (!ta && tb)
      go16(F{}, T{});
    else
      go16(T{}, T{});
  } else if (prec == PREC_F32) {
    go(0.0f);
  } else {
    go(0.0);
  }
  RUTV_TRY(hipGetLastError());
  // algorithmic bytes: op(A) and op(B) read, C read when beta != 0 (or
  // accumulated onto), C written
  if (tm)
    tm->end(st, cls, 2.0 * (double)M * (double)N * (double)K,
            8.0 * ((double)M * K + (double)K * N + (beta != 0.0 ? 2.0 : 1.0) * (double)M * N));
  if (part) {
    const i64 MN = M * N;
    const int blocks = (int)std::min<i64>(cdiv(MN, 256), 4096);
    if (tm) tm->begin(st, K_SPLITK);
    splitk_reduce_kernel<<<blocks, 256, 0, st>>>((int)M, (int)N, p.splits, part, beta, C, ldc);
    RUTV_TRY(hipGetLastError());
    if (tm) tm->end(st, K_SPLITK, 0.0, 0.0);
  }
  return RANDUTV_OK;
}

}  // namespace rutv
