// Sketch generator and small memory kernels.
#include <algorithm>

#include "kernels.hpp"

namespace rutv {

// ---------------------------------------------------------------------------
// Gaussian sketch G(i) (Section 3.1: i.i.d. standard normal entries).
// Philox4x64-10 (Salmon, Moraes, Dror & Shaw, SC'11): 64-bit multiplies by
// the two round constants, key schedule bumped by the two Weyl constants
// between rounds.  Key (seed, step); block k at counter (k, 0, 0, 0); each
// block's words x0..x3 give four normals by Box-Muller:
//   u0 = ((x >> 11) + 1) 2^-53 in (0, 1], u1 = (x' >> 11) 2^-53 in [0, 1),
//   z = sqrt(-2 ln u0) cos(2 pi u1), z' = sqrt(-2 ln u0) sin(2 pi u1).
// Normal number e lands at G(e % rows, e / rows) (column-major fill).
// ---------------------------------------------------------------------------
struct u64x4 {
  uint64_t v[4];
};

__device__ __forceinline__ u64x4 philox4x64_10(u64x4 ctr, uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  constexpr uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t lo0 = M0 * ctr.v[0], hi0 = __umul64hi(M0, ctr.v[0]);
    const uint64_t lo1 = M1 * ctr.v[2], hi1 = __umul64hi(M1, ctr.v[2]);
    u64x4 o;
    o.v[0] = hi1 ^ ctr.v[1] ^ k0;
    o.v[1] = lo1;
    o.v[2] = hi0 ^ ctr.v[3] ^ k1;
    o.v[3] = lo0;
    ctr = o;
  }
  return ctr;
}

__global__ __launch_bounds__(256) void sketch_kernel(uint64_t seed, uint64_t step, i64 rows, i64 cols,
                                                     double* __restrict__ G, i64 ldg) {
  const i64 count = rows * cols;
  const i64 nblocks = (count + 3) / 4;
  for (i64 b = (i64)blockIdx.x * 256 + threadIdx.x; b < nblocks; b += (i64)gridDim.x * 256) {
    u64x4 c{{(uint64_t)b, 0ull, 0ull, 0ull}};
    const u64x4 x = philox4x64_10(c, seed, step);
    double z[4];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const double u0 = ((double)(x.v[2 * h] >> 11) + 1.0) * 0x1p-53;
      const double u1 = (double)(x.v[2 * h + 1] >> 11) * 0x1p-53;
      const double r = sqrt(-2.0 * log(u0));
      const double ang = 2.0 * 3.141592653589793 * u1;
      z[2 * h] = r * cos(ang);
      z[2 * h + 1] = r * sin(ang);
    }
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const i64 e = 4 * b + l;
      if (e < count) G[(e % rows) + (e / rows) * ldg] = z[l];
    }
  }
}

int sketch(hipStream_t st, uint64_t seed, uint64_t step, i64 rows, i64 cols, double* G, i64 ldg) {
  if (rows <= 0 || cols <= 0) return RANDUTV_OK;
  const i64 nb = (rows * cols + 3) / 4;
  const int blocks = (int)std::min<i64>(cdiv(nb, 256), 16384);
  LaunchTimer* tm = launch_timer();
  if (tm) tm->begin(st, K_SKETCH);
  sketch_kernel<<<blocks, 256, 0, st>>>(seed, step, rows, cols, G, ldg);
  RUTV_TRY(hipGetLastError());
  if (tm) tm->end(st, K_SKETCH, 0.0, 0.0);
  return RANDUTV_OK;
}

// raw generator words of blocks first .. first + nblocks - 1 (for bit-exact
// checks of the integer stream)
__global__ __launch_bounds__(256) void sketch_words_kernel(uint64_t seed, uint64_t step,
                                                           uint64_t first, i64 nblocks,
                                                           uint64_t* __restrict__ out) {
  for (i64 j = (i64)blockIdx.x * 256 + threadIdx.x; j < nblocks; j += (i64)gridDim.x * 256) {
    u64x4 c{{first + (uint64_t)j, 0ull, 0ull, 0ull}};
    const u64x4 x = philox4x64_10(c, seed, step);
#pragma unroll
    for (int w = 0; w < 4; ++w) out[4 * j + w] = x.v[w];
  }
}

int sketch_words(hipStream_t st, uint64_t seed, uint64_t step, uint64_t first, i64 nblocks,
                 uint64_t* out) {
  if (nblocks <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(nblocks, 256), 16384);
  sketch_words_kernel<<<blocks, 256, 0, st>>>(seed, step, first, nblocks, out);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void identity_kernel(i64 rows, i64 cols, double* __restrict__ X,
                                                      i64 ldx) {
  const i64 total = rows * cols;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 r = e % rows, c = e / rows;
    X[r + c * ldx] = r == c ? 1.0 : 0.0;
  }
}

int set_eye(hipStream_t st, i64 rows, i64 cols, double* X, i64 ldx) {
  if (rows <= 0 || cols <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(rows * cols, 256), 16384);
  identity_kernel<<<blocks, 256, 0, st>>>(rows, cols, X, ldx);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

int set_identity(hipStream_t st, i64 n, double* X, i64 ldx) { return set_eye(st, n, n, X, ldx); }

// inverse of the k x k upper triangular R by back substitution, one column of
// the inverse per thread (R^{-1} e_j needs rows 0..j of column j only); the
// lower triangle is written as zeros
__global__ __launch_bounds__(64) void tri_inverse_kernel(int k, const double* __restrict__ R,
                                                         i64 ldr, double* __restrict__ X, i64 ldx,
                                                         int* __restrict__ flag) {
  const int j = blockIdx.x * 64 + threadIdx.x;
  if (j >= k) return;
  double* x = X + (i64)j * ldx;
  bool bad = false;
  for (int i = k - 1; i > j; --i) x[i] = 0.0;
  for (int i = j; i >= 0; --i) {
    double s = i == j ? 1.0 : 0.0;
    for (int l = i + 1; l <= j; ++l) s -= R[i + (i64)l * ldr] * x[l];
    const double r = R[i + (i64)i * ldr];
    const double v = s / r;
    bad |= r == 0.0 || !isfinite(v);
    x[i] = v;
  }
  if (bad) atomicOr(flag, 1);
}

int tri_inverse(hipStream_t st, i64 k, const double* R, i64 ldr, double* X, i64 ldx, int* flag) {
  if (k <= 0) return RANDUTV_OK;
  tri_inverse_kernel<<<(int)cdiv(k, 64), 64, 0, st>>>((int)k, R, ldr, X, ldx, flag);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

__global__ __launch_bounds__(256) void copy_check_kernel(i64 m, i64 n, const double* __restrict__ A,
                                                         i64 lda, double* __restrict__ B, i64 ldb,
                                                         int* __restrict__ flag) {
  const i64 total = m * n;
  int bad = 0;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 r = e % m, c = e / m;
    const double v = A[r + c * lda];
    if (!isfinite(v)) bad = 1;
    if (B) B[r + c * ldb] = v;
  }
  if (flag && bad) atomicOr(flag, 1);
}

int copy_check(hipStream_t st, i64 m, i64 n, const double* A, i64 lda, double* B, i64 ldb,
               int* flag) {
  if (m <= 0 || n <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(m * n, 256), 16384);
  copy_check_kernel<<<blocks, 256, 0, st>>>(m, n, A, lda, B, ldb, flag);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

int check_finite(hipStream_t st, i64 m, i64 n, const double* A, i64 lda, int* flag) {
  return copy_check(st, m, n, A, lda, nullptr, 0, flag);
}

__global__ void fill_u32_kernel(unsigned* p, i64 n) {
  const i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

int fill_zero_u32(hipStream_t st, unsigned* p, i64 n) {
  if (n <= 0) return RANDUTV_OK;
  fill_u32_kernel<<<(int)cdiv(n, 256), 256, 0, st>>>(p, n);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

__global__ __launch_bounds__(256) void diag_block_kernel(i64 k, const double* __restrict__ d,
                                                         double* __restrict__ D, i64 ldd) {
  const i64 total = k * k;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 r = e % k, c = e / k;
    D[r + c * ldd] = r == c ? d[r] : 0.0;
  }
}

int set_diag_block(hipStream_t st, i64 k, const double* d, double* D, i64 ldd) {
  if (k <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(k * k, 256), 1024);
  diag_block_kernel<<<blocks, 256, 0, st>>>(k, d, D, ldd);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

__global__ __launch_bounds__(256) void copy_matrix_kernel(i64 rows, i64 cols, const double* __restrict__ Y,
                                                          i64 ldy, double* __restrict__ X, i64 ldx) {
  const i64 total = rows * cols;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 r = e % rows, c = e / rows;
    X[r + c * ldx] = Y[r + c * ldy];
  }
}

int copy_matrix(hipStream_t st, i64 rows, i64 cols, const double* Y, i64 ldy, double* X, i64 ldx) {
  if (rows <= 0 || cols <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(rows * cols, 256), 16384);
  copy_matrix_kernel<<<blocks, 256, 0, st>>>(rows, cols, Y, ldy, X, ldx);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// X(:, i) *= c / lam[i] for i < cols (rows x cols, ld ldx); flag[0] |= 1 where
// lam[i] is zero or the result is not finite
__global__ __launch_bounds__(256) void scale_cols_kernel(i64 rows, i64 cols, double* __restrict__ X,
                                                         i64 ldx, const double* __restrict__ lam,
                                                         double c, int* __restrict__ flag) {
  const i64 total = rows * cols;
  int bad = 0;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 r = e % rows, i = e / rows;
    const double l = lam[i];
    const double v = X[r + i * ldx] * (c / l);
    if (l == 0.0 || !isfinite(v)) bad = 1;
    X[r + i * ldx] = v;
  }
  if (bad) atomicOr(flag, 1);
}

int scale_cols(hipStream_t st, i64 rows, i64 cols, double* X, i64 ldx, const double* lam,
               double c, int* flag) {
  if (rows <= 0 || cols <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(rows * cols, 256), 16384);
  scale_cols_kernel<<<blocks, 256, 0, st>>>(rows, cols, X, ldx, lam, c, flag);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// X (r x k, ld ldx): X[j, i] *= 2 / (d_i^2 - d_{k+j}^2), the eigenvalue gaps of
// d (descending singular values); flag[0] |= 1 on a zero gap or a
// non-finite result
__global__ __launch_bounds__(256) void gap_divide_kernel(i64 r, i64 k, double* __restrict__ X,
                                                         i64 ldx, const double* __restrict__ d,
                                                         int* __restrict__ flag) {
  const i64 total = r * k;
  int bad = 0;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 j = e % r, i = e / r;
    const double gap = d[i] * d[i] - d[k + j] * d[k + j];
    const double v = X[j + i * ldx] * (2.0 / gap);
    if (gap == 0.0 || !isfinite(v)) bad = 1;
    X[j + i * ldx] = v;
  }
  if (bad) atomicOr(flag, 1);
}

int gap_divide(hipStream_t st, i64 r, i64 k, double* X, i64 ldx, const double* d, int* flag) {
  if (r <= 0 || k <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(r * k, 256), 16384);
  gap_divide_kernel<<<blocks, 256, 0, st>>>(r, k, X, ldx, d, flag);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// lam[i] := d[i]^2
__global__ void square_kernel(i64 n, const double* __restrict__ d, double* __restrict__ lam) {
  const i64 i = (i64)blockIdx.x * 256 + threadIdx.x;
  if (i < n) lam[i] = d[i] * d[i];
}

int square_vec(hipStream_t st, i64 n, const double* d, double* lam) {
  if (n <= 0) return RANDUTV_OK;
  square_kernel<<<(int)cdiv(n, 256), 256, 0, st>>>(n, d, lam);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// Triangular combinations of k x k matrices (ld k), for the reverse passes of
// QR and LU factorizations:
//   mode 0: out = P_L(X - X^T)                  (P_L: strictly lower part)
//   mode 1: out = P_L(X) - triu(Y)               (triu: upper part with the diagonal)
//   mode 2: out = P_L(X)
__global__ __launch_bounds__(256) void tri_combine_kernel(int k, const double* __restrict__ X,
                                                          const double* __restrict__ Y,
                                                          double* __restrict__ out, int mode) {
  const int total = k * k;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
    const int i = e % k, j = e / k;
    double v = 0.0;
    if (mode == 0) {
      v = i > j ? X[i + j * k] - X[j + i * k] : 0.0;
    } else if (mode == 1) {
      v = i > j ? X[i + j * k] : -Y[i + j * k];
    } else {
      v = i > j ? X[i + j * k] : 0.0;
    }
    out[i + j * k] = v;
  }
}

int tri_combine(hipStream_t st, i64 k, const double* X, const double* Y, double* out, int mode) {
  if (k <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(k * k, 256), 1024);
  tri_combine_kernel<<<blocks, 256, 0, st>>>((int)k, X, Y, out, mode);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// X (k x k, ld k) := Y^T
__global__ __launch_bounds__(256) void transpose_kernel(int k, const double* __restrict__ Y,
                                                        double* __restrict__ X) {
  const int total = k * k;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < total; e += gridDim.x * 256) {
    const int i = e % k, j = e / k;
    X[i + j * k] = Y[j + i * k];
  }
}

int transpose_square(hipStream_t st, i64 k, const double* Y, double* X) {
  if (k <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(k * k, 256), 1024);
  transpose_kernel<<<blocks, 256, 0, st>>>((int)k, Y, X);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// X (rows x cols, ld ldx) := 0
__global__ __launch_bounds__(256) void zero_matrix_kernel(i64 rows, i64 cols, double* __restrict__ X,
                                                          i64 ldx) {
  const i64 total = rows * cols;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256)
    X[e % rows + (e / rows) * ldx] = 0.0;
}

int zero_matrix(hipStream_t st, i64 rows, i64 cols, double* X, i64 ldx) {
  if (rows <= 0 || cols <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(rows * cols, 256), 16384);
  zero_matrix_kernel<<<blocks, 256, 0, st>>>(rows, cols, X, ldx);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// Y += alpha X (rows x cols)
__global__ __launch_bounds__(256) void axpy_matrix_kernel(i64 rows, i64 cols, double alpha,
                                                          const double* __restrict__ X, i64 ldx,
                                                          double* __restrict__ Y, i64 ldy) {
  const i64 total = rows * cols;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 r = e % rows, c = e / rows;
    Y[r + c * ldy] += alpha * X[r + c * ldx];
  }
}

int axpy_matrix(hipStream_t st, i64 rows, i64 cols, double alpha, const double* X, i64 ldx, double* Y,
                i64 ldy) {
  if (rows <= 0 || cols <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(rows * cols, 256), 16384);
  axpy_matrix_kernel<<<blocks, 256, 0, st>>>(rows, cols, alpha, X, ldx, Y, ldy);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

}  // namespace rutv
