// Host-side launchers of the gfx950 kernels (all enqueue on the given stream).
#pragma once

#include "common.hpp"

namespace rutv {

// Per-launch accounting hook (kernel timing); implemented by the driver.
struct LaunchTimer {
  virtual void begin(hipStream_t st, int cls) = 0;
  // flops: algorithmic flops of the launch; bytes: its algorithmic memory
  // traffic (every operand read once, every result written once; 0 where not
  // counted)
  virtual void end(hipStream_t st, int cls, double flops, double bytes) = 0;
  virtual ~LaunchTimer() = default;
};
void set_launch_timer(LaunchTimer* t);
LaunchTimer* launch_timer();

enum KernelClass : int {
  K_GEMM_NN = 0, K_GEMM_TN, K_GEMM_NT, K_GEMM_TT, K_SPLITK, K_PANEL, K_LARFT,
  K_JACOBI, K_SKETCH, K_EXTRACT, K_UTIL, K_APPLY_US, K_NUM_CLASSES
};
const char* kernel_class_name(int cls);

// ---- GEMM (gemm.hip) ------------------------------------------------------
// Arithmetic of a product (operands and result are FP64 in memory):
//   PREC_F64    FP64 matrix cores;
//   PREC_F32    operands rounded to FP32, FP32 matrix cores;
//   PREC_BF16   operands rounded to BF16 (via FP32), BF16 matrix cores;
//   PREC_BF16X3 each operand split into two BF16 parts x = hi + lo, product
//               hi*hi + hi*lo + lo*hi on the BF16 matrix cores.
// The reduced-precision forms accumulate in FP32 within a K split.
enum GemmPrec : int { PREC_F64 = 0, PREC_F32, PREC_BF16, PREC_BF16X3 };
// C = alpha op(A) op(B) + beta C.  'work' (work_elems doubles) holds split-K
// partial tiles; the launcher picks fewer splits when it is too small.
int dgemm(hipStream_t st, bool ta, bool tb, i64 M, i64 N, i64 K, double alpha,
          const double* A, i64 lda, const double* B, i64 ldb, double beta,
          double* C, i64 ldc, double* work, i64 work_elems, int prec = PREC_F64);
// split-K partial buffer size (doubles) that lets dgemm use its preferred plan
i64 dgemm_work_elems(i64 M, i64 N, i64 K);

// ---- Householder panel QR and compact-WY factor (householder.hip) ----------
constexpr int kPanelMaxCols = 256;
struct PanelWork {
  unsigned long long* xch = nullptr;  // exchange words between workgroups
  int* err = nullptr;                 // device status word
  unsigned spin_limit = 0;            // polls before a wait gives up (0: built-in limit)
};
// size (64-bit words) of PanelWork::xch for panels of up to m rows
i64 panel_work_elems(i64 m);
// shared_cus: the kernel variant that fits beside a GEMM workgroup on a CU
// (for a panel that runs while other streams keep the chip busy); otherwise
// each workgroup takes a CU for itself
int panel_qr(hipStream_t st, i64 m, i64 k, double* A, i64 lda, double* tau,
             const PanelWork& w, bool shared_cus = false);
// W (m x k, ld ldw) := explicit unit lower trapezoidal part of the factored
// panel P; R (k x k, ld ldr, may be null) := its upper triangle; if zero_panel
// the panel is overwritten with zeros afterwards.
int extract_reflectors(hipStream_t st, i64 m, i64 k, double* P, i64 ldp, double* W,
                       i64 ldw, double* R, i64 ldr, bool zero_panel);
// Tf (k x k, ld ldt) from the Gram matrix G = W^T W (k x k, ld ldg) and tau.
int larft_from_gram(hipStream_t st, i64 k, const double* G, i64 ldg,
                    const double* tau, double* Tf, i64 ldt);

// ---- Jacobi SVD (jacobi.hip) ------------------------------------------------
constexpr int kJacobiMaxN = 256;
constexpr int kJacobiMaxSweeps = 30;
i64 jacobi_work_elems(i64 k);
// status[0] = sweeps, status[1] = converged flag, status[2] = barrier error (device ints)
// max_sweeps: sweep cap (0: kJacobiMaxSweeps); spin_limit: polls before a
// grid-barrier wait gives up (0: built-in limit)
int jacobi_svd(hipStream_t st, i64 k, const double* R, i64 ldr, double* d, double* Us,
               double* Vs, double* work, int* status, int max_sweeps = 0,
               unsigned spin_limit = 0);
// count independent SVDs in one launch: problem p is R + p*rs (k x k, ld ldr;
// the last one k_last x k_last), outputs d + p*ds, Us/Vs + p*us (ld = its k),
// work + p*jacobi_work_elems(k), status + 3p.
int jacobi_svd_batched(hipStream_t st, int count, i64 k, i64 k_last, const double* R, i64 ldr,
                       i64 rs, double* d, i64 ds, double* Us, double* Vs, i64 us, double* work,
                       int* status, int max_sweeps = 0, unsigned spin_limit = 0);

// ---- HQRRP pivoting (hqrrp.hip) ---------------------------------------------
struct CpqrWork {
  double* sval = nullptr;     // 2 * 256 per-workgroup best norms (by step parity)
  int* sidx = nullptr;        // 2 * 256 their columns
  double* scol = nullptr;     // 2 * 256 * 256 the candidate columns (LDS variant)
  unsigned* counter = nullptr;  // grid barrier counter
  int* err = nullptr;         // device status word
};
struct ExchangeWork {
  int* idx = nullptr;                    // N entries
  int *chg = nullptr, *cnt = nullptr;    // 2k entries, 1
  double* tmp = nullptr;                 // m x 2k
  int64_t* jtmp = nullptr;               // 2k
};
// J[0..k) := the columns chosen by k steps of Householder column-pivoted QR of
// Y (k x N, ld ldy, k <= 256; Y is overwritten): largest residual norm first,
// the lowest column on ties
int cpqr_pivots(hipStream_t st, i64 k, i64 N, double* Y, i64 ldy, int* J, CpqrWork& w);
// exchange, in A (m rows, columns 0..N-1, ld lda) and jp, the column holding
// J[t] with column t for t = 0..k-1 in turn (N <= 32768)
int exchange_columns(hipStream_t st, i64 m, i64 k, i64 N, const int* J, double* A, i64 lda,
                     int64_t* jp, ExchangeWork& w);
int set_iota(hipStream_t st, i64 n, int64_t* x);

// ---- sketch and utilities (util.hip) ----------------------------------------
int sketch(hipStream_t st, uint64_t seed, uint64_t step, i64 rows, i64 cols, double* G,
           i64 ldg);
// out[4 j + w] := word w of the generator block first + j, j < nblocks
int sketch_words(hipStream_t st, uint64_t seed, uint64_t step, uint64_t first, i64 nblocks,
                 uint64_t* out);
int set_identity(hipStream_t st, i64 n, double* X, i64 ldx);
// X (rows x cols, ld ldx) := the first cols columns of the rows x rows identity
int set_eye(hipStream_t st, i64 rows, i64 cols, double* X, i64 ldx);
// X (k x k, ld ldx) := R^{-1} for the upper triangular R (k x k, ld ldr);
// flag[0] |= 1 if a diagonal entry is zero or the result is not finite
int tri_inverse(hipStream_t st, i64 k, const double* R, i64 ldr, double* X, i64 ldx, int* flag);
// B := A (m x n) and flag[0] |= 1 if A holds a non-finite value (flag may be null)
int copy_check(hipStream_t st, i64 m, i64 n, const double* A, i64 lda, double* B, i64 ldb,
               int* flag);
int check_finite(hipStream_t st, i64 m, i64 n, const double* A, i64 lda, int* flag);
int fill_zero_u32(hipStream_t st, unsigned* p, i64 n);
// write diag(d) into the k x k block D (ld ldd) (off-diagonal entries := 0)
int set_diag_block(hipStream_t st, i64 k, const double* d, double* D, i64 ldd);
// X (rows x cols, ld ldx) := Y (same shape, ld ldy)
int copy_matrix(hipStream_t st, i64 rows, i64 cols, const double* Y, i64 ldy, double* X,
                i64 ldx);
// X(:, i) *= c / lam[i] (rows x cols); flag[0] |= 1 on lam[i] == 0 or a non-finite result
int scale_cols(hipStream_t st, i64 rows, i64 cols, double* X, i64 ldx, const double* lam,
               double c, int* flag);
// X (r x k): X[j, i] *= 2 / (d_i^2 - d_{k+j}^2); flag[0] |= 1 on a zero gap
int gap_divide(hipStream_t st, i64 r, i64 k, double* X, i64 ldx, const double* d, int* flag);
// lam[i] := d[i]^2
int square_vec(hipStream_t st, i64 n, const double* d, double* lam);
// k x k (ld k): mode 0 out = P_L(X - X^T), mode 1 out = P_L(X) - triu(Y), mode 2
// out = P_L(X), with P_L the strictly lower part and triu the upper part
int tri_combine(hipStream_t st, i64 k, const double* X, const double* Y, double* out, int mode);
// X (k x k, ld k) := Y^T
int transpose_square(hipStream_t st, i64 k, const double* Y, double* X);
// X (rows x cols, ld ldx) := 0
int zero_matrix(hipStream_t st, i64 rows, i64 cols, double* X, i64 ldx);
// Y += alpha X (rows x cols)
int axpy_matrix(hipStream_t st, i64 rows, i64 cols, double alpha, const double* X, i64 ldx, double* Y,
                i64 ldy);

// ---- truncation of the first block and its reverse pass (truncation.hip) ----
struct TruncJob {
  i64 m = 0, n = 0, lda = 0, b = 0, k = 0;  // 0 < k <= min(b, n)
  int q = 0;
  uint64_t seed = 0;
  const double* A = nullptr;
  const double* Gbar = nullptr;  // reverse pass only
  i64 ldg = 0;
  double* out = nullptr;         // A_k (forward) or dL/dA (reverse)
  i64 ldo = 0;
  bool reverse = false;
};
// device workspace (bytes) of one job
size_t trunc_ws_bytes(const TruncJob& j);
// enqueue one job on st with its workspace at base; status: 8 device ints
int trunc_enqueue(const TruncJob& j, hipStream_t st, char* base, int* status);
// the job's status code from its 8 status ints (copied to the host)
int trunc_status(const int* flags, const TruncJob& j);

// ---- out-of-core factorization (ooc.hip) -------------------------------------
struct OocCfg {
  i64 m = 0, n = 0, b = 0;
  int q = 0;
  uint64_t seed = 0;
  const double* A = nullptr;  // host
  i64 lda = 0;
  double *U = nullptr, *T = nullptr, *V = nullptr;  // host (U, V may be null)
  i64 ldu = 0, ldt = 0, ldv = 0;
  size_t budget = 0;          // bytes of HBM for the tile cache
  int mode = 2;               // 0 traditional, 1 cached, 2 overlapped
  bool finite_check = true;
  int max_sweeps = 0;
  unsigned spin_limit = 0;
};
// the factorization with the matrices in host memory: cs computes, xs copies
// tiles in, ws writes them back
int ooc_factor(const OocCfg& c, hipStream_t cs, hipStream_t xs, hipStream_t ws,
               randutv_ooc_stats* stats);

}  // namespace rutv
