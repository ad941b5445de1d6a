/*
 * randutv.h -- C ABI of the MI355X (gfx950) randUTV library.
 *
 * Rank-revealing UTV factorization A = U T V^T (Heavner, Martinsson &
 * Quintana-Orti, arXiv 2002.06960, Section 1.1 eq. (1) and Section 3.1):
 * U (m x m) and V (n x n) orthogonal, T (m x n) upper triangular, computed by
 * the blocked randomized algorithm of Section 3.1 / Figure 2 (sketch with
 * power iteration, Householder QR of the sketch, right transform of all rows,
 * panel Householder QR, left transform, SVD of each diagonal b x b block).
 *
 * Conventions shared by every entry point:
 *   - real FP64, column-major storage;
 *   - every matrix/vector pointer is a DEVICE (HBM) pointer owned by the
 *     caller, unless the comment says "host";
 *   - calls run on the library's own HIP streams on the current device and
 *     return after the device work has finished (synchronous), unless noted;
 *   - return value: 0 on success; -k when the k-th argument is invalid
 *     (LAPACK style); RANDUTV_ERR_* (> 0) for run-time failures.  Outputs are
 *     undefined on a non-zero return.
 */
#ifndef RANDUTV_H
#define RANDUTV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RANDUTV_OK 0
#define RANDUTV_ERR_HIP 1          /* HIP runtime error or no usable device */
#define RANDUTV_ERR_NOMEM 2        /* device workspace allocation failed */
#define RANDUTV_ERR_NONFINITE 3    /* A holds NaN or Inf */
#define RANDUTV_ERR_NOCONV 4       /* a b x b Jacobi SVD exceeded its sweep cap */
#define RANDUTV_ERR_SYNC 5         /* a multi-workgroup kernel's bounded wait expired */
#define RANDUTV_ERR_TOO_LARGE 6    /* a dimension exceeds a documented kernel limit */
#define RANDUTV_ERR_RANK 7         /* the first block's sketch is rank deficient */
#define RANDUTV_ERR_SCRATCH 8      /* beyond the fixed scratch of randutv_factor_noalloc */

/*
 * randutv_factor -- A = U T V^T (Section 3.1, Figure 2).
 *   m, n    : rows and columns, m >= n >= 0 (the paper assumes m >= n).
 *   A, lda  : input m x n, lda >= max(1, m).  Read only, unless T == A.
 *   b       : block size, b >= 1 (clamped to n).  Kernel limit b <= 256.
 *   q       : power-iteration count, q >= 0 (Y = (B^T B)^q B^T G per step).
 *   seed    : key of the sketch stream: step i draws G(i), (m - i b) x b_i,
 *             i.i.d. N(0,1) from Philox4x64-10 keyed (seed, i), block k at
 *             counter (k, 0, 0, 0), four normals per block by Box-Muller,
 *             column-major fill (see randutv_sketch).
 *   U       : m x m output, ld = m; or NULL to skip building U.
 *   T       : m x n output, ld = m; may alias A when lda == m.
 *   V       : n x n output, ld = n; or NULL to skip building V.
 * Each diagonal b x b block of T is diagonal with non-negative, descending
 * entries (the singular values of that block's triangular factor).
 * m == 0 or n == 0 returns 0 without touching memory.  A holding NaN or Inf
 * returns RANDUTV_ERR_NONFINITE before any factorization work.
 * Errors: -1 m, -2 n (n < 0 or n > m), -3 A NULL, -4 lda, -5 b, -6 q,
 * -8 U aliases T or V, -9 T NULL (or T == A with lda != m), -10 V aliases T,
 * RANDUTV_ERR_TOO_LARGE for min(b, n) > 256 or m > 32768 (panel kernel
 * limit), checked before any device work; RANDUTV_ERR_* at run time (the
 * library drains its streams before returning an error).
 */
int randutv_factor(int64_t m, int64_t n, const double* A, int64_t lda,
                   int64_t b, int32_t q, uint64_t seed,
                   double* U, double* T, double* V);

/*
 * randutv_factor_ex -- the factorization of randutv_factor (Section 3.1,
 * Figure 2) with every option of the method exposed through one argument
 * structure.  Fields (the caller zero-initializes the structure, sets
 * struct_size = sizeof(randutv_args), then fills what it needs; a zero field
 * takes the default noted):
 *   m, n, A, lda, b, q, seed : as randutv_factor.
 *   U, ldu : m x m output (ldu >= m; 0 means m), or U = NULL to skip it.
 *   T, ldt : m x n output (ldt >= m; 0 means m); T == A needs ldt == lda.
 *   V, ldv : n x n output (ldv >= n; 0 means n), or V = NULL to skip it.
 *   stream : with RANDUTV_FLAG_STREAM, the caller's HIP stream (a
 *            hipStream_t; NULL is the null stream).  The library's work
 *            starts after everything enqueued on it before the call, and
 *            everything enqueued on it after the call starts after the
 *            library's work; the host thread still returns only when the
 *            factorization has finished (to report its status).  Without the
 *            flag the field is ignored and the library waits for nothing the
 *            caller enqueued (as randutv_factor).
 *   G      : NULL: the library draws the sketches itself (as randutv_factor).
 *            Otherwise the caller's sketches, which the algorithm uses
 *            instead: G(0), G(1), ..., G(p-1) stored one after the other,
 *            G(i) (m - i b) x b_i column-major with leading dimension
 *            m - i b, b_i = min(b, n - i b) (b clamped to n), so G(i) starts
 *            at element sum_{j<i} (m - j b) b_j; randutv_sketch_host writes
 *            this layout.  Device memory, or host memory with
 *            RANDUTV_FLAG_G_HOST (page-locked memory keeps the copies
 *            asynchronous).  Section 3.1 only asks for i.i.d. N(0,1) entries.
 *   sketch_bits : arithmetic of the sketch and power-iteration products
 *            Y = (B^T B)^q B^T G (0 means 64):
 *              RANDUTV_SKETCH_FP64 (64) FP64 matrix cores;
 *              RANDUTV_SKETCH_FP32 (32) operands rounded to FP32, FP32
 *                matrix cores (FP32 accumulation within a K split);
 *              RANDUTV_SKETCH_BF16 (16) operands rounded to BF16 (via FP32),
 *                BF16 matrix cores, FP32 accumulation;
 *              RANDUTV_SKETCH_BF16X3 (48) each operand split into BF16 parts
 *                x = hi + lo, product hi*hi + hi*lo + lo*hi (about 16
 *                significant bits per operand), FP32 accumulation.
 *            These products only choose the subspace that each step's V^
 *            spans: A = U T V^T and the orthogonality of U and V keep FP64
 *            accuracy in every mode.
 *   update_bits : arithmetic (same codes; 0 means 64) of the compact-WY
 *            updates of T, U and V (T V^, V V^, U U^, U^^T T and the
 *            products with W inside them).  Householder vectors, tau, the
 *            block factors and the b x b SVDs stay FP64 in every mode.  With
 *            reduced-precision updates A = U T V^T and the orthogonality of
 *            U and V hold only to about that precision times the number of
 *            steps (for FP32: ||A - U T V^T||_F / ||A||_F and max|U^T U - I|
 *            of order 1e-6 at n = 16000).
 *   flags  : RANDUTV_FLAG_STREAM       order the call on `stream`;
 *            RANDUTV_FLAG_G_HOST       G is in host memory;
 *            RANDUTV_FLAG_NO_FINITE_CHECK  skip the NaN/Inf scan of A (one
 *            read of A and one host round trip fewer; outputs are then
 *            undefined for such an A);
 *            RANDUTV_FLAG_ASYNC (with RANDUTV_FLAG_STREAM only) return as
 *            soon as the work is enqueued, with no host synchronization
 *            (the caller's host thread goes on while the GPU works); the
 *            run-time outcome (a non-finite A included: the kernels then run
 *            on it) is read afterwards by randutv_factor_status.
 *            Consecutive calls share the workspace and must be ordered
 *            through the caller's stream (or events on it); a call is not
 *            timed.  Capturing such a call into a HIP graph is not
 *            supported (ending the capture crashed in the runtime).
 *   jacobi_max_sweeps : sweep cap of each b x b Jacobi SVD (0 means 30);
 *            exceeding it returns RANDUTV_ERR_NOCONV.
 *   spin_limit : polls before a multi-workgroup kernel gives up a wait and
 *            reports RANDUTV_ERR_SYNC (0 means the built-in limit).  A small
 *            value makes the waits give up early: every kernel still ends,
 *            the outputs are garbage and the call returns RANDUTV_ERR_SYNC.
 *   max_workspace_bytes : largest device workspace the call may hold
 *            (0 means no limit); a call that needs more returns
 *            RANDUTV_ERR_NOMEM before any device work.
 * Errors: -1 m, -2 n, -3 A, -4 lda, -5 b, -6 q, -8 U/ldu, -9 T/ldt,
 * -10 V/ldv, -11 sketch_bits, -12 update_bits, -13 flags,
 * -14 jacobi_max_sweeps (< 0 or > 1000), -15 args NULL or struct_size
 * smaller than the structure of this header; RANDUTV_ERR_TOO_LARGE for
 * min(b, n) > 256 or m > 32768; RANDUTV_ERR_* at run time.  On a run-time
 * error the library drains its streams before it returns: no work of the
 * call is left running on the caller's buffers.
 */
#define RANDUTV_SKETCH_FP64 64
#define RANDUTV_SKETCH_FP32 32
#define RANDUTV_SKETCH_BF16 16
#define RANDUTV_SKETCH_BF16X3 48
#define RANDUTV_FLAG_G_HOST 1u
#define RANDUTV_FLAG_NO_FINITE_CHECK 2u
#define RANDUTV_FLAG_STREAM 4u
#define RANDUTV_FLAG_ASYNC 8u
struct ihipStream_t;
typedef struct randutv_args {
  int64_t struct_size;
  int64_t m, n;
  const double* A;
  int64_t lda;
  int64_t b;
  int32_t q;
  int32_t sketch_bits;
  uint64_t seed;
  double* U;
  int64_t ldu;
  double* T;
  int64_t ldt;
  double* V;
  int64_t ldv;
  struct ihipStream_t* stream;
  const double* G;
  int32_t update_bits;
  uint32_t flags;
  int32_t jacobi_max_sweeps;
  uint32_t spin_limit;
  int64_t max_workspace_bytes;
} randutv_args;
int randutv_factor_ex(const randutv_args* args);

/*
 * randutv_factor_status -- waits for all work on the current device and
 * returns the run-time outcome of the library's last factorization
 * (randutv_factor_ex or randutv_factor_noalloc with RANDUTV_FLAG_ASYNC; for a
 * synchronous call the value it already returned): RANDUTV_OK,
 * RANDUTV_ERR_NONFINITE (only if
 * the call checked A), RANDUTV_ERR_SYNC or RANDUTV_ERR_NOCONV, read from
 * the status words in the library's workspace; RANDUTV_OK when another
 * library call has used the workspace since (its words are gone).
 */
int randutv_factor_status(void);

/*
 * randutv_factor_noalloc -- randutv_factor_ex for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same factorization and kernels, with
 * every temporary carved out of a fixed device array of
 * RANDUTV_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs
 * on until the process ends.  The call makes no hipMalloc, hipFree or other
 * allocating call (the library's first call on a device still creates its
 * streams and events).  Arguments as randutv_factor_ex, except that
 * max_workspace_bytes must be 0.  The split-K partial sums get what the
 * fixed scratch leaves, so a large problem may use fewer K splits than
 * randutv_factor_ex (same arithmetic per split, different summation order).
 * What fits: about 4096 x 4096 at b = 128 or 2048 x 2048 at b = 256 with U
 * and V built; a problem whose other temporaries exceed the scratch returns
 * RANDUTV_ERR_SCRATCH before any device work.  Every call on a GPU shares
 * that GPU's scratch and leaves the last call's contents in it (each call
 * clears what must start at zero).  Two calls whose device work overlapped
 * on one GPU would race on it; the library prevents that within a process
 * (calls take one lock and return only after their device work has ended).
 * Errors: as randutv_factor_ex (-15 also for max_workspace_bytes != 0);
 * RANDUTV_ERR_SCRATCH.
 */
#define RANDUTV_NOALLOC_SCRATCH_BYTES (128ull << 20)
int randutv_factor_noalloc(const randutv_args* args);

/*
 * randutv_factor_ooc -- the factorization of randutv_factor (Section 3.1,
 * Figure 2) for matrices that stay in HOST memory, computed out of core as in
 * Section 3.2: HBM holds a cache of tiles (block columns of b columns, all
 * rows, of T, U and V) of at most hbm_budget_bytes, and a copy stream moves
 * tiles between host and HBM while the compute stream works on them
 * (Section 3.2.4; copies in and write-backs run on two streams, so both
 * directions of the host link work at once).  The result equals
 * randutv_factor's up to the summation
 * order of the products (sums over tiles instead of over whole columns).
 *   m, n, b, q, seed : as randutv_factor (same sketches G(i)).
 *   A, lda  : HOST m x n input, lda >= m.  Read only, unless T == A (then
 *             lda == ldt and A is factored in place).
 *   U, ldu  : HOST m x m output (ldu >= m), or NULL to skip it.
 *   T, ldt  : HOST m x n output (ldt >= m).
 *   V, ldv  : HOST n x n output (ldv >= n), or NULL to skip it.
 *   hbm_budget_bytes : device memory for the tile cache; it holds
 *             floor(budget / (8 max(m, n) b)) tiles and must hold at least 2.
 *             The fixed buffers of a step (sketch, reflectors, products of
 *             max(m, n) x b) come on top (stats->fixed_bytes).
 *   mode    : RANDUTV_OOC_TRADITIONAL (0) every access reads its tile from
 *             host memory and writes a changed tile straight back;
 *             RANDUTV_OOC_CACHED (1) least-recently-used cache with dirty
 *             bits, tiles copied when a miss needs them;
 *             RANDUTV_OOC_OVERLAPPED (2) the cache plus prefetch of the next
 *             tile of each sweep on the copy stream.
 *   stats   : NULL, or filled on return (struct_size set by the caller):
 *             wall time, time of the compute tasks and of the copies (HIP
 *             events on their streams), bytes and tiles moved, cache hits.
 * Page-locked host memory (hipHostMalloc) lets the copies run beside the
 * computation; pageable memory works but serializes them.  The call is
 * synchronous.  b <= 256 and m <= 32768 as in randutv_factor.
 * Errors: -1 m, -2 n, -3 A, -4 lda, -5 b, -6 q, -8 U/ldu, -9 T/ldt,
 * -10 V/ldv, -11 hbm_budget_bytes (< 2 tiles), -12 mode;
 * RANDUTV_ERR_TOO_LARGE, RANDUTV_ERR_NONFINITE, RANDUTV_ERR_* at run time.
 */
#define RANDUTV_OOC_TRADITIONAL 0
#define RANDUTV_OOC_CACHED 1
#define RANDUTV_OOC_OVERLAPPED 2
typedef struct randutv_ooc_stats {
  int64_t struct_size;
  double real_ms;      /* wall time of the call */
  double compute_ms;   /* sum of the compute tasks' durations */
  double io_ms;        /* h2d_ms + d2h_ms */
  double h2d_ms;       /* sum of the host -> HBM copies' durations */
  double d2h_ms;       /* sum of the HBM -> host write-backs' durations */
  int64_t h2d_bytes, d2h_bytes;
  int64_t tile_loads, tile_writebacks, tile_hits;
  int64_t slots, slot_bytes, fixed_bytes;
} randutv_ooc_stats;
int randutv_factor_ooc(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                       int32_t q, uint64_t seed, double* U, int64_t ldu, double* T,
                       int64_t ldt, double* V, int64_t ldv, int64_t hbm_budget_bytes,
                       int32_t mode, randutv_ooc_stats* stats);

/*
 * randutv_sketch_host -- every sketch G(0), ..., G(p-1) that randutv_factor
 * (m, n, ..., b, ..., seed) draws, written to HOST memory in the layout that
 * randutv_factor_ex takes as a caller's G (G(i) of (m - i b) x b_i,
 * column-major, ld m - i b, one after the other; b clamped to n, p =
 * ceil(n / b)): sum_i (m - i b) b_i doubles.  The values are generated on the
 * device by the generator described at randutv_factor, then copied out.
 * Errors: -2 m (m < 0), -3 n (n < 0 or n > m), -4 b, -5 G_host;
 * RANDUTV_ERR_NOMEM, RANDUTV_ERR_HIP.
 */
int randutv_sketch_host(uint64_t seed, int64_t m, int64_t n, int64_t b, double* G_host);

/*
 * randutv_sketch_words -- the raw 64-bit Philox4x64-10 words behind the
 * sketch of step `step` (key (seed, step), counter (k, 0, 0, 0) for block
 * k = first_block, ..., first_block + nblocks - 1): out[4 j + w] is word w of
 * block first_block + j (device memory, 4 nblocks words).  Exported so that
 * the integer stream can be compared bit for bit with an independent
 * implementation of the published generator.
 * Errors: -4 nblocks (< 0), -5 out.
 */
int randutv_sketch_words(uint64_t seed, uint64_t step, uint64_t first_block, int64_t nblocks,
                         uint64_t* out);

/*
 * randutv_truncate -- rank-k truncation A_k = U(:, 0:k) T(0:k, :) V^T
 * (Section 1.1).  U m x m (ld m), T m x n (ld m), V n x n (ld n), Ak m x n
 * (ld m), all device pointers from a previous randutv_factor.
 * 0 <= k <= n; k == 0 writes zeros.  Errors: -1 m, -2 n, -3 k, -4 U, -5 T,
 * -6 V, -7 Ak.
 */
int randutv_truncate(int64_t m, int64_t n, int64_t k, const double* U,
                     const double* T, const double* V, double* Ak);

/*
 * randutv_hqrrp -- randomized blocked column-pivoted QR A P = Q R (HQRRP,
 * Section 2, with the sketch of each step drawn as randutv_factor's step i:
 * Y = G^T A(s:m, s:n), G (m - s) x b_i; b_i steps of Householder CPQR on Y
 * choose the pivots (largest residual norm, lowest column on ties); the
 * column holding the t-th pivot is exchanged with column s + t; unpivoted
 * Householder QR of the b_i-column panel; compact-WY update of the rest).
 *   A    : m x n (ld lda), overwritten in the LAPACK dgeqp3 layout: R on and
 *          above the diagonal, the reflector vectors (v(0) = 1 implied) below.
 *   tau  : n reflector scalars (device).
 *   jpvt : n int64 (device): column j of A P is column jpvt[j] of A.
 * m >= n, n <= 32768.  b > n is clamped to n.  Synchronous.  Errors: -1 m,
 * -2 n, -3 A, -4 lda, -5 b, -7 tau, -8 jpvt, RANDUTV_ERR_TOO_LARGE for
 * min(b, n) > 256 or n > 32768,
 * RANDUTV_ERR_NONFINITE (A untouched), RANDUTV_ERR_SYNC.
 */
int randutv_hqrrp(int64_t m, int64_t n, double* A, int64_t lda, int64_t b,
                  uint64_t seed, double* tau, int64_t* jpvt);

/*
 * randutv_geqrf_blocked -- unpivoted blocked Householder QR A = Q R (LAPACK
 * dgeqrf's operation): randutv_hqrrp's step loop without the sketch, the
 * pivots and the exchanges (panel QR of b columns, compact-WY update of the
 * rest).  Section 2 weighs HQRRP's cost against this factorization; the
 * entry point is its baseline.
 *   A   : m x n (ld lda), overwritten in the LAPACK dgeqrf layout: R on and
 *         above the diagonal, the reflector vectors (v(0) = 1 implied) below.
 *   tau : n reflector scalars (device).
 * m >= n, m <= 32768.  b > n is clamped to n.  Device pointers, column-major
 * FP64, synchronous.  Errors: -1 m, -2 n, -3 A, -4 lda, -5 b, -6 tau,
 * RANDUTV_ERR_TOO_LARGE for min(b, n) > 256 or m > 32768,
 * RANDUTV_ERR_NONFINITE (A untouched), RANDUTV_ERR_SYNC.
 */
int randutv_geqrf_blocked(int64_t m, int64_t n, double* A, int64_t lda, int64_t b,
                          double* tau);

/*
 * randutv_truncate_first_block -- the first-block truncation A_k,
 * k = min(b, n), of randutv_factor(m, n, A, lda, b, q, seed, ...) computed
 * without the rest of the factorization: A_k = Q Q^T A with Q an orthonormal
 * basis of the range of M = (A A^T)^(q+1) G(0) (Section 3.1's first step;
 * why this equals U_k T(0:k, :) V^T is explained at randutv_truncate_grad).
 * Ak: m x n output (ld ldak), must not alias A.  Device pointers, column-major
 * FP64, synchronous.  Errors: -1 m, -2 n, -3 A, -4 lda, -5 b, -6 q, -8 Ak,
 * -9 ldak, RANDUTV_ERR_TOO_LARGE for min(b, n) > 256, RANDUTV_ERR_NONFINITE.
 */
int randutv_truncate_first_block(int64_t m, int64_t n, const double* A, int64_t lda,
                                 int64_t b, int32_t q, uint64_t seed, double* Ak,
                                 int64_t ldak);

/*
 * randutv_truncate_grad -- reverse pass (vector-Jacobian product) of the
 * first-block truncation A_k, k = min(b, n), of randutv_factor(m, n, A, lda,
 * b, q, seed, ...) with the sketch G(0) held fixed (Section 3.1 for the first
 * step; A_k as in randutv_truncate, Section 1.1).
 * Since T(0:k, :) V^T = U_k^T A, A_k = U_k U_k^T A, and step 0 makes range(U_k)
 * the range of M = (A A^T)^(q+1) G(0); A_k is the projection of A onto it.
 *   Gbar : m x n (ld ldg), dL/dA_k of some scalar L.
 *   Abar : m x n (ld ldab) output, dL/dA; must not alias A or Gbar.
 * All device pointers, column-major FP64; the call is synchronous.  The
 * sketch and power products are recomputed (nothing is kept from the
 * forward call).  Errors: -1 m, -2 n (n < 0 or n > m), -3 A, -4 lda, -5 b,
 * -6 q (q < 0 or q > 64: every power-iteration product is kept), -8 Gbar,
 * -9 ldg, -10 Abar (NULL or aliasing), -11 ldab,
 * RANDUTV_ERR_TOO_LARGE for min(b, n) > 256, RANDUTV_ERR_NONFINITE for NaN/Inf
 * in A or Gbar, RANDUTV_ERR_RANK when M has a zero pivot (the projector is
 * not differentiable there).
 */
int randutv_truncate_grad(int64_t m, int64_t n, const double* A, int64_t lda,
                          int64_t b, int32_t q, uint64_t seed, const double* Gbar,
                          int64_t ldg, double* Abar, int64_t ldab);

/*
 * randutv_truncate_grad_k -- reverse pass of the truncation A_k of
 * randutv_factor(m, n, A, lda, b, q, seed, ...) for any
 * 0 < k <= b_0 + b_1 (b_0 = min(b, n), b_1 = min(b, n - b_0): the first two
 * blocks of U), with the sketches G(0) and G(1) held fixed (Section 1.1 for
 * A_k, Section 3.1 for the steps).
 * k <= b_0: after step 0, U's first b_0 columns are the leading left singular
 * vectors of C = A Q_Y, Q_Y an orthonormal basis of Y = (A^T A)^q A^T G(0)
 * (the panel Q of C times the b x b SVD's left factor), so A_k = U_k U_k^T A
 * projects A onto C's leading k left singular vectors; the reverse pass
 * differentiates that projector (the eigenvalue gaps d_i^2 - d_j^2 of the
 * first block enter for i < k <= j) and the power chain.  k = b_0 gives
 * randutv_truncate_grad's value.
 * b_0 < k <= b_0 + b_1: A_k = Q_H Q_H^T A + U_2 U_2^T A with Q_H step 0's
 * panel Q and U_2 the leading k - b_0 left singular vectors of step 1's
 * C_1 = (I - Q_H Q_H^T) A Q_t, Q_t orthonormal for step 1's powered sketch of
 * the trailing matrix; that sketch is drawn in the coordinates of step 0's
 * Householder complements, so the reverse pass also runs through the
 * reflectors (an unpivoted LU of [I; 0] - Q_H) and both thin QRs of step 0.
 *   Gbar : m x n (ld ldg), dL/dA_k.   Abar : m x n (ld ldab) output, dL/dA.
 * Device pointers, column-major FP64, synchronous.  Errors: -1 m, -2 n,
 * -3 A, -4 lda, -5 b, -6 q (q < 0 or q > 64), -8 k, -9 Gbar, -10 ldg,
 * -11 Abar (NULL or aliasing), -12 ldab; RANDUTV_ERR_TOO_LARGE for
 * min(b, n) > 256; RANDUTV_ERR_NONFINITE; RANDUTV_ERR_RANK when a singular
 * value that enters is zero, a gap d_k = d_{k+1} is zero (no derivative
 * there) or a triangular factor is singular; RANDUTV_ERR_NOCONV /
 * RANDUTV_ERR_SYNC from a b x b SVD.
 */
int randutv_truncate_grad_k(int64_t m, int64_t n, const double* A, int64_t lda,
                            int64_t b, int32_t q, uint64_t seed, int64_t k,
                            const double* Gbar, int64_t ldg, double* Abar, int64_t ldab);

/*
 * randutv_truncate_first_block_k -- the forward value of the truncation A_k,
 * 0 < k <= b_0 + b_1 (b_0 = min(b, n), b_1 = min(b, n - b_0)), of
 * randutv_factor(m, n, A, lda, b, q, seed, ...) from its first step (k <= b_0)
 * or first two steps alone: A_k = U_k U_k^T A as described at
 * randutv_truncate_grad_k (Section 1.1, Section 3.1).  Ak: m x n output
 * (ld ldak), must not alias A.  Device
 * pointers, column-major FP64, synchronous.  Errors: -1 m, -2 n, -3 A,
 * -4 lda, -5 b, -6 q, -8 k, -9 Ak, -10 ldak; RANDUTV_ERR_TOO_LARGE,
 * RANDUTV_ERR_NONFINITE, RANDUTV_ERR_NOCONV, RANDUTV_ERR_SYNC.
 */
int randutv_truncate_first_block_k(int64_t m, int64_t n, const double* A, int64_t lda,
                                   int64_t b, int32_t q, uint64_t seed, int64_t k,
                                   double* Ak, int64_t ldak);

/*
 * randutv_truncate_batched -- randutv_truncate_first_block_k (reverse == 0)
 * or randutv_truncate_grad_k (reverse == 1) for `batch` matrices of the same
 * shape and the same (b, q, seed, k) in one call (Section 1.1, Section 3.1):
 * matrix t is A + t stride_a (ld lda), its Gbar is Gbar + t stride_g (ld ldg,
 * reverse only), and its result goes to out + t stride_o (ld ldo).  The
 * matrices are spread over the library's streams, each with a workspace of
 * its own, so that their launches overlap; every result equals the
 * single-matrix call's bit for bit.  Device pointers, column-major FP64,
 * synchronous.  Errors: -1 batch, -2 reverse, -3 m, -4 n, -5 A, -6 lda,
 * -7 stride_a (< lda n with batch > 1), -8 b, -9 q, -11 k, -12 Gbar, -13 ldg,
 * -14 stride_g, -15 out (NULL or aliasing A or Gbar), -16 ldo, -17 stride_o;
 * then the run-time errors of the single calls (the first one met, in batch
 * order).
 */
int randutv_truncate_batched(int64_t batch, int32_t reverse, int64_t m, int64_t n,
                             const double* A, int64_t lda, int64_t stride_a, int64_t b,
                             int32_t q, uint64_t seed, int64_t k, const double* Gbar,
                             int64_t ldg, int64_t stride_g, double* out, int64_t ldo,
                             int64_t stride_o);

/*
 * randutv_sketch -- write the sketch G(step) (rows x cols, ld = ldg) that
 * randutv_factor draws at that step (Section 3.1, "draw a random matrix with
 * i.i.d. standard normal entries"; generator as described at randutv_factor).
 * Element (r, c) is normal number r + c*rows of the (seed, step) stream.
 * Errors: -3 rows, -4 cols, -5 G, -6 ldg.
 */
int randutv_sketch(uint64_t seed, uint64_t step, int64_t rows, int64_t cols,
                   double* G, int64_t ldg);

/*
 * Building blocks of the step loop, exported for per-kernel checks.
 */

/* C = alpha op(A) op(B) + beta C with op(X) = X (trans 'N') or X^T ('T');
 * op(A) M x K, op(B) K x N, C M x N.  FP64 MFMA kernels.  C must not overlap
 * A or B.  Errors: -1 transa, -2 transb, -3 M, -4 N, -5 K, -8 lda, -10 ldb,
 * -13 ldc. */
int randutv_dgemm(char transa, char transb, int64_t M, int64_t N, int64_t K,
                  double alpha, const double* A, int64_t lda, const double* B,
                  int64_t ldb, double beta, double* C, int64_t ldc);

/* Same operation and arguments as randutv_dgemm, FP64 operands and result,
 * with the operands rounded to FP32 and multiplied on the FP32 matrix cores
 * (the product used by randutv_factor_ex with RANDUTV_SKETCH_FP32). */
int randutv_gemm_f32(char transa, char transb, int64_t M, int64_t N, int64_t K,
                     double alpha, const double* A, int64_t lda, const double* B,
                     int64_t ldb, double beta, double* C, int64_t ldc);

/* Same operation and arguments as randutv_dgemm, FP64 operands and result,
 * on the BF16 matrix cores with FP32 accumulation (the products used by
 * randutv_factor_ex with RANDUTV_SKETCH_BF16 / RANDUTV_SKETCH_BF16X3):
 * terms = 1 rounds each operand to BF16 (via FP32); terms = 3 splits each
 * operand x (rounded to FP32) into BF16 parts hi + lo and forms
 * hi*hi + hi*lo + lo*hi.  Errors as randutv_dgemm, plus -14 for terms other
 * than 1 or 3. */
int randutv_gemm_bf16(char transa, char transb, int64_t M, int64_t N, int64_t K,
                      double alpha, const double* A, int64_t lda, const double* B,
                      int64_t ldb, double beta, double* C, int64_t ldc, int32_t terms);

/* Householder QR of the m x k matrix A (m >= k, k <= 256) in place, LAPACK
 * dgeqr2 conventions (Figure 2's "unpivoted QR"): on return R is in the upper
 * triangle, reflector vectors (v(0) = 1 implied) below it, tau (k) holds the
 * scalars: A_in = H_0 ... H_{k-1} [R; 0], H_j = I - tau_j v_j v_j^T.
 * Errors: -1 m, -2 k, -3 A, -4 lda, -5 tau. */
int randutv_geqrf(int64_t m, int64_t k, double* A, int64_t lda, double* tau);

/* Forward column-wise compact-WY factor (LAPACK dlarft): from the reflectors
 * stored below the diagonal of W (m x k, ld ldw; diagonal and upper part are
 * ignored and read as 1 and 0) and tau, write the k x k upper triangular Tf
 * (ld ldt) with H_0 ... H_{k-1} = I - W Tf W^T (Figure 2's T_V, T_U).
 * Errors: -1 m, -2 k, -3 W, -4 ldw, -5 tau, -6 Tf, -7 ldt. */
int randutv_larft(int64_t m, int64_t k, const double* W, int64_t ldw,
                  const double* tau, double* Tf, int64_t ldt);

/* SVD of the k x k matrix R (k <= 256, ld ldr) by one-sided Jacobi
 * (Figure 2's "SVD(A_11)"): R = Us diag(d) Vs^T, d >= 0 descending (ties keep
 * column order), Us/Vs k x k (ld k); each (u_j, v_j) is signed so that the
 * largest-magnitude entry of v_j (lowest index on ties) is positive; u_j is
 * completed by Gram-Schmidt over e_1, e_2, ... where d_j == 0.  *sweeps
 * (host pointer, may be NULL) receives the sweep count.  Errors: -1 k, -2 R,
 * -3 ldr, -4 d, -5 Us, -6 Vs, RANDUTV_ERR_NONFINITE if R holds NaN/Inf,
 * RANDUTV_ERR_NOCONV after 30 sweeps. */
int randutv_gesvj(int64_t k, const double* R, int64_t ldr, double* d,
                  double* Us, double* Vs, int32_t* sweeps);

/* Per-kernel timing.  randutv_set_timing(1) clears the counters and makes
 * every later randutv_factor call record a HIP event pair around each kernel
 * launch on the stream it is launched on; randutv_set_timing(2) does the same
 * for the GEMM launches only (half the event records); randutv_set_timing(3)
 * times the GEMM launches only and runs each of them alone (the host waits
 * for all queued work before the launch and for the launch after it), so
 * that the recorded durations are the kernel's own rather than shares of a
 * chip that other streams' kernels also occupy; randutv_set_timing(0) stops
 * it.  Other values return -1.
 * randutv_kernel_stats writes, per kernel class, the number of launches, the
 * summed device time in ms and the algorithmic FP64 flops accumulated since
 * timing was enabled.  Returns the number of classes written (at most cap);
 * names: host array of cap pointers to static strings. */
int randutv_set_timing(int32_t enable);
int randutv_kernel_stats(int32_t cap, const char** names, int64_t* launches,
                         double* ms, double* flops);
/* The algorithmic memory traffic per kernel class, in the class order of
 * randutv_kernel_stats, accumulated over the same launches: for the GEMM
 * classes 8 (M K + K N + M N) bytes per launch, plus 8 M N when beta != 0 (C
 * read as well as written); 0 for classes that do not count it.  Returns the
 * number of classes written (at most cap); bytes: host array of cap doubles. */
int randutv_kernel_bytes(int32_t cap, double* bytes);
/* The per-launch record of the last randutv_factor call made with timing on
 * (the library's counterpart of a task-by-task execution trace): for launch i,
 * in the order the host enqueued them, its kernel class (index in
 * randutv_kernel_stats' order), the library stream it ran on (0: the critical
 * chain of sketch, power iteration, sketch panel, right and left transforms;
 * 1: block factors and the column-block panel; 2: the U and V updates and the
 * rows above the block row; 3: the b x b SVDs and their factors), its start
 * in ms after the call's first work was enqueued, and its duration in ms.
 * With GEMM-only timing only the GEMM launches are recorded.  Host arrays of
 * cap entries (any may be NULL); returns the number of records (at most cap
 * are written), -1 for cap < 0. */
int randutv_kernel_trace(int32_t cap, int32_t* cls, int32_t* stream, double* start_ms,
                         double* dur_ms);

/* Jacobi sweep counts of each step of the last randutv_factor call (host
 * array of cap entries); returns the number of steps. */
int randutv_last_sweeps(int32_t cap, int32_t* sweeps);

/* Text of the last HIP runtime error met by the calling thread inside the
 * library ("" if none), for diagnosing RANDUTV_ERR_HIP / RANDUTV_ERR_NOMEM. */
const char* randutv_last_hip_error(void);

/* Releases the library's streams, events and device workspace on the current
 * device after waiting for its work (the next call creates them again).
 * Meant for an orderly process exit: the Python binding calls it at
 * interpreter shutdown, before the HIP runtime is torn down.  Returns 0. */
int randutv_finalize(void);

/* Human-readable text for a return code (static storage). */
const char* randutv_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* RANDUTV_H */
