// randUTV driver and C ABI (see include/randutv.h).
//
// Step loop (Section 3.1, Figure 2; 0-based step i, s = i b, b_i = min(b, n-s)):
//   G     <- sketch(seed, i)                      (m-s) x b_i
//   Y     <- B^T G, then q times Y <- B^T (B Y)   B = T(s:m, s:n)
//   (W_V, tau_V) <- QR(Y);  T_V <- larft;  Z_V <- W_V T_V^T
//   T(:, s:n) -= (T(:, s:n) W_V) Z_V^T            all m rows
//   V(:, s:n) -= (V(:, s:n) W_V) Z_V^T
//   (W_U, tau_U, R) <- QR(T(s:m, s:s+b_i));  T_U;  Z_U <- W_U T_U^T
//   T(s:m, s+b_i:n) -= Z_U (W_U^T T(s:m, s+b_i:n))  (= H_U^T C)
//   U(:, s:m) -= (U(:, s:m) W_U) Z_U^T
//   T(s:m, s:s+b_i) <- 0;  R = U_S diag(d) V_S^T;  T(s:s+b_i, s:s+b_i) <- diag(d)
//   T(0:s, s:s+b_i) <- T(0:s, s:s+b_i) V_S;  V(:, s:s+b_i) <- V(:, s:s+b_i) V_S
//   U(:, s:s+b_i) <- U(:, s:s+b_i) U_S
// The left factors U_S^T of the rows T(s:s+b_i, s+b_i:n) are applied after
// the loop: later steps only multiply those rows from the right, and left and
// right factors commute, so the result is the same while the SVD stays off
// the path that feeds the next step.
#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "kernels.hpp"

namespace rutv {

// ---------------------------------------------------------------------------
// kernel timing (HIP events on the launching stream)
// ---------------------------------------------------------------------------
static thread_local char g_hip_error[256] = "";
void note_hip_error(hipError_t e) {
  snprintf(g_hip_error, sizeof(g_hip_error), "%s (%d): %s", hipGetErrorName(e), (int)e,
           hipGetErrorString(e));
}

static LaunchTimer* g_timer = nullptr;
void set_launch_timer(LaunchTimer* t) { g_timer = t; }
LaunchTimer* launch_timer() { return g_timer; }

static const char* kClassNames[K_NUM_CLASSES] = {
    "dgemm_nn", "dgemm_tn", "dgemm_nt", "dgemm_tt", "splitk_reduce", "panel_qr",
    "larft", "jacobi_svd", "sketch", "extract_reflectors", "util", "apply_us"};
const char* kernel_class_name(int cls) {
  return (cls >= 0 && cls < K_NUM_CLASSES) ? kClassNames[cls] : "?";
}

struct EventTimer final : LaunchTimer {
  struct Rec {
    hipEvent_t a, b;
    int cls;
    double flops, bytes;
    hipStream_t st;
  };
  // per-launch record of the last timed call: class, stream, start after the
  // call's reference event, duration
  struct TraceRec {
    int cls;
    hipStream_t st;
    float start, dur;
  };
  std::vector<TraceRec> trace;
  hipEvent_t ref = nullptr;
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  std::vector<hipEvent_t> open;  // begin events awaiting their end (one per class nesting level)
  bool gemm_only = false;  // time the GEMM launches alone (fewer event records)
  // run every GEMM launch alone: wait for all queued work before it and for
  // the launch itself after it, so that its duration is the kernel's own
  bool serialize = false;
  int64_t launches[K_NUM_CLASSES] = {};
  double ms[K_NUM_CLASSES] = {};
  double flops[K_NUM_CLASSES] = {};
  double bytes[K_NUM_CLASSES] = {};

  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  void start_call() {
    used = 0;
    recs.clear();
    open.clear();
    trace.clear();
    ref = nullptr;
  }
  // the reference event of the per-launch starts, on stream st before the
  // call's first work
  void mark(hipStream_t st) {
    ref = take();
    if (ref) (void)hipEventRecord(ref, st);
  }
  void clear_counts() {
    for (int c = 0; c < K_NUM_CLASSES; ++c) launches[c] = 0, ms[c] = 0.0, flops[c] = 0.0, bytes[c] = 0.0;
  }
  void destroy() {
    for (auto e : pool) (void)hipEventDestroy(e);
    pool.clear();
    used = 0;
    recs.clear();
    open.clear();
  }
  static bool is_gemm(int cls) { return cls >= K_GEMM_NN && cls <= K_GEMM_TT; }
  void begin(hipStream_t st, int cls) override {
    if (serialize && is_gemm(cls)) (void)hipDeviceSynchronize();
    hipEvent_t e = gemm_only && !is_gemm(cls) ? nullptr : take();
    if (e) (void)hipEventRecord(e, st);
    open.push_back(e);
  }
  void end(hipStream_t st, int cls, double f, double by) override {
    hipEvent_t a = open.empty() ? nullptr : open.back();
    if (!open.empty()) open.pop_back();
    hipEvent_t b = a ? take() : nullptr;
    if (a && b) {
      (void)hipEventRecord(b, st);
      recs.push_back({a, b, cls, f, by, st});
    }
    if (serialize && is_gemm(cls)) (void)hipStreamSynchronize(st);
  }
  void collect() {
    for (auto& r : recs) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.cls] += t;
        launches[r.cls] += 1;
        flops[r.cls] += r.flops;
        bytes[r.cls] += r.bytes;
        float t0 = 0.f;
        if (ref && hipEventElapsedTime(&t0, ref, r.a) == hipSuccess) trace.push_back({r.cls, r.st, t0, t});
      }
    }
    recs.clear();
    used = 0;
  }
};

// ---------------------------------------------------------------------------
// per-process library state: streams, events, workspace, timing
// ---------------------------------------------------------------------------
enum { ST_T = 0, ST_P, ST_UV, ST_S, NSTREAMS };
constexpr int kEvRing = 4;  // events of a kind are reused every kEvRing steps
#ifndef RUTV_TOP_ON_UV
#define RUTV_TOP_ON_UV 1
#endif
// the right transform of the rows above the current block row on stream UV
constexpr bool kTopOnUV = RUTV_TOP_ON_UV != 0;
// reflector buffers (W, Z of V^ and of U^) by step: stream T may run this many
// steps ahead of the U/V updates that read them
#ifndef RUTV_WY_BUFFERS
#define RUTV_WY_BUFFERS 2
#endif
constexpr int kWyBuf = RUTV_WY_BUFFERS;
static_assert(kWyBuf >= 2 && kWyBuf - 2 < kEvRing, "an awaited event must not be re-recorded first");
enum { EV_V = 0, EV_COLS, EV_U, EV_UV, EV_PRE, EV_WV, EV_WU, EV_LEFT, EV_TOP, EV_KINDS };

// Device scratch of the allocation-free factorization entry point: file-scope
// device memory, one copy per GPU, resolved to a device address per device
// at set-up (host code never passes the array's name to a kernel).
static __device__ __align__(256) char scratch[RANDUTV_NOALLOC_SCRATCH_BYTES];

// one library lock: calls are serialized across threads and devices (the
// launch timer is process-wide)
static std::mutex g_mu;

struct Context {
  int device = -1;
  char* scratch_ptr = nullptr;  // this device's copy of `scratch`
  hipStream_t st = nullptr;  // == streams[ST_T]
  hipStream_t streams[NSTREAMS] = {};
  hipEvent_t ev[EV_KINDS][kEvRing] = {};
  hipEvent_t ev_misc[4] = {};
  hipEvent_t ev_tail[2][NSTREAMS] = {};  // the end of the factorization: two joins of all streams
  int* last_status = nullptr;  // status words of the last factorization (in the workspace)
  i64 last_nsteps = 0;
  bool last_finite_check = false;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool timing = false;
  EventTimer timer;
  std::vector<int> sweeps;

  // set-up on the current device (each device has a Context of its own)
  int init() {
    int dev = 0;
    RUTV_TRY(hipGetDevice(&dev));
    if (st) return RANDUTV_OK;
    device = dev;
    RUTV_TRY(hipGetSymbolAddress(reinterpret_cast<void**>(&scratch_ptr), HIP_SYMBOL(scratch)));
    // Streams created with a CU mask (here: every CU) get a hardware queue of
    // their own; pooled streams share the few queues a process has by default,
    // and a long kernel (a batch of Jacobi SVDs) then holds up every kernel of
    // the other streams queued behind it on the same queue.
    {
      hipDeviceProp_t prop;
      RUTV_TRY(hipGetDeviceProperties(&prop, dev));
      const int words = (prop.multiProcessorCount + 31) / 32;
      std::vector<uint32_t> mask(words, 0xffffffffu);
      if (prop.multiProcessorCount % 32) mask[words - 1] = (1u << (prop.multiProcessorCount % 32)) - 1u;
      for (auto& x : streams)
        if (hipExtStreamCreateWithCUMask(&x, (uint32_t)words, mask.data()) != hipSuccess) {
          (void)hipGetLastError();
          RUTV_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        }
    }
    for (auto& kind : ev)
      for (auto& e : kind) RUTV_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& e : ev_misc) RUTV_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    for (auto& row : ev_tail)
      for (auto& e : row) RUTV_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    st = streams[ST_T];
    return RANDUTV_OK;
  }
  // release streams, events and the workspace (explicit teardown, before the
  // HIP runtime itself is torn down at process exit)
  void release() {
    if (!st) return;
    for (auto& x : streams) (void)hipStreamSynchronize(x);
    for (auto& x : streams) (void)hipStreamDestroy(x);
    for (auto& kind : ev)
      for (auto& e : kind) (void)hipEventDestroy(e);
    for (auto& e : ev_misc) (void)hipEventDestroy(e);
    for (auto& row : ev_tail)
      for (auto& e : row) (void)hipEventDestroy(e);
    timer.destroy();
    if (ws) (void)hipFree(ws);
    ws = nullptr;
    ws_bytes = 0;
    last_status = nullptr;
    st = nullptr;
    for (auto& x : streams) x = nullptr;
    device = -1;
    scratch_ptr = nullptr;
  }
  // wait for everything the library enqueued (used before returning an error,
  // so that no kernel of a failed call keeps running on the caller's buffers)
  void drain() {
    for (auto& x : streams)
      if (x) (void)hipStreamSynchronize(x);
  }
  int reserve(size_t bytes) {
    last_status = nullptr;  // every call that takes the workspace may overwrite it
    if (bytes <= ws_bytes) return RANDUTV_OK;
    if (ws) {
      RUTV_TRY(hipDeviceSynchronize());
      (void)hipFree(ws);
      ws = nullptr;
      ws_bytes = 0;
    }
    hipError_t e = hipMalloc((void**)&ws, bytes);
    if (e != hipSuccess) {
      ws = nullptr;
      (void)hipGetLastError();
      return RANDUTV_ERR_NOMEM;
    }
    ws_bytes = bytes;
    return RANDUTV_OK;
  }
};

constexpr int kMaxDevices = 64;
static Context g_ctx[kMaxDevices];

// the current device's library state
static Context& ctx() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) dev = 0;
  return g_ctx[dev];
}

// carve aligned regions out of one allocation
struct Carver {
  size_t off = 0;
  char* base = nullptr;
  template <class T>
  T* take(i64 count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (size_t)std::max<i64>(count, 1);
    return p;
  }
};

// scratch owned by one stream
struct StreamWS {
  double* splitk = nullptr;
  i64 splitk_elems = 0;
  double* Gram = nullptr;  // b x b
  double* Tf = nullptr;    // b x b block factor (stream P)
  double* X = nullptr;     // max(m, n) x b
  PanelWork pw;
};

// the column-block panel takes the CU-sharing kernel variant while the
// trailing update beside it is at least this wide (below that the GEMMs leave
// CUs free and the faster exclusive variant gets them)
#ifndef RUTV_SHARED_PANEL_MIN_COLS
#define RUTV_SHARED_PANEL_MIN_COLS 6000
#endif
#ifndef RUTV_SVD_GROUP
#define RUTV_SVD_GROUP 8
#endif
constexpr int kSvdGroup = RUTV_SVD_GROUP;  // SVDs per batched launch
// the panel kernel's row limit (its workgroups times their slab)
constexpr i64 kMaxRows = 32768;

struct FactorWS {
  StreamWS sw[NSTREAMS];
  double *G, *Y, *Zp, *tauV, *tauU, *X3;
  // reflectors W and Z = W Tf^T (Tf their block factor), one set per step in
  // turn (kWyBuf sets)
  double *WV[kWyBuf], *ZV[kWyBuf], *WU[kWyBuf], *ZU[kWyBuf];
  double *Rall, *dall, *Usall, *Vsall, *jwork;
  int* status;  // [0] finite flag, [1] panel sync error, [2 + 3i ..] sweeps, converged, sync error
};

static i64 splitk_need(i64 m, i64 n, i64 b, int q, bool wantU, bool wantV) {
  i64 need = 0;
  auto upd = [&](i64 M, i64 N, i64 K) { need = std::max(need, dgemm_work_elems(M, N, K)); };
  for (i64 s = 0; s < n; s += b) {
    const i64 bi = std::min(b, n - s), mi = m - s, ni = n - s;
    upd(ni, bi, mi);
    if (q > 0) upd(mi, bi, ni);
    upd(bi, bi, ni);
    upd(ni, bi, bi);
    upd(m, bi, ni);
    upd(m, bi, bi);
    upd(m, ni - bi, bi);
    if (s > 0) {  // rows s.. on stream T, rows ..s on stream UV
      upd(m - s, bi, ni);
      upd(m - s, bi, bi);
      upd(m - s, ni - bi, bi);
      upd(s, bi, ni);
      upd(s, ni, bi);
    }
    if (wantV) {
      upd(n, bi, ni);
      upd(n, ni, bi);
      upd(n, bi, bi);
    }
    upd(bi, bi, mi);
    upd(mi, bi, bi);
    if (ni > bi) {
      upd(bi, ni - bi, mi);
      upd(mi, ni - bi, bi);
      upd(bi, ni - bi, bi);
    }
    if (wantU) {
      upd(m, bi, mi);
      upd(m, mi, bi);
      upd(m, bi, bi);
    }
    if (s > 0) upd(s, bi, bi);
  }
  return need;
}

// sk_cap >= 0 bounds each stream's split-K partial space (in doubles); the
// GEMMs then take as many K splits as fit (none when it is 0)
static size_t layout(Carver& c, FactorWS& w, i64 m, i64 n, i64 b, int q, bool wantU, bool wantV,
                     i64 sk_cap = -1) {
  const i64 nsteps = cdiv(n, b);
  const i64 mx = std::max(m, n);
  i64 sk = splitk_need(m, n, b, q, wantU, wantV);
  if (sk_cap >= 0) sk = std::min(sk, sk_cap);
  for (int t = 0; t < NSTREAMS; ++t) {
    StreamWS& x = w.sw[t];
    x.splitk_elems = sk;
    x.splitk = c.take<double>(sk);
    x.Gram = c.take<double>(b * b);
    x.X = c.take<double>(mx * b);
    x.Tf = c.take<double>(b * b);
    x.pw.xch = c.take<unsigned long long>(panel_work_elems(mx));
  }
  w.G = c.take<double>(m * b);
  w.Y = c.take<double>(n * b);
  w.Zp = c.take<double>(m * b);
  w.tauV = c.take<double>(b);
  w.tauU = c.take<double>(b);
  w.X3 = c.take<double>(b * n);
  for (int t = 0; t < kWyBuf; ++t) {
    w.WV[t] = c.take<double>(n * b);
    w.ZV[t] = c.take<double>(n * b);
    w.WU[t] = c.take<double>(m * b);
    w.ZU[t] = c.take<double>(m * b);
  }
  w.Rall = c.take<double>(nsteps * b * b);
  w.dall = c.take<double>(nsteps * b);
  w.Usall = c.take<double>(nsteps * b * b);
  w.Vsall = c.take<double>(nsteps * b * b);
  w.jwork = c.take<double>(kSvdGroup * jacobi_work_elems(b));
  w.status = c.take<int>(2 + 3 * nsteps);
  return c.off;
}

static int gemm(hipStream_t st, const StreamWS& x, bool ta, bool tb, i64 M, i64 N, i64 K,
                double alpha, const double* A, i64 lda, const double* B, i64 ldb, double beta,
                double* C, i64 ldc, int prec = PREC_F64) {
  return dgemm(st, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, x.splitk, x.splitk_elems,
               prec);
}

// Z (rows x k, ld rows) := W Tf^T, Tf the block factor of the reflectors W
// (rows x k, unit lower trapezoidal, ld rows), formed from the Gram matrix
// W^T W: H_1 ... H_k = I - W Tf W^T = I - W Z^T, and its transpose is
// I - Z W^T.  Every later use of the block reflector needs Z only.
static int t_factor(hipStream_t st, const StreamWS& x, i64 rows, i64 k, const double* W,
                    const double* tau, double* Z) {
  RUTV_CHECK(gemm(st, x, true, false, k, k, rows, 1.0, W, rows, W, rows, 0.0, x.Gram, k));
  RUTV_CHECK(larft_from_gram(st, k, x.Gram, k, tau, x.Tf, k));
  RUTV_CHECK(gemm(st, x, false, true, rows, k, k, 1.0, W, rows, x.Tf, k, 0.0, Z, rows));
  return RANDUTV_OK;
}

// C(rows x cols, ld ldc) <- C (I - W Tf W^T) = C - (C W) Z^T, W and Z: cols x k
// (ld cols)
static int right_apply(hipStream_t st, const StreamWS& x, i64 rows, i64 cols, i64 k, double* C,
                       i64 ldc, const double* W, const double* Z, int prec = PREC_F64) {
  RUTV_CHECK(gemm(st, x, false, false, rows, k, cols, 1.0, C, ldc, W, cols, 0.0, x.X, rows, prec));
  RUTV_CHECK(gemm(st, x, false, true, rows, cols, k, -1.0, x.X, rows, Z, cols, 1.0, C, ldc, prec));
  return RANDUTV_OK;
}

// C(rows x k, ld ldc) <- C S (S: k x k, ld k), through the stream's X buffer
static int right_mul_small(hipStream_t st, const StreamWS& x, i64 rows, i64 k, double* C, i64 ldc,
                           const double* S) {
  if (rows <= 0) return RANDUTV_OK;
  RUTV_CHECK(gemm(st, x, false, false, rows, k, k, 1.0, C, ldc, S, k, 0.0, x.X, rows));
  RUTV_CHECK(copy_matrix(st, rows, k, x.X, rows, C, ldc));
  return RANDUTV_OK;
}

// sketch_prec: arithmetic of the sketch and power-iteration products
// Y = (B^T B)^q B^T G (a GemmPrec; FP64 storage either way); every transform
// of T, U and V stays FP64
// Everything a factorization call needs (validated by the entry points).
struct FactorCfg {
  i64 m = 0, n = 0;
  const double* A = nullptr;
  i64 lda = 0, b = 0;
  int q = 0;
  uint64_t seed = 0;
  double *U = nullptr, *T = nullptr, *V = nullptr;
  i64 ldu = 0, ldt = 0, ldv = 0;
  bool has_caller = false;       // order the call on the caller's stream
  hipStream_t caller = nullptr;  // that stream (null: the null stream)
  const double* G = nullptr;     // the caller's sketches (concatenated), or null
  bool g_host = false;           // G is host memory
  bool finite_check = true;
  int sketch_prec = PREC_F64;    // sketch and power-iteration products
  int update_prec = PREC_F64;    // compact-WY updates of T, U and V
  int max_sweeps = 0;            // Jacobi sweep cap (0: default)
  unsigned spin_limit = 0;       // bounded waits (0: default)
  size_t max_ws = 0;             // workspace cap (0: none)
  bool noalloc = false;          // carve the workspace out of the device's `scratch`
  bool async = false;            // return once enqueued (status: randutv_factor_status)
};

static int factor_run(const FactorCfg& c, Context& cx);

// the outcome of the last factorization from its device status words (after
// its work has finished): [0] non-finite input, [1] panel sync error, then
// per step sweeps, converged, Jacobi sync error
static int read_status(Context& cx, bool check_finite) {
  if (!cx.last_status) return RANDUTV_OK;
  const i64 nsteps = cx.last_nsteps;
  std::vector<int> stat(2 + 3 * nsteps);
  RUTV_TRY(hipMemcpy(stat.data(), cx.last_status, sizeof(int) * stat.size(), hipMemcpyDeviceToHost));
  cx.sweeps.assign(nsteps, 0);
  for (i64 i = 0; i < nsteps; ++i) cx.sweeps[i] = stat[2 + 3 * i];
  if (check_finite && stat[0]) return RANDUTV_ERR_NONFINITE;
  if (stat[1]) return RANDUTV_ERR_SYNC;
  for (i64 i = 0; i < nsteps; ++i)
    if (stat[4 + 3 * i]) return RANDUTV_ERR_SYNC;
  for (i64 i = 0; i < nsteps; ++i)
    if (!stat[3 + 3 * i]) return RANDUTV_ERR_NOCONV;
  return RANDUTV_OK;
}

static int factor_impl(const FactorCfg& c) {
  Context& cx = ctx();
  RUTV_CHECK(cx.init());
  const int rc = factor_run(c, cx);
  if (rc != RANDUTV_OK) cx.drain();
  return rc;
}

static int factor_run(const FactorCfg& c, Context& cx) {
  hipStream_t sT = cx.streams[ST_T], sP = cx.streams[ST_P], sUV = cx.streams[ST_UV],
              sS = cx.streams[ST_S];
  const i64 m = c.m, n = c.n, lda = c.lda, ldt = c.ldt, ldu = c.ldu, ldv = c.ldv;
  const double* A = c.A;
  double *U = c.U, *T = c.T, *V = c.V;
  const int q = c.q;
  const uint64_t seed = c.seed;
  const int sketch_prec = c.sketch_prec, update_prec = c.update_prec;
  const bool wantU = U != nullptr, wantV = V != nullptr;
  i64 b = c.b;
  if (b > n) b = n;
  const i64 nsteps = cdiv(n, b);
  const i64 b_last = n - (nsteps - 1) * b;

  FactorWS w{};
  Carver real;
  i64 sk_cap = -1;
  if (c.noalloc) {
    // the fixed scratch: everything but the split-K partials must fit; the
    // partials get what is left (fewer K splits, same arithmetic per split)
    constexpr size_t cap = RANDUTV_NOALLOC_SCRATCH_BYTES;
    Carver p0, pf;
    const size_t fixed = layout(p0, w, m, n, b, q, wantU, wantV, 0);
    if (fixed > cap) return RANDUTV_ERR_SCRATCH;
    if (layout(pf, w, m, n, b, q, wantU, wantV) > cap)
      sk_cap = std::max<i64>(0, (i64)((cap - fixed) / (NSTREAMS * sizeof(double))) - 64);
    Carver pc;
    if (layout(pc, w, m, n, b, q, wantU, wantV, sk_cap) > cap) return RANDUTV_ERR_SCRATCH;
    if (!cx.scratch_ptr) return RANDUTV_ERR_HIP;
    real.base = cx.scratch_ptr;
  } else {
    Carver probe;
    const size_t bytes = layout(probe, w, m, n, b, q, wantU, wantV);
    if (c.max_ws && bytes > c.max_ws) return RANDUTV_ERR_NOMEM;
    RUTV_CHECK(cx.reserve(bytes));
    real.base = cx.ws;
  }
  layout(real, w, m, n, b, q, wantU, wantV, sk_cap);
  for (auto& x : w.sw) {
    x.pw.err = &w.status[1];
    x.pw.spin_limit = c.spin_limit;
  }
  const StreamWS &xT = w.sw[ST_T], &xP = w.sw[ST_P], &xUV = w.sw[ST_UV];
  // the caller's sketch of step i: offset of G(i) in the concatenation
  auto g_offset = [&](i64 i) {
    i64 off = 0;
    for (i64 j = 0; j < i; ++j) off += (m - j * b) * std::min(b, n - j * b);
    return off;
  };

  cx.timer.start_call();
  const bool timed = cx.timing && !c.async;  // an asynchronous call is not timed
  set_launch_timer(timed ? &cx.timer : nullptr);
  struct Reset {
    ~Reset() { set_launch_timer(nullptr); }
  } reset_timer;
  auto ev = [&](int kind, i64 i) { return cx.ev[kind][i % kEvRing]; };

  // ---- the caller's stream: the library's streams start after the work
  // enqueued on it so far
  if (c.has_caller) {
    RUTV_TRY(hipEventRecord(cx.ev_misc[3], c.caller));
    for (auto x : cx.streams) RUTV_TRY(hipStreamWaitEvent(x, cx.ev_misc[3], 0));
  }
  if (timed) cx.timer.mark(sT);
  // ---- prologue (stream T): status, T := A with a finiteness check
  RUTV_CHECK(fill_zero_u32(sT, reinterpret_cast<unsigned*>(w.status), 2 + 3 * nsteps));
  if (T != A)
    RUTV_CHECK(copy_check(sT, m, n, A, lda, T, ldt, c.finite_check ? &w.status[0] : nullptr));
  else if (c.finite_check)
    RUTV_CHECK(check_finite(sT, m, n, T, ldt, &w.status[0]));
  if (c.finite_check && !c.async) {
    int flag = 0;
    RUTV_TRY(hipMemcpyAsync(&flag, &w.status[0], sizeof(int), hipMemcpyDeviceToHost, sT));
    RUTV_TRY(hipStreamSynchronize(sT));
    if (flag) return RANDUTV_ERR_NONFINITE;
  }
  if (wantU) RUTV_CHECK(set_identity(sUV, m, U, ldu));
  if (wantV) RUTV_CHECK(set_identity(sUV, n, V, ldv));

  i64 g0 = 0;
  // stream S: once step j's U/V update is enqueued, the SVD group that ends
  // at step j (every kSvdGroup steps, and the last), then its right factors
  auto svd_group = [&](i64 j) -> int {
    const i64 sj = j * b, bj = std::min(b, n - sj);
    const bool last = sj + bj >= n;
    if ((j + 1 - g0) != kSvdGroup && !last) return RANDUTV_OK;
    const int cnt = (int)(j + 1 - g0);
    RUTV_TRY(hipStreamWaitEvent(sS, ev(EV_U, j), 0));
    // the rows above each block of the group have had their last right
    // transform (stream UV) before V_S is applied to them
    if (kTopOnUV && j >= 1) RUTV_TRY(hipStreamWaitEvent(sS, ev(EV_TOP, j), 0));
    RUTV_CHECK(jacobi_svd_batched(sS, cnt, b, last ? b_last : b, w.Rall + g0 * b * b, b, b * b,
                                  w.dall + g0 * b, b, w.Usall + g0 * b * b, w.Vsall + g0 * b * b,
                                  b * b, w.jwork, &w.status[2 + 3 * g0], c.max_sweeps,
                                  c.spin_limit));
    // the right factors of each block (its columns of T, V and U).  After the
    // last group every stream is free: the blocks are spread over all four
    // (they touch disjoint columns), each stream with its own buffers
    if (last) RUTV_TRY(hipEventRecord(cx.ev_misc[0], sS));
    for (i64 t = g0; t <= j; ++t) {
      const int sx = last ? (int)((t - g0 + ST_S) % NSTREAMS) : ST_S;
      hipStream_t sa = cx.streams[sx];
      const StreamWS& xa = w.sw[sx];
      if (last && t - g0 < NSTREAMS && sx != ST_S)
        RUTV_TRY(hipStreamWaitEvent(sa, cx.ev_misc[0], 0));
      const i64 st_ = t * b, bt = std::min(b, n - st_);
      const double* d = w.dall + t * b;
      const double* Vs = w.Vsall + t * b * b;
      const double* Us = w.Usall + t * b * b;
      RUTV_CHECK(set_diag_block(sa, bt, d, T + st_ + st_ * ldt, ldt));
      RUTV_CHECK(right_mul_small(sa, xa, st_, bt, T + st_ * ldt, ldt, Vs));
      RUTV_TRY(hipStreamWaitEvent(sa, ev(EV_UV, t), 0));
      if (wantV) RUTV_CHECK(right_mul_small(sa, xa, n, bt, V + st_ * ldv, ldv, Vs));
      if (wantU) RUTV_CHECK(right_mul_small(sa, xa, m, bt, U + st_ * ldu, ldu, Us));
    }
    g0 = j + 1;
    return RANDUTV_OK;
  };
  // stream UV: the V and U updates of step j.  They are enqueued one step
  // late, behind the event that marks the end of the next step's power
  // iteration, so that they fill the chip during the next QR of the sketch (a
  // latency-bound kernel on few CUs) instead of competing with the power
  // iteration.
  auto uv_updates = [&](i64 j, bool wait_pre) -> int {
    const i64 sj = j * b, bj = std::min(b, n - sj), mj = m - sj, nj = n - sj;
    const int bf = (int)(j % kWyBuf);
    if (wait_pre) RUTV_TRY(hipStreamWaitEvent(sUV, ev(EV_PRE, j + 1), 0));
    RUTV_TRY(hipStreamWaitEvent(sUV, ev(EV_V, j), 0));
    if (wantV)
      RUTV_CHECK(right_apply(sUV, xUV, n, nj, bj, V + sj * ldv, ldv, w.WV[bf], w.ZV[bf], update_prec));
    RUTV_TRY(hipStreamWaitEvent(sUV, ev(EV_U, j), 0));
    if (wantU)
      RUTV_CHECK(right_apply(sUV, xUV, m, mj, bj, U + sj * ldu, ldu, w.WU[bf], w.ZU[bf], update_prec));
    RUTV_TRY(hipEventRecord(ev(EV_UV, j), sUV));
    return svd_group(j);
  };

  i64 s = 0;
  for (i64 i = 0; s < n; ++i) {
    const i64 bi = std::min(b, n - s), e = s + bi, mi = m - s, ni = n - s;
    const int buf = (int)(i % kWyBuf);
    double* Bm = T + s + s * ldt;
    // ---- stream T: sketch, power iteration, QR(Y), compact WY of V^
    if (i >= kWyBuf) RUTV_TRY(hipStreamWaitEvent(sT, ev(EV_UV, i - kWyBuf), 0));  // WV[buf] free
    const double* Gi = w.G;
    if (!c.G) {
      RUTV_CHECK(sketch(sT, seed, (uint64_t)i, mi, bi, w.G, mi));
    } else if (c.g_host) {
      RUTV_TRY(hipMemcpyAsync(w.G, c.G + g_offset(i), sizeof(double) * mi * bi,
                              hipMemcpyHostToDevice, sT));
    } else {
      Gi = c.G + g_offset(i);
    }
    RUTV_CHECK(gemm(sT, xT, true, false, ni, bi, mi, 1.0, Bm, ldt, Gi, mi, 0.0, w.Y, ni, sketch_prec));
    for (int it = 0; it < q; ++it) {
      RUTV_CHECK(gemm(sT, xT, false, false, mi, bi, ni, 1.0, Bm, ldt, w.Y, ni, 0.0, w.Zp, mi, sketch_prec));
      RUTV_CHECK(gemm(sT, xT, true, false, ni, bi, mi, 1.0, Bm, ldt, w.Zp, mi, 0.0, w.Y, ni, sketch_prec));
    }
    RUTV_TRY(hipEventRecord(ev(EV_PRE, i), sT));
    if (i >= 1) RUTV_CHECK(uv_updates(i - 1, true));
    RUTV_CHECK(panel_qr(sT, ni, bi, w.Y, ni, w.tauV, xT.pw));
    RUTV_CHECK(extract_reflectors(sT, ni, bi, w.Y, ni, w.WV[buf], ni, nullptr, 0, false));
    RUTV_TRY(hipEventRecord(ev(EV_WV, i), sT));
    // stream P: block factor of V^ while stream T forms X = T W
    RUTV_TRY(hipStreamWaitEvent(sP, ev(EV_WV, i), 0));
    if (i >= kWyBuf) RUTV_TRY(hipStreamWaitEvent(sP, ev(EV_UV, i - kWyBuf), 0));  // ZV/WU/ZU[buf] free
    RUTV_CHECK(t_factor(sP, xP, ni, bi, w.WV[buf], w.tauV, w.ZV[buf]));
    RUTV_TRY(hipEventRecord(ev(EV_V, i), sP));
    // right transform, T <- T - (T W) Z^T.  Stream T transforms rows s..m-1
    // (the trailing matrix the next steps sketch): first the current column
    // block (it feeds the panel QR on stream P), then the rest.  Rows 0..s-1
    // are read by no later step, only transformed again from the right: their
    // transform runs on stream UV, after the left transform of step i - 1
    // (which last wrote block row i - 1 there)
    const i64 r0 = kTopOnUV ? s : 0, mr = m - r0;
    RUTV_CHECK(gemm(sT, xT, false, false, mr, bi, ni, 1.0, T + r0 + s * ldt, ldt, w.WV[buf], ni, 0.0,
                    xT.X, m, update_prec));
    RUTV_TRY(hipStreamWaitEvent(sT, ev(EV_V, i), 0));
    RUTV_CHECK(gemm(sT, xT, false, true, mr, bi, bi, -1.0, xT.X, m, w.ZV[buf], ni, 1.0, T + r0 + s * ldt,
                    ldt, update_prec));
    RUTV_TRY(hipEventRecord(ev(EV_COLS, i), sT));
    if (e < n)
      RUTV_CHECK(gemm(sT, xT, false, true, mr, ni - bi, bi, -1.0, xT.X, m, w.ZV[buf] + bi, ni, 1.0,
                      T + r0 + e * ldt, ldt, update_prec));
    if (kTopOnUV && s > 0) {
      RUTV_TRY(hipStreamWaitEvent(sUV, ev(EV_V, i), 0));
      RUTV_TRY(hipStreamWaitEvent(sUV, ev(EV_LEFT, i - 1), 0));
      RUTV_CHECK(right_apply(sUV, xUV, s, ni, bi, T + s * ldt, ldt, w.WV[buf], w.ZV[buf], update_prec));
      RUTV_TRY(hipEventRecord(ev(EV_TOP, i), sUV));
    }
    // ---- stream P: panel QR of the column block, its reflectors, then their
    // block factor while stream T forms W^T C
    RUTV_TRY(hipStreamWaitEvent(sP, ev(EV_COLS, i), 0));
    // (the trailing update on stream T and the U/V updates keep every CU busy
    // meanwhile: while that update is wide, this panel takes the variant that
    // shares CUs with them)
    RUTV_CHECK(panel_qr(sP, mi, bi, Bm, ldt, w.tauU, xP.pw, ni - bi >= RUTV_SHARED_PANEL_MIN_COLS));
    RUTV_CHECK(extract_reflectors(sP, mi, bi, Bm, ldt, w.WU[buf], mi, w.Rall + i * b * b, b, true));
    RUTV_TRY(hipEventRecord(ev(EV_WU, i), sP));
    RUTV_CHECK(t_factor(sP, xP, mi, bi, w.WU[buf], w.tauU, w.ZU[buf]));
    RUTV_TRY(hipEventRecord(ev(EV_U, i), sP));
    // ---- stream T: left transform of the remaining columns,
    // C <- C - Z (W^T C)
    RUTV_TRY(hipStreamWaitEvent(sT, ev(EV_WU, i), 0));
    if (e < n) {
      double* C = T + s + e * ldt;
      RUTV_CHECK(gemm(sT, xT, true, false, bi, ni - bi, mi, 1.0, w.WU[buf], mi, C, ldt, 0.0, w.X3, bi,
                      update_prec));
      RUTV_TRY(hipStreamWaitEvent(sT, ev(EV_U, i), 0));
      RUTV_CHECK(gemm(sT, xT, false, false, mi, ni - bi, bi, -1.0, w.ZU[buf], mi, w.X3, bi, 1.0, C, ldt,
                      update_prec));
    } else {
      RUTV_TRY(hipStreamWaitEvent(sT, ev(EV_U, i), 0));
    }
    RUTV_TRY(hipEventRecord(ev(EV_LEFT, i), sT));
    s = e;
  }
  RUTV_CHECK(uv_updates(nsteps - 1, false));
  // ---- join all streams (the right factors of the last blocks act on
  // columns that every block row's left factor touches), then the deferred
  // left factors T(s:e, e:n) <- U_S^T T(s:e, e:n), block rows spread over the
  // four streams (disjoint rows), then join on stream T
  auto join = [&](int k) -> int {
    for (int x = 0; x < NSTREAMS; ++x) RUTV_TRY(hipEventRecord(cx.ev_tail[k][x], cx.streams[x]));
    return RANDUTV_OK;
  };
  RUTV_CHECK(join(1));
  for (int x = 0; x < NSTREAMS; ++x)
    for (int y = 0; y < NSTREAMS; ++y)
      if (x != y) RUTV_TRY(hipStreamWaitEvent(cx.streams[x], cx.ev_tail[1][y], 0));
  s = 0;
  for (i64 i = 0; s < n; ++i) {
    const i64 bi = std::min(b, n - s), e = s + bi;
    if (e < n) {
      const int sx = (int)(i % NSTREAMS);
      const double* Us = w.Usall + i * b * b;
      double* C = T + s + e * ldt;
      double* X = w.sw[sx].X;
      RUTV_CHECK(gemm(cx.streams[sx], w.sw[sx], true, false, bi, n - e, bi, 1.0, Us, bi, C, ldt, 0.0, X, bi));
      RUTV_CHECK(copy_matrix(cx.streams[sx], bi, n - e, X, bi, C, ldt));
    }
    s = e;
  }
  RUTV_CHECK(join(0));
  for (int x = 0; x < NSTREAMS; ++x)
    if (x != ST_T) RUTV_TRY(hipStreamWaitEvent(sT, cx.ev_tail[0][x], 0));
  if (c.has_caller) {
    RUTV_TRY(hipEventRecord(cx.ev_misc[3], sT));
    RUTV_TRY(hipStreamWaitEvent(c.caller, cx.ev_misc[3], 0));
  }
  cx.last_status = w.status;
  cx.last_nsteps = nsteps;
  cx.last_finite_check = c.finite_check;
  if (c.async) return RANDUTV_OK;  // randutv_factor_status reads the outcome later
  RUTV_TRY(hipStreamSynchronize(sT));
  if (cx.timing) cx.timer.collect();
  return read_status(cx, false);
}

// host-side allocation failures (std::vector and the like) must not cross the
// C ABI as C++ exceptions
template <class F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return RANDUTV_ERR_NOMEM;
  } catch (...) {
    return RANDUTV_ERR_HIP;
  }
}

// an entry point's device work: on any failure after work was enqueued, wait
// for the library's streams before returning, so that no kernel of the call
// is left running on the caller's buffers
template <class F>
static int drained(Context& cx, F&& f) {
  int rc;
  try {
    rc = f();
  } catch (const std::bad_alloc&) {
    rc = RANDUTV_ERR_NOMEM;
  } catch (...) {
    rc = RANDUTV_ERR_HIP;
  }
  if (rc != RANDUTV_OK) cx.drain();
  return rc;
}

}  // namespace rutv

using namespace rutv;

extern "C" {

static int prec_of_bits(int32_t bits, int& prec) {
  switch (bits) {
    case 0:
    case RANDUTV_SKETCH_FP64: prec = PREC_F64; return 0;
    case RANDUTV_SKETCH_FP32: prec = PREC_F32; return 0;
    case RANDUTV_SKETCH_BF16: prec = PREC_BF16; return 0;
    case RANDUTV_SKETCH_BF16X3: prec = PREC_BF16X3; return 0;
    default: return -1;
  }
}

// checks shared by both factorization entry points; returns 0, a negative
// argument code, or RANDUTV_ERR_TOO_LARGE
static int check_factor(const FactorCfg& c) {
  if (c.m < 0) return -1;
  if (c.n < 0 || c.n > c.m) return -2;
  if (c.m == 0 || c.n == 0) return RANDUTV_OK;
  if (!c.A) return -3;
  if (c.lda < std::max<int64_t>(1, c.m)) return -4;
  if (c.b < 1) return -5;
  if (c.q < 0) return -6;
  if (c.U && c.ldu < c.m) return -8;
  if (!c.T || c.ldt < c.m) return -9;
  if (c.T == c.A && c.lda != c.ldt) return -9;
  if (c.V && c.ldv < c.n) return -10;
  if (c.U && (c.U == c.T || c.U == c.V)) return -8;
  if (c.V && c.V == c.T) return -10;
  if (std::min(c.b, c.n) > kPanelMaxCols) return RANDUTV_ERR_TOO_LARGE;
  if (c.m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return RANDUTV_OK;
}

static int factor_entry(const FactorCfg& c) {
  const int rc = check_factor(c);
  if (rc != RANDUTV_OK || c.m == 0 || c.n == 0) return rc;
  std::lock_guard<std::mutex> lk(g_mu);
  return guarded([&] { return factor_impl(c); });
}

int randutv_factor(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                   uint64_t seed, double* U, double* T, double* V) {
  FactorCfg c;
  c.m = m, c.n = n, c.A = A, c.lda = lda, c.b = b, c.q = q, c.seed = seed;
  c.U = U, c.T = T, c.V = V, c.ldu = m, c.ldt = m, c.ldv = n;
  return factor_entry(c);
}

static int cfg_from_args(const randutv_args* a, FactorCfg& c) {
  c.m = a->m, c.n = a->n, c.A = a->A, c.lda = a->lda, c.b = a->b, c.q = a->q, c.seed = a->seed;
  c.U = a->U, c.T = a->T, c.V = a->V;
  c.ldu = a->ldu ? a->ldu : a->m;
  c.ldt = a->ldt ? a->ldt : a->m;
  c.ldv = a->ldv ? a->ldv : a->n;
  constexpr uint32_t kKnown =
      RANDUTV_FLAG_G_HOST | RANDUTV_FLAG_NO_FINITE_CHECK | RANDUTV_FLAG_STREAM | RANDUTV_FLAG_ASYNC;
  if (a->flags & ~kKnown) return -13;
  if ((a->flags & RANDUTV_FLAG_ASYNC) && !(a->flags & RANDUTV_FLAG_STREAM)) return -13;
  if ((a->flags & RANDUTV_FLAG_G_HOST) && !a->G) return -13;
  if (prec_of_bits(a->sketch_bits, c.sketch_prec)) return -11;
  if (prec_of_bits(a->update_bits, c.update_prec)) return -12;
  if (a->jacobi_max_sweeps < 0 || a->jacobi_max_sweeps > 1000) return -14;
  c.has_caller = (a->flags & RANDUTV_FLAG_STREAM) != 0;
  c.caller = c.has_caller ? reinterpret_cast<hipStream_t>(a->stream) : nullptr;
  c.G = a->G;
  c.g_host = (a->flags & RANDUTV_FLAG_G_HOST) != 0;
  c.finite_check = (a->flags & RANDUTV_FLAG_NO_FINITE_CHECK) == 0;
  c.async = (a->flags & RANDUTV_FLAG_ASYNC) != 0;
  c.max_sweeps = a->jacobi_max_sweeps;
  c.spin_limit = a->spin_limit;
  c.max_ws = a->max_workspace_bytes > 0 ? (size_t)a->max_workspace_bytes : 0;
  return RANDUTV_OK;
}

int randutv_factor_ex(const randutv_args* a) {
  if (!a || a->struct_size < (int64_t)sizeof(randutv_args)) return -15;
  FactorCfg c;
  const int rc = cfg_from_args(a, c);
  if (rc != RANDUTV_OK) return rc;
  return factor_entry(c);
}

int randutv_factor_status(void) {
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return guarded([&]() -> int {
    if (!cx.st) return RANDUTV_OK;
    RUTV_TRY(hipDeviceSynchronize());
    return read_status(cx, cx.last_finite_check);
  });
}

int randutv_factor_noalloc(const randutv_args* a) {
  if (!a || a->struct_size < (int64_t)sizeof(randutv_args)) return -15;
  if (a->max_workspace_bytes != 0) return -15;
  FactorCfg c;
  const int rc = cfg_from_args(a, c);
  if (rc != RANDUTV_OK) return rc;
  c.noalloc = true;
  return factor_entry(c);
}

int randutv_factor_ooc(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                       uint64_t seed, double* U, int64_t ldu, double* T, int64_t ldt, double* V,
                       int64_t ldv, int64_t hbm_budget_bytes, int32_t mode,
                       randutv_ooc_stats* stats) {
  if (m < 0) return -1;
  if (n < 0 || n > m) return -2;
  if (m == 0 || n == 0) return RANDUTV_OK;
  if (!A) return -3;
  if (lda < m) return -4;
  if (b < 1) return -5;
  if (q < 0) return -6;
  if (U && (ldu < m || U == T || U == V)) return -8;
  if (!T || ldt < m || (T == A && lda != ldt)) return -9;
  if (V && (ldv < n || V == T)) return -10;
  const i64 bb = std::min<i64>(b, n);
  if (hbm_budget_bytes < 0 || (uint64_t)hbm_budget_bytes / (8ull * (uint64_t)m * (uint64_t)bb) < 2)
    return -11;
  if (mode < RANDUTV_OOC_TRADITIONAL || mode > RANDUTV_OOC_OVERLAPPED) return -12;
  if (bb > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  OocCfg c;
  c.m = m, c.n = n, c.b = b, c.q = q, c.seed = seed, c.A = A, c.lda = lda;
  c.U = U, c.T = T, c.V = V, c.ldu = ldu, c.ldt = ldt, c.ldv = ldv;
  c.budget = (size_t)hbm_budget_bytes;
  c.mode = mode;
  std::lock_guard<std::mutex> lk(g_mu);
  Context& cx = ctx();
  return drained(cx, [&]() -> int {
    RUTV_CHECK(cx.init());
    set_launch_timer(nullptr);
    return ooc_factor(c, cx.streams[ST_T], cx.streams[ST_P], cx.streams[ST_UV], stats);
  });
}

int randutv_truncate(int64_t m, int64_t n, int64_t k, const double* U, const double* T,
                     const double* V, double* Ak) {
  if (m < 0) return -1;
  if (n < 0 || n > m) return -2;
  if (k < 0 || k > n) return -3;
  if (m == 0 || n == 0) return RANDUTV_OK;
  if (!U) return -4;
  if (!T) return -5;
  if (!V) return -6;
  if (!Ak) return -7;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return drained(cx, [&]() -> int {
  RUTV_CHECK(cx.init());
  hipStream_t st = cx.st;
  if (k == 0) {
    RUTV_TRY(hipMemsetAsync(Ak, 0, sizeof(double) * m * n, st));
    RUTV_TRY(hipStreamSynchronize(st));
    return RANDUTV_OK;
  }
  // M1 = T(0:k, :) V^T  (k x n), then Ak = U(:, 0:k) M1
  const i64 sk1 = dgemm_work_elems(k, n, n), sk2 = dgemm_work_elems(m, n, k);
  const i64 sk = std::max(sk1, sk2);
  Carver c;
  c.take<double>(k * n);
  c.take<double>(sk);
  RUTV_CHECK(cx.reserve(c.off));
  Carver r;
  r.base = cx.ws;
  double* M1 = r.take<double>(k * n);
  double* wk = r.take<double>(sk);
  set_launch_timer(nullptr);
  RUTV_CHECK(dgemm(st, false, true, k, n, n, 1.0, T, m, V, n, 0.0, M1, k, wk, sk));
  RUTV_CHECK(dgemm(st, false, false, m, n, k, 1.0, U, m, M1, k, 0.0, Ak, m, wk, sk));
  RUTV_TRY(hipStreamSynchronize(st));
  return RANDUTV_OK;
  });
}

// HQRRP (Section 2): A P = Q R by blocks of b columns.  Step i (s = i b):
// Y = G^T A(s:m, s:n) with G the (m - s) x b_i sketch of randUTV's step i;
// b_i steps of CPQR on Y choose the pivots; the chosen columns are exchanged
// to the front (all m rows); Householder QR of the b_i-column panel; the
// remaining columns of rows s..m-1 get Q22^T = H^T (compact WY).
// The same step loop without the sketch, the pivots and the exchanges
// (pivot == false) is the unpivoted blocked Householder QR (LAPACK dgeqrf's
// operation), the baseline HQRRP is measured against.
static int blocked_qr(int64_t m, int64_t n, double* A, int64_t lda, int64_t b, uint64_t seed,
                      double* tau, int64_t* jpvt, bool pivot) {
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return drained(cx, [&]() -> int {
  RUTV_CHECK(cx.init());
  hipStream_t st = cx.st;
  i64 sk = 0;
  for (i64 s0 = 0; s0 < n; s0 += b) {
    const i64 bi = std::min(b, n - s0), mi = m - s0, ni = n - s0;
    for (auto s3 : {std::array<i64, 3>{bi, ni, mi}, {bi, bi, mi}, {mi, bi, bi}, {bi, ni - bi, mi},
                    {mi, ni - bi, bi}})
      if (s3[1] > 0) sk = std::max(sk, dgemm_work_elems(s3[0], s3[1], s3[2]));
  }
  StreamWS x;
  double *G, *Y, *W, *Z, *X3;
  int *J, *status;
  CpqrWork cw;
  ExchangeWork ew;
  unsigned long long* xch;
  auto lay = [&](Carver& c) {
    x.splitk_elems = sk;
    x.splitk = c.take<double>(sk);
    x.Gram = c.take<double>(b * b);
    x.Tf = c.take<double>(b * b);
    G = c.take<double>(m * b);
    Y = c.take<double>(b * n);
    W = c.take<double>(m * b);
    Z = c.take<double>(m * b);
    X3 = c.take<double>(b * n);
    J = c.take<int>(b);
    cw.sval = c.take<double>(2 * 256);
    cw.sidx = c.take<int>(2 * 256);
    cw.scol = c.take<double>(2 * 256 * kPanelMaxCols);
    cw.counter = c.take<unsigned>(1);
    ew.idx = c.take<int>(n);
    ew.chg = c.take<int>(2 * b);
    ew.cnt = c.take<int>(1);
    ew.tmp = c.take<double>(m * 2 * b);
    ew.jtmp = c.take<int64_t>(2 * b);
    status = c.take<int>(4);
    xch = c.take<unsigned long long>(panel_work_elems(m));
  };
  Carver probe;
  lay(probe);
  RUTV_CHECK(cx.reserve(probe.off));
  Carver real;
  real.base = cx.ws;
  lay(real);
  cw.err = &status[0];
  PanelWork pw;
  pw.xch = xch;
  pw.err = &status[1];
  set_launch_timer(nullptr);
  RUTV_CHECK(fill_zero_u32(st, reinterpret_cast<unsigned*>(status), 4));
  RUTV_CHECK(check_finite(st, m, n, A, lda, &status[2]));
  {
    int flag = 0;
    RUTV_TRY(hipMemcpyAsync(&flag, &status[2], sizeof(int), hipMemcpyDeviceToHost, st));
    RUTV_TRY(hipStreamSynchronize(st));
    if (flag) return RANDUTV_ERR_NONFINITE;
  }
  if (pivot) RUTV_CHECK(set_iota(st, n, jpvt));
  i64 s = 0;
  for (i64 i = 0; s < n; ++i) {
    const i64 bi = std::min(b, n - s), mi = m - s, ni = n - s;
    double* As = A + s * lda;  // columns s..n-1, all rows
    if (pivot) {
      RUTV_CHECK(sketch(st, seed, (uint64_t)i, mi, bi, G, mi));
      RUTV_CHECK(gemm(st, x, true, false, bi, ni, mi, 1.0, G, mi, As + s, lda, 0.0, Y, bi));
      RUTV_CHECK(cpqr_pivots(st, bi, ni, Y, bi, J, cw));
      RUTV_CHECK(exchange_columns(st, m, bi, ni, J, As, lda, jpvt + s, ew));
    }
    double* Pn = As + s;  // the panel, rows s..m-1
    RUTV_CHECK(panel_qr(st, mi, bi, Pn, lda, tau + s, pw));
    if (ni > bi) {
      RUTV_CHECK(extract_reflectors(st, mi, bi, Pn, lda, W, mi, nullptr, 0, false));
      RUTV_CHECK(t_factor(st, x, mi, bi, W, tau + s, Z));
      double* C = Pn + bi * lda;
      RUTV_CHECK(gemm(st, x, true, false, bi, ni - bi, mi, 1.0, W, mi, C, lda, 0.0, X3, bi));
      RUTV_CHECK(gemm(st, x, false, false, mi, ni - bi, bi, -1.0, Z, mi, X3, bi, 1.0, C, lda));
    }
    s += bi;
  }
  int flags[4] = {0, 0, 0, 0};
  RUTV_TRY(hipMemcpyAsync(flags, status, sizeof(flags), hipMemcpyDeviceToHost, st));
  RUTV_TRY(hipStreamSynchronize(st));
  if (flags[0] || flags[1]) return RANDUTV_ERR_SYNC;
  return RANDUTV_OK;
  });
}

int randutv_hqrrp(int64_t m, int64_t n, double* A, int64_t lda, int64_t b, uint64_t seed,
                  double* tau, int64_t* jpvt) {
  if (m < 0) return -1;
  if (n < 0 || n > m) return -2;
  if (m == 0 || n == 0) return RANDUTV_OK;
  if (!A) return -3;
  if (lda < std::max<int64_t>(1, m)) return -4;
  if (b < 1) return -5;
  if (!tau) return -7;
  if (!jpvt) return -8;
  if (b > n) b = n;
  if (b > kPanelMaxCols) return RANDUTV_ERR_TOO_LARGE;
  if (n > 32768) return RANDUTV_ERR_TOO_LARGE;  // the exchange plan's LDS index arrays
  if (m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return blocked_qr(m, n, A, lda, b, seed, tau, jpvt, true);
}

int randutv_geqrf_blocked(int64_t m, int64_t n, double* A, int64_t lda, int64_t b, double* tau) {
  if (m < 0) return -1;
  if (n < 0 || n > m) return -2;
  if (m == 0 || n == 0) return RANDUTV_OK;
  if (!A) return -3;
  if (lda < std::max<int64_t>(1, m)) return -4;
  if (b < 1) return -5;
  if (!tau) return -6;
  if (b > n) b = n;
  if (b > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return blocked_qr(m, n, A, lda, b, 0, tau, nullptr, false);
}

// Truncation jobs (forward value or reverse pass of A_k, see truncation.hip):
// job t runs on stream t mod S with a workspace slice of its own, so that the
// matrices of a batch overlap; the call waits for all of them.
static int run_trunc(Context& cx, const std::vector<TruncJob>& jobs) {
  const int S = (int)std::min<size_t>(jobs.size(), NSTREAMS);
  size_t slice = 0;
  for (const auto& j : jobs) slice = std::max(slice, trunc_ws_bytes(j));
  slice = (slice + 255) & ~size_t(255);
  RUTV_CHECK(cx.reserve(slice * (size_t)S + sizeof(int) * 8 * jobs.size()));
  int* status = reinterpret_cast<int*>(cx.ws + slice * (size_t)S);
  set_launch_timer(nullptr);
  for (size_t t = 0; t < jobs.size(); ++t) {
    const int s = (int)(t % (size_t)S);
    RUTV_CHECK(trunc_enqueue(jobs[t], cx.streams[s], cx.ws + slice * (size_t)s, status + 8 * t));
  }
  for (int s = 0; s < S; ++s) RUTV_TRY(hipStreamSynchronize(cx.streams[s]));
  std::vector<int> flags(8 * jobs.size());
  RUTV_TRY(hipMemcpy(flags.data(), status, sizeof(int) * flags.size(), hipMemcpyDeviceToHost));
  for (size_t t = 0; t < jobs.size(); ++t) RUTV_CHECK(trunc_status(&flags[8 * t], jobs[t]));
  return RANDUTV_OK;
}

static int run_trunc_entry(const std::vector<TruncJob>& jobs) {
  std::lock_guard<std::mutex> lk(g_mu);
  Context& cx = ctx();
  return drained(cx, [&]() -> int {
    RUTV_CHECK(cx.init());
    return run_trunc(cx, jobs);
  });
}

constexpr int32_t kGradMaxQ = 64;

// argument checks shared by the truncation entry points (positions 1..6)
static int check_trunc_args(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                            int32_t q, bool reverse) {
  if (m < 0) return -1;
  if (n < 0 || n > m) return -2;
  if (m == 0 || n == 0) return RANDUTV_OK;
  if (!A) return -3;
  if (lda < std::max<int64_t>(1, m)) return -4;
  if (b < 1) return -5;
  if (q < 0 || (reverse && q > kGradMaxQ)) return -6;  // the reverse pass keeps every product
  return RANDUTV_OK;
}

static TruncJob make_job(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b, int32_t q,
                         uint64_t seed, int64_t k, const double* Gbar, int64_t ldg, double* out,
                         int64_t ldo, bool reverse) {
  TruncJob j;
  j.m = m, j.n = n, j.A = A, j.lda = lda, j.b = b, j.q = q, j.seed = seed, j.k = k;
  j.Gbar = Gbar, j.ldg = ldg, j.out = out, j.ldo = ldo, j.reverse = reverse;
  return j;
}

int randutv_truncate_first_block(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                                 int32_t q, uint64_t seed, double* Ak, int64_t ldak) {
  int rc = check_trunc_args(m, n, A, lda, b, q, false);
  if (rc != RANDUTV_OK || m == 0 || n == 0) return rc;
  if (!Ak || Ak == A) return -8;
  if (ldak < std::max<int64_t>(1, m)) return -9;
  const i64 k = std::min<i64>(b, n);
  if (k > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return guarded([&] {
    return run_trunc_entry({make_job(m, n, A, lda, b, q, seed, k, nullptr, 0, Ak, ldak, false)});
  });
}

int randutv_truncate_first_block_k(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                                   int32_t q, uint64_t seed, int64_t k, double* Ak, int64_t ldak) {
  int rc = check_trunc_args(m, n, A, lda, b, q, false);
  if (rc != RANDUTV_OK || m == 0 || n == 0) return rc;
  const i64 bb = std::min<i64>(b, n);
  if (k < 1 || k > bb + std::min<i64>(b, n - bb)) return -8;
  if (!Ak || Ak == A) return -9;
  if (ldak < std::max<int64_t>(1, m)) return -10;
  if (bb > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return guarded([&] {
    return run_trunc_entry({make_job(m, n, A, lda, b, q, seed, k, nullptr, 0, Ak, ldak, false)});
  });
}

int randutv_truncate_grad(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                          int32_t q, uint64_t seed, const double* Gbar, int64_t ldg,
                          double* Abar, int64_t ldab) {
  int rc = check_trunc_args(m, n, A, lda, b, q, true);
  if (rc != RANDUTV_OK || m == 0 || n == 0) return rc;
  if (!Gbar) return -8;
  if (ldg < std::max<int64_t>(1, m)) return -9;
  if (!Abar || Abar == A || Abar == Gbar) return -10;
  if (ldab < std::max<int64_t>(1, m)) return -11;
  const i64 k = std::min<i64>(b, n);
  if (k > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return guarded([&] {
    return run_trunc_entry({make_job(m, n, A, lda, b, q, seed, k, Gbar, ldg, Abar, ldab, true)});
  });
}

int randutv_truncate_grad_k(int64_t m, int64_t n, const double* A, int64_t lda, int64_t b,
                            int32_t q, uint64_t seed, int64_t k, const double* Gbar, int64_t ldg,
                            double* Abar, int64_t ldab) {
  int rc = check_trunc_args(m, n, A, lda, b, q, true);
  if (rc != RANDUTV_OK || m == 0 || n == 0) return rc;
  const i64 bb = std::min<i64>(b, n);
  if (k < 1 || k > bb + std::min<i64>(b, n - bb)) return -8;
  if (!Gbar) return -9;
  if (ldg < std::max<int64_t>(1, m)) return -10;
  if (!Abar || Abar == A || Abar == Gbar) return -11;
  if (ldab < std::max<int64_t>(1, m)) return -12;
  if (bb > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return guarded([&] {
    return run_trunc_entry({make_job(m, n, A, lda, b, q, seed, k, Gbar, ldg, Abar, ldab, true)});
  });
}

int randutv_truncate_batched(int64_t batch, int32_t reverse, int64_t m, int64_t n, const double* A,
                             int64_t lda, int64_t stride_a, int64_t b, int32_t q, uint64_t seed,
                             int64_t k, const double* Gbar, int64_t ldg, int64_t stride_g,
                             double* out, int64_t ldo, int64_t stride_o) {
  if (batch < 0) return -1;
  if (reverse != 0 && reverse != 1) return -2;
  if (m < 0) return -3;
  if (n < 0 || n > m) return -4;
  if (batch == 0 || m == 0 || n == 0) return RANDUTV_OK;
  if (!A) return -5;
  if (lda < std::max<int64_t>(1, m)) return -6;
  if (batch > 1 && stride_a < lda * n) return -7;
  if (b < 1) return -8;
  if (q < 0 || (reverse && q > kGradMaxQ)) return -9;
  const i64 bb = std::min<i64>(b, n);
  if (k < 1 || k > bb + std::min<i64>(b, n - bb)) return -11;
  if (reverse) {
    if (!Gbar) return -12;
    if (ldg < std::max<int64_t>(1, m)) return -13;
    if (batch > 1 && stride_g < ldg * n) return -14;
  }
  if (!out || out == A || (reverse && out == Gbar)) return -15;
  if (ldo < std::max<int64_t>(1, m)) return -16;
  if (batch > 1 && stride_o < ldo * n) return -17;
  if (bb > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  return guarded([&] {
    std::vector<TruncJob> jobs;
    jobs.reserve((size_t)batch);
    for (int64_t t = 0; t < batch; ++t)
      jobs.push_back(make_job(m, n, A + t * stride_a, lda, b, q, seed, k,
                              reverse ? Gbar + t * stride_g : nullptr, ldg, out + t * stride_o, ldo,
                              reverse != 0));
    return run_trunc_entry(jobs);
  });
}

int randutv_sketch(uint64_t seed, uint64_t step, int64_t rows, int64_t cols, double* G,
                   int64_t ldg) {
  if (rows < 0) return -3;
  if (cols < 0) return -4;
  if (rows == 0 || cols == 0) return RANDUTV_OK;
  if (!G) return -5;
  if (ldg < std::max<int64_t>(1, rows)) return -6;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return drained(cx, [&]() -> int {
  RUTV_CHECK(cx.init());
  set_launch_timer(nullptr);
  RUTV_CHECK(sketch(cx.st, seed, step, rows, cols, G, ldg));
  RUTV_TRY(hipStreamSynchronize(cx.st));
  return RANDUTV_OK;
  });
}

int randutv_sketch_host(uint64_t seed, int64_t m, int64_t n, int64_t b, double* G_host) {
  if (m < 0) return -2;
  if (n < 0 || n > m) return -3;
  if (m == 0 || n == 0) return RANDUTV_OK;
  if (b < 1) return -4;
  if (!G_host) return -5;
  if (b > n) b = n;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return guarded([&]() -> int {
    RUTV_CHECK(cx.init());
    RUTV_CHECK(cx.reserve(sizeof(double) * (size_t)(m * b)));
    double* G = reinterpret_cast<double*>(cx.ws);
    set_launch_timer(nullptr);
    i64 off = 0;
    for (i64 i = 0, s = 0; s < n; ++i, s += b) {
      const i64 bi = std::min(b, n - s), mi = m - s;
      int rc = sketch(cx.st, seed, (uint64_t)i, mi, bi, G, mi);
      if (rc == RANDUTV_OK) {
        const hipError_t e =
            hipMemcpyAsync(G_host + off, G, sizeof(double) * mi * bi, hipMemcpyDeviceToHost, cx.st);
        if (e == hipSuccess) {
          const hipError_t e2 = hipStreamSynchronize(cx.st);
          rc = e2 == hipSuccess ? RANDUTV_OK : hip_code(e2);
        } else {
          rc = hip_code(e);
        }
      }
      if (rc != RANDUTV_OK) {
        cx.drain();
        return rc;
      }
      off += mi * bi;
    }
    return RANDUTV_OK;
  });
}

int randutv_sketch_words(uint64_t seed, uint64_t step, uint64_t first_block, int64_t nblocks,
                         uint64_t* out) {
  if (nblocks < 0) return -4;
  if (nblocks == 0) return RANDUTV_OK;
  if (!out) return -5;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return guarded([&]() -> int {
    RUTV_CHECK(cx.init());
    set_launch_timer(nullptr);
    RUTV_CHECK(sketch_words(cx.st, seed, step, first_block, nblocks, out));
    RUTV_TRY(hipStreamSynchronize(cx.st));
    return RANDUTV_OK;
  });
}

int randutv_finalize(void) {
  std::lock_guard<std::mutex> lk(g_mu);
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) cur = -1;
  for (Context& cx : g_ctx) {
    if (!cx.st) continue;
    const int dev = cx.device;
    if (dev != cur) (void)hipSetDevice(dev);
    cx.release();
  }
  if (cur >= 0) (void)hipSetDevice(cur);
  return RANDUTV_OK;
}

static int gemm_entry(char transa, char transb, int64_t M, int64_t N, int64_t K, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                      double* C, int64_t ldc, int prec) {
  const bool ta = transa == 'T' || transa == 't', tb = transb == 'T' || transb == 't';
  if (!ta && transa != 'N' && transa != 'n') return -1;
  if (!tb && transb != 'N' && transb != 'n') return -2;
  if (M < 0) return -3;
  if (N < 0) return -4;
  if (K < 0) return -5;
  if (M == 0 || N == 0) return RANDUTV_OK;
  if (K > 0 && !A) return -7;
  if (lda < std::max<int64_t>(1, ta ? K : M)) return -8;
  if (K > 0 && !B) return -9;
  if (ldb < std::max<int64_t>(1, tb ? N : K)) return -10;
  if (!C) return -12;
  if (ldc < std::max<int64_t>(1, M)) return -13;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return drained(cx, [&]() -> int {
  RUTV_CHECK(cx.init());
  const i64 sk = dgemm_work_elems(M, N, K);
  RUTV_CHECK(cx.reserve(sizeof(double) * std::max<i64>(sk, 1)));
  set_launch_timer(nullptr);
  RUTV_CHECK(dgemm(cx.st, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                   reinterpret_cast<double*>(cx.ws), sk, prec));
  RUTV_TRY(hipStreamSynchronize(cx.st));
  return RANDUTV_OK;
  });
}

int randutv_dgemm(char transa, char transb, int64_t M, int64_t N, int64_t K, double alpha,
                  const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                  double* C, int64_t ldc) {
  return gemm_entry(transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, PREC_F64);
}

int randutv_gemm_f32(char transa, char transb, int64_t M, int64_t N, int64_t K, double alpha,
                     const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                     double* C, int64_t ldc) {
  return gemm_entry(transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, PREC_F32);
}

int randutv_gemm_bf16(char transa, char transb, int64_t M, int64_t N, int64_t K, double alpha,
                      const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                      double* C, int64_t ldc, int32_t terms) {
  if (terms != 1 && terms != 3) return -14;
  return gemm_entry(transa, transb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc,
                    terms == 3 ? PREC_BF16X3 : PREC_BF16);
}

int randutv_geqrf(int64_t m, int64_t k, double* A, int64_t lda, double* tau) {
  if (m < 0) return -1;
  if (k < 0 || k > m) return -2;
  if (m == 0 || k == 0) return RANDUTV_OK;
  if (!A) return -3;
  if (lda < std::max<int64_t>(1, m)) return -4;
  if (!tau) return -5;
  if (k > kPanelMaxCols || m > kMaxRows) return RANDUTV_ERR_TOO_LARGE;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return drained(cx, [&]() -> int {
  RUTV_CHECK(cx.init());
  Carver c;
  c.take<unsigned long long>(panel_work_elems(m));
  c.take<int>(4);
  RUTV_CHECK(cx.reserve(c.off));
  Carver r;
  r.base = cx.ws;
  PanelWork pw;
  pw.xch = r.take<unsigned long long>(panel_work_elems(m));
  pw.err = r.take<int>(4);
  set_launch_timer(nullptr);
  RUTV_CHECK(fill_zero_u32(cx.st, reinterpret_cast<unsigned*>(pw.err), 1));
  RUTV_CHECK(panel_qr(cx.st, m, k, A, lda, tau, pw));
  int err = 0;
  RUTV_TRY(hipMemcpyAsync(&err, pw.err, sizeof(int), hipMemcpyDeviceToHost, cx.st));
  RUTV_TRY(hipStreamSynchronize(cx.st));
  return err ? RANDUTV_ERR_SYNC : RANDUTV_OK;
  });
}

int randutv_larft(int64_t m, int64_t k, const double* W, int64_t ldw, const double* tau,
                  double* Tf, int64_t ldt) {
  if (m < 0) return -1;
  if (k < 0 || k > m) return -2;
  if (k == 0) return RANDUTV_OK;
  if (!W) return -3;
  if (ldw < std::max<int64_t>(1, m)) return -4;
  if (!tau) return -5;
  if (!Tf) return -6;
  if (ldt < k) return -7;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return drained(cx, [&]() -> int {
  RUTV_CHECK(cx.init());
  const i64 sk = dgemm_work_elems(k, k, m);
  Carver c;
  c.take<double>(m * k);
  c.take<double>(k * k);
  c.take<double>(sk);
  RUTV_CHECK(cx.reserve(c.off));
  Carver r;
  r.base = cx.ws;
  double* We = r.take<double>(m * k);
  double* G = r.take<double>(k * k);
  double* wk = r.take<double>(sk);
  set_launch_timer(nullptr);
  RUTV_CHECK(extract_reflectors(cx.st, m, k, const_cast<double*>(W), ldw, We, m, nullptr, 0, false));
  RUTV_CHECK(dgemm(cx.st, true, false, k, k, m, 1.0, We, m, We, m, 0.0, G, k, wk, sk));
  RUTV_CHECK(larft_from_gram(cx.st, k, G, k, tau, Tf, ldt));
  RUTV_TRY(hipStreamSynchronize(cx.st));
  return RANDUTV_OK;
  });
}

int randutv_gesvj(int64_t k, const double* R, int64_t ldr, double* d, double* Us, double* Vs,
                  int32_t* sweeps) {
  if (k < 0) return -1;
  if (k == 0) return RANDUTV_OK;
  if (!R) return -2;
  if (ldr < k) return -3;
  if (!d) return -4;
  if (!Us) return -5;
  if (!Vs) return -6;
  if (k > kJacobiMaxN) return RANDUTV_ERR_TOO_LARGE;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  return drained(cx, [&]() -> int {
  RUTV_CHECK(cx.init());
  Carver c;
  c.take<double>(jacobi_work_elems(k));
  c.take<int>(4);
  RUTV_CHECK(cx.reserve(c.off));
  Carver r;
  r.base = cx.ws;
  double* wk = r.take<double>(jacobi_work_elems(k));
  int* status = r.take<int>(4);
  set_launch_timer(nullptr);
  {
    int flag = 0;
    RUTV_CHECK(fill_zero_u32(cx.st, reinterpret_cast<unsigned*>(status), 1));
    RUTV_CHECK(check_finite(cx.st, k, k, R, ldr, status));
    RUTV_TRY(hipMemcpyAsync(&flag, status, sizeof(int), hipMemcpyDeviceToHost, cx.st));
    RUTV_TRY(hipStreamSynchronize(cx.st));
    if (flag) return RANDUTV_ERR_NONFINITE;
  }
  RUTV_CHECK(jacobi_svd(cx.st, k, R, ldr, d, Us, Vs, wk, status));
  int hs[3] = {0, 0, 0};
  RUTV_TRY(hipMemcpyAsync(hs, status, sizeof(hs), hipMemcpyDeviceToHost, cx.st));
  RUTV_TRY(hipStreamSynchronize(cx.st));
  if (sweeps) *sweeps = hs[0];
  if (hs[2]) return RANDUTV_ERR_SYNC;
  return hs[1] ? RANDUTV_OK : RANDUTV_ERR_NOCONV;
  });
}

int randutv_set_timing(int32_t enable) {
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  if (enable < 0 || enable > 3) return -1;
  cx.timing = enable != 0;
  cx.timer.gemm_only = enable >= 2;
  cx.timer.serialize = enable == 3;
  cx.timer.clear_counts();
  return RANDUTV_OK;
}

int randutv_kernel_stats(int32_t cap, const char** names, int64_t* launches, double* ms,
                         double* flops) {
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  int nout = 0;
  for (int c = 0; c < K_NUM_CLASSES && nout < cap; ++c) {
    if (names) names[nout] = kernel_class_name(c);
    if (launches) launches[nout] = cx.timer.launches[c];
    if (ms) ms[nout] = cx.timer.ms[c];
    if (flops) flops[nout] = cx.timer.flops[c];
    ++nout;
  }
  return nout;
}

int randutv_kernel_trace(int32_t cap, int32_t* cls, int32_t* stream, double* start_ms,
                         double* dur_ms) {
  if (cap < 0) return -1;
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  const auto& tr = cx.timer.trace;
  const int n = (int)std::min<size_t>(tr.size(), (size_t)cap);
  for (int i = 0; i < n; ++i) {
    int sx = -1;
    for (int x = 0; x < NSTREAMS; ++x)
      if (cx.streams[x] == tr[i].st) sx = x;
    if (cls) cls[i] = tr[i].cls;
    if (stream) stream[i] = sx;
    if (start_ms) start_ms[i] = tr[i].start;
    if (dur_ms) dur_ms[i] = tr[i].dur;
  }
  return (int)tr.size();
}

int randutv_kernel_bytes(int32_t cap, double* bytes) {
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  int nout = 0;
  for (int c = 0; c < K_NUM_CLASSES && nout < cap; ++c) {
    if (bytes) bytes[nout] = cx.timer.bytes[c];
    ++nout;
  }
  return nout;
}

int randutv_last_sweeps(int32_t cap, int32_t* sweeps) {
  Context& cx = ctx();
  std::lock_guard<std::mutex> lk(g_mu);
  const int n = (int)cx.sweeps.size();
  for (int i = 0; i < n && i < cap; ++i) sweeps[i] = cx.sweeps[i];
  return n;
}

const char* randutv_last_hip_error(void) { return g_hip_error; }

const char* randutv_strerror(int code) {
  switch (code) {
    case RANDUTV_OK: return "success";
    case RANDUTV_ERR_HIP: return "HIP runtime error or no usable device";
    case RANDUTV_ERR_NOMEM: return "device workspace allocation failed";
    case RANDUTV_ERR_NONFINITE: return "input holds NaN or Inf";
    case RANDUTV_ERR_NOCONV: return "Jacobi SVD did not converge within 30 sweeps";
    case RANDUTV_ERR_SYNC: return "multi-workgroup kernel wait expired";
    case RANDUTV_ERR_TOO_LARGE: return "dimension exceeds a kernel limit";
    case RANDUTV_ERR_RANK: return "the first block's sketch is rank deficient (no derivative)";
    case RANDUTV_ERR_SCRATCH:
      return "the problem needs more device scratch than the allocation-free entry point's fixed "
             "RANDUTV_NOALLOC_SCRATCH_BYTES";
    default: return code < 0 ? "invalid argument" : "unknown error";
  }
}

}  // extern "C"
