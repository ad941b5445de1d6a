// Out-of-core randUTV on one GPU (Section 3.2): the matrices live in host
// memory (the paper's external device), HBM holds a cache of their tiles
// (the paper's in-RAM block cache), and a copy stream moves tiles while the
// compute stream works (the paper's I/O thread overlapping the computation).
//
// Tiles are block columns: tile j of a matrix holds its columns
// [j b, j b + b_j) for every row, so that each operation of a block step
// (Section 3.1, Figure 2) splits into one FP64 matrix-core GEMM per tile:
//
//   sketch        Y_j = T_j(s:m, :)^T G                         j >= i
//   power         Z = sum_j T_j(s:m, :) Y_j;  Y_j = T_j(s:m, :)^T Z
//   right update  X = sum_j T_j W_j;  T_j -= X Z_j^T           all m rows
//   V update      X = sum_j V_j W_j;  V_j -= X Z_j^T
//   panel         Householder QR of T_i(s:m, :)
//   left update   X3 = W_U^T T_j(s:m, :);  T_j(s:m, :) -= Z_U X3   j > i
//   U update      X = sum_j U_j W_Uj;  U_j -= X Z_Uj^T
//   SVD           T_i, V_i, U_i times the b x b factors
//
// with W, Z, X and the sketch in fixed HBM buffers.  The arithmetic is that of
// the in-core path (same kernels, same reflector conventions); only the
// summation order of the sums over tiles differs.
//
// Cache (Section 3.2.4's three variants, chosen by `mode`):
//   traditional  every access reads its tile from host memory and a tile
//                that was written goes back at once (no reuse);
//   cached       least-recently-used HBM slots with a dirty bit: a hit costs
//                nothing, a miss waits for its copy, a dirty victim is written
//                back first;
//   overlapped   the cache plus prefetch: while the compute stream works on
//                tile t of a sweep, the copy stream already brings in tile
//                t + 1 (evicting and writing back as needed).
// Sweeps over the tiles of one matrix alternate their direction, so that the
// tiles a sweep touched last are still cached when the next one starts.
//
// Copies into HBM and write-backs to host memory run on two streams of their
// own, so that both directions of the host link work at once.  Ordering is by
// events only: a slot's write-back waits for the compute stream's last use of
// the slot (`used`); a copy into the slot waits for that use and for the
// write-back of its previous contents (`wb`); the compute stream waits for the
// copy that filled it (`ready`); and a copy of a tile from host memory waits
// for that tile's last write-back there (write-backs all run on one stream,
// so the latest record of the slot event that covered it is enough).
#include <algorithm>
#include <chrono>
#include <vector>

#include "kernels.hpp"

namespace rutv {

namespace {

// X (rows x cols, ld ldx) := columns [c0, c0 + cols) of the rows x rows identity
__global__ __launch_bounds__(256) void eye_block_kernel(i64 rows, i64 cols, i64 c0,
                                                        double* __restrict__ X, i64 ldx) {
  const i64 total = rows * cols;
  for (i64 e = (i64)blockIdx.x * 256 + threadIdx.x; e < total; e += (i64)gridDim.x * 256) {
    const i64 r = e % rows, c = e / rows;
    X[r + c * ldx] = r == c0 + c ? 1.0 : 0.0;
  }
}

int eye_block(hipStream_t st, i64 rows, i64 cols, i64 c0, double* X, i64 ldx) {
  if (rows <= 0 || cols <= 0) return RANDUTV_OK;
  const int blocks = (int)std::min<i64>(cdiv(rows * cols, 256), 16384);
  eye_block_kernel<<<blocks, 256, 0, st>>>(rows, cols, c0, X, ldx);
  RUTV_TRY(hipGetLastError());
  return RANDUTV_OK;
}

// a matrix in host memory, cut into block columns of width tw
struct HostMat {
  double* dst = nullptr;        // where its tiles are written back (ld ld)
  i64 ld = 0;
  const double* src = nullptr;  // first contents (ld ld_src); null: identity
  i64 ld_src = 0;
  i64 rows = 0, cols = 0, tw = 0;
  std::vector<char> fresh;      // tile not yet written back to dst
  std::vector<int> wb_slot;     // slot whose `wb` event covers the tile's last write-back (-1: none)
  i64 tiles() const { return cdiv(cols, tw); }
  i64 width(i64 j) const { return std::min(tw, cols - j * tw); }
};

// HIP events around copies or compute tasks, summed at the end
struct Intervals {
  std::vector<hipEvent_t> pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> recs;
  size_t used = 0;
  hipEvent_t take() {
    if (used == pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return nullptr;
      pool.push_back(e);
    }
    return pool[used++];
  }
  hipEvent_t begin(hipStream_t st) {
    hipEvent_t a = take();
    if (a) (void)hipEventRecord(a, st);
    return a;
  }
  void end(hipStream_t st, hipEvent_t a) {
    hipEvent_t b = a ? take() : nullptr;
    if (!b) return;
    (void)hipEventRecord(b, st);
    recs.push_back({a, b});
  }
  double total_ms() const {
    double s = 0.0;
    for (auto& r : recs) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, r.first, r.second) == hipSuccess) s += t;
    }
    return s;
  }
  ~Intervals() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

class TileCache {
 public:
  struct Slot {
    int mat = -1;
    i64 tile = -1;
    bool dirty = false;
    bool pending = false;  // a copy into the slot is in flight (`ready` marks its end)
    uint64_t stamp = 0;
    hipEvent_t ready = nullptr, used = nullptr, wb = nullptr;
  };

  TileCache(hipStream_t cs, hipStream_t xs, hipStream_t ws, int mode, std::vector<HostMat>& mats)
      : cs_(cs), xs_(xs), ws_(ws), mode_(mode), mats_(mats) {}
  ~TileCache() {
    for (auto& s : slots_) {
      if (s.ready) (void)hipEventDestroy(s.ready);
      if (s.used) (void)hipEventDestroy(s.used);
      if (s.wb) (void)hipEventDestroy(s.wb);
    }
    if (mem_) (void)hipFree(mem_);
  }

  int init(i64 nslots, i64 slot_elems) {
    slot_elems_ = slot_elems;
    RUTV_TRY(hipMalloc((void**)&mem_, sizeof(double) * (size_t)(nslots * slot_elems)));
    slots_.resize(nslots);
    for (auto& s : slots_) {
      RUTV_TRY(hipEventCreateWithFlags(&s.ready, hipEventDisableTiming));
      RUTV_TRY(hipEventCreateWithFlags(&s.used, hipEventDisableTiming));
      RUTV_TRY(hipEventCreateWithFlags(&s.wb, hipEventDisableTiming));
    }
    where_.resize(mats_.size());
    for (size_t k = 0; k < mats_.size(); ++k) where_[k].assign(mats_[k].tiles(), -1);
    return RANDUTV_OK;
  }

  // device pointer of tile j of matrix `mat` (ld = the matrix's rows); the
  // compute stream is ordered after the copy that brings it in
  int acquire(int mat, i64 j, bool write, double** out) {
    int k = where_[mat][j];
    if (k >= 0) {
      ++hits;
    } else {
      RUTV_CHECK(bring(mat, j, &k));
    }
    Slot& s = slots_[k];
    if (s.pending) {
      RUTV_TRY(hipStreamWaitEvent(cs_, s.ready, 0));
      s.pending = false;
    }
    s.stamp = ++clock_;
    if (write) s.dirty = true;
    *out = ptr(k);
    return RANDUTV_OK;
  }
  // after the compute stream's work on the tile has been enqueued
  int release(int mat, i64 j) {
    const int k = where_[mat][j];
    if (k < 0) return RANDUTV_OK;
    RUTV_TRY(hipEventRecord(slots_[k].used, cs_));
    if (mode_ == 0) RUTV_CHECK(evict(k));  // traditional: no reuse
    return RANDUTV_OK;
  }
  // start bringing in a tile that a later acquire will need (overlapped mode)
  int prefetch(int mat, i64 j) {
    if (mode_ != 2) return RANDUTV_OK;
    int k = where_[mat][j];
    if (k >= 0) {
      slots_[k].stamp = ++clock_;
      return RANDUTV_OK;
    }
    RUTV_CHECK(bring(mat, j, &k));
    slots_[k].stamp = ++clock_;
    return RANDUTV_OK;
  }
  // write every dirty tile back and forget the cached copies
  int flush() {
    for (int k = 0; k < (int)slots_.size(); ++k) RUTV_CHECK(evict(k));
    return RANDUTV_OK;
  }

  int64_t hits = 0, loads = 0, writebacks = 0, inits = 0, h2d_bytes = 0, d2h_bytes = 0;
  Intervals io_in, io_out;

 private:
  double* ptr(int k) const { return mem_ + (i64)k * slot_elems_; }

  int victim() const {
    int best = 0;
    for (int k = 1; k < (int)slots_.size(); ++k)
      if (slots_[k].stamp < slots_[best].stamp) best = k;
    return best;
  }

  // copy-stream write-back of a dirty slot, then the slot is free
  int evict(int k) {
    Slot& s = slots_[k];
    if (s.tile < 0) return RANDUTV_OK;
    HostMat& M = mats_[s.mat];
    if (s.dirty) {
      const i64 w = M.width(s.tile);
      RUTV_TRY(hipStreamWaitEvent(ws_, s.used, 0));
      hipEvent_t a = io_out.begin(ws_);
      RUTV_TRY(hipMemcpy2DAsync(M.dst + s.tile * M.tw * M.ld, sizeof(double) * M.ld, ptr(k),
                                sizeof(double) * M.rows, sizeof(double) * M.rows, w,
                                hipMemcpyDeviceToHost, ws_));
      io_out.end(ws_, a);
      RUTV_TRY(hipEventRecord(s.wb, ws_));
      M.fresh[s.tile] = 0;
      M.wb_slot[s.tile] = k;
      ++writebacks;
      d2h_bytes += (int64_t)sizeof(double) * M.rows * w;
    }
    where_[s.mat][s.tile] = -1;
    s.mat = -1;
    s.tile = -1;
    s.dirty = false;
    return RANDUTV_OK;
  }

  // a slot for tile j of `mat`, filled: from host memory on the copy stream,
  // or (identity start of U and V) by a kernel on the compute stream
  int bring(int mat, i64 j, int* slot) {
    const int k = victim();
    RUTV_CHECK(evict(k));
    Slot& s = slots_[k];
    HostMat& M = mats_[mat];
    const i64 w = M.width(j);
    if (M.fresh[j] && !M.src) {
      // after the write-back of the previous tile (and any copy still
      // filling the slot), on the compute stream, which orders itself after
      // its own earlier use
      RUTV_TRY(hipStreamWaitEvent(cs_, s.wb, 0));
      if (s.pending) RUTV_TRY(hipStreamWaitEvent(cs_, s.ready, 0));
      RUTV_CHECK(eye_block(cs_, M.rows, w, j * M.tw, ptr(k), M.rows));
      s.pending = false;
      ++inits;
    } else {
      const double* from = M.fresh[j] ? M.src + j * M.tw * M.ld_src : M.dst + j * M.tw * M.ld;
      const i64 ldf = M.fresh[j] ? M.ld_src : M.ld;
      // nothing may write the slot before the compute stream is done with it
      // and its previous contents are back in host memory
      RUTV_TRY(hipStreamWaitEvent(xs_, s.used, 0));
      RUTV_TRY(hipStreamWaitEvent(xs_, s.wb, 0));
      if (!M.fresh[j] && M.wb_slot[j] >= 0)
        RUTV_TRY(hipStreamWaitEvent(xs_, slots_[M.wb_slot[j]].wb, 0));
      hipEvent_t a = io_in.begin(xs_);
      RUTV_TRY(hipMemcpy2DAsync(ptr(k), sizeof(double) * M.rows, from, sizeof(double) * ldf,
                                sizeof(double) * M.rows, w, hipMemcpyHostToDevice, xs_));
      io_in.end(xs_, a);
      RUTV_TRY(hipEventRecord(s.ready, xs_));
      s.pending = true;
      ++loads;
      h2d_bytes += (int64_t)sizeof(double) * M.rows * w;
    }
    s.mat = mat;
    s.tile = j;
    s.dirty = false;
    where_[mat][j] = k;
    *slot = k;
    return RANDUTV_OK;
  }

  hipStream_t cs_, xs_, ws_;
  int mode_;
  std::vector<HostMat>& mats_;
  std::vector<Slot> slots_;
  std::vector<std::vector<int>> where_;
  double* mem_ = nullptr;
  i64 slot_elems_ = 0;
  uint64_t clock_ = 0;
};

}  // namespace

int ooc_factor(const OocCfg& c, hipStream_t cs, hipStream_t xs, hipStream_t ws,
               randutv_ooc_stats* stats) {
  const auto t_start = std::chrono::steady_clock::now();
  const i64 m = c.m, n = c.n;
  const i64 b = std::min(c.b, n);
  const int q = c.q;
  const i64 p = cdiv(n, b);
  const bool wantU = c.U != nullptr, wantV = c.V != nullptr;
  enum { MT = 0, MU = 1, MV = 2 };
  std::vector<HostMat> mats(3);
  mats[MT] = HostMat{c.T, c.ldt, c.A, c.lda, m, n, b, {}};
  mats[MU] = HostMat{c.U, c.ldu, nullptr, 0, m, wantU ? m : 0, b, {}};
  mats[MV] = HostMat{c.V, c.ldv, nullptr, 0, n, wantV ? n : 0, b, {}};
  for (auto& M : mats) {
    M.fresh.assign(M.tiles(), 1);
    M.wb_slot.assign(M.tiles(), -1);
  }
  // in place (T == A): T's tiles start as what its host memory holds
  if (c.T == c.A) std::fill(mats[MT].fresh.begin(), mats[MT].fresh.end(), 0);

  // ---- fixed HBM buffers (outside the tile budget)
  const i64 mx = std::max(m, n);
  const i64 sk = std::max(dgemm_work_elems(b, b, mx), dgemm_work_elems(mx, b, b));
  struct Bufs {
    double *G, *Y, *Zp, *X, *X3, *WV, *ZV, *WU, *ZU, *tauV, *tauU, *R, *d, *Us, *Vs, *Usall, *jwork,
        *splitk, *Gram, *Tf;
    int* status;
    unsigned long long* xch;
  } w{};
  size_t off = 0;
  char* base = nullptr;
  auto take = [&](auto*& p_, i64 count) {
    using Tp = std::remove_reference_t<decltype(*p_)>;
    off = (off + 255) & ~size_t(255);
    p_ = base ? reinterpret_cast<Tp*>(base + off) : nullptr;
    off += sizeof(Tp) * (size_t)std::max<i64>(count, 1);
  };
  auto lay = [&]() {
    off = 0;
    take(w.G, m * b);
    take(w.Y, n * b);
    take(w.Zp, m * b);
    take(w.X, mx * b);
    take(w.X3, b * b);
    take(w.WV, n * b);
    take(w.ZV, n * b);
    take(w.WU, m * b);
    take(w.ZU, m * b);
    take(w.tauV, b);
    take(w.tauU, b);
    take(w.R, b * b);
    take(w.d, b);
    take(w.Us, b * b);
    take(w.Vs, b * b);
    take(w.Usall, p * b * b);
    take(w.jwork, jacobi_work_elems(b));
    take(w.splitk, sk);
    take(w.Gram, b * b);
    take(w.Tf, b * b);
    take(w.status, 4 + 3 * p);
    take(w.xch, panel_work_elems(mx));
  };
  lay();
  const size_t fixed_bytes = off;
  struct DevMem {
    char* p = nullptr;
    ~DevMem() {
      if (p) (void)hipFree(p);
    }
  } fixed;
  RUTV_TRY(hipMalloc((void**)&fixed.p, fixed_bytes));
  base = fixed.p;
  lay();
  PanelWork pw;
  pw.xch = w.xch;
  pw.err = &w.status[1];

  // ---- tile cache: as many block-column slots as the budget holds
  const i64 slot_elems = mx * b;
  const i64 nslots = (i64)(c.budget / (sizeof(double) * (size_t)slot_elems));
  if (nslots < 2) return RANDUTV_ERR_TOO_LARGE;
  TileCache cache(cs, xs, ws, c.mode, mats);
  RUTV_CHECK(cache.init(nslots, slot_elems));
  Intervals comp;

  auto gemm = [&](bool ta, bool tb, i64 M, i64 N, i64 K, double alpha, const double* A, i64 lda,
                  const double* B, i64 ldb, double beta, double* C, i64 ldc) {
    return dgemm(cs, ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, w.splitk, sk);
  };
  // one sweep over tiles [j0, j1) of a matrix, in the direction that starts
  // where the previous sweep over that matrix ended
  bool fwd[3] = {true, true, true};
  auto sweep = [&](int mat, i64 j0, i64 j1, bool write, auto&& body) -> int {
    if (j1 <= j0) return RANDUTV_OK;
    const bool f = fwd[mat];
    fwd[mat] = !f;
    const i64 cnt = j1 - j0;
    auto at = [&](i64 t) { return f ? j0 + t : j1 - 1 - t; };
    for (i64 t = 0; t < cnt; ++t) {
      const i64 j = at(t);
      double* tile = nullptr;
      RUTV_CHECK(cache.acquire(mat, j, write, &tile));
      // the next tile of the sweep comes in while this one is worked on (it
      // takes the least recently used slot, never this one)
      if (t + 1 < cnt) RUTV_CHECK(cache.prefetch(mat, at(t + 1)));
      hipEvent_t a = comp.begin(cs);
      RUTV_CHECK(body(j, tile));
      comp.end(cs, a);
      RUTV_CHECK(cache.release(mat, j));
    }
    return RANDUTV_OK;
  };

  // the step loop; on an error the streams are drained before the cache
  // slots and buffers are freed
  auto run = [&]() -> int {
  RUTV_CHECK(fill_zero_u32(cs, reinterpret_cast<unsigned*>(w.status), 4 + 3 * p));
  for (i64 i = 0; i < p; ++i) {
    const i64 s = i * b, bi = std::min(b, n - s), mi = m - s, ni = n - s;
    // ---- sketch and power iteration over the trailing tiles (step 0's
    // sweep also checks each tile of A for NaN/Inf as it first arrives)
    {
      hipEvent_t a = comp.begin(cs);
      RUTV_CHECK(sketch(cs, c.seed, (uint64_t)i, mi, bi, w.G, mi));
      comp.end(cs, a);
    }
    RUTV_CHECK(sweep(MT, i, p, false, [&](i64 j, double* tile) {
      const i64 bj = mats[MT].width(j);
      if (i == 0 && c.finite_check) RUTV_CHECK(check_finite(cs, m, bj, tile, m, &w.status[0]));
      return gemm(true, false, bj, bi, mi, 1.0, tile + s, m, w.G, mi, 0.0, w.Y + (j * b - s), ni);
    }));
    if (i == 0 && c.finite_check) {
      int flag = 0;
      RUTV_TRY(hipMemcpyAsync(&flag, &w.status[0], sizeof(int), hipMemcpyDeviceToHost, cs));
      RUTV_TRY(hipStreamSynchronize(cs));
      if (flag) return RANDUTV_ERR_NONFINITE;
    }
    for (int it = 0; it < q; ++it) {
      // Z = sum_j T_j(s:m) Y_j: the first tile of the sweep writes, the rest add
      bool first = true;
      RUTV_CHECK(sweep(MT, i, p, false, [&](i64 j, double* tile) {
        const i64 bj = mats[MT].width(j);
        const double beta = first ? 0.0 : 1.0;
        first = false;
        return gemm(false, false, mi, bi, bj, 1.0, tile + s, m, w.Y + (j * b - s), ni, beta, w.Zp, mi);
      }));
      RUTV_CHECK(sweep(MT, i, p, false, [&](i64 j, double* tile) {
        const i64 bj = mats[MT].width(j);
        return gemm(true, false, bj, bi, mi, 1.0, tile + s, m, w.Zp, mi, 0.0, w.Y + (j * b - s), ni);
      }));
    }
    // ---- QR of the sketch and the block factor of V^
    {
      hipEvent_t a = comp.begin(cs);
      RUTV_CHECK(panel_qr(cs, ni, bi, w.Y, ni, w.tauV, pw));
      RUTV_CHECK(extract_reflectors(cs, ni, bi, w.Y, ni, w.WV, ni, nullptr, 0, false));
      RUTV_CHECK(gemm(true, false, bi, bi, ni, 1.0, w.WV, ni, w.WV, ni, 0.0, w.Gram, bi));
      RUTV_CHECK(larft_from_gram(cs, bi, w.Gram, bi, w.tauV, w.Tf, bi));
      RUTV_CHECK(gemm(false, true, ni, bi, bi, 1.0, w.WV, ni, w.Tf, bi, 0.0, w.ZV, ni));
      comp.end(cs, a);
    }
    // ---- right transform of T (all m rows) and of V: X = sum_j M_j W_j,
    // then M_j -= X Z_j^T
    auto right = [&](int mat, const double* W, const double* Z, i64 ldw) -> int {
      HostMat& M = mats[mat];
      bool first = true;
      RUTV_CHECK(sweep(mat, i, M.tiles(), false, [&](i64 j, double* tile) {
        const double beta = first ? 0.0 : 1.0;
        first = false;
        return gemm(false, false, M.rows, bi, M.width(j), 1.0, tile, M.rows, W + (j * b - s), ldw,
                    beta, w.X, M.rows);
      }));
      RUTV_CHECK(sweep(mat, i, M.tiles(), true, [&](i64 j, double* tile) {
        return gemm(false, true, M.rows, M.width(j), bi, -1.0, w.X, M.rows, Z + (j * b - s), ldw, 1.0,
                    tile, M.rows);
      }));
      return RANDUTV_OK;
    };
    RUTV_CHECK(right(MT, w.WV, w.ZV, ni));
    if (wantV) RUTV_CHECK(right(MV, w.WV, w.ZV, ni));
    // ---- panel QR of T_i(s:m), its reflectors, R, and the block factor of U^
    {
      double* tile = nullptr;
      RUTV_CHECK(cache.acquire(MT, i, true, &tile));
      hipEvent_t a = comp.begin(cs);
      RUTV_CHECK(panel_qr(cs, mi, bi, tile + s, m, w.tauU, pw));
      RUTV_CHECK(extract_reflectors(cs, mi, bi, tile + s, m, w.WU, mi, w.R, b, true));
      comp.end(cs, a);
      RUTV_CHECK(cache.release(MT, i));
    }
    {
      hipEvent_t a = comp.begin(cs);
      RUTV_CHECK(gemm(true, false, bi, bi, mi, 1.0, w.WU, mi, w.WU, mi, 0.0, w.Gram, bi));
      RUTV_CHECK(larft_from_gram(cs, bi, w.Gram, bi, w.tauU, w.Tf, bi));
      RUTV_CHECK(gemm(false, true, mi, bi, bi, 1.0, w.WU, mi, w.Tf, bi, 0.0, w.ZU, mi));
      comp.end(cs, a);
    }
    // ---- left transform of the later tiles' rows s:m, C <- C - Z_U (W_U^T C)
    RUTV_CHECK(sweep(MT, i + 1, p, true, [&](i64 j, double* tile) {
      const i64 bj = mats[MT].width(j);
      RUTV_CHECK(gemm(true, false, bi, bj, mi, 1.0, w.WU, mi, tile + s, m, 0.0, w.X3, bi));
      return gemm(false, false, mi, bj, bi, -1.0, w.ZU, mi, w.X3, bi, 1.0, tile + s, m);
    }));
    // ---- U update (columns s:m of U)
    if (wantU) RUTV_CHECK(right(MU, w.WU, w.ZU, mi));
    // ---- b x b SVD of R and its factors on T_i, V_i, U_i
    {
      hipEvent_t a = comp.begin(cs);
      RUTV_CHECK(jacobi_svd(cs, bi, w.R, b, w.d, w.Us, w.Vs, w.jwork, &w.status[4 + 3 * i],
                            c.max_sweeps, c.spin_limit));
      RUTV_CHECK(copy_matrix(cs, bi, bi, w.Us, bi, w.Usall + i * b * b, bi));
      comp.end(cs, a);
    }
    auto right_small = [&](int mat, i64 rows, const double* S) -> int {
      if (rows <= 0) return RANDUTV_OK;
      double* tile = nullptr;
      RUTV_CHECK(cache.acquire(mat, i, true, &tile));
      hipEvent_t a = comp.begin(cs);
      RUTV_CHECK(gemm(false, false, rows, bi, bi, 1.0, tile, mats[mat].rows, S, bi, 0.0, w.X, rows));
      RUTV_CHECK(copy_matrix(cs, rows, bi, w.X, rows, tile, mats[mat].rows));
      comp.end(cs, a);
      return cache.release(mat, i);
    };
    {
      double* tile = nullptr;
      RUTV_CHECK(cache.acquire(MT, i, true, &tile));
      RUTV_CHECK(set_diag_block(cs, bi, w.d, tile + s, m));
      RUTV_CHECK(cache.release(MT, i));
    }
    RUTV_CHECK(right_small(MT, s, w.Vs));
    if (wantV) RUTV_CHECK(right_small(MV, n, w.Vs));
    if (wantU) RUTV_CHECK(right_small(MU, m, w.Us));
  }
  // ---- the deferred left factors: T_j(s_i : s_i + b_i, :) <- U_S(i)^T (...)
  // for every step i < j (later right transforms commute with them)
  RUTV_CHECK(sweep(MT, 1, p, true, [&](i64 j, double* tile) {
    const i64 bj = mats[MT].width(j);
    for (i64 i = 0; i < j; ++i) {
      const i64 s = i * b, bi = std::min(b, n - s);
      RUTV_CHECK(gemm(true, false, bi, bj, bi, 1.0, w.Usall + i * b * b, bi, tile + s, m, 0.0, w.X3, bi));
      RUTV_CHECK(copy_matrix(cs, bi, bj, w.X3, bi, tile + s, m));
    }
    return RANDUTV_OK;
  }));
  RUTV_CHECK(cache.flush());
  RUTV_TRY(hipStreamSynchronize(cs));
  RUTV_TRY(hipStreamSynchronize(xs));
  RUTV_TRY(hipStreamSynchronize(ws));
  return RANDUTV_OK;
  };
  const int rc = run();
  if (rc != RANDUTV_OK) {
    (void)hipStreamSynchronize(cs);
    (void)hipStreamSynchronize(xs);
    (void)hipStreamSynchronize(ws);
    return rc;
  }
  std::vector<int> st(4 + 3 * p);
  RUTV_TRY(hipMemcpy(st.data(), w.status, sizeof(int) * st.size(), hipMemcpyDeviceToHost));
  if (stats && stats->struct_size >= (int64_t)sizeof(randutv_ooc_stats)) {
    stats->real_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    stats->compute_ms = comp.total_ms();
    stats->h2d_ms = cache.io_in.total_ms();
    stats->d2h_ms = cache.io_out.total_ms();
    stats->io_ms = stats->h2d_ms + stats->d2h_ms;
    stats->h2d_bytes = cache.h2d_bytes;
    stats->d2h_bytes = cache.d2h_bytes;
    stats->tile_loads = cache.loads;
    stats->tile_writebacks = cache.writebacks;
    stats->tile_hits = cache.hits;
    stats->slots = nslots;
    stats->slot_bytes = (int64_t)sizeof(double) * slot_elems;
    stats->fixed_bytes = (int64_t)fixed_bytes;
  }
  if (st[1]) return RANDUTV_ERR_SYNC;
  for (i64 i = 0; i < p; ++i)
    if (st[6 + 3 * i]) return RANDUTV_ERR_SYNC;
  for (i64 i = 0; i < p; ++i)
    if (!st[5 + 3 * i]) return RANDUTV_ERR_NOCONV;
  return RANDUTV_OK;
}

}  // namespace rutv
