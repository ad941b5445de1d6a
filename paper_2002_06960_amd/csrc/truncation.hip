// The rank-k truncation A_k = U_k U_k^T A of the factorization (Section 1.1:
// T(0:k, :) V^T = U_k^T A since T = U^T A V) for 0 < k <= b_0 = min(b, n),
// where the first step (Section 3.1) already fixes U's first b_0 columns: its
// forward value from that step alone and its reverse pass (vector-Jacobian
// product) with the sketch G(0) held fixed.  One job is enqueued on a stream
// with a workspace slice of its own, so that a batch of matrices can run on
// several streams at once.
//
// k = b_0: range(U_k) = range(M), M = (A A^T)^(q+1) G(0) (the sketch and power
// iteration choose V's first block, A times that block spans range(M), the
// panel QR and the b x b SVD only rotate inside it).  With M = Q R and
// P = Q Q^T: A_k = P A, and
//   dP = (I - P) dM M^+ + (M^+)^T dM^T (I - P),  M^+ = R^{-1} Q^T,
//   Abar = P Gbar + [the chain of M reversed from Mbar = (I - P)(W + W^T) Q R^{-T}],
// W = Gbar A^T (never formed), the chain M_{j+1} = A (A^T M_j) recomputed.
//
// k < b_0: U_k holds the leading k left singular vectors of C = A Q_Y, Q_Y an
// orthonormal basis of Y = (A^T A)^q A^T G(0) (the panel Q of C times the
// b x b SVD's U_S).  With U_C = [U_1 U_2], d and lambda = d^2, the
// eigenprojector derivative of S = C C^T gives
//   Abar  = P_k Gbar + L Q_Y^T + (the power chain reversed from Ybar),
//   E     = sym(Gbar A^T) U_1,
//   H     = U_2 F + 2 (I - U_C U_C^T) E Lambda_1^-1,  F_ji = 2 (U_2^T E)_ji / (lambda_i - lambda_j),
//   L     = H (U_1^T C) + U_1 (H^T C),
//   Ybar  = (I - Q_Y Q_Y^T) A^T [H (U_1^T D) + U_1 (H^T D)],  D = C R_Y^-T,
// and the chain Z_j = A^T M_j, M_{j+1} = A Z_j (M_0 = G(0), Y = Z_q) reversed:
// Abar += M_j Zbar_j^T, Mbar_j = A Zbar_j, Abar += Mbar_j Z_{j-1}^T,
// Zbar_{j-1} = A^T Mbar_j.
//
// b_0 < k <= b_0 + b_1: U's second block comes from step 1, which sketches
// B_1 = U_perp^T A V_perp in the coordinates of step 0's Householder
// complements (U_perp = H(:, b_0:) of the panel QR of C_0 = A Q_V, V_perp of
// the QR of Y_0).  In A's space its sketch is Gamma = U_perp G(1) =
// [0; G(1)] - W T W_2^T G(1) (W, T the reflectors and block factor of C_0), its
// powered sketch Yt = Pi_V (A^T Pi_U A Pi_V)^q A^T Gamma (Pi_U = I - Q_H Q_H^T,
// Pi_V = I - Q_V Q_V^T), and U's second block holds the left singular vectors
// of C_1 = Pi_U A orth(Yt): A_k = Q_H Q_H^T A + U_2 U_2^T A, U_2 the leading
// k - b_0 of them.  The reverse pass runs every piece backwards: the
// eigenprojector of C_1 C_1^T as above, the projections Pi_U and Pi_V, the
// power chain of Yt, Gamma through the unpivoted LU [I; 0] - Q_H = W (T W_1^T)
// that ties the reflectors to Q_H (Gamma = [0; G(1)] - M W_1^{-T} W_2^T G(1),
// M = [I; 0] - Q_H), the thin QRs of C_0 and Y_0 (for C = Q R with Rbar = 0:
// Cbar = [Qbar - Q (N - P_L(N - N^T))] R^{-T}, N = Q^T Qbar, P_L the strictly
// lower part), and the chain of Y_0.
#include <algorithm>
#include <array>
#include <vector>

#include "kernels.hpp"

namespace rutv {

namespace {

struct Carve {
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

// the second block's buffers (b_0 < k <= b_0 + b_1)
struct TwoWS {
  double *G1, *Qv, *Rv, *RvInv, *C0, *Qh, *Rh, *RhInv, *Wh, *Tfh, *Ulu, *UluInv, *W1T, *W1TInv, *Xg,
      *Vg, *Gam, *Qt, *Rt, *RtInv, *D1, *C1, *Qc, *Rc, *d, *lam, *Us, *Vs, *Uc, *QhB, *QvB, *E2, *H2,
      *X1, *P1, *P2, *C1B, *D1B, *NB, *NB2, *MB, *MB2, *Mbar, *SQ, *SQ2, *SQ3, *Y2b, *W1b, *W2b, *BigM,
      *BigN;
  std::vector<double*> Yt, Vt, At, Ut;
};

struct TruncWS {
  std::vector<double*> Mj, Zj;
  double *Qy, *Ry, *RyInv, *C, *Fp, *tau, *Wr, *Gram, *Tf, *X, *Rc, *Qc, *d, *lam, *Us, *Vs, *jw,
      *Uc, *T1, *E, *H, *X1, *W1, *W2, *L, *D, *Yb, *Zb, *Mb, *Cn, *S, *wk;
  unsigned long long* xch;
  i64 sk;
  TwoWS two;
};

i64 trunc_splitk(i64 m, i64 n, i64 bb, i64 k, i64 b1, i64 k2) {
  i64 sk = 0;
  for (auto s3 : {std::array<i64, 3>{n, bb, m}, {m, bb, n}, {bb, bb, m}, {bb, bb, n}, {bb, bb, bb},
                  {m, bb, bb}, {n, bb, bb}, {k, n, m}, {m, n, k}, {m, n, bb}, {n, k, m}, {m, k, n},
                  {bb, k, m}, {m, k, bb}, {k, bb, m}, {m, bb, k}, {bb, n, m}})
    sk = std::max(sk, dgemm_work_elems(s3[0], s3[1], s3[2]));
  if (b1 > 0) {
    for (auto s3 : {std::array<i64, 3>{n, b1, m}, {m, b1, n}, {b1, b1, m}, {b1, b1, n},
                    {bb, b1, m - bb}, {bb, b1, bb}, {m, b1, bb}, {bb, b1, m}, {bb, b1, n},
                    {n, k2, m}, {m, k2, n}, {b1, k2, m}, {m, k2, b1}, {k2, b1, m}, {m, b1, k2},
                    {k2, n, m}, {m, n, k2}, {m, n, b1}, {n, bb, m}, {m, bb, b1}, {n, bb, b1},
                    {bb, bb, m}, {m - bb, bb, b1}, {bb, bb, m - bb}})
      sk = std::max(sk, dgemm_work_elems(s3[0], s3[1], s3[2]));
  }
  return sk;
}

size_t trunc_layout(Carve& c, const TruncJob& j, TruncWS& w) {
  const i64 m = j.m, n = j.n, bb = std::min(j.b, n), k = j.k, mx = std::max(m, n);
  // the reverse pass keeps every product of the power chain; the forward
  // value needs two of each
  const int nm = j.reverse ? j.q + 2 : 2, nz = j.reverse ? j.q + 1 : 2;
  w.Mj.assign(nm, nullptr);
  w.Zj.assign(nz, nullptr);
  for (int t = 0; t < nm; ++t) w.Mj[t] = c.take<double>(m * bb);
  for (int t = 0; t < nz; ++t) w.Zj[t] = c.take<double>(n * bb);
  w.Qy = c.take<double>(mx * bb);
  w.Ry = c.take<double>(bb * bb);
  w.RyInv = c.take<double>(bb * bb);
  w.C = c.take<double>(m * bb);
  w.Fp = c.take<double>(mx * bb);
  w.tau = c.take<double>(bb);
  w.Wr = c.take<double>(mx * bb);
  w.Gram = c.take<double>(bb * bb);
  w.Tf = c.take<double>(bb * bb);
  w.X = c.take<double>(bb * bb);
  w.Rc = c.take<double>(bb * bb);
  w.Qc = c.take<double>(m * bb);
  w.d = c.take<double>(bb);
  w.lam = c.take<double>(bb);
  w.Us = c.take<double>(bb * bb);
  w.Vs = c.take<double>(bb * bb);
  w.jw = c.take<double>(jacobi_work_elems(bb));
  w.Uc = c.take<double>(m * bb);
  w.T1 = c.take<double>(n * bb);
  w.E = c.take<double>(m * k);
  w.H = c.take<double>(m * k);
  w.X1 = c.take<double>(bb * k);
  w.W1 = c.take<double>(k * bb);
  w.W2 = c.take<double>(k * bb);
  w.L = c.take<double>(m * bb);
  w.D = c.take<double>(m * bb);
  w.Yb = c.take<double>(n * bb);
  w.Zb = c.take<double>(n * bb);
  w.Mb = c.take<double>(m * bb);
  w.Cn = c.take<double>(bb * n);
  w.S = c.take<double>(m * bb);
  const i64 b1_ = k > bb ? std::min(j.b, n - bb) : 0;
  w.sk = trunc_splitk(m, n, bb, k, b1_, k > bb ? k - bb : 0);
  w.wk = c.take<double>(w.sk);
  w.xch = c.take<unsigned long long>(panel_work_elems(mx));
  if (k > bb) {  // the second block (step 1)
    const i64 b1 = std::min(j.b, n - bb);
    TwoWS& t = w.two;
    t.G1 = c.take<double>((m - bb) * b1);
    t.Qv = c.take<double>(n * bb);
    t.Rv = c.take<double>(bb * bb);
    t.RvInv = c.take<double>(bb * bb);
    t.C0 = c.take<double>(m * bb);
    t.Qh = c.take<double>(m * bb);
    t.Rh = c.take<double>(bb * bb);
    t.RhInv = c.take<double>(bb * bb);
    t.Wh = c.take<double>(m * bb);
    t.Tfh = c.take<double>(bb * bb);
    t.Ulu = c.take<double>(bb * bb);
    t.UluInv = c.take<double>(bb * bb);
    t.W1T = c.take<double>(bb * bb);
    t.W1TInv = c.take<double>(bb * bb);
    t.Xg = c.take<double>(bb * b1);
    t.Vg = c.take<double>(bb * b1);
    t.Gam = c.take<double>(m * b1);
    t.Yt.assign(j.q + 1, nullptr);
    t.Vt.assign(j.q + 1, nullptr);
    t.At.assign(std::max(j.q, 1), nullptr);
    t.Ut.assign(std::max(j.q, 1), nullptr);
    for (int r = 0; r <= j.q; ++r) t.Yt[r] = c.take<double>(n * b1);
    for (int r = 0; r <= j.q; ++r) t.Vt[r] = c.take<double>(n * b1);
    for (int r = 0; r < std::max(j.q, 1); ++r) t.At[r] = c.take<double>(m * b1);
    for (int r = 0; r < std::max(j.q, 1); ++r) t.Ut[r] = c.take<double>(m * b1);
    t.Qt = c.take<double>(n * b1);
    t.Rt = c.take<double>(b1 * b1);
    t.RtInv = c.take<double>(b1 * b1);
    t.D1 = c.take<double>(m * b1);
    t.C1 = c.take<double>(m * b1);
    t.Qc = c.take<double>(m * b1);
    t.Rc = c.take<double>(b1 * b1);
    t.d = c.take<double>(b1);
    t.lam = c.take<double>(b1);
    t.Us = c.take<double>(b1 * b1);
    t.Vs = c.take<double>(b1 * b1);
    t.Uc = c.take<double>(m * b1);
    t.QhB = c.take<double>(m * bb);
    t.QvB = c.take<double>(n * bb);
    t.E2 = c.take<double>(m * b1);
    t.H2 = c.take<double>(m * b1);
    t.X1 = c.take<double>(b1 * b1);
    t.P1 = c.take<double>(b1 * b1);
    t.P2 = c.take<double>(b1 * b1);
    t.C1B = c.take<double>(m * b1);
    t.D1B = c.take<double>(m * b1);
    t.NB = c.take<double>(n * b1);
    t.NB2 = c.take<double>(n * b1);
    t.MB = c.take<double>(m * b1);
    t.MB2 = c.take<double>(m * b1);
    t.Mbar = c.take<double>(m * bb);
    t.SQ = c.take<double>(std::max(bb, b1) * std::max(bb, b1));
    t.SQ2 = c.take<double>(std::max(bb, b1) * std::max(bb, b1));
    t.SQ3 = c.take<double>(std::max(bb, b1) * std::max(bb, b1));
    t.Y2b = c.take<double>(bb * b1);
    t.W1b = c.take<double>(bb * bb);
    t.W2b = c.take<double>((m - bb) * bb);
    t.BigM = c.take<double>(mx * bb);
    t.BigN = c.take<double>(mx * bb);
  }
  return c.off;
}

}  // namespace

size_t trunc_ws_bytes(const TruncJob& j) {
  Carve c;
  TruncWS w;
  return trunc_layout(c, j, w);
}

// b_0 < k <= b_0 + b_1 (see the notes at the top of the file)
template <class MM, class QR, class MT, class ZT>
static int two_blocks(const TruncJob& j, hipStream_t st, TruncWS& w, int* status, MM& mm, QR& qr_explicit,
                      MT& Mt, ZT& Zt) {
  const i64 m = j.m, n = j.n, bb = std::min(j.b, n), b1 = std::min(j.b, n - bb), k2 = j.k - bb,
            r3 = b1 - k2;
  const int q = j.q;
  const double* A = j.A;
  const i64 lda = j.lda;
  TwoWS& t = w.two;
  // ---- forward: Y_0 chain, Q_V, C_0 = A Q_V, Q_H with its reflectors
  for (int r = 0; r <= q; ++r) {
    RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, Mt(r), m, 0.0, Zt(r), n));
    if (r < q) RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, Zt(r), n, 0.0, Mt(r + 1), m));
  }
  RUTV_CHECK(qr_explicit(n, Zt(q), t.Qv, t.Rv));
  RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, t.Qv, n, 0.0, t.C0, m));
  RUTV_CHECK(qr_explicit(m, t.C0, t.Qh, t.Rh));
  RUTV_CHECK(copy_matrix(st, m, bb, w.Wr, m, t.Wh, m));  // the reflectors of C_0 and their factor
  RUTV_CHECK(copy_matrix(st, bb, bb, w.Tf, bb, t.Tfh, bb));
  // Gamma = U_perp G(1) = [0; G(1)] - W (T (W_2^T G(1)))
  RUTV_CHECK(sketch(st, j.seed, 1, m - bb, b1, t.G1, m - bb));
  RUTV_CHECK(mm(true, false, bb, b1, m - bb, 1.0, t.Wh + bb, m, t.G1, m - bb, 0.0, t.Y2b, bb));
  RUTV_CHECK(mm(false, false, bb, b1, bb, 1.0, t.Tfh, bb, t.Y2b, bb, 0.0, t.Vg, bb));
  RUTV_CHECK(zero_matrix(st, bb, b1, t.Gam, m));
  RUTV_CHECK(copy_matrix(st, m - bb, b1, t.G1, m - bb, t.Gam + bb, m));
  RUTV_CHECK(mm(false, false, m, b1, bb, -1.0, t.Wh, m, t.Vg, bb, 1.0, t.Gam, m));
  // projections Pi(X) = X - Q (Q^T X) (cols columns of rows rows)
  auto proj = [&](const double* Q, i64 rows, i64 qcols, const double* X, double* Y, i64 cols) -> int {
    if (Y != X) RUTV_CHECK(copy_matrix(st, rows, cols, X, rows, Y, rows));
    RUTV_CHECK(mm(true, false, qcols, cols, rows, 1.0, Q, rows, X, rows, 0.0, t.SQ3, qcols));
    return mm(false, false, rows, cols, qcols, -1.0, Q, rows, t.SQ3, qcols, 1.0, Y, rows);
  };
  // Yt chain: V_0 = A^T Gamma, Yt_0 = Pi_V V_0; A_r = A Yt_r, U_r = Pi_U A_r,
  // V_{r+1} = A^T U_r, Yt_{r+1} = Pi_V V_{r+1}
  RUTV_CHECK(mm(true, false, n, b1, m, 1.0, A, lda, t.Gam, m, 0.0, t.Vt[0], n));
  RUTV_CHECK(proj(t.Qv, n, bb, t.Vt[0], t.Yt[0], b1));
  for (int r = 0; r < q; ++r) {
    RUTV_CHECK(mm(false, false, m, b1, n, 1.0, A, lda, t.Yt[r], n, 0.0, t.At[r], m));
    RUTV_CHECK(proj(t.Qh, m, bb, t.At[r], t.Ut[r], b1));
    RUTV_CHECK(mm(true, false, n, b1, m, 1.0, A, lda, t.Ut[r], m, 0.0, t.Vt[r + 1], n));
    RUTV_CHECK(proj(t.Qv, n, bb, t.Vt[r + 1], t.Yt[r + 1], b1));
  }
  // Q_t = orth(Yt_q); D_1 = A Q_t; C_1 = Pi_U D_1; its SVD through QR + Jacobi
  PanelWork pw;
  pw.xch = w.xch;
  pw.err = &status[1];
  auto qr_cols = [&](i64 rows, i64 cols, const double* P, double* Qo, double* Ro) -> int {
    RUTV_CHECK(copy_matrix(st, rows, cols, P, rows, w.Fp, rows));
    RUTV_CHECK(panel_qr(st, rows, cols, w.Fp, rows, w.tau, pw));
    RUTV_CHECK(extract_reflectors(st, rows, cols, w.Fp, rows, w.Wr, rows, Ro, cols, false));
    RUTV_CHECK(mm(true, false, cols, cols, rows, 1.0, w.Wr, rows, w.Wr, rows, 0.0, w.Gram, cols));
    RUTV_CHECK(larft_from_gram(st, cols, w.Gram, cols, w.tau, w.Tf, cols));
    RUTV_CHECK(mm(false, true, cols, cols, cols, 1.0, w.Tf, cols, w.Wr, rows, 0.0, w.X, cols));
    RUTV_CHECK(set_eye(st, rows, cols, Qo, rows));
    return mm(false, false, rows, cols, cols, -1.0, w.Wr, rows, w.X, cols, 1.0, Qo, rows);
  };
  RUTV_CHECK(qr_cols(n, b1, t.Yt[q], t.Qt, t.Rt));
  RUTV_CHECK(mm(false, false, m, b1, n, 1.0, A, lda, t.Qt, n, 0.0, t.D1, m));
  RUTV_CHECK(proj(t.Qh, m, bb, t.D1, t.C1, b1));
  RUTV_CHECK(qr_cols(m, b1, t.C1, t.Qc, t.Rc));
  RUTV_CHECK(jacobi_svd(st, b1, t.Rc, b1, t.d, t.Us, t.Vs, w.jw, &status[4]));
  RUTV_CHECK(square_vec(st, b1, t.d, t.lam));
  RUTV_CHECK(mm(false, false, m, b1, b1, 1.0, t.Qc, m, t.Us, b1, 0.0, t.Uc, m));
  const double* U2 = t.Uc;
  const double* U3 = t.Uc + k2 * m;
  if (!j.reverse) {  // A_k = Q_H (Q_H^T A) + U_2 (U_2^T A)
    RUTV_CHECK(mm(true, false, bb, n, m, 1.0, t.Qh, m, A, lda, 0.0, w.Cn, bb));
    RUTV_CHECK(mm(false, false, m, n, bb, 1.0, t.Qh, m, w.Cn, bb, 0.0, j.out, j.ldo));
    RUTV_CHECK(mm(true, false, k2, n, m, 1.0, U2, m, A, lda, 0.0, w.Cn, k2));
    return mm(false, false, m, n, k2, 1.0, U2, m, w.Cn, k2, 1.0, j.out, j.ldo);
  }
  double* Abar = j.out;
  const i64 ldab = j.ldo;
  const double* Gbar = j.Gbar;
  const i64 ldg = j.ldg;
  // ---- reverse
  // Abar = Q_H (Q_H^T Gbar) + U_2 (U_2^T Gbar); Qbar_H = Gbar (A^T Q_H) + A (Gbar^T Q_H)
  RUTV_CHECK(mm(true, false, bb, n, m, 1.0, t.Qh, m, Gbar, ldg, 0.0, w.Cn, bb));
  RUTV_CHECK(mm(false, false, m, n, bb, 1.0, t.Qh, m, w.Cn, bb, 0.0, Abar, ldab));
  RUTV_CHECK(mm(true, false, k2, n, m, 1.0, U2, m, Gbar, ldg, 0.0, w.Cn, k2));
  RUTV_CHECK(mm(false, false, m, n, k2, 1.0, U2, m, w.Cn, k2, 1.0, Abar, ldab));
  RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, t.Qh, m, 0.0, t.BigN, n));
  RUTV_CHECK(mm(false, false, m, bb, n, 1.0, Gbar, ldg, t.BigN, n, 0.0, t.QhB, m));
  RUTV_CHECK(mm(true, false, n, bb, m, 1.0, Gbar, ldg, t.Qh, m, 0.0, t.BigN, n));
  RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, t.BigN, n, 1.0, t.QhB, m));
  RUTV_CHECK(zero_matrix(st, n, bb, t.QvB, n));
  // eigenprojector of C_1 C_1^T: E_2 = sym(Gbar A^T) U_2; H_2; Cbar_1
  RUTV_CHECK(mm(true, false, n, k2, m, 1.0, A, lda, U2, m, 0.0, t.NB, n));
  RUTV_CHECK(mm(false, false, m, k2, n, 0.5, Gbar, ldg, t.NB, n, 0.0, t.E2, m));
  RUTV_CHECK(mm(true, false, n, k2, m, 1.0, Gbar, ldg, U2, m, 0.0, t.NB, n));
  RUTV_CHECK(mm(false, false, m, k2, n, 0.5, A, lda, t.NB, n, 1.0, t.E2, m));
  RUTV_CHECK(mm(true, false, b1, k2, m, 1.0, t.Uc, m, t.E2, m, 0.0, t.X1, b1));
  RUTV_CHECK(copy_matrix(st, m, k2, t.E2, m, t.H2, m));
  RUTV_CHECK(mm(false, false, m, k2, b1, -1.0, t.Uc, m, t.X1, b1, 1.0, t.H2, m));
  RUTV_CHECK(scale_cols(st, m, k2, t.H2, m, t.lam, 2.0, &status[2]));
  if (r3 > 0) {
    RUTV_CHECK(gap_divide(st, r3, k2, t.X1 + k2, b1, t.d, &status[2]));
    RUTV_CHECK(mm(false, false, m, k2, r3, 1.0, U3, m, t.X1 + k2, b1, 1.0, t.H2, m));
  }
  RUTV_CHECK(mm(true, false, k2, b1, m, 1.0, U2, m, t.C1, m, 0.0, t.P1, k2));
  RUTV_CHECK(mm(true, false, k2, b1, m, 1.0, t.H2, m, t.C1, m, 0.0, t.P2, k2));
  RUTV_CHECK(mm(false, false, m, b1, k2, 1.0, t.H2, m, t.P1, k2, 0.0, t.C1B, m));
  RUTV_CHECK(mm(false, false, m, b1, k2, 1.0, U2, m, t.P2, k2, 1.0, t.C1B, m));
  // C_1 = Pi_U D_1: Dbar_1 = Pi_U Cbar_1, Qbar_H -= Cbar_1 (D_1^T Q_H) + D_1 (Cbar_1^T Q_H)
  auto proj_bar = [&](const double* Q, double* QB, i64 rows, i64 qcols, const double* Xbar,
                      const double* X, i64 cols) -> int {
    RUTV_CHECK(mm(true, false, cols, qcols, rows, 1.0, X, rows, Q, rows, 0.0, t.SQ, cols));
    RUTV_CHECK(mm(false, false, rows, qcols, cols, -1.0, Xbar, rows, t.SQ, cols, 1.0, QB, rows));
    RUTV_CHECK(mm(true, false, cols, qcols, rows, 1.0, Xbar, rows, Q, rows, 0.0, t.SQ2, cols));
    return mm(false, false, rows, qcols, cols, -1.0, X, rows, t.SQ2, cols, 1.0, QB, rows);
  };
  RUTV_CHECK(proj(t.Qh, m, bb, t.C1B, t.D1B, b1));
  RUTV_CHECK(proj_bar(t.Qh, t.QhB, m, bb, t.C1B, t.D1, b1));
  // D_1 = A Q_t: Abar += Dbar_1 Q_t^T; Qbar_t = A^T Dbar_1; Ytbar = (I - Q_t Q_t^T) Qbar_t R_t^{-T}
  RUTV_CHECK(mm(false, true, m, n, b1, 1.0, t.D1B, m, t.Qt, n, 1.0, Abar, ldab));
  RUTV_CHECK(mm(true, false, n, b1, m, 1.0, A, lda, t.D1B, m, 0.0, t.NB, n));
  RUTV_CHECK(tri_inverse(st, b1, t.Rt, b1, t.RtInv, b1, &status[2]));
  RUTV_CHECK(mm(false, true, n, b1, b1, 1.0, t.NB, n, t.RtInv, b1, 0.0, t.NB2, n));
  double* Ytb = t.NB;
  RUTV_CHECK(proj(t.Qt, n, b1, t.NB2, Ytb, b1));
  // the Yt chain reversed
  for (int r = q - 1; r >= 0; --r) {
    // Yt_{r+1} = Pi_V V_{r+1}
    double* Vb = t.NB2;
    RUTV_CHECK(proj(t.Qv, n, bb, Ytb, Vb, b1));
    RUTV_CHECK(proj_bar(t.Qv, t.QvB, n, bb, Ytb, t.Vt[r + 1], b1));
    // V_{r+1} = A^T U_r
    RUTV_CHECK(mm(false, true, m, n, b1, 1.0, t.Ut[r], m, Vb, n, 1.0, Abar, ldab));
    RUTV_CHECK(mm(false, false, m, b1, n, 1.0, A, lda, Vb, n, 0.0, t.MB, m));
    // U_r = Pi_U A_r
    RUTV_CHECK(proj(t.Qh, m, bb, t.MB, t.MB2, b1));
    RUTV_CHECK(proj_bar(t.Qh, t.QhB, m, bb, t.MB, t.At[r], b1));
    // A_r = A Yt_r
    RUTV_CHECK(mm(false, true, m, n, b1, 1.0, t.MB2, m, t.Yt[r], n, 1.0, Abar, ldab));
    RUTV_CHECK(mm(true, false, n, b1, m, 1.0, A, lda, t.MB2, m, 0.0, Ytb, n));
  }
  // Yt_0 = Pi_V V_0, V_0 = A^T Gamma
  RUTV_CHECK(proj(t.Qv, n, bb, Ytb, t.NB2, b1));
  RUTV_CHECK(proj_bar(t.Qv, t.QvB, n, bb, Ytb, t.Vt[0], b1));
  RUTV_CHECK(mm(false, true, m, n, b1, 1.0, t.Gam, m, t.NB2, n, 1.0, Abar, ldab));
  double* GamB = t.MB;
  RUTV_CHECK(mm(false, false, m, b1, n, 1.0, A, lda, t.NB2, n, 0.0, GamB, m));
  // Gamma = [0; G(1)] - M X, M = [I; 0] - Q_H, X = W_1^{-T} (W_2^T G(1)):
  // Mbar = -Gammabar X^T, Xbar = -M^T Gammabar
  RUTV_CHECK(copy_matrix(st, bb, bb, t.Wh, m, t.SQ, bb));
  RUTV_CHECK(transpose_square(st, bb, t.SQ, t.W1T));
  RUTV_CHECK(tri_inverse(st, bb, t.W1T, bb, t.W1TInv, bb, &status[3]));
  RUTV_CHECK(mm(false, false, bb, b1, bb, 1.0, t.W1TInv, bb, t.Y2b, bb, 0.0, t.Xg, bb));
  RUTV_CHECK(mm(false, true, m, bb, b1, -1.0, GamB, m, t.Xg, bb, 0.0, t.Mbar, m));
  // Xbar = Q_H^T Gammabar - Gammabar(0:b_0) (into SQ2, bb x b1)
  RUTV_CHECK(mm(true, false, bb, b1, m, 1.0, t.Qh, m, GamB, m, 0.0, t.SQ2, bb));
  RUTV_CHECK(axpy_matrix(st, bb, b1, -1.0, GamB, m, t.SQ2, bb));
  // X = W_1^{-T} Y_2: Ybar_2 = W_1^{-1} Xbar; W_1bar = P_L(-X Ybar_2^T); Y_2 = W_2^T G(1): W_2bar = G(1) Ybar_2^T
  double* Yb2 = t.Vg;
  RUTV_CHECK(mm(true, false, bb, b1, bb, 1.0, t.W1TInv, bb, t.SQ2, bb, 0.0, Yb2, bb));
  RUTV_CHECK(mm(false, true, bb, bb, b1, -1.0, t.Xg, bb, Yb2, bb, 0.0, t.SQ, bb));
  RUTV_CHECK(tri_combine(st, bb, t.SQ, nullptr, t.W1b, 2));
  RUTV_CHECK(mm(false, true, m - bb, bb, b1, 1.0, t.G1, m - bb, Yb2, bb, 0.0, t.W2b, m - bb));
  // the unpivoted LU M = W U (U = T W_1^T) backwards:
  // Psi = P_L(W_1^T W_1bar) - triu(W_2^T W_2bar), Mbar_1 += W_1^{-T} Psi U^{-T}, Mbar_2 += W_2bar U^{-T}
  RUTV_CHECK(mm(true, false, bb, bb, bb, 1.0, t.Wh, m, t.W1b, bb, 0.0, t.SQ, bb));
  RUTV_CHECK(mm(true, false, bb, bb, m - bb, 1.0, t.Wh + bb, m, t.W2b, m - bb, 0.0, t.SQ2, bb));
  RUTV_CHECK(tri_combine(st, bb, t.SQ, t.SQ2, t.SQ3, 1));
  RUTV_CHECK(mm(false, false, bb, bb, bb, 1.0, t.Tfh, bb, t.W1T, bb, 0.0, t.Ulu, bb));
  RUTV_CHECK(tri_inverse(st, bb, t.Ulu, bb, t.UluInv, bb, &status[2]));
  RUTV_CHECK(mm(false, true, bb, bb, bb, 1.0, t.SQ3, bb, t.UluInv, bb, 0.0, t.SQ, bb));
  RUTV_CHECK(mm(false, false, bb, bb, bb, 1.0, t.W1TInv, bb, t.SQ, bb, 1.0, t.Mbar, m));
  RUTV_CHECK(mm(false, true, m - bb, bb, bb, 1.0, t.W2b, m - bb, t.UluInv, bb, 1.0, t.Mbar + bb, m));
  // M = [I; 0] - Q_H: Qbar_H -= Mbar
  RUTV_CHECK(axpy_matrix(st, m, bb, -1.0, t.Mbar, m, t.QhB, m));
  // thin QR backwards (Rbar = 0): Cbar = [Qbar - Q (N - P_L(N - N^T))] R^{-T}, N = Q^T Qbar
  auto qr_bar = [&](i64 rows, const double* Q, const double* QB, const double* R, double* RInv,
                    double* out) -> int {
    RUTV_CHECK(mm(true, false, bb, bb, rows, 1.0, Q, rows, QB, rows, 0.0, t.SQ, bb));
    RUTV_CHECK(tri_combine(st, bb, t.SQ, nullptr, t.SQ2, 0));
    RUTV_CHECK(axpy_matrix(st, bb, bb, -1.0, t.SQ2, bb, t.SQ, bb));
    RUTV_CHECK(copy_matrix(st, rows, bb, QB, rows, t.BigM, rows));
    RUTV_CHECK(mm(false, false, rows, bb, bb, -1.0, Q, rows, t.SQ, bb, 1.0, t.BigM, rows));
    RUTV_CHECK(tri_inverse(st, bb, R, bb, RInv, bb, &status[2]));
    return mm(false, true, rows, bb, bb, 1.0, t.BigM, rows, RInv, bb, 0.0, out, rows);
  };
  double* C0B = t.Mbar;
  RUTV_CHECK(qr_bar(m, t.Qh, t.QhB, t.Rh, t.RhInv, C0B));
  // C_0 = A Q_V: Abar += Cbar_0 Q_V^T; Qbar_V += A^T Cbar_0
  RUTV_CHECK(mm(false, true, m, n, bb, 1.0, C0B, m, t.Qv, n, 1.0, Abar, ldab));
  RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, C0B, m, 1.0, t.QvB, n));
  // Q_V of Y_0 = Z_q, then the chain of Y_0 reversed
  RUTV_CHECK(qr_bar(n, t.Qv, t.QvB, t.Rv, t.RvInv, t.BigN));
  for (int r = q; r >= 0; --r) {
    RUTV_CHECK(mm(false, true, m, n, bb, 1.0, Mt(r), m, t.BigN, n, 1.0, Abar, ldab));
    if (r == 0) break;
    RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, t.BigN, n, 0.0, t.BigM, m));
    RUTV_CHECK(mm(false, true, m, n, bb, 1.0, t.BigM, m, Zt(r - 1), n, 1.0, Abar, ldab));
    RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, t.BigM, m, 0.0, t.BigN, n));
  }
  return RANDUTV_OK;
}

int trunc_enqueue(const TruncJob& j, hipStream_t st, char* base, int* status) {
  const i64 m = j.m, n = j.n, bb = std::min(j.b, n), k = j.k;
  const int q = j.q;
  const double* A = j.A;
  const i64 lda = j.lda;
  Carve c;
  c.base = base;
  TruncWS w;
  trunc_layout(c, j, w);
  auto mm = [&](bool ta, bool tb, i64 M_, i64 N_, i64 K_, double alpha, const double* A_, i64 la,
                const double* B_, i64 lb, double beta, double* C_, i64 lc) {
    return dgemm(st, ta, tb, M_, N_, K_, alpha, A_, la, B_, lb, beta, C_, lc, w.wk, w.sk);
  };
  PanelWork pw;
  pw.xch = w.xch;
  pw.err = &status[1];
  // Householder QR of P (rows x bb, ld rows, copied to Fp): explicit Q (rows x
  // bb) = [I; 0] - W (Tf W_1^T), and R (bb x bb)
  auto qr_explicit = [&](i64 rows, const double* P, double* Qo, double* Ro) -> int {
    RUTV_CHECK(copy_matrix(st, rows, bb, P, rows, w.Fp, rows));
    RUTV_CHECK(panel_qr(st, rows, bb, w.Fp, rows, w.tau, pw));
    RUTV_CHECK(extract_reflectors(st, rows, bb, w.Fp, rows, w.Wr, rows, Ro, bb, false));
    RUTV_CHECK(mm(true, false, bb, bb, rows, 1.0, w.Wr, rows, w.Wr, rows, 0.0, w.Gram, bb));
    RUTV_CHECK(larft_from_gram(st, bb, w.Gram, bb, w.tau, w.Tf, bb));
    RUTV_CHECK(mm(false, true, bb, bb, bb, 1.0, w.Tf, bb, w.Wr, rows, 0.0, w.X, bb));
    RUTV_CHECK(set_eye(st, rows, bb, Qo, rows));
    return mm(false, false, rows, bb, bb, -1.0, w.Wr, rows, w.X, bb, 1.0, Qo, rows);
  };
  RUTV_CHECK(fill_zero_u32(st, reinterpret_cast<unsigned*>(status), 8));
  RUTV_CHECK(check_finite(st, m, n, A, lda, &status[0]));
  if (j.reverse) RUTV_CHECK(check_finite(st, m, n, j.Gbar, j.ldg, &status[0]));
  RUTV_CHECK(sketch(st, j.seed, 0, m, bb, w.Mj[0], m));
  // buffers of M_t and Z_t: all kept for the reverse pass, alternating for
  // the forward value
  auto Mt = [&](int t) { return j.reverse ? w.Mj[t] : w.Mj[t & 1]; };
  auto Zt = [&](int t) { return j.reverse ? w.Zj[t] : w.Zj[t & 1]; };

  if (k == bb) {
    // chain M_{t+1} = A (A^T M_t); M = M_{q+1} = Q R
    for (int t = 0; t <= q; ++t) {
      RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, Mt(t), m, 0.0, Zt(t), n));
      RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, Zt(t), n, 0.0, Mt(t + 1), m));
    }
    RUTV_CHECK(qr_explicit(m, Mt(q + 1), w.Qc, w.Rc));
    const double* Q = w.Qc;
    if (!j.reverse) {  // A_k = Q (Q^T A)
      RUTV_CHECK(mm(true, false, bb, n, m, 1.0, Q, m, A, lda, 0.0, w.Cn, bb));
      return mm(false, false, m, n, bb, 1.0, Q, m, w.Cn, bb, 0.0, j.out, j.ldo);
    }
    // Qt = Q R^{-T} = (M^+)^T
    RUTV_CHECK(tri_inverse(st, bb, w.Rc, bb, w.RyInv, bb, &status[2]));
    double* Qt = w.D;
    RUTV_CHECK(mm(false, true, m, bb, bb, 1.0, Q, m, w.RyInv, bb, 0.0, Qt, m));
    // S = (W + W^T) Qt = Gbar (A^T Qt) + A (Gbar^T Qt); Mbar = S - Q (Q^T S)
    double* S = w.S;
    RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, Qt, m, 0.0, w.T1, n));
    RUTV_CHECK(mm(false, false, m, bb, n, 1.0, j.Gbar, j.ldg, w.T1, n, 0.0, S, m));
    RUTV_CHECK(mm(true, false, n, bb, m, 1.0, j.Gbar, j.ldg, Qt, m, 0.0, w.T1, n));
    RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, w.T1, n, 1.0, S, m));
    RUTV_CHECK(mm(true, false, bb, bb, m, 1.0, Q, m, S, m, 0.0, w.X, bb));
    RUTV_CHECK(mm(false, false, m, bb, bb, -1.0, Q, m, w.X, bb, 1.0, S, m));
    // Abar = P Gbar, then the chain of M in reverse
    RUTV_CHECK(mm(true, false, bb, n, m, 1.0, Q, m, j.Gbar, j.ldg, 0.0, w.Cn, bb));
    RUTV_CHECK(mm(false, false, m, n, bb, 1.0, Q, m, w.Cn, bb, 0.0, j.out, j.ldo));
    for (int t = q; t >= 0; --t) {
      RUTV_CHECK(mm(false, true, m, n, bb, 1.0, S, m, w.Zj[t], n, 1.0, j.out, j.ldo));
      RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, S, m, 0.0, w.Zb, n));
      RUTV_CHECK(mm(false, true, m, n, bb, 1.0, w.Mj[t], m, w.Zb, n, 1.0, j.out, j.ldo));
      if (t > 0) RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, w.Zb, n, 0.0, S, m));
    }
    return RANDUTV_OK;
  }

  if (k > bb) return two_blocks(j, st, w, status, mm, qr_explicit, Mt, Zt);

  // ---- k < b_0: Z_t = A^T M_t, M_{t+1} = A Z_t; Y = Z_q
  for (int t = 0; t <= q; ++t) {
    RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, Mt(t), m, 0.0, Zt(t), n));
    if (t < q) RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, Zt(t), n, 0.0, Mt(t + 1), m));
  }
  RUTV_CHECK(qr_explicit(n, Zt(q), w.Qy, w.Ry));
  if (j.reverse) RUTV_CHECK(tri_inverse(st, bb, w.Ry, bb, w.RyInv, bb, &status[2]));
  RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, w.Qy, n, 0.0, w.C, m));
  RUTV_CHECK(qr_explicit(m, w.C, w.Qc, w.Rc));
  RUTV_CHECK(jacobi_svd(st, bb, w.Rc, bb, w.d, w.Us, w.Vs, w.jw, &status[4]));
  RUTV_CHECK(square_vec(st, bb, w.d, w.lam));
  RUTV_CHECK(mm(false, false, m, bb, bb, 1.0, w.Qc, m, w.Us, bb, 0.0, w.Uc, m));
  const i64 r2 = bb - k;
  const double* U1 = w.Uc;
  const double* U2 = w.Uc + k * m;
  if (!j.reverse) {  // A_k = U_1 (U_1^T A)
    RUTV_CHECK(mm(true, false, k, n, m, 1.0, U1, m, A, lda, 0.0, w.Cn, k));
    return mm(false, false, m, n, k, 1.0, U1, m, w.Cn, k, 0.0, j.out, j.ldo);
  }
  double* Abar = j.out;
  const i64 ldab = j.ldo;
  const double* Gbar = j.Gbar;
  const i64 ldg = j.ldg;
  // Abar = U_1 (U_1^T Gbar)
  RUTV_CHECK(mm(true, false, k, n, m, 1.0, U1, m, Gbar, ldg, 0.0, w.Cn, k));
  RUTV_CHECK(mm(false, false, m, n, k, 1.0, U1, m, w.Cn, k, 0.0, Abar, ldab));
  // E = (Gbar (A^T U_1) + A (Gbar^T U_1)) / 2
  RUTV_CHECK(mm(true, false, n, k, m, 1.0, A, lda, U1, m, 0.0, w.T1, n));
  RUTV_CHECK(mm(false, false, m, k, n, 0.5, Gbar, ldg, w.T1, n, 0.0, w.E, m));
  RUTV_CHECK(mm(true, false, n, k, m, 1.0, Gbar, ldg, U1, m, 0.0, w.T1, n));
  RUTV_CHECK(mm(false, false, m, k, n, 0.5, A, lda, w.T1, n, 1.0, w.E, m));
  // H = 2 (E - U_C (U_C^T E)) Lambda_1^-1 + U_2 F
  RUTV_CHECK(mm(true, false, bb, k, m, 1.0, w.Uc, m, w.E, m, 0.0, w.X1, bb));
  RUTV_CHECK(copy_matrix(st, m, k, w.E, m, w.H, m));
  RUTV_CHECK(mm(false, false, m, k, bb, -1.0, w.Uc, m, w.X1, bb, 1.0, w.H, m));
  RUTV_CHECK(scale_cols(st, m, k, w.H, m, w.lam, 2.0, &status[2]));
  if (r2 > 0) {
    RUTV_CHECK(gap_divide(st, r2, k, w.X1 + k, bb, w.d, &status[2]));
    RUTV_CHECK(mm(false, false, m, k, r2, 1.0, U2, m, w.X1 + k, bb, 1.0, w.H, m));
  }
  // L = H (U_1^T C) + U_1 (H^T C);  Abar += L Q_Y^T
  RUTV_CHECK(mm(true, false, k, bb, m, 1.0, U1, m, w.C, m, 0.0, w.W1, k));
  RUTV_CHECK(mm(true, false, k, bb, m, 1.0, w.H, m, w.C, m, 0.0, w.W2, k));
  RUTV_CHECK(mm(false, false, m, bb, k, 1.0, w.H, m, w.W1, k, 0.0, w.L, m));
  RUTV_CHECK(mm(false, false, m, bb, k, 1.0, U1, m, w.W2, k, 1.0, w.L, m));
  RUTV_CHECK(mm(false, true, m, n, bb, 1.0, w.L, m, w.Qy, n, 1.0, Abar, ldab));
  // D = C R_Y^-T; L2 = H (U_1^T D) + U_1 (H^T D) (into L)
  RUTV_CHECK(mm(false, true, m, bb, bb, 1.0, w.C, m, w.RyInv, bb, 0.0, w.D, m));
  RUTV_CHECK(mm(true, false, k, bb, m, 1.0, U1, m, w.D, m, 0.0, w.W1, k));
  RUTV_CHECK(mm(true, false, k, bb, m, 1.0, w.H, m, w.D, m, 0.0, w.W2, k));
  RUTV_CHECK(mm(false, false, m, bb, k, 1.0, w.H, m, w.W1, k, 0.0, w.L, m));
  RUTV_CHECK(mm(false, false, m, bb, k, 1.0, U1, m, w.W2, k, 1.0, w.L, m));
  // Ybar = (I - Q_Y Q_Y^T) A^T L2
  RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, w.L, m, 0.0, w.Yb, n));
  RUTV_CHECK(mm(true, false, bb, bb, n, 1.0, w.Qy, n, w.Yb, n, 0.0, w.X, bb));
  RUTV_CHECK(mm(false, false, n, bb, bb, -1.0, w.Qy, n, w.X, bb, 1.0, w.Yb, n));
  // the chain reversed: Zbar_q = Ybar
  double* Zbar = w.Yb;
  for (int t = q; t >= 0; --t) {
    RUTV_CHECK(mm(false, true, m, n, bb, 1.0, w.Mj[t], m, Zbar, n, 1.0, Abar, ldab));
    if (t == 0) break;
    RUTV_CHECK(mm(false, false, m, bb, n, 1.0, A, lda, Zbar, n, 0.0, w.Mb, m));
    RUTV_CHECK(mm(false, true, m, n, bb, 1.0, w.Mb, m, w.Zj[t - 1], n, 1.0, Abar, ldab));
    double* next = Zbar == w.Yb ? w.Zb : w.Yb;
    RUTV_CHECK(mm(true, false, n, bb, m, 1.0, A, lda, w.Mb, m, 0.0, next, n));
    Zbar = next;
  }
  return RANDUTV_OK;
}

int trunc_status(const int* flags, const TruncJob& j) {
  if (flags[0]) return RANDUTV_ERR_NONFINITE;
  if (flags[1] || flags[6]) return RANDUTV_ERR_SYNC;
  const bool svd = j.k != std::min(j.b, j.n);  // k = b_0 needs no b x b SVD
  if (svd && !flags[5]) return RANDUTV_ERR_NOCONV;
  if (j.reverse && flags[2]) return RANDUTV_ERR_RANK;
  return RANDUTV_OK;
}

}  // namespace rutv
