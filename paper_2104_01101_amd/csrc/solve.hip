// Exact sketched rank-constrained solve of one Tucker subproblem (Sec. 4
// theorems; Sec. 2.2 for the roles of A^(n) and C_(n)^T):
//
//   [Z^T Z ; Y^T Z]      one MFMA Gram launch in the operands' precision
//   X^T = (Y^T Z)(Z^T Z)^{-1}     FP64: inverse of the r x r Gram by sweeps (in
//                                 LDS when r fits, else block sweeps with MFMA
//                                 tile updates), then an FP64 MFMA product
//   A   = leading R right singular vectors of X
//         r <= s: eigenvectors U of X X^T (r x r), A = X^T U Lambda^{-1/2}
//         r >  s: eigenvectors of X^T X (s x s)
//   A  <- CholeskyQR(A), largest-magnitude entry of each column positive
//   W   = X A = C_(n)^T
// All FP64 after the Gram products; no host synchronisation.

#include <mutex>

#include "common.h"
#include "kernels.h"

namespace tsk {

tsk_status rc_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s, int R,
                    int prec, double* A, double* W, int* info, Ws& ws, hipStream_t st) {
  double* GH = ws.take<double>(size_t(r + s) * r);
  double* G = GH;
  double* Xt = GH + size_t(r) * r;  // s x r, holds Y^T Z then X^T
  const bool small_r = r <= s;
  const int64_t q = small_r ? r : s;
  double* Mq = ws.take<double>(size_t(q) * q);
  double* lam = ws.take<double>(R);
  double* U = small_r ? ws.take<double>(size_t(r) * R) : nullptr;
  double* X = small_r ? nullptr : ws.take<double>(size_t(r) * s);
  const bool gj = spd_inverse_fits(r);
  // Y^T Z kept for the product X^T = (Y^T Z) B; B = G^{-1} in place (one
  // workgroup) when it fits in LDS, else by block sweeps into Bi
  double* Ht = ws.take<double>(size_t(s) * r);
  double* Bi = gj ? G : ws.take<double>(size_t(r) * r);
  const bool run = !ws.measuring();
  {
    ProfScope prof(run ? "gram" : "", st);
    TSK_TRY(gemm_tn(prec, r + s, r, m, Z, r, r, Y, s, Z, r, GH, r, ws, st));
  }
  {
    ProfScope prof(run ? "solve_la" : "", st);
    if (run) TSK_HIP(hipMemcpyAsync(Ht, Xt, size_t(s) * r * 8, hipMemcpyDeviceToDevice, st));
    if (gj) {
      if (run) TSK_TRY(spd_inverse(G, r, r, info, st));
    } else {
      TSK_TRY(spd_inverse_blocked(G, r, r, Bi, r, info, ws, st));
    }
    TSK_TRY(gemm_nn_f64(s, r, r, Ht, r, Bi, r, Xt, r, ws, st));
  }
  if (small_r) {
    TSK_TRY(gemm_tn(TSK_PREC_F64, r, r, s, Xt, r, r, nullptr, 0, Xt, r, Mq, r, ws, st));
    TSK_TRY(sym_eig_top(Mq, r, R, lam, U, ws, st));
    TSK_TRY(gemm_nn_f64(s, R, r, Xt, r, U, R, A, R, ws, st));
    if (run) TSK_TRY(scale_columns_inv_sqrt(A, s, R, lam, st, info + 3));
  } else {
    if (run) TSK_TRY(transpose_f64(Xt, s, r, X, st));
    TSK_TRY(gemm_tn(TSK_PREC_F64, s, s, r, X, s, s, nullptr, 0, X, s, Mq, s, ws, st));
    TSK_TRY(sym_eig_top(Mq, s, R, lam, A, ws, st));
  }
  TSK_TRY(cholqr(A, s, R, info + 1, ws, st));
  TSK_TRY(sign_fix_columns(A, s, R, ws, st));
  TSK_TRY(gemm_tn(TSK_PREC_F64, r, R, s, Xt, r, r, nullptr, 0, A, R, W, R, ws, st));
  return TSK_OK;
}


// RSVD-LRLS (Alg. 5), the randomized low-rank least-squares solve that Alg. 4
// calls for each subproblem, with the s x k Gaussian test matrix Om:
//
//   [Z^T Z ; Y^T Z]                 one MFMA Gram launch (as the exact solve)
//   B = (Z^T Z)^{-1}                sweeps in LDS when r fits, else block sweeps
//   C^T = (Om^T H^T) B              H = Z^T Y;  C = B Z^T Y Om  (r x k)
//   Q = thin Householder QR of C
//   D^T = H^T (B Q)                 D = Q^T B Z^T Y  (k x s)
//   U, S: leading R eigenpairs of D D^T (k x k);  A = D^T U S^{-1} = V(:, :R)
//   sign rule on A (A is not re-orthonormalised)
//   W = Q (D A)                     = Q U S with the signs of A
namespace {

// The same solve with the products ordered for the cost of Sec. 6.1, O(m s k)
// in Y instead of O(m s r): Z^T Y (r x s) is never formed.
//   G = Z^T Z;  Y Omega (m x k);  C0 = Z^T (Y Omega)
//   B = G^{-1};  C^T = C0^T B;  Q = qr(C);  P = B Q
//   D^T = Y^T (Z P)  (s x k)
// The two products with Y run in the operands' precision (Omega and Z P
// rounded to it); the products with Z in FP64.
tsk_status rsvd_solve_yside(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s, int R,
                            int prec, const double* Om, int64_t k, double* A, double* W, int* info,
                            Ws& ws, hipStream_t st) {
  const bool f64 = prec == TSK_PREC_F64;
  const size_t eb = prec_bytes(prec);
  // the rounded copies of Omega and Z P get rows of a multiple of 4 elements
  // (vector loads in the FP32 products)
  const int64_t kp = ceil_div(k, 4) * 4;
  // FP32 operands with aligned rows of Y: the skinny products streaming Y,
  // with Omega and Z P transposed (rows along the contraction)
  const int64_t lds_t = ceil_div(s, 16) * 16, ldm_t = ceil_div(m, 16) * 16;
  const bool ysk = prec == TSK_PREC_F32 && yskinny_fits(true, k, s, Y, s, nullptr, lds_t) &&
                   yskinny_fits(false, k, m, Y, s, nullptr, ldm_t);
  double* G = ws.take<double>(size_t(r) * r);
  void* Om_e = f64 ? static_cast<void*>(const_cast<double*>(Om))
               : ysk ? static_cast<void*>(ws.take<float>(size_t(k) * lds_t))
                     : static_cast<void*>(ws.take<char>(size_t(s) * kp * eb));
  double* YO = ws.take<double>(size_t(m) * k);
  const double* Z64 = f64 ? static_cast<const double*>(Z) : ws.take<double>(size_t(m) * r);
  double* C0 = ws.take<double>(size_t(r) * k);
  double* Ct = ws.take<double>(size_t(k) * r);
  double* Qt = ws.take<double>(size_t(k) * r);
  double* Pt = ws.take<double>(size_t(k) * r);
  double* P = ws.take<double>(size_t(r) * k);
  double* ZP = ws.take<double>(size_t(m) * k);
  void* ZP_e = f64   ? static_cast<void*>(ZP)
               : ysk ? static_cast<void*>(ws.take<float>(size_t(k) * ldm_t))
                     : static_cast<void*>(ws.take<char>(size_t(m) * kp * eb));
  double* Dt = ws.take<double>(size_t(s) * k);
  double* Mk = ws.take<double>(size_t(k) * k);
  double* lam = ws.take<double>(R);
  double* U = ws.take<double>(size_t(k) * R);
  double* sgn = ws.take<double>(R);
  const bool gj = spd_inverse_fits(r);
  double* Bi = gj ? G : ws.take<double>(size_t(r) * r);
  const bool run = !ws.measuring();
  // the blocked inverse of G goes to a side stream as soon as G is formed;
  // the caller's stream waits for it before C^T = C0^T B
  SideJob inv(st);
  hipStream_t side = nullptr;
  if (run && !gj && !ws.serial) TSK_TRY(side_stream(&side));
  {
    ProfScope prof(run ? "gram" : "", st);
    TSK_TRY(gemm_tn(prec, r, r, m, Z, r, r, nullptr, 0, Z, r, G, r, ws, st));
    if (side) {
      TSK_TRY(inv.fork(side));
      TSK_TRY(spd_inverse_blocked(G, r, r, Bi, r, info, ws, side));
      TSK_TRY(inv.done());
    }
    if (ysk) {
      if (run) TSK_TRY(convert_from_f64_t(Om, s, k, static_cast<float*>(Om_e), lds_t, st));
      TSK_TRY(gemm_yskinny_f32(true, m, k, s, static_cast<const float*>(Y), s,
                               static_cast<const float*>(Om_e), lds_t, YO, k, ws, st));
    } else {
      if (run && !f64) TSK_TRY(convert_from_f64(Om, s, k, Om_e, kp, prec, st));
      TSK_TRY(gemm_nn(prec, m, k, s, Y, s, Om_e, f64 ? k : kp, YO, k, ws, st));
    }
  }
  {
    ProfScope prof(run ? "solve_la" : "", st);
    if (run && !f64) TSK_TRY(convert_to_f64(Z, int(eb), m * r, const_cast<double*>(Z64), st));
    TSK_TRY(gemm_tn(TSK_PREC_F64, r, k, m, Z64, r, r, nullptr, 0, YO, k, C0, k, ws, st));
    if (gj) {
      if (run) TSK_TRY(spd_inverse(G, r, r, info, st));
    } else if (side) {
      TSK_TRY(inv.join());
    } else {
      TSK_TRY(spd_inverse_blocked(G, r, r, Bi, r, info, ws, st));
    }
    TSK_TRY(gemm_tn(TSK_PREC_F64, k, r, r, C0, k, k, nullptr, 0, Bi, r, Ct, r, ws, st));
    TSK_TRY(qr_rows(Ct, k, r, Qt, ws, st));
    TSK_TRY(gemm_nn_f64(k, r, r, Qt, r, Bi, r, Pt, r, ws, st));
    if (run) TSK_TRY(transpose_f64(Pt, k, r, P, st));
    TSK_TRY(gemm_nn_f64(m, k, r, Z64, r, P, k, ZP, k, ws, st));
  }
  {
    ProfScope prof(run ? "gram" : "", st);
    if (ysk) {
      if (run) TSK_TRY(convert_from_f64_t(ZP, m, k, static_cast<float*>(ZP_e), ldm_t, st));
      TSK_TRY(gemm_yskinny_f32(false, s, k, m, static_cast<const float*>(Y), s,
                               static_cast<const float*>(ZP_e), ldm_t, Dt, k, ws, st));
    } else {
      if (run && !f64) TSK_TRY(convert_from_f64(ZP, m, k, ZP_e, kp, prec, st));
      TSK_TRY(gemm_tn(prec, s, k, m, Y, s, s, nullptr, 0, ZP_e, f64 ? k : kp, Dt, k, ws, st));
    }
  }
  TSK_TRY(gemm_tn(TSK_PREC_F64, k, k, s, Dt, k, k, nullptr, 0, Dt, k, Mk, k, ws, st));
  TSK_TRY(sym_eig_top(Mk, k, R, lam, U, ws, st));
  if (run) TSK_TRY(scale_columns_inv_sqrt(U, k, R, lam, st, info + 3));
  TSK_TRY(gemm_nn_f64(s, R, k, Dt, k, U, R, A, R, ws, st));
  TSK_TRY(sign_fix_columns(A, s, R, ws, st, sgn));
  if (run) TSK_TRY(rsvd_w(Qt, false, U, lam, sgn, k, r, R, W, st));
  return TSK_OK;
}

constexpr int kMaxSideDevices = 64;
hipStream_t g_side[kMaxSideDevices];
std::mutex g_side_mu;

}  // namespace

tsk_status side_stream(hipStream_t* out) {
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  *out = nullptr;
  if (dev < 0 || dev >= kMaxSideDevices) return TSK_OK;
  std::lock_guard<std::mutex> lock(g_side_mu);
  if (!g_side[dev]) TSK_HIP(hipStreamCreateWithFlags(&g_side[dev], hipStreamNonBlocking));
  *out = g_side[dev];
  return TSK_OK;
}

// The Y-side order pays when Z^T Y (2 m s r flops) costs well over the two
// products with Y (4 m s k) and the one-workgroup fused chain does not apply.
bool rsvd_uses_yside(int64_t r, int64_t k) {
  return !(spd_inverse_fits(r) && range_basis_fits(r, k) && c0_inverse_fits(r)) && r >= 4 * k;
}

tsk_status rsvd_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s, int R,
                      int prec, const double* Om, int64_t k, double* A, double* W, int* info,
                      Ws& ws, hipStream_t st) {
  if (rsvd_uses_yside(r, k))
    return rsvd_solve_yside(Z, Y, m, r, s, R, prec, Om, k, A, W, info, ws, st);
  double* GH = ws.take<double>(size_t(r + s) * r);
  double* G = GH;
  const double* Ht = GH + size_t(r) * r;  // s x r: Y^T Z = H^T
  double* C0t = ws.take<double>(size_t(k) * r);
  double* Ct = ws.take<double>(size_t(k) * r);
  double* Qt = ws.take<double>(size_t(k) * r);
  double* Pt = ws.take<double>(size_t(k) * r);
  double* P = ws.take<double>(size_t(r) * k);
  double* Dt = ws.take<double>(size_t(s) * k);
  double* Mk = ws.take<double>(size_t(k) * k);
  double* lam = ws.take<double>(R);
  double* U = ws.take<double>(size_t(k) * R);
  double* sgn = ws.take<double>(R);
  const bool gj = spd_inverse_fits(r);
  const bool run = !ws.measuring();
  {
    ProfScope prof(run ? "gram" : "", st);
    TSK_TRY(gemm_tn(prec, r + s, r, m, Z, r, r, Y, s, Z, r, GH, r, ws, st));
  }
  if (gj && range_basis_fits(r, k) && c0_inverse_fits(r)) {
    // fused chain: C0 = H Omega beside B = G^{-1} (one launch), then C = B C0,
    // Q = qr(C), P = B Q (one launch); D^T = H^T P and the Gram D D^T
    double* Q = Qt;  // r x k here
    double* C0 = C0t;
    {
      ProfScope prof(run ? "solve_la" : "", st);
      if (run) TSK_TRY(c0_and_inverse(r, k, s, Ht, r, Om, k, C0, k, G, r, r, info, st));
      if (run) TSK_TRY(range_basis(C0, G, r, k, Q, P, st));
      TSK_TRY(gemm_nn_f64(s, k, r, Ht, r, P, k, Dt, k, ws, st));
      TSK_TRY(gemm_tn(TSK_PREC_F64, k, k, s, Dt, k, k, nullptr, 0, Dt, k, Mk, k, ws, st));
    }
    TSK_TRY(sym_eig_top(Mk, k, R, lam, U, ws, st));
    if (run) TSK_TRY(rsvd_finish(Dt, U, lam, Q, s, k, r, R, A, W, info + 3, st));
    return TSK_OK;
  }
  {
    ProfScope prof(run ? "solve_la" : "", st);
    TSK_TRY(gemm_tn(TSK_PREC_F64, k, r, s, Om, k, k, nullptr, 0, Ht, r, C0t, r, ws, st));
    // B = G^{-1}: in place (one workgroup) when it fits in LDS, else by block
    // sweeps into Bi
    double* Bi = G;
    if (gj) {
      if (run) TSK_TRY(spd_inverse(G, r, r, info, st));
    } else {
      Bi = ws.take<double>(size_t(r) * r);
      TSK_TRY(spd_inverse_blocked(G, r, r, Bi, r, info, ws, st));
    }
    TSK_TRY(gemm_nn_f64(k, r, r, C0t, r, Bi, r, Ct, r, ws, st));
    TSK_TRY(qr_rows(Ct, k, r, Qt, ws, st));
    TSK_TRY(gemm_nn_f64(k, r, r, Qt, r, Bi, r, Pt, r, ws, st));
    if (run) TSK_TRY(transpose_f64(Pt, k, r, P, st));
    TSK_TRY(gemm_nn_f64(s, k, r, Ht, r, P, k, Dt, k, ws, st));
    TSK_TRY(gemm_tn(TSK_PREC_F64, k, k, s, Dt, k, k, nullptr, 0, Dt, k, Mk, k, ws, st));
  }
  // SVD of D = Q^T B Z^T Y (k x s) from the eigenpairs of D D^T = Dt^T Dt:
  // right singular vectors A = D^T U Sigma^{-1} = Dt (U lam^{-1/2}), left
  // factor W = Q U Sigma, both in the column signs that make the largest
  // entry of each column of A positive
  TSK_TRY(sym_eig_top(Mk, k, R, lam, U, ws, st));
  if (run) TSK_TRY(scale_columns_inv_sqrt(U, k, R, lam, st, info + 3));
  TSK_TRY(gemm_nn_f64(s, R, k, Dt, k, U, R, A, R, ws, st));
  TSK_TRY(sign_fix_columns(A, s, R, ws, st, sgn));
  if (run) TSK_TRY(rsvd_w(Qt, false, U, lam, sgn, k, r, R, W, st));
  return TSK_OK;
}

}  // namespace tsk
