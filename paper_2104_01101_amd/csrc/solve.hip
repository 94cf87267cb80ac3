// Exact sketched rank-constrained solve of one Tucker subproblem (Sec. 4
// theorems; Sec. 2.2 for the roles of A^(n) and C_(n)^T):
//
//   [Z^T Z ; Y^T Z]      one MFMA Gram launch in the operands' precision
//   X^T = (Y^T Z)(Z^T Z)^{-1}     FP64: Gauss-Jordan inverse of the r x r Gram in
//                                 LDS and an FP64 MFMA product when r fits, else
//                                 Cholesky + row-block triangular solves
//   A   = leading R right singular vectors of X
//         r <= s: eigenvectors U of X X^T (r x r), A = X^T U Lambda^{-1/2}
//         r >  s: eigenvectors of X^T X (s x s)
//   A  <- CholeskyQR(A), largest-magnitude entry of each column positive
//   W   = X A = C_(n)^T
// All FP64 after the Gram products; no host synchronisation.

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
  double* Ht = gj ? ws.take<double>(size_t(s) * r) : nullptr;  // Y^T Z kept for the product
  const bool run = !ws.measuring();
  {
    ProfScope prof(run ? "gram" : "", st);
    TSK_TRY(gemm_tn(prec, r + s, r, m, Z, r, r, Y, s, Z, r, GH, r, ws, st));
  }
  if (gj) {
    // G^{-1} in place (Gauss-Jordan), then X^T = (Y^T Z) G^{-1} on the matrix cores
    ProfScope prof(run ? "solve_la" : "", st);
    if (run) TSK_HIP(hipMemcpyAsync(Ht, Xt, size_t(s) * r * 8, hipMemcpyDeviceToDevice, st));
    if (run) TSK_TRY(spd_inverse(G, r, r, info, st));
    TSK_TRY(gemm_nn_f64(s, r, r, Ht, r, G, r, Xt, r, ws, st));
  } else {
    ProfScope prof(run ? "solve_la" : "", st);
    if (run) TSK_TRY(cholesky(G, r, r, info, st));
    if (run) TSK_TRY(chol_solve_rows(G, r, r, Xt, s, r, false, st));
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
  if (run) TSK_TRY(sign_fix_columns(A, s, R, st));
  TSK_TRY(gemm_tn(TSK_PREC_F64, r, R, s, Xt, r, r, nullptr, 0, A, R, W, R, ws, st));
  return TSK_OK;
}


// RSVD-LRLS (Alg. 5), the randomized low-rank least-squares solve that Alg. 4
// calls for each subproblem, with the s x k Gaussian test matrix Om:
//
//   [Z^T Z ; Y^T Z]                 one MFMA Gram launch (as the exact solve)
//   B = (Z^T Z)^{-1}                Gauss-Jordan when r fits, else Cholesky solves
//   C^T = (Om^T H^T) B              H = Z^T Y;  C = B Z^T Y Om  (r x k)
//   Q = thin Householder QR of C
//   D^T = H^T (B Q)                 D = Q^T B Z^T Y  (k x s)
//   U, S: leading R eigenpairs of D D^T (k x k);  A = D^T U S^{-1} = V(:, :R)
//   A <- CholeskyQR(A), sign rule
//   W = Q (D A)                     = Q U S with the signs of A
tsk_status rsvd_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s, int R,
                      int prec, const double* Om, int64_t k, double* A, double* W, int* info,
                      Ws& ws, hipStream_t st) {
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
    if (gj) {
      if (run) TSK_TRY(spd_inverse(G, r, r, info, st));
      TSK_TRY(gemm_nn_f64(k, r, r, C0t, r, G, r, Ct, r, ws, st));
    } else {
      if (run) TSK_TRY(cholesky(G, r, r, info, st));
      if (run) TSK_HIP(hipMemcpyAsync(Ct, C0t, size_t(k) * r * 8, hipMemcpyDeviceToDevice, st));
      if (run) TSK_TRY(chol_solve_rows(G, r, r, Ct, k, r, false, st));
    }
    TSK_TRY(qr_rows(Ct, k, r, Qt, ws, st));
    if (gj) {
      TSK_TRY(gemm_nn_f64(k, r, r, Qt, r, G, r, Pt, r, ws, st));
    } else {
      if (run) TSK_HIP(hipMemcpyAsync(Pt, Qt, size_t(k) * r * 8, hipMemcpyDeviceToDevice, st));
      if (run) TSK_TRY(chol_solve_rows(G, r, r, Pt, k, r, false, st));
    }
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
  if (run) TSK_TRY(sign_fix_columns(A, s, R, st, sgn));
  if (run) TSK_TRY(rsvd_w(Qt, false, U, lam, sgn, k, r, R, W, st));
  return TSK_OK;
}

}  // namespace tsk
