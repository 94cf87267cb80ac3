// Internal interfaces between the host driver and the kernel translation units.
#pragma once

#include "common.h"

namespace tsk {

// A tensor as seen by the kernels (copied from tsk_tensor after validation).
struct TensorView {
  int order;
  int64_t dims[TSK_MAX_ORDER];
  int dtype;
  int layout;
  const void* values;
  int64_t nnz;  // number of stored entries (prod dims for DENSE)
  const int32_t* idx[TSK_MAX_ORDER];
};

// ---- sketch pass (sketch_pass.hip) ----
// type 0: Y[(sum_{k != col_mode} h[k][i_k]) mod rows, i_col] += prod sg[k][i_k] * v
// type 1: Y[g(j), i_col] += tau(j) * v, (g, tau) from draw(key, j), j = row-major
//         index of the other modes
struct PassJob {
  int type;
  int col_mode;
  int64_t rows;
  const int32_t* const* h;  // host array of device pointers (type 0)
  const int8_t* const* sg;
  uint64_t key;  // type 1
  void* out;     // device rows x dims[col_mode], dtype of the tensor
};
tsk_status sketch_pass(const TensorView& T, const PassJob* jobs, int njobs, Ws& ws,
                       hipStream_t st);

// ---- dense range-finder pass (rrf_dense.hip) ----
// B (s_n x k1, FP64) = T_(n) Omega^T G for a dense T: CountSketch (g, tau) of
// the other-mode row-major index from draw(key, j), G k2 x k1 (device FP64);
// one structured GEMM over T in the operand precision (FP64 for FP64 tensors
// or prec = F64, BF16 with FP32 accumulation for prec = BF16, else FP32).
bool rrf_dense_supported(const TensorView& T, int64_t k1);
tsk_status rrf_dense(const TensorView& T, int n, int64_t k1, int64_t k2, uint64_t key,
                     const double* G, int prec, double* B, Ws& ws, hipStream_t st);

// ---- random tables (rng.hip) ----
// h[i] = bucket_m(draw(key, i)), sg[i] = sign(draw(key, i)), i < s
tsk_status launch_hash_table(uint64_t key, int64_t s, int64_t m, int32_t* h, int8_t* sg,
                             hipStream_t st);
// out[i] = scale * gauss(key, i), i < count (FP64)
tsk_status launch_gauss(uint64_t key, int64_t count, double scale, double* out, hipStream_t st);
// Several Gaussian arrays in one launch: out[b][i] = gauss(key[b], i), i < count[b]
constexpr int kGaussBatch = 64;
struct GaussBatch {
  int n;
  uint64_t key[kGaussBatch];
  int64_t count[kGaussBatch];
  double* out[kGaussBatch];
};
tsk_status launch_gauss_batch(const GaussBatch& b, hipStream_t st);

// ---- TensorSketch of the Kronecker chain (ts_lhs.hip) ----
struct CsrTable {  // inverse hash of one mode: bucket b holds items[ptr[b] .. ptr[b+1])
  int32_t* ptr;    // m + 1
  int32_t* items;  // s, increasing within a bucket
};
tsk_status build_inverse_hash(const int32_t* h, int64_t s, int64_t m, CsrTable csr, Ws& ws,
                              hipStream_t st);
// Hash tables h, sg (as launch_hash_table) and their inverse-hash tables for
// several (n, k) pairs: one launch for all tables, one for all inverses.
constexpr int kTableBatch = 16;
struct TableBatch {
  int n;
  uint64_t key[kTableBatch];
  int64_t s[kTableBatch];
  int32_t* h[kTableBatch];
  int8_t* sg[kTableBatch];
  CsrTable csr[kTableBatch];
};
bool table_batch_fits(int64_t s, int64_t m);
tsk_status hash_tables_batch(const TableBatch& b, int64_t m, hipStream_t st);
// Z (m x r row-major, precision prec) = TensorSketch of kron_{k in modes} A^(k)
struct LhsMode {
  const double* A;  // s_k x R_k
  int64_t s, R;
  const int8_t* sg;
  CsrTable csr;
};
tsk_status ts_lhs(const LhsMode* modes, int nmodes, int64_t m, int prec, void* Z, Ws& ws,
                  hipStream_t st);
// Pieces of ts_lhs shared with the adjoint.  CS: m x sum R_k (mode blocks,
// each m x R_k row-major); spec: complex FFT of every CS column (column-major
// blocks of m complex); tw: m complex twiddles.
tsk_status ts_lhs_spectra(const LhsMode* modes, int nmodes, int64_t m, double* CS,
                          double* spec, double* tw, Ws& ws, hipStream_t st);
tsk_status ts_compose(const LhsMode* modes, int nmodes, int64_t m, const double* spec,
                      const double* tw, int prec, void* Z, hipStream_t st);
tsk_status fft_columns(const double* X, int64_t m, int64_t cols, const double* tw, double* spec,
                       hipStream_t st);
tsk_status ts_conv_adjoint(const LhsMode* modes, int nmodes, int64_t m, const double* spec,
                           const double* gspec, const double* tw, double* gCS, hipStream_t st);

// ---- GEMM (gemm.hip) ----
// C (M x N, FP64) = A^T B with A = [A1 | A2] (K x M1, K x (M - M1), row-major,
// leading dims lda1/lda2) and B (K x N, ldb), all of element type `prec`.
// `ldc` leading dimension of C.  Deterministic split-K.
// Grams C[p] = A[p]^T A[p] (A[p] row-major K[p] x R[p], R[p] <= 64, FP64) of up to
// TSK_MAX_ORDER matrices in one launch (skinny tiles).  With `part` (room for
// gram_batch_splits(n, K) * sum_p R[p]^2 doubles) the rows are split into
// ranges whose partial Grams are summed in range order by a second launch;
// with part = NULL one workgroup per tile covers all rows.
constexpr int kGramSplitsMax = 32;
int gram_batch_splits(int n, const int64_t* K);
tsk_status gram_batch_f64(int n, const int64_t* R, const int64_t* K, const double* const* A,
                          double* const* C, double* part, hipStream_t st);
// C (M x N, FP64) = A B for FP32 A (M x K row-major when a_mk, else K x M)
// and B given transposed (Bt: N x K, row stride ldbt, zero from K up to
// ldbt), N <= 32: the products with Y in the randomized solve, streaming A
// once (matrix cores, deterministic range split).  yskinny_fits tells whether
// the shapes and alignments allow it (ldbt a multiple of 4 and at least K
// rounded up to a multiple of 16, 16-byte aligned Bt; for a_mk also K and lda
// multiples of 4 and a 16-byte aligned A).
bool yskinny_fits(bool a_mk, int64_t N, int64_t K, const void* A, int64_t lda, const void* Bt,
                  int64_t ldbt);
tsk_status gemm_yskinny_f32(bool a_mk, int64_t M, int64_t N, int64_t K, const float* A,
                            int64_t lda, const float* Bt, int64_t ldbt, double* C, int64_t ldc,
                            Ws& ws, hipStream_t st);
// dst (cols x ldd, FP32) = src^T (src rows x cols, FP64), zero beyond rows
tsk_status convert_from_f64_t(const double* src, int64_t rows, int64_t cols, float* dst,
                              int64_t ldd, hipStream_t st);
tsk_status gemm_tn(int prec, int64_t M, int64_t N, int64_t K, const void* A1, int64_t lda1,
                   int64_t M1, const void* A2, int64_t lda2, const void* B, int64_t ldb,
                   double* C, int64_t ldc, Ws& ws, hipStream_t st);
// C (M x N, FP64) = A B, A (M x K) and B (K x N) row-major FP64 (matrix cores)
tsk_status gemm_nn_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double* C, int64_t ldc, Ws& ws,
                       hipStream_t st);
// C (M x N) = alpha * op(A) op(B) + beta * C, FP64, small sizes; op given by
// strides: A(i,k) = A[i*sai + k*sak], B(k,j) = B[k*sbk + j*sbj], C(i,j) = C[i*ldc + j]
tsk_status gemm_small(int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                      int64_t sai, int64_t sak, const double* B, int64_t sbk, int64_t sbj,
                      double beta, double* C, int64_t ldc, hipStream_t st);
tsk_status convert_to_f64(const void* src, int dtype_or_prec_bytes, int64_t count, double* dst,
                          hipStream_t st);
// dst (rows x ldd elements of precision prec) = src (rows x cols, FP64)
// rounded to that precision, columns cols..ldd-1 set to 0
tsk_status convert_from_f64(const double* src, int64_t rows, int64_t cols, void* dst,
                            int64_t ldd, int prec, hipStream_t st);
// C (M x N, FP64) = A B, A (M x K) and B (K x N) row-major, element type prec
tsk_status gemm_nn(int prec, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                   const void* B, int64_t ldb, double* C, int64_t ldc, Ws& ws, hipStream_t st);

// ---- FP64 dense linear algebra (linalg.hip) ----
// In-place lower Cholesky of the n x n matrix G (row-major, lda); sets *info
// (device int) to j+1 at the first non-positive pivot j (0 = success).
tsk_status cholesky(double* G, int64_t n, int64_t lda, int* info, hipStream_t st);
// Rows of X (rows x n, ldx) <- rows of X G^{-1} with G = L L^T (L from
// cholesky); forward_only: X <- X L^{-T}.
tsk_status chol_solve_rows(const double* L, int64_t n, int64_t ldl, double* X, int64_t rows,
                           int64_t ldx, bool forward_only, hipStream_t st);
// Leading R eigenpairs (descending) of the symmetric q x q matrix M (row-major);
// M is overwritten.  lam: R doubles, V: q x R row-major.
tsk_status sym_eig_top(double* M, int64_t q, int64_t R, double* lam, double* V, Ws& ws,
                       hipStream_t st);
// In-place inverse of the SPD n x n matrix G (row-major, lda) by Gauss-Jordan
// elimination without pivoting (single workgroup, LDS); *info = j+1 at the first
// non-positive pivot.  Returns EUNSUPPORTED if G does not fit in LDS.
tsk_status spd_inverse(double* G, int64_t n, int64_t lda, int* info, hipStream_t st);
bool spd_inverse_fits(int64_t n);
// Ginv (n x n, ldi) = G^{-1} for an SPD G (n x n, ldg) of any order: block
// sweeps of 32 or 64 pivots, one launch per block, FP64 MFMA tile updates.
// Ginv must not alias G.  *info = j+1 at the first non-positive pivot j when
// it was 0.
tsk_status spd_inverse_blocked(const double* G, int64_t n, int64_t ldg, double* Ginv,
                               int64_t ldi, int* info, Ws& ws, hipStream_t st);
// Make the entry of largest magnitude of every column of A (rows x R) positive.
// sgn (optional, R entries) receives the sign applied to each column
tsk_status sign_fix_columns(double* A, int64_t rows, int64_t R, hipStream_t st,
                            double* sgn = nullptr);
// The same, for tall A in two launches over ranges of rows (partial results in
// ws; call in the measuring pass too)
tsk_status sign_fix_columns(double* A, int64_t rows, int64_t R, Ws& ws, hipStream_t st,
                            double* sgn = nullptr);
// C = A^T B (A: K x M, B: K x N, row-major FP64) beside the in-place SPD
// inverse of G (n x n, n <= 128) in one launch (c0_inverse_fits)
bool c0_inverse_fits(int64_t n);
tsk_status c0_and_inverse(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                          const double* B, int64_t ldb, double* C, int64_t ldc, double* G,
                          int64_t n, int64_t ldg, int* info, hipStream_t st);
// Range basis of the randomized solve: C = B C0 (r x k), Q = qr(C), P = B Q
// (r x k row-major); r <= 128, k <= 24 (range_basis_fits).
bool range_basis_fits(int64_t r, int64_t k);
tsk_status range_basis(const double* C0, const double* B, int64_t r, int64_t k, double* Q,
                       double* P, hipStream_t st);
// A = Dt U lam^{-1/2} (s x R), sign rule on its columns, W = Q U lam^{1/2} in
// the same signs (Q r x k row-major); k <= 64; one launch; *bad = 1 when some
// lam_c <= 0 (or NaN)
tsk_status rsvd_finish(const double* Dt, const double* U, const double* lam, const double* Q,
                       int64_t s, int64_t k, int64_t r, int64_t R, double* A, double* W,
                       int* bad, hipStream_t st);
// W = Q U diag(lam * sgn), Q given as r x k (q_rows) or as Q^T (k x r), U (k x R)
tsk_status rsvd_w(const double* Qm, bool q_rows, const double* U, const double* lam,
                  const double* sgn, int64_t k, int64_t r, int64_t R, double* W, hipStream_t st);
// A (rows x R): A <- A * diag(scale) with scale[c] = 1/sqrt(lam[c]); *bad = 1
// (when bad is given) if some lam[c] <= 0 (or NaN)
tsk_status scale_columns_inv_sqrt(double* A, int64_t rows, int64_t R, const double* lam,
                                  hipStream_t st, int* bad = nullptr);
tsk_status transpose_f64(const double* A, int64_t rows, int64_t cols, double* At,
                         hipStream_t st);
// Thin Householder QR: Ct (k x r) holds the columns of C (r x k) as rows; Qt
// (k x r) receives the columns of Q as rows.  k <= 64.
tsk_status qr_rows(const double* Ct, int64_t k, int64_t r, double* Qt, Ws& ws, hipStream_t st);
// A (rows x R) <- A chol(A^T A)^{-T} (one CholeskyQR pass, FP64)
tsk_status cholqr(double* A, int64_t rows, int64_t R, int* info, Ws& ws, hipStream_t st);

// ---- rank-constrained solves (solve.hip) ----
tsk_status rc_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s, int R,
                    int prec, double* A, double* W, int* info, Ws& ws, hipStream_t st);
// RSVD-LRLS (Alg. 5) with the s x k Gaussian test matrix Om (device).
tsk_status rsvd_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s, int R,
                      int prec, const double* Om, int64_t k, double* A, double* W, int* info,
                      Ws& ws, hipStream_t st);

}  // namespace tsk
