/*
 * tsk.h -- C ABI of the MI355X (gfx950) sketched Tucker-ALS library.
 *
 * Method: L. Ma, E. Solomonik, "Fast and accurate randomized algorithms for
 * low-rank tensor decompositions" (arXiv 2104.01101).  The library computes the
 * sketched mode-n rank-constrained least-squares subproblems of Tucker-ALS
 * (Alg. 4) with TensorSketch (Sec. 3.1) or leverage-score sampling (Sec. 3.2),
 * the randomized-range-finder initialisation (Alg. 3, composite sketch of
 * Sec. 5) and CP-ALS on the Tucker core (Alg. 6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - "device" pointers are HIP device allocations owned by the caller; the
 *    library never frees or retains them after a call returns.  "host"
 *    pointers are ordinary host memory.
 *  - Tensors, matrices and cores are row-major (last index fastest).  A factor
 *    A^(n) is s_n x R_n; the core C is R_1 x ... x R_N.  For mode n the other
 *    modes are linearised row-major in increasing k: this is the row order of
 *    the Kronecker chain kron_{k != n} A^(k), the column order of Z = S P and
 *    the row order of W = C_(n)^T (r x R_n, r = prod_{k != n} R_k).
 *  - Random objects (hash maps, signs, Gaussian matrices, leverage-sampling
 *    uniforms, random initial factors) are drawn from SplitMix64 (Steele, Lea
 *    & Flood 2014) streams keyed by (seed, purpose, a, b, c); see tsk_draw.
 *  - The library allocates no device memory.  Entry points that need scratch
 *    take a workspace: pass ws == NULL to query its size in *ws_bytes (no work
 *    is done), then call again with a device buffer of at least that size.
 *    Workspaces must be 256-byte aligned.
 *  - Component entry points enqueue their work on `stream` (a hipStream_t;
 *    NULL = the null stream) and return after validating arguments; execution
 *    errors surface as TSK_EHIP from a later synchronising call.  Entry points
 *    documented as synchronous synchronise `stream` before returning.
 *  - No C++ exception crosses the ABI.  On error the outputs are undefined and
 *    tsk_last_error() (thread-local) describes the failure.
 *  - Calls on different streams with different workspaces are independent.
 *    Global state: the thread-local error message; one internal stream per
 *    device (default priority, created on first use) on which the randomized
 *    solve and the driver run work beside their own (the blocked Gram
 *    inverse, the residual's sort), always joined back into `stream` before
 *    the work that reads it, so ordering on `stream` is as if all ran there;
 *    and the static scratch of tsk_rsvd_solve_noalloc.
 */
#ifndef TSK_H
#define TSK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TSK_MAX_ORDER 8
#define TSK_ABI_VERSION 5

typedef enum {
  TSK_OK = 0,
  TSK_EINVAL = -1,       /* invalid argument (message says which) */
  TSK_EUNSUPPORTED = -2, /* valid but not supported by this library */
  TSK_ENOMEM = -3,       /* workspace too small */
  TSK_EHIP = -4,         /* HIP runtime / kernel launch failure */
  TSK_ENUMERIC = -5      /* numerical breakdown: a Gram pivot or a singular value not positive */
} tsk_status;

typedef enum { TSK_F32 = 0, TSK_F64 = 1 } tsk_dtype;
typedef enum { TSK_DENSE = 0, TSK_COO = 1 } tsk_layout;
/* Sketch of every subproblem: TensorSketch (Sec. 3.1), leverage-score
 * importance sampling (Sec. 3.2), or the deterministic leverage selection of
 * Sec. 3.2 (the m rows of largest score, weights 1; needs m <= prod_{k != n} s_k). */
typedef enum { TSK_SKETCH_TS = 0, TSK_SKETCH_LEV = 1, TSK_SKETCH_LEV_DET = 2 } tsk_sketch;
typedef enum { TSK_INIT_RRF = 0, TSK_INIT_RANDOM = 1, TSK_INIT_USER = 2 } tsk_init;
/* Arithmetic of the sketched operands Z, Y and of their Gram products:
 * F64; F32; BF16 operands with FP32 accumulation.  Factorisations (Cholesky,
 * eigen-decomposition, re-orthonormalisation) are FP64 in every mode. */
typedef enum { TSK_PREC_F64 = 0, TSK_PREC_F32 = 1, TSK_PREC_BF16 = 2 } tsk_prec;
/* Subproblem solver: the exact best rank-R approximation of Z^+ Y (truncated
 * SVD), or RSVD-LRLS (Alg. 5), the randomized solver that Alg. 4 calls. */
typedef enum { TSK_SOLVE_EXACT = 0, TSK_SOLVE_RSVD = 1 } tsk_solve;

/* Relative residual (Sec. 7 fitness, evaluation only: not a step of Alg. 4).
 * RECORD_FIT: after every sweep; FINAL_FIT: after the last sweep only (the
 * earlier entries of fit_history are set to NaN).  FINAL_FIT wins when both are
 * set.  The sign rule on the factors (largest-magnitude entry of each column
 * positive) is always applied; there is no flag for it. */
#define TSK_FLAG_RECORD_FIT 1u
#define TSK_FLAG_FINAL_FIT 2u

/* An order-N tensor.  DENSE: `values` holds prod(dims) entries, row-major.
 * COO: `values` holds nnz entries and idx[k][e] (int32, 0-based) is the mode-k
 * index of entry e; entries are unsorted and duplicates add (the sketches are
 * linear).  All pointers are device pointers. */
typedef struct {
  int32_t order;
  int64_t dims[TSK_MAX_ORDER];
  int32_t dtype;  /* tsk_dtype of values */
  int32_t layout; /* tsk_layout */
  const void* values;
  int64_t nnz; /* COO only */
  const int32_t* idx[TSK_MAX_ORDER];
} tsk_tensor;

/* Inputs of Alg. 4 beyond the tensor and the ranks.  The paper's sketching
 * tolerance eps enters through the sketch size m (m = K prod_{k != n} R_k in the
 * experiments of Sec. 7) and the range-finder sizes k1 = O(R/eps),
 * k2 = O(R^2 + R/eps) (Def. composite sketch); rrf_k1 = 0 / rrf_k2 = 0 select
 * k1 = ceil(sqrt(m / prod_{k != n} R_k) R_n) and k2 = R_n^2 + k1. */
typedef struct {
  int32_t sketch; /* tsk_sketch */
  int64_t m;      /* sketch size, >= prod_{k != n} R_k for every n */
  int32_t init;   /* tsk_init */
  int32_t rrf_k1, rrf_k2;
  int32_t sweeps; /* I_max */
  int32_t prec;   /* tsk_prec */
  uint64_t seed;
  void* stream; /* hipStream_t */
  void* workspace;
  size_t workspace_bytes;
  uint32_t flags; /* TSK_FLAG_* */
  int32_t solve;  /* tsk_solve */
  int32_t rsvd_k; /* RSVD-LRLS test-matrix columns, O(R) in Alg. 5; 0 = min(R_n + 10, r) */
  /* Absolute index of the first sweep.  The per-sweep random streams (leverage
   * samples, RSVD test matrices) are keyed by the absolute sweep, so a run with
   * init = USER from the factors after sweep i and first_sweep = i + 1 continues
   * that run exactly (checkpoint / resume of the sweep loop of Alg. 4). */
  int32_t first_sweep;
  /* Convergence test of the sweep loop (the "until converged" of Alg. 1; Alg. 4
   * fixes I_max = sweeps): stop after sweep i >= 1 when
   * |residual_i - residual_{i-1}| < tol.  0 = run all sweeps.  tol > 0 needs
   * TSK_FLAG_RECORD_FIT (and not FINAL_FIT) and synchronises the stream once per
   * sweep. */
  double tol;
} tsk_options;

/* ---------------------------------------------------------------------- */
/* Library information                                                     */
/* ---------------------------------------------------------------------- */
int32_t tsk_abi_version(void);
/* Message of the last failure on this thread (empty string if none). */
const char* tsk_last_error(void);

/* Keyed SplitMix64 draw, host side (the device kernels evaluate the same
 * function).  key = stream key of (seed, purpose, a, b, c):
 *   k0 = seed; k_{t+1} = mix64(k_t + (tag_t + 1) * 0x9E3779B97F4A7C15)
 *   for tag in (purpose, a, b, c);  tsk_draw returns mix64(key + (i + 1) * GAMMA).
 * purpose < 0 means "no tags" (key = seed).  Used by tests and bindings. */
uint64_t tsk_stream_key(uint64_t seed, int32_t purpose, int64_t a, int64_t b, int64_t c);
uint64_t tsk_draw(uint64_t key, uint64_t counter);

/* Launch timing for measurement.  tsk_profile_enable(name) makes the library
 * record HIP events on the launching stream around every launch group called
 * `name` ("sketch_pass", "rrf_pass", "gram", "ts_lhs", "solve_la", "eig", "fit", "rrf",
 * "leverage", "cp_core", "adjoint_pass" (the pass over Y of the sketched
 * residual and its adjoint); the driver's phases "phase_prep" (maps and
 * sketched right-hand sides), "phase_init" (initialisation), "phase_sweeps"
 * (one per sweep, the subproblems only) and "phase_fit"; a comma-separated list
 * selects several;
 * "*" = all; NULL or "" = off, the default)
 * and clears earlier records.  tsk_profile_read(name) waits for the recorded
 * events and returns the summed milliseconds and the number of groups (name
 * NULL = all).  Not thread-safe with respect to concurrent library calls that
 * record events. */
tsk_status tsk_profile_enable(const char* name);
tsk_status tsk_profile_read(const char* name, double* total_ms, int64_t* launches);

/* ---------------------------------------------------------------------- */
/* Drivers                                                                 */
/* ---------------------------------------------------------------------- */
/* Workspace size of tsk_tucker_sketch_als for this tensor, ranks and options.
 * Validation errors are reported without touching the device.  Leverage
 * sampling of a COO tensor, deterministic selection, and the residual of an
 * order-3 COO tensor of ranks (16, 16, 16) with at least 2^16 entries (a
 * copy of the entries sorted by their last index) include the scratch of a
 * device radix sort, whose size depends on the current device: on a host
 * without one that part of the query fails with EHIP. */
tsk_status tsk_workspace_size(const tsk_tensor* T, const int32_t* ranks,
                              const tsk_options* opt, size_t* bytes);

/* Sketch-Tucker-ALS (Alg. 4).  C <- 0; A^(n) <- Init-RRF(T_(n), R_n) for
 * n = 2..N (Alg. 3; or a random orthonormal / user initialisation); then
 * opt->sweeps sweeps, each solving for n = 1..N the sketched subproblem
 * min ||S^(n) P^(n) B - S^(n) T_(n)^T|| s.t. rank(B) <= R_n (eq. tucker_ls):
 * B~ = best rank-R_n approximation of (S P)^+ (S T_(n)^T), A^(n) = its leading
 * right singular vectors, C_(n)^T = B~ A^(n) (Sec. 2.2, Sec. 4 theorems).
 * TensorSketch maps are drawn once and S^(n) T_(n)^T is formed once for all
 * sweeps; leverage samples (or the deterministic selection) are redrawn for
 * every subproblem (Sec. 6.1); for a
 * COO tensor the mode-n fibre indices (tsk_fiber_index) are built once, in
 * the workspace, and every sampled right-hand side is gathered through them.
 *   ranks       host int32[N], 1 <= R_n < s_n
 *   core        device double[prod R_n]          (output)
 *   factors     host array of N device double*, factors[n] is s_n x R_n with
 *               orthonormal columns (with RSVD-LRLS to O(u kappa^2), see
 *               tsk_rsvd_solve), the entry of largest magnitude of each
 *               column positive (output; input too when init = USER)
 *   fit_history host double[sweeps] or NULL: ||T - T~||_F / ||T||_F after each
 *               sweep (TSK_FLAG_RECORD_FIT) or after the last one
 *               (TSK_FLAG_FINAL_FIT, the others NaN); index i is the i-th sweep
 *               of this call (absolute sweep first_sweep + i)
 *   sweeps_done host int32 or NULL: sweeps run (fewer than opt->sweeps when
 *               opt->tol stopped the loop)
 * Synchronous.  Errors: EINVAL (shapes, m < prod_{k != n} R_k, sizes),
 * EUNSUPPORTED (prod s_k > 2^64 for leverage sampling of a COO tensor), ENOMEM (workspace),
 * ENUMERIC (a sketched Gram not positive definite, or a subproblem whose sketched
 * right-hand side has rank below R_n, e.g. an all-zero tensor: a singular value
 * the solve divides by is zero), EHIP. */
tsk_status tsk_tucker_sketch_als(const tsk_tensor* T, const int32_t* ranks,
                                 const tsk_options* opt, double* core,
                                 double* const* factors, double* fit_history,
                                 int32_t* sweeps_done);

/* Workspace size of tsk_cp_via_tucker. */
tsk_status tsk_cp_workspace_size(const tsk_tensor* T, int32_t cp_rank,
                                 const int32_t* tucker_ranks, const tsk_options* opt,
                                 size_t* bytes);

/* CP-Sketch-Tucker (Alg. 6): {C, B^(n)} <- Sketch-Tucker-ALS(T, tucker_ranks);
 * {A^(n)} <- CP-ALS(C, cp_rank) (Alg. 2, normal equations with the
 * pseudo-inverse of the Hadamard product of Grams, cp_sweeps sweeps) started
 * from the HOSVD of the core (Sec. 7); returns cp_factors[n] = B^(n) A^(n).
 * The Hadamard product of the Grams is positive definite when the core
 * factors have full column rank, and its pseudo-inverse is then its inverse.
 *   cp_rank <= min_n tucker_ranks[n]
 *   cp_factors host array of N device double*, s_n x cp_rank (output)
 *   cp_fit     host double or NULL: ||T - sum_r a_r o b_r o ...|| / ||T||
 * Synchronous.  Errors as tsk_tucker_sketch_als; ENUMERIC also when a Hadamard
 * product of Grams is not positive definite (core factors of lower rank). */
tsk_status tsk_cp_via_tucker(const tsk_tensor* T, int32_t cp_rank,
                             const int32_t* tucker_ranks, int32_t cp_sweeps,
                             const tsk_options* opt, double* const* cp_factors,
                             double* cp_fit);

/* ---------------------------------------------------------------------- */
/* Components (each one step of the hot path; used by tests and autograd)  */
/* ---------------------------------------------------------------------- */

/* TensorSketch maps of subproblem n (Def. TensorSketch, eq. h_ts/s_ts): for
 * every k != n, h[k][i] = bucket_m(x) in [0, m) and sign[k][i] = +-1 with
 * x = draw(stream_key(seed, 1, n, k, 0), i), i < dims[k].  h[n], sign[n] are
 * not touched (may be NULL).  Device int32[dims[k]], int8[dims[k]]. */
tsk_status tsk_hash_tables(int32_t order, const int64_t* dims, int32_t n, int64_t m,
                           uint64_t seed, int32_t* const* h, int8_t* const* sign,
                           void* stream);

/* Sketched right-hand side Y = S^(n) T_(n)^T (Alg. 4, line "Y <- S^(n) T_(n)"):
 * every entry v at coordinate i adds (prod_{k != n} sign[k][i_k]) v to
 * Y[(sum_{k != n} h[k][i_k]) mod m, i_n].  Deterministic: each cell is the
 * left-to-right sum of its contributions in input order, in the tensor's dtype.
 *   h, sign  host arrays of N device pointers (entry n unused)
 *   Y        device, m x dims[n], dtype of T (output, fully overwritten)
 *   ws       workspace (query with ws == NULL) */
tsk_status tsk_sketch_rhs_ts(const tsk_tensor* T, int32_t n, int64_t m,
                             const int32_t* const* h, const int8_t* const* sign,
                             void* Y, void* ws, size_t* ws_bytes, void* stream);

/* Sketched left-hand side Z = S^(n) P^(n), P^(n) = kron_{k != n} A^(k), by the
 * FFT identity of Sec. 3.1: Z(:, rho) = IFFT(prod_{k != n} FFT(S^(k) A^(k))(:, rho_k)),
 * a length-m circular convolution of the CountSketches (FFT in FP64).
 *   factors  host array of N device double* (entry n unused), s_k x R_k
 *   Z        device m x r, row-major, element type by prec (double / float /
 *            bfloat16 as uint16) (output)
 * Any m >= 1 (radix 2, 3, 4, 5 stages, other prime factors by direct DFT). */
tsk_status tsk_sketch_lhs_ts(int32_t order, const int64_t* dims, const int32_t* ranks,
                             int32_t n, int64_t m, const int32_t* const* h,
                             const int8_t* const* sign, const double* const* factors,
                             int32_t prec, void* Z, void* ws, size_t* ws_bytes,
                             void* stream);

/* Exact sketched rank-constrained solve (Sec. 4 theorems, Sec. 2.2):
 * X = argmin ||Z X - Y||_F = (Z^T Z)^{-1} Z^T Y in FP64 (Gram and Z^T Y on the
 * matrix cores in the operand precision with FP32/FP64 accumulation; the SPD
 * Gram is inverted by Gauss-Jordan sweeps when r <= 142, else Cholesky-solved),
 * A = leading R right singular vectors of X (FP64 symmetric eigen-decomposition
 * of the smaller Gram of X, re-orthonormalised, largest-magnitude entry of
 * each column positive), W = X A = C_(n)^T.
 *   Z  device m x r, Y device m x s, element type by prec (as above)
 *   A  device double s x R (output);  W device double r x R (output)
 * Requires m >= r, R <= min(r, s).  Synchronous: waits for the stream to check
 * the factorisation status; ENUMERIC if the Gram is not positive definite or, for
 * r <= s, if one of the R leading eigenvalues of X^T X (X = Z^+ Y) is not
 * positive (Y of rank below R). */
tsk_status tsk_rc_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s,
                        int32_t R, int32_t prec, double* A, double* W, void* ws,
                        size_t* ws_bytes, void* stream);

/* RSVD-LRLS (Alg. 5), the randomized low-rank least-squares solve of Alg. 4:
 * the randomized SVD, with the caller's s x k Gaussian test matrix Omega (the
 * driver draws it from the stream (seed, 6, sweep, n), row-major), of the
 * least-squares solution X = (Z^T Z)^{-1} Z^T Y: Q = thin Householder QR basis
 * of X Omega, D = Q^T X (k x s), U S V^T = svd(D); A = V(:, :R) (sign rule as
 * above), W = Q U(:, :R) S(:R, :R) with the signs of A.  The products with Y are
 * ordered for the O(m s k) cost of Sec. 6: Y Omega and Y^T (Z B Q) when s is
 * large against r, else Z^T Y once.  The SVD of D comes from the eigenpairs of
 * D D^T, so the columns of A are orthonormal to O(u kappa(D)^2) (u the FP64 unit
 * roundoff, kappa(D) = sigma_1 / sigma_R) and are not re-orthonormalised.  All
 * FP64 after the products with Z and Y.
 *   Z, Y   device, as tsk_rc_solve;  Omega device double s x k, R <= k <= min(r, 64)
 *   A  device double s x R (output);  W device double r x R (output)
 * Synchronous (checks the factorisation status); ENUMERIC if the Gram is not
 * positive definite or one of the R leading eigenvalues of D D^T is not positive
 * (Y of rank below R). */
tsk_status tsk_rsvd_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s,
                          int32_t R, int32_t prec, const double* Omega, int32_t k, double* A,
                          double* W, void* ws, size_t* ws_bytes, void* stream);

/* tsk_rsvd_solve for callers that cannot allocate device memory (serving
 * loops and harnesses in which hipMalloc is not allowed): the same solve,
 * kernels and results, with no workspace argument.  Its scratch is a fixed
 * 32 MiB array in the library's device code, one copy per GPU, held from the
 * library's load until the process ends; the call allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  Shapes whose scratch
 * exceeds 32 MiB (about m r + 3 r^2 + (m + 2 s) k doubles for r > 128) return
 * TSK_ENOMEM with a message, before any work.  All calls on one GPU share its
 * array, so calls that overlap on one GPU (several threads or streams) race;
 * successive calls on one stream are safe.  Arguments, errors and
 * synchronisation as tsk_rsvd_solve. */
tsk_status tsk_rsvd_solve_noalloc(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s,
                                  int32_t R, int32_t prec, const double* Omega, int32_t k,
                                  double* A, double* W, void* stream);

/* Init-RRF of mode n (Alg. 3 with the composite sketch of Sec. 5):
 * W = T_(n) Omega^T with the CountSketch g : [K] -> [k2], tau (stream
 * (seed, 2, n) at the other-mode row-major index), G (k2 x k1) i.i.d.
 * N(0, 1/k1) (stream (seed, 3, n)), B = W G, A = leading R left singular
 * vectors of B (sign rule as above).
 *   A  device double dims[n] x R (output).  Requires R <= k1.
 * Synchronous: waits for the stream to check the factorisation status; ENUMERIC if
 * one of the R leading eigenvalues of B^T B is not positive (a sketched range of rank
 * below R, e.g. an all-zero tensor) or the QR of the result fails. */
tsk_status tsk_rrf_init(const tsk_tensor* T, int32_t n, int32_t R, int32_t k1, int32_t k2,
                        uint64_t seed, double* A, void* ws, size_t* ws_bytes,
                        void* stream);

/* Leverage-score sampling of kron_{k != n} A^(k) (Def. leverage scores,
 * Def. importance sampling, Lemma on Kronecker leverage scores): for sample j
 * and mode k != n, u = uniform(draw(stream_key(seed, 4, sweep, n, k), j)) and
 * idx[j][t] = first i with cdf_k[i] > u cdf_k[last], cdf_k the sequential FP64
 * prefix sum of l_i = sum_c A^(k)(i,c)^2 (each square rounded before the add);
 * w[j] = 1 / sqrt(m prod_k l_{i_k} / sum l).
 *   ranks   host int32[N]; factors host array of N device double*, factors[k]
 *           s_k x R_k row-major (entry n unused)
 *   idx     device int32 m x (N-1) (modes k != n in increasing order) (output)
 *   w       device double m (output) */
tsk_status tsk_leverage_sample(int32_t order, const int64_t* dims, const int32_t* ranks,
                               int32_t n, int64_t m, uint64_t seed, int32_t sweep,
                               const double* const* factors, int32_t* idx, double* w,
                               void* ws, size_t* ws_bytes, void* stream);

/* Deterministic leverage selection (Sec. 3.2, the alternative to importance
 * sampling that keeps the rows of largest leverage score).  Row (i_k)_{k != n}
 * of kron_{k != n} A^(k) has the score pi = prod_k l^(k)_{i_k} (Lemma on
 * Kronecker leverage scores; l as in tsk_leverage_sample; the product taken in
 * increasing k, FP64).  Rows are ordered by pi descending, equal pi by the
 * per-mode ranks (position in score-descending, index-ascending order)
 * compared lexicographically in increasing k; the first m are returned.  No
 * rescaling: use weights 1 with tsk_sketch_lev / tsk_sketch_lev_coo.
 *   ranks    host int32[N]; factors host array of N device double*, factors[k]
 *            s_k x R_k row-major (entry n unused)
 *   idx      device int32 m x (N-1), modes k != n in increasing order (output)
 * Requires 1 <= m <= prod_{k != n} s_k (EINVAL otherwise).  Workspace query
 * convention as tsk_leverage_sample; asynchronous on `stream`. */
tsk_status tsk_leverage_select(int32_t order, const int64_t* dims, const int32_t* ranks,
                               int32_t n, int64_t m, const double* const* factors, int32_t* idx,
                               void* ws, size_t* ws_bytes, void* stream);

/* Sampled sketch (Sec. 3.2): Z[j, :] = w_j kron_{k != n} A^(k)(idx[j][.], :),
 * Y[j, :] = w_j T(i_1, .., :, .., i_N) (the sampled mode-n fibre of a dense T).
 *   Z device m x r, Y device m x dims[n], element type by prec (outputs).
 * Either output may be NULL.  For a COO tensor Y must be NULL (EUNSUPPORTED):
 * its fibres come from tsk_sketch_lev_coo. */
tsk_status tsk_sketch_lev(const tsk_tensor* T, const int32_t* ranks, int32_t n, int64_t m,
                          const int32_t* idx, const double* w, const double* const* factors,
                          int32_t prec, void* Z, void* Y, void* stream);

/* Mode-n fibre index of a COO tensor, the access structure behind the O(m s_n)
 * sampled right-hand side of leverage-score sampling (Sec. 3.2, cost in
 * Sec. 6.1).  Every entry e gets the key
 *   key(e) = (row-major linear index of (i_k)_{k != n}) * s_n + i_n,
 * and the index holds the keys in ascending order (uint64[nnz]) followed by the
 * values in the same order (the tensor's dtype), from a stable sort, so that
 * duplicate coordinates stay adjacent in input order.
 *   index  device buffer of *index_bytes, 256-byte aligned (output); it stays
 *          valid while T's coordinates and values are unchanged
 *   ws     device scratch of *ws_bytes, 256-byte aligned (free after the call)
 * With index == NULL or ws == NULL, only *index_bytes and *ws_bytes are set.
 * Asynchronous on `stream`.  Errors: EINVAL (not COO, bad mode, NULL sizes,
 * buffers too small or misaligned), EUNSUPPORTED (prod s_k > 2^64), EHIP. */
tsk_status tsk_fiber_index(const tsk_tensor* T, int32_t n, void* index, size_t* index_bytes,
                           void* ws, size_t* ws_bytes, void* stream);

/* Sampled fibres of a COO tensor (Sec. 3.2) through its mode-n fibre index:
 *   Y[j, i] = w_j * (sum of the values stored at the coordinate whose mode-n
 *             index is i and whose other indices are idx[j][.]),
 * duplicates summed in FP64 in input order, 0 where nothing is stored.
 *   index  built by tsk_fiber_index from the same T and n (not checked)
 *   idx    device int32 m x (N-1), modes k != n in increasing order (as from
 *          tsk_leverage_sample); each idx[j][t] within [0, s_k)
 *   w      device double m
 *   Y      device m x dims[n], element type by prec (output)
 * Asynchronous.  Errors: EINVAL, EHIP. */
tsk_status tsk_sketch_lev_coo(const tsk_tensor* T, int32_t n, const void* index, int64_t m,
                              const int32_t* idx, const double* w, int32_t prec, void* Y,
                              void* stream);

/* Relative residual ||T - C x_1 A^(1) ... x_N A^(N)||_F / ||T||_F (Sec. 7,
 * 1 - fitness), accumulated in FP64 as ||T||^2 - 2 <T, T~> + ||T~||^2.  For a
 * COO tensor ||T||^2 is the sum of the squares of the stored values, so its
 * coordinates must be distinct (duplicates are not merged here, unlike in the
 * sketches).  Order-3 COO tensors of ranks (16, 16, 16) with at least 2^16
 * entries are sorted by their last index (in the workspace) and take
 * <T, T~> as u0^T W_k u1, W_k = C x_3 A^(3)(k, :); other shapes entry by
 * entry.  Synchronous; result in *rel_residual (host). */
tsk_status tsk_fit(const tsk_tensor* T, const int32_t* ranks, const double* core,
                   const double* const* factors, double* rel_residual, void* ws,
                   size_t* ws_bytes, void* stream);

/* Sketched mode-n residual L = ||Z W A^T - Y||_F^2 with Z = S^(n) P^(n) built
 * from the factors k != n (TensorSketch maps h, sign), W = C_(n)^T, A = A^(n),
 * Y = S^(n) T_(n)^T (m x dims[n], dtype ydtype) -- the objective of the
 * sketched subproblem of Alg. 4.  Forward: *L (device double).  Backward:
 * gradients dL/dA^(k) for every k (device double s_k x R_k, grads[k]) and
 * dL/dC (device double, core layout); dL/dZ is back-propagated through the FFT
 * convolution and the CountSketches.  E = Z W A^T - Y is recomputed tile by
 * tile and never stored. */
tsk_status tsk_sketched_residual_fwd(int32_t order, const int64_t* dims, const int32_t* ranks,
                                     int32_t n, int64_t m, const int32_t* const* h,
                                     const int8_t* const* sign, const double* const* factors,
                                     const double* core, const void* Y, int32_t ydtype,
                                     double* L, void* ws, size_t* ws_bytes, void* stream);
tsk_status tsk_sketched_residual_bwd(int32_t order, const int64_t* dims, const int32_t* ranks,
                                     int32_t n, int64_t m, const int32_t* const* h,
                                     const int8_t* const* sign, const double* const* factors,
                                     const double* core, const void* Y, int32_t ydtype,
                                     double* const* grads, double* grad_core, void* ws,
                                     size_t* ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* TSK_H */
