// FP64 dense linear algebra of the sketched solve, on the GPU.
//
//   cholesky          in-place lower Cholesky of the sketched Gram Z^T Z
//   chol_solve_rows   X <- X G^{-1} row block by row block (X^T = (Z^T Z)^{-1} Z^T Y)
//   sym_eig_top       leading R eigenpairs of a symmetric q x q matrix:
//                     Householder tridiagonalisation, eigenvalues by Sturm-count
//                     multisection (64 points per wave per step), eigenvectors by
//                     inverse iteration on the tridiagonal (partial-pivoting LU),
//                     modified Gram-Schmidt in eigenvalue order, back-transform
//   sign_fix_columns  largest-magnitude entry of every column made positive
//   cholqr            one CholeskyQR pass, A <- A chol(A^T A)^{-T}
//
// These problems are small (q <= ~1000) and latency-bound; every kernel is a
// single workgroup (or one workgroup per row block) so that the whole solve
// stays on the device without host round trips.

#include <cfloat>

#include "common.h"
#include "kernels.h"

namespace tsk {

namespace {

// ------------------------------------------------------------ reductions ----
template <int NT>
__device__ double block_sum(double v, double* red) {
  // fixed-order: wave shuffles then waves in order (deterministic)
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

__device__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// -------------------------------------------------------------- cholesky ----
constexpr int kCholT = 512;
__global__ __launch_bounds__(kCholT) void k_cholesky(double* G, int64_t n, int64_t lda,
                                                     int* info, int use_lds) {
  extern __shared__ double smem[];
  __shared__ double diag;
  double* a = G;
  int64_t ld = lda;
  if (use_lds) {
    a = smem;
    ld = n;
    for (int64_t t = threadIdx.x; t < n * n; t += kCholT) smem[t] = G[(t / n) * lda + t % n];
    __syncthreads();
  }
  if (threadIdx.x == 0) *info = 0;
  for (int64_t j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      double d = a[j * ld + j];
      if (!(d > 0.0) && *info == 0) *info = int(j + 1);
      d = sqrt(d);
      a[j * ld + j] = d;
      diag = d;
    }
    __syncthreads();
    const double d = diag;
    for (int64_t i = j + 1 + threadIdx.x; i < n; i += kCholT) a[i * ld + j] /= d;
    __syncthreads();
    const int64_t L = n - j - 1;
    for (int64_t t = threadIdx.x; t < L * L; t += kCholT) {
      int64_t i = j + 1 + t / L, k = j + 1 + t % L;
      if (k <= i) a[i * ld + k] -= a[i * ld + j] * a[k * ld + j];
    }
    __syncthreads();
  }
  if (use_lds)
    for (int64_t t = threadIdx.x; t < n * n; t += kCholT) {
      int64_t i = t / n, k = t % n;
      G[i * lda + k] = k <= i ? smem[t] : 0.0;
    }
  else
    for (int64_t t = threadIdx.x; t < n * n; t += kCholT) {
      int64_t i = t / n, k = t % n;
      if (k > i) G[i * lda + k] = 0.0;
    }
}

// rows of X <- rows of X L^{-T} (forward) then X L^{-1} (backward): X G^{-1}
constexpr int kSolveT = 256;
__global__ __launch_bounds__(kSolveT) void k_chol_solve_rows(const double* L, int64_t n,
                                                             int64_t ldl, double* X,
                                                             int64_t rows, int64_t ldx,
                                                             int64_t rb, int forward_only) {
  extern __shared__ double xs[];  // rb x n
  const int64_t r0 = int64_t(blockIdx.x) * rb;
  const int64_t nr = rows - r0 < rb ? rows - r0 : rb;
  for (int64_t t = threadIdx.x; t < nr * n; t += kSolveT) xs[t] = X[(r0 + t / n) * ldx + t % n];
  __syncthreads();
  // forward: y L^T = x  ->  y_j = (x_j - sum_{i<j} L_ji y_i) / L_jj, column-oriented
  for (int64_t j = 0; j < n; ++j) {
    const double djj = L[j * ldl + j];
    for (int64_t rr = threadIdx.x; rr < nr; rr += kSolveT) xs[rr * n + j] /= djj;
    __syncthreads();
    const int64_t rem = n - j - 1;
    for (int64_t t = threadIdx.x; t < nr * rem; t += kSolveT) {
      int64_t rr = t / rem, i = j + 1 + t % rem;
      xs[rr * n + i] -= L[i * ldl + j] * xs[rr * n + j];
    }
    __syncthreads();
  }
  if (!forward_only) {
    // backward: x L = y  ->  x_j = (y_j - sum_{i>j} x_i L_ij) / L_jj
    for (int64_t j = n - 1; j >= 0; --j) {
      const double djj = L[j * ldl + j];
      for (int64_t rr = threadIdx.x; rr < nr; rr += kSolveT) xs[rr * n + j] /= djj;
      __syncthreads();
      for (int64_t t = threadIdx.x; t < nr * j; t += kSolveT) {
        int64_t rr = t / j, i = t % j;
        xs[rr * n + i] -= L[j * ldl + i] * xs[rr * n + j];
      }
      __syncthreads();
    }
  }
  for (int64_t t = threadIdx.x; t < nr * n; t += kSolveT) X[(r0 + t / n) * ldx + t % n] = xs[t];
}

// ----------------------------------------------------------- eigen (top R) ----
constexpr int kEigT = 512;
constexpr int kEigWaves = kEigT / 64;

// number of eigenvalues of the tridiagonal (d, e2 = e^2) smaller than x
__device__ int sturm_count(const double* d, const double* e2, int q, double x, double pivmin) {
  int c = 0;
  double t = d[0] - x;
  if (t < 0.0) ++c;
  for (int i = 1; i < q; ++i) {
    if (fabs(t) <= pivmin) t = -pivmin;
    t = d[i] - x - e2[i - 1] / t;
    if (t < 0.0) ++c;
  }
  return c;
}

// Solve (T - lam I) x = b by LU with partial pivoting (tridiagonal, fill in
// the second superdiagonal).  Factors in u0,u1,u2,mu, piv; b overwritten by x.
__device__ void tri_factor(const double* d, const double* e, int q, double lam, double tiny,
                           double* u0, double* u1, double* u2, double* mu, int8_t* piv) {
  double p = d[0] - lam, qq = q > 1 ? e[0] : 0.0, rr = 0.0;
  for (int i = 0; i < q - 1; ++i) {
    const double c = e[i], a1 = d[i + 1] - lam, b1 = i + 1 < q - 1 ? e[i + 1] : 0.0;
    if (fabs(p) >= fabs(c)) {
      double pv = p == 0.0 ? tiny : p;
      u0[i] = pv, u1[i] = qq, u2[i] = rr, piv[i] = 0;
      double mlt = c / pv;
      mu[i] = mlt;
      p = a1 - mlt * qq;
      qq = b1 - mlt * rr;
      rr = 0.0;
    } else {
      u0[i] = c, u1[i] = a1, u2[i] = b1, piv[i] = 1;
      double mlt = p / c;
      mu[i] = mlt;
      double np = qq - mlt * a1, nq = rr - mlt * b1;
      p = np;
      qq = nq;
      rr = 0.0;
    }
  }
  u0[q - 1] = p == 0.0 ? tiny : p;
  u1[q - 1] = 0.0;
  u2[q - 1] = 0.0;
}

__device__ void tri_solve(int q, const double* u0, const double* u1, const double* u2,
                          const double* mu, const int8_t* piv, double* x) {
  for (int i = 0; i < q - 1; ++i) {
    if (piv[i]) {
      double t = x[i];
      x[i] = x[i + 1];
      x[i + 1] = t;
    }
    x[i + 1] -= mu[i] * x[i];
  }
  for (int i = q - 1; i >= 0; --i) {
    double s = x[i];
    if (i + 1 < q) s -= u1[i] * x[i + 1];
    if (i + 2 < q) s -= u2[i] * x[i + 2];
    x[i] = s / u0[i];
  }
}

__global__ __launch_bounds__(kEigT) void k_sym_eig_top(double* Mg, int q, int R, double* lam,
                                                       double* V, double* scratch,
                                                       int8_t* pivs, int use_lds) {
  extern __shared__ double smem[];
  __shared__ double red[kEigWaves];
  __shared__ double sh[4];
  double* M = use_lds ? smem : Mg;
  double* d = (use_lds ? smem + size_t(q) * q : smem);
  double* e = d + q;
  double* e2 = e + q;
  double* pw = e2 + q;  // p then w
  double* bet = pw + q;
  if (use_lds) {
    for (int t = threadIdx.x; t < q * q; t += kEigT) M[t] = Mg[t];
    __syncthreads();
  }
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  // ---- Householder tridiagonalisation (lower) ----
  for (int k = 0; k + 2 < q; ++k) {
    const int L = q - k - 1;
    const double* x = M + size_t(k + 1) * q + k;  // stride q
    double part = 0.0;
    for (int i = tid; i < L; i += kEigT) part += x[size_t(i) * q] * x[size_t(i) * q];
    const double norm2 = block_sum<kEigT>(part, red);
    const double x0 = x[0];
    const double alpha = norm2 > 0.0 ? -copysign(sqrt(norm2), x0) : 0.0;
    const double v0 = x0 - alpha;
    const double vtv = norm2 - x0 * x0 + v0 * v0;
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    __syncthreads();
    if (tid == 0) {
      d[k] = M[size_t(k) * q + k];
      e[k] = norm2 > 0.0 ? alpha : x0;
      bet[k] = beta;
      M[size_t(k + 1) * q + k] = v0;  // v stored in column k below the diagonal
    }
    __syncthreads();
    if (beta != 0.0) {
      double* A22 = M + size_t(k + 1) * q + (k + 1);
      // p_i = beta sum_j A22[j][i] v_j
      for (int i = tid; i < L; i += kEigT) {
        double s = 0.0;
        for (int j = 0; j < L; ++j) s += A22[size_t(j) * q + i] * x[size_t(j) * q];
        pw[i] = beta * s;
      }
      __syncthreads();
      double part2 = 0.0;
      for (int i = tid; i < L; i += kEigT) part2 += x[size_t(i) * q] * pw[i];
      const double K = 0.5 * beta * block_sum<kEigT>(part2, red);
      __syncthreads();
      for (int i = tid; i < L; i += kEigT) pw[i] = pw[i] - K * x[size_t(i) * q];
      __syncthreads();
      for (int t = tid; t < L * L; t += kEigT) {
        int i = t / L, j = t % L;
        A22[size_t(i) * q + j] -= x[size_t(i) * q] * pw[j] + pw[i] * x[size_t(j) * q];
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (q >= 2) {
      d[q - 2] = M[size_t(q - 2) * q + (q - 2)];
      e[q - 2] = M[size_t(q - 1) * q + (q - 2)];
      if (q >= 3) bet[q - 2] = 0.0;
    }
    d[q - 1] = M[size_t(q - 1) * q + (q - 1)];
    double lo = DBL_MAX, hi = -DBL_MAX, emax2 = 0.0, onenrm = 0.0;
    for (int i = 0; i < q; ++i) {
      double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < q ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      onenrm = fmax(onenrm, fabs(d[i]) + r);
      if (i + 1 < q) {
        e2[i] = e[i] * e[i];
        emax2 = fmax(emax2, e2[i]);
      }
    }
    double pad = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + DBL_MIN;
    sh[0] = lo - pad;
    sh[1] = hi + pad;
    sh[2] = DBL_MIN * fmax(1.0, emax2);
    sh[3] = onenrm;
  }
  __syncthreads();
  const double glo = sh[0], ghi = sh[1], pivmin = sh[2], onenrm = sh[3];

  // ---- eigenvalues: multisection, one wave per eigenvalue ----
  for (int t = wave; t < R; t += kEigWaves) {
    const int target = q - 1 - t;  // ascending index
    double lo = glo, hi = ghi;
    for (int it = 0; it < 64; ++it) {
      const double width = hi - lo;
      if (width <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
      const double xl = lo + width * double(lane + 1) / 65.0;
      const int c = sturm_count(d, e2, q, xl, pivmin);
      const uint64_t above = __ballot(c > target);
      double nlo, nhi;
      if (above == 0ull) {
        nlo = __shfl(xl, 63);
        nhi = hi;
      } else {
        const int f = __ffsll((unsigned long long)above) - 1;
        nhi = __shfl(xl, f);
        nlo = f > 0 ? __shfl(xl, f - 1) : lo;
      }
      if (nlo == lo && nhi == hi) break;
      lo = nlo;
      hi = nhi;
    }
    if (lane == 0) lam[t] = 0.5 * (lo + hi);
  }
  __syncthreads();

  // ---- eigenvectors of the tridiagonal: inverse iteration, one lane each ----
  double* y = scratch;                       // R x q
  double* lu = scratch + size_t(R) * q;      // R x 4q
  const double tiny = DBL_EPSILON * fmax(onenrm, DBL_MIN);
  for (int t = tid; t < R; t += kEigT) {
    double* yt = y + size_t(t) * q;
    double* u0 = lu + size_t(t) * 4 * q;
    double* u1 = u0 + q;
    double* u2 = u1 + q;
    double* mu = u2 + q;
    int8_t* pv = pivs + size_t(t) * q;
    tri_factor(d, e, q, lam[t], tiny, u0, u1, u2, mu, pv);
    for (int i = 0; i < q; ++i) {
      uint32_t hsh = uint32_t(i) * 2654435761u + uint32_t(t + 1) * 40503u;
      yt[i] = 1.0 + double((hsh >> 8) & 1023u) / 2048.0;
    }
    for (int it = 0; it < 4; ++it) {
      tri_solve(q, u0, u1, u2, mu, pv, yt);
      double nrm = 0.0, mx = 0.0;
      for (int i = 0; i < q; ++i) mx = fmax(mx, fabs(yt[i]));
      mx = mx > 0.0 ? mx : 1.0;
      for (int i = 0; i < q; ++i) {
        yt[i] /= mx;
        nrm += yt[i] * yt[i];
      }
      nrm = 1.0 / sqrt(nrm);
      for (int i = 0; i < q; ++i) yt[i] *= nrm;
    }
  }
  __syncthreads();
  // ---- modified Gram-Schmidt in eigenvalue order (wave 0) ----
  if (wave == 0) {
    for (int t = 0; t < R; ++t) {
      double* yt = y + size_t(t) * q;
      for (int u = 0; u < t; ++u) {
        const double* yu = y + size_t(u) * q;
        double s = 0.0;
        for (int i = lane; i < q; i += 64) s += yu[i] * yt[i];
        s = wave_sum(s);
        for (int i = lane; i < q; i += 64) yt[i] -= s * yu[i];
      }
      double s = 0.0;
      for (int i = lane; i < q; i += 64) s += yt[i] * yt[i];
      s = 1.0 / sqrt(wave_sum(s));
      for (int i = lane; i < q; i += 64) yt[i] *= s;
    }
  }
  __syncthreads();
  // ---- back-transform y <- H_0 H_1 ... H_{q-3} y, one wave per vector ----
  for (int t = wave; t < R; t += kEigWaves) {
    double* yt = y + size_t(t) * q;
    for (int k = q - 3; k >= 0; --k) {
      const double beta = bet[k];
      if (beta == 0.0) continue;
      const int L = q - k - 1;
      const double* v = M + size_t(k + 1) * q + k;
      double s = 0.0;
      for (int i = lane; i < L; i += 64) s += v[size_t(i) * q] * yt[k + 1 + i];
      s = beta * wave_sum(s);
      for (int i = lane; i < L; i += 64) yt[k + 1 + i] -= s * v[size_t(i) * q];
    }
    for (int i = lane; i < q; i += 64) V[size_t(i) * R + t] = yt[i];
  }
}

// -------------------------------------------------------------- sign fix ----
__global__ void k_sign_fix(double* A, int64_t rows, int64_t R) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int64_t c = blockIdx.x;
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    double a = fabs(A[i * R + c]);
    if (a > best) best = a, bidx = i;  // first maximum within the thread's stride
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (threadIdx.x < off) {
      double o = bv[threadIdx.x + off];
      int64_t oi = bi[threadIdx.x + off];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x]))
        bv[threadIdx.x] = o, bi[threadIdx.x] = oi;
    }
    __syncthreads();
  }
  const bool flip = A[bi[0] * R + c] < 0.0;
  __syncthreads();
  if (flip)
    for (int64_t i = threadIdx.x; i < rows; i += 256) A[i * R + c] = -A[i * R + c];
}

__global__ void k_scale_inv_sqrt(double* A, int64_t rows, int64_t R, const double* lam) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= rows * R) return;
  A[t] /= sqrt(lam[t % R]);
}

__global__ void k_transpose(const double* A, int64_t rows, int64_t cols, double* At) {
  __shared__ double tile[32][33];
  int64_t bx = int64_t(blockIdx.x) * 32, by = int64_t(blockIdx.y) * 32;
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    int64_t r = by + yy, c = bx + threadIdx.x;
    if (r < rows && c < cols) tile[yy][threadIdx.x] = A[r * cols + c];
  }
  __syncthreads();
  for (int yy = threadIdx.y; yy < 32; yy += 8) {
    int64_t c = bx + yy, r = by + threadIdx.x;
    if (r < rows && c < cols) At[c * rows + r] = tile[threadIdx.x][yy];
  }
}

int max_lds_bytes() {
  static int v = -1;
  if (v < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
  }
  return v;
}

}  // namespace

tsk_status cholesky(double* G, int64_t n, int64_t lda, int* info, hipStream_t st) {
  size_t bytes = size_t(n) * n * 8;
  int use_lds = bytes <= size_t(max_lds_bytes()) - 1024 ? 1 : 0;
  hipLaunchKernelGGL(k_cholesky, dim3(1), dim3(kCholT), use_lds ? bytes : 0, st, G, n, lda, info,
                     use_lds);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status chol_solve_rows(const double* L, int64_t n, int64_t ldl, double* X, int64_t rows,
                           int64_t ldx, bool forward_only, hipStream_t st) {
  if (rows == 0 || n == 0) return TSK_OK;
  int64_t budget = (max_lds_bytes() - 1024) / 8;
  int64_t rb = budget / n;
  if (rb > 64) rb = 64;
  if (rb < 1) {
    set_error("triangular solve of order %lld exceeds the LDS budget", (long long)n);
    return TSK_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(k_chol_solve_rows, dim3(ceil_div(rows, rb)), dim3(kSolveT),
                     size_t(rb * n * 8), st, L, n, ldl, X, rows, ldx, rb, forward_only ? 1 : 0);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status sym_eig_top(double* M, int64_t q, int64_t R, double* lam, double* V, Ws& ws,
                       hipStream_t st) {
  double* scratch = ws.take<double>(size_t(R) * q * 5);
  int8_t* pivs = ws.take<int8_t>(size_t(R) * q);
  if (ws.measuring()) return TSK_OK;
  size_t small = size_t(5) * q * 8;
  size_t full = size_t(q) * q * 8 + small;
  int use_lds = full + 2048 <= size_t(max_lds_bytes()) ? 1 : 0;
  if (!use_lds && small + 2048 > size_t(max_lds_bytes())) {
    set_error("eigenproblem of order %lld exceeds the LDS budget", (long long)q);
    return TSK_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(k_sym_eig_top, dim3(1), dim3(kEigT), use_lds ? full : small, st, M, int(q),
                     int(R), lam, V, scratch, pivs, use_lds);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status sign_fix_columns(double* A, int64_t rows, int64_t R, hipStream_t st) {
  hipLaunchKernelGGL(k_sign_fix, dim3(R), dim3(256), 0, st, A, rows, R);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status scale_columns_inv_sqrt(double* A, int64_t rows, int64_t R, const double* lam,
                                  hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(ceil_div(rows * R, 256)), dim3(256), 0, st, A, rows,
                     R, lam);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status transpose_f64(const double* A, int64_t rows, int64_t cols, double* At,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_transpose, dim3(ceil_div(cols, 32), ceil_div(rows, 32)), dim3(32, 8), 0,
                     st, A, rows, cols, At);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status cholqr(double* A, int64_t rows, int64_t R, int* info, Ws& ws, hipStream_t st) {
  double* G = ws.take<double>(R * R);
  TSK_TRY(gemm_tn(TSK_PREC_F64, R, R, rows, A, R, R, nullptr, 0, A, R, G, R, ws, st));
  if (ws.measuring()) return TSK_OK;
  TSK_TRY(cholesky(G, R, R, info, st));
  TSK_TRY(chol_solve_rows(G, R, R, A, rows, R, true, st));
  return TSK_OK;
}

}  // namespace tsk
