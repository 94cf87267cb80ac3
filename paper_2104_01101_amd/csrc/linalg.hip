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
#include <type_traits>

#include "common.h"
#include "kernels.h"
#include "skinny.h"
#include "wave.h"

namespace tsk {

namespace {

typedef double dx4 __attribute__((ext_vector_type(4)));  // FP64 MFMA accumulator

// ------------------------------------------------------------ reductions ----
template <int NT>
__device__ double block_sum(double v, double* red) {
  // fixed-order: wave sum then waves in order (deterministic)
  v = wave_allsum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NT / 64; ++w) s += red[w];
  return s;
}

__device__ double wave_sum(double v) { return wave_allsum(v); }

// f(integral_constant<int, I>) for I = B, B+1, ..., E-1 (or downwards when
// DOWN): loop bodies whose register-array indices must be constants.
template <int B, int E, bool DOWN = false, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    if constexpr (DOWN) {
      f(std::integral_constant<int, E - 1>{});
      static_for<B, E - 1, true>(f);
    } else {
      f(std::integral_constant<int, B>{});
      static_for<B + 1, E, false>(f);
    }
  }
}

// -------------------------------------------------------------- cholesky ----
constexpr int kCholT = 256;
constexpr int kCholWaves = kCholT / 64;
template <bool LDS>
__global__ __launch_bounds__(kCholT) void k_cholesky(double* G, int n, int lda, int* info) {
  extern __shared__ double smem[];
  double* a = LDS ? smem : G;
  const int ld = LDS ? n : lda;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (LDS) {
    for (int i = wave; i < n; i += kCholWaves)
      for (int k = lane; k <= i; k += 64) smem[i * n + k] = G[i * lda + k];
    __syncthreads();
  }
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    const double piv = a[j * ld + j];
    if (!(piv > 0.0) && bad == 0) bad = j + 1;
    const double dj = sqrt(piv), rj = 1.0 / dj;
    // column j below the diagonal
    for (int i = j + 1 + tid; i < n; i += kCholT) a[i * ld + j] *= rj;
    __syncthreads();
    if (tid == 0) a[j * ld + j] = dj;
    // trailing lower triangle: rows by wave, columns by lane
    for (int i = j + 1 + wave; i < n; i += kCholWaves) {
      const double lij = a[i * ld + j];
      for (int k = j + 1 + lane; k <= i; k += 64) a[i * ld + k] -= lij * a[k * ld + j];
    }
    __syncthreads();
  }
  if (tid == 0 && bad) *info = bad;  // sticky: the caller zeroes info once per job
  for (int i = wave; i < n; i += kCholWaves)
    for (int k = lane; k < n; k += 64) G[i * lda + k] = k <= i ? a[i * ld + k] : 0.0;
}

// ------------------------------------------------------ SPD inverse (GJ) ----
// Gauss-Jordan on an SPD matrix needs no pivoting; the pivots are the
// Cholesky pivots squared, so a non-positive one flags a non-SPD Gram.
constexpr int kGjT = 512;
__global__ __launch_bounds__(kGjT) void k_spd_inverse(double* G, int n, int lda, int* info) {
  extern __shared__ double a[];  // n x n
  constexpr int NW = kGjT / 64;
  __shared__ double prow_inv;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = wave; i < n; i += NW)
    for (int k = lane; k < n; k += 64) a[i * n + k] = G[i * lda + k];
  __syncthreads();
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    const double piv = a[j * n + j];
    if (!(piv > 0.0) && bad == 0) bad = j + 1;
    const double pinv = 1.0 / piv;
    __syncthreads();  // everyone has read the pivot
    for (int k = tid; k < n; k += kGjT) a[j * n + k] = k == j ? pinv : a[j * n + k] * pinv;
    __syncthreads();
    for (int i = wave; i < n; i += NW) {
      if (i == j) continue;
      const double f = a[i * n + j];
      for (int k = lane; k < n; k += 64) {
        const double rk = a[j * n + k];
        a[i * n + k] = k == j ? -f * pinv : a[i * n + k] - f * rk;
      }
    }
    __syncthreads();
  }
  (void)prow_inv;
  if (tid == 0 && bad) *info = bad;  // sticky: the caller zeroes info once per job
  for (int i = wave; i < n; i += NW)
    for (int k = lane; k < n; k += 64) G[i * lda + k] = a[i * n + k];
}

// rows of X <- rows of X G^{-1} (X L^{-T} then L^{-1}); forward_only: X L^{-T}.
// Thread per row with L in LDS (used when L and the row block fit).
constexpr int kRowT = 64;
__global__ __launch_bounds__(kRowT) void k_chol_solve_rows_lds(const double* Lg, int n, int ldl,
                                                               double* X, int rows, int ldx,
                                                               int forward_only) {
  extern __shared__ double smem[];
  double* L = smem;                 // n x n (lower)
  double* xs = smem + n * n;        // kRowT rows, stride n + 1
  const int stride = n + 1;
  for (int t = threadIdx.x; t < n * n; t += kRowT) {
    const int i = t / n, k = t - (t / n) * n;
    L[t] = k <= i ? Lg[i * ldl + k] : 0.0;
  }
  const int r0 = blockIdx.x * kRowT;
  const int nr = rows - r0 < kRowT ? rows - r0 : kRowT;
  for (int t = threadIdx.x; t < nr * n; t += kRowT) {
    const int rr = t / n, c = t - (t / n) * n;
    xs[rr * stride + c] = X[int64_t(r0 + rr) * ldx + c];
  }
  __syncthreads();
  const int rr = threadIdx.x;
  if (rr < nr) {
    double* x = xs + rr * stride;
    for (int j = 0; j < n; ++j) {  // y L^T = x
      const double* lj = L + j * n;
      double a0 = x[j], a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int i = 0;
      for (; i + 3 < j; i += 4) {
        a0 -= lj[i] * x[i];
        a1 -= lj[i + 1] * x[i + 1];
        a2 -= lj[i + 2] * x[i + 2];
        a3 -= lj[i + 3] * x[i + 3];
      }
      for (; i < j; ++i) a0 -= lj[i] * x[i];
      x[j] = ((a0 + a1) + (a2 + a3)) / lj[j];
    }
    if (!forward_only)
      for (int j = n - 1; j >= 0; --j) {  // x L = y
        double a0 = x[j], a1 = 0.0, a2 = 0.0, a3 = 0.0;
        int i = j + 1;
        for (; i + 3 < n; i += 4) {
          a0 -= L[i * n + j] * x[i];
          a1 -= L[(i + 1) * n + j] * x[i + 1];
          a2 -= L[(i + 2) * n + j] * x[i + 2];
          a3 -= L[(i + 3) * n + j] * x[i + 3];
        }
        for (; i < n; ++i) a0 -= L[i * n + j] * x[i];
        x[j] = ((a0 + a1) + (a2 + a3)) / L[j * n + j];
      }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nr * n; t += kRowT) {
    const int q = t / n, c = t - (t / n) * n;
    X[int64_t(r0 + q) * ldx + c] = xs[q * stride + c];
  }
}

// same, column-oriented over a row block, L read from global memory (large n)
constexpr int kSolveT = 256;
__global__ __launch_bounds__(kSolveT) void k_chol_solve_rows(const double* L, int n, int ldl,
                                                             double* X, int rows, int ldx, int rb,
                                                             int forward_only) {
  extern __shared__ double xs[];  // rb x n
  const int r0 = blockIdx.x * rb;
  const int nr = rows - r0 < rb ? rows - r0 : rb;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = kSolveT / 64;
  for (int q = wave; q < nr; q += nw)
    for (int c = lane; c < n; c += 64) xs[q * n + c] = X[int64_t(r0 + q) * ldx + c];
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double djj = L[j * ldl + j];
    for (int q = tid; q < nr; q += kSolveT) xs[q * n + j] /= djj;
    __syncthreads();
    for (int q = wave; q < nr; q += nw) {
      const double xj = xs[q * n + j];
      for (int i = j + 1 + lane; i < n; i += 64) xs[q * n + i] -= L[i * ldl + j] * xj;
    }
    __syncthreads();
  }
  if (!forward_only) {
    for (int j = n - 1; j >= 0; --j) {
      const double djj = L[j * ldl + j];
      for (int q = tid; q < nr; q += kSolveT) xs[q * n + j] /= djj;
      __syncthreads();
      for (int q = wave; q < nr; q += nw) {
        const double xj = xs[q * n + j];
        for (int i = lane; i < j; i += 64) xs[q * n + i] -= L[j * ldl + i] * xj;
      }
      __syncthreads();
    }
  }
  for (int q = wave; q < nr; q += nw)
    for (int c = lane; c < n; c += 64) X[int64_t(r0 + q) * ldx + c] = xs[q * n + c];
}

// ----------------------------------------------------------- eigen (top R) ----
constexpr int kEigT = 512;

// 1/t from the hardware reciprocal plus one Newton step (close to full FP64
// accuracy, no division sequence).
__device__ inline double rcp64(double t) {
  const double r = __builtin_amdgcn_rcp(t);
  return fma(r, fma(-t, r, 1.0), r);
}

// number of eigenvalues of the tridiagonal (d, e2 = e^2) smaller than x; the
// pivot recurrence uses rcp64, i.e. it counts for a tridiagonal perturbed in
// the last bits, which moves eigenvalue boundaries by O(eps ||T||).
__device__ int sturm_count(const double* d, const double* e2, int q, double x, double pivmin) {
  int c = 0;
  double t = d[0] - x;
  if (t < 0.0) ++c;
  int i = 1;
  for (; i + 3 < q; i += 4) {  // loads batched ahead of the dependent chain
    const double d0 = d[i] - x, d1 = d[i + 1] - x, d2 = d[i + 2] - x, d3 = d[i + 3] - x;
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
    if (fabs(t) <= pivmin) t = -pivmin;
    t = d0 - f0 * rcp64(t);
    c += t < 0.0;
    if (fabs(t) <= pivmin) t = -pivmin;
    t = d1 - f1 * rcp64(t);
    c += t < 0.0;
    if (fabs(t) <= pivmin) t = -pivmin;
    t = d2 - f2 * rcp64(t);
    c += t < 0.0;
    if (fabs(t) <= pivmin) t = -pivmin;
    t = d3 - f3 * rcp64(t);
    c += t < 0.0;
  }
  for (; i < q; ++i) {
    if (fabs(t) <= pivmin) t = -pivmin;
    t = (d[i] - x) - e2[i - 1] * rcp64(t);
    if (t < 0.0) ++c;
  }
  return c;
}

// Solve (T - lam I) x = b by LU with partial pivoting (tridiagonal, fill in
// the second superdiagonal).  Factors in u0 (reciprocal pivots), u1, u2, mu,
// piv; b overwritten by x.
__device__ void tri_factor(const double* d, const double* e, int q, double lam, double tiny,
                           double* u0, double* u1, double* u2, double* mu, int8_t* piv) {
  double p = d[0] - lam, qq = q > 1 ? e[0] : 0.0, rr = 0.0;
  for (int i = 0; i < q - 1; ++i) {
    const double c = e[i], a1 = d[i + 1] - lam, b1 = i + 1 < q - 1 ? e[i + 1] : 0.0;
    if (fabs(p) >= fabs(c)) {
      double pv = p == 0.0 ? tiny : p;
      u0[i] = 1.0 / pv, u1[i] = qq, u2[i] = rr, piv[i] = 0;
      double mlt = c / pv;
      mu[i] = mlt;
      p = a1 - mlt * qq;
      qq = b1 - mlt * rr;
      rr = 0.0;
    } else {
      u0[i] = 1.0 / c, u1[i] = a1, u2[i] = b1, piv[i] = 1;
      double mlt = p / c;
      mu[i] = mlt;
      double np = qq - mlt * a1, nq = rr - mlt * b1;
      p = np;
      qq = nq;
      rr = 0.0;
    }
  }
  u0[q - 1] = 1.0 / (p == 0.0 ? tiny : p);
  u1[q - 1] = 0.0;
  u2[q - 1] = 0.0;
}

// x <- (T - lam I)^{-1} (scale * x); returns ||x||^2
__device__ double tri_solve(int q, const double* u0, const double* u1, const double* u2,
                            const double* mu, const int8_t* piv, double* x, double scale) {
  double prev = x[0] * scale;
  for (int i = 0; i < q - 1; ++i) {
    double nx = x[i + 1] * scale;
    if (piv[i]) {
      const double t = prev;
      prev = nx;
      nx = t;
    }
    x[i] = prev;
    prev = nx - mu[i] * prev;
  }
  x[q - 1] = prev;
  double n2 = 0.0, x1 = 0.0, x2 = 0.0;
  for (int i = q - 1; i >= 0; --i) {
    const double xi = (x[i] - u1[i] * x1 - u2[i] * x2) * u0[i];
    x[i] = xi;
    n2 += xi * xi;
    x2 = x1;
    x1 = xi;
  }
  return n2;
}

// Layout of the kernel's working set: M (q x q) and the vector scratch
// (d, e, e2, p, beta: 5q; y: R q; LU factors: 4 R q; pivots: R q bytes) each
// live in LDS when they fit, else in the global scratch.  `timers` (optional)
// receives wall-clock stamps at the phase boundaries.
// Eigenvalues and eigenvectors from the tridiagonal (d, e) and the stored
// reflectors (reflector k: v in column k of Vr below the diagonal, stride q,
// beta in bet[k]): multisection, inverse iteration, Gram-Schmidt, back-transform.
template <int NT>
__device__ void eig_tail(int q, int R, double* d, double* e, double* e2, const double* bet,
                         const double* Vr, double* y, double* lu, int8_t* pivs, double* sh,
                         double* lam, double* V, uint64_t* timers) {
  constexpr int NW = NT / 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // d, e complete (d[q-1], e[q-2] included), bet[k] for k <= q-3, bet[q-2] = 0
  if (timers && tid == 0) timers[1] = wall_clock64();
  if (tid == 0) {
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

  // ---- eigenvalues: multisection; G lanes per eigenvalue (G = 64, 32 or 16,
  // chosen so that all R eigenvalues are bracketed in as few rounds as
  // possible), G points per step ----
  {
    const int per_wave = R <= NW ? 1 : (R <= 2 * NW ? 2 : 4);
    const int G = 64 / per_wave;
    const int gi = lane / G, gl = lane % G;
    const uint64_t gmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    for (int t0 = 0; t0 < R; t0 += NW * per_wave) {
      const int t = t0 + wave * per_wave + gi;
      const int target = q - 1 - (t < R ? t : 0);  // ascending index
      double lo = glo, hi = ghi;
      bool done = t >= R;
      for (int it = 0; it < 64; ++it) {
        const double width = hi - lo;
        if (width <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) done = true;
        if (__ballot(!done) == 0ull) break;
        const double xl = lo + width * double(gl + 1) / double(G + 1);
        const int c = done ? 0 : sturm_count(d, e2, q, xl, pivmin);
        const uint64_t above = (__ballot(c > target) >> (gi * G)) & gmask;
        double nlo, nhi;
        if (above == 0ull) {
          nlo = __shfl(xl, gi * G + G - 1);
          nhi = hi;
        } else {
          const int f = __ffsll((unsigned long long)above) - 1;
          nhi = __shfl(xl, gi * G + f);
          nlo = f > 0 ? __shfl(xl, gi * G + f - 1) : lo;
        }
        if (!done) {
          if (nlo == lo && nhi == hi) done = true;
          lo = nlo;
          hi = nhi;
        }
      }
      if (t < R && gl == 0) lam[t] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();
  if (timers && tid == 0) timers[2] = wall_clock64();

  // ---- eigenvectors of the tridiagonal: inverse iteration, one lane each ----
  const double tiny = DBL_EPSILON * fmax(onenrm, DBL_MIN);
  for (int t = tid; t < R; t += NT) {
    double* yt = y + t * q;
    double* u0 = lu + t * 4 * q;
    double* u1 = u0 + q;
    double* u2 = u1 + q;
    double* mu = u2 + q;
    int8_t* pv = pivs + t * q;
    tri_factor(d, e, q, lam[t], tiny, u0, u1, u2, mu, pv);
    for (int i = 0; i < q; ++i) {
      uint32_t hsh = uint32_t(i) * 2654435761u + uint32_t(t + 1) * 40503u;
      yt[i] = 1.0 + double((hsh >> 8) & 1023u) / 2048.0;
    }
    double scale = 1.0;
    for (int it = 0; it < 3; ++it) scale = 1.0 / sqrt(tri_solve(q, u0, u1, u2, mu, pv, yt, scale));
    for (int i = 0; i < q; ++i) yt[i] *= scale;
  }
  __syncthreads();
  if (timers && tid == 0) timers[3] = wall_clock64();
  // ---- modified Gram-Schmidt in eigenvalue order (wave 0) ----
  if (wave == 0) {
    for (int t = 0; t < R; ++t) {
      double* yt = y + t * q;
      for (int u = 0; u < t; ++u) {
        const double* yu = y + u * q;
        double sdot = 0.0;
        for (int i = lane; i < q; i += 64) sdot += yu[i] * yt[i];
        sdot = wave_sum(sdot);
        for (int i = lane; i < q; i += 64) yt[i] -= sdot * yu[i];
      }
      double sn = 0.0;
      for (int i = lane; i < q; i += 64) sn += yt[i] * yt[i];
      sn = 1.0 / sqrt(wave_sum(sn));
      for (int i = lane; i < q; i += 64) yt[i] *= sn;
    }
  }
  __syncthreads();
  // ---- back-transform y <- H_0 H_1 ... H_{q-3} y: 16 lanes per vector, the
  // vectors of a wave are independent, so no block barrier per reflector ----
  {
    const int seg = lane & 15;
    for (int t0 = wave * 4; t0 < R; t0 += NW * 4) {
      const int t = t0 + (lane >> 4);
      double* yt = y + (t < R ? t : 0) * q;
      for (int k = q - 3; k >= 0; --k) {
        const double beta = bet[k];
        if (beta == 0.0) continue;
        const int L = q - k - 1;
        const double* v = Vr + (k + 1) * q + k;
        double sdot = 0.0;
        for (int i = seg; i < L; i += 16) sdot += v[i * q] * yt[k + 1 + i];
        sdot += __shfl_xor(sdot, 1);
        sdot += __shfl_xor(sdot, 2);
        sdot += __shfl_xor(sdot, 4);
        sdot += __shfl_xor(sdot, 8);
        sdot *= beta;
        if (t < R)
          for (int i = seg; i < L; i += 16) yt[k + 1 + i] -= sdot * v[i * q];
      }
      if (t < R)
        for (int i = seg; i < q; i += 16) V[i * R + t] = yt[i];
    }
  }
  if (timers) {
    __syncthreads();
    if (tid == 0) timers[4] = wall_clock64();
  }
}

template <int NT, bool MLDS, bool VLDS>
__global__ __launch_bounds__(NT) void k_sym_eig_top(double* Mg, int q, int R, double* lam,
                                                    double* V, double* gscratch, int8_t* gpivs,
                                                    uint64_t* timers) {
  constexpr int NW = NT / 64;
  extern __shared__ double smem[];
  __shared__ double redK[NW];
  __shared__ double redN[2][NW];
  __shared__ double sh[4];
  // small vectors always in LDS: d, e, e2, p, beta (5q); then M (q^2) and the
  // inverse-iteration vectors/factors (5 R q doubles + R q bytes) if they fit
  double* d = smem;
  double* e = d + q;
  double* e2 = e + q;
  double* pw = e2 + q;
  double* bet = pw + q;
  double* M = MLDS ? smem + 5 * q : Mg;
  double* y = VLDS ? smem + 5 * q + (MLDS ? q * q : 0) : gscratch;  // R x q
  double* lu = y + R * q;                                            // R x 4q
  int8_t* pivs = VLDS ? reinterpret_cast<int8_t*>(lu + 4 * R * q) : gpivs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (timers && tid == 0) timers[0] = wall_clock64();
  if (MLDS) {
    for (int t = tid; t < q * q; t += NT) M[t] = Mg[t];
    __syncthreads();
  }

  // ---- Householder tridiagonalisation (lower); reflector k: I - beta v v^T on
  // indices k+1.., v stored in column k below the diagonal.  Two barriers per
  // step: p = beta A22 v (wave per row, lane-parallel dot products) with v^T p,
  // then the rank-2 update, which also accumulates the squared norm of the
  // next column. ----
  if (q >= 3) {
    double part = 0.0;
    for (int i = 1 + tid; i < q; i += NT) part += M[i * q] * M[i * q];
    part = wave_sum(part);
    if (lane == 0) redN[0][wave] = part;
    __syncthreads();
  }
  for (int k = 0; k + 2 < q; ++k) {
    const int L = q - k - 1;
    const double* x = M + (k + 1) * q + k;  // stride q
    double norm2 = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) norm2 += redN[k & 1][w];
    const double x0 = x[0];
    const double alpha = norm2 > 0.0 ? -copysign(sqrt(norm2), x0) : 0.0;
    const double v0 = x0 - alpha;
    const double vtv = norm2 - x0 * x0 + v0 * v0;
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    double* A22 = M + (k + 1) * q + (k + 1);
    double nxt = 0.0;
    if (beta != 0.0) {
      // p_i = beta sum_j A22[j][i] v_j: tpc threads per column (all threads busy
      // while L <= NT), loads issued eight at a time; v_j read from column k
      // (v_0 = x0 - alpha)
      const int tpc = L <= NT / 8 ? 8 : L <= NT / 4 ? 4 : L <= NT / 2 ? 2 : 1;
      const int cpp = NT / tpc;
      double pp = 0.0;
      for (int c0 = 0; c0 < L; c0 += cpp) {
        const int i = c0 + tid / tpc, h = tid % tpc;
        double a8[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a8[u] = 0.0;
        if (i < L) {
          int j = h;
          for (; j + 7 * tpc < L; j += 8 * tpc) {
            double av[8], vv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int jj = j + u * tpc;
              av[u] = A22[jj * q + i];
              vv[u] = x[jj * q];
            }
            if (j == 0) vv[0] = v0;
#pragma unroll
            for (int u = 0; u < 8; ++u) a8[u] += av[u] * vv[u];
          }
          for (; j < L; j += tpc) a8[0] += A22[j * q + i] * (j == 0 ? v0 : x[j * q]);
        }
        double sacc = ((a8[0] + a8[1]) + (a8[2] + a8[3])) + ((a8[4] + a8[5]) + (a8[6] + a8[7]));
        for (int o = 1; o < tpc; o <<= 1) sacc += __shfl_xor(sacc, o);
        if (i < L && h == 0) {
          const double pi = beta * sacc;
          pw[i] = pi;
          pp += (i == 0 ? v0 : x[i * q]) * pi;
        }
      }
      pp = wave_sum(pp);
      if (lane == 0) redK[wave] = pp;
      __syncthreads();
      double vp = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) vp += redK[w];
      const double K = 0.5 * beta * vp;
      // rank-2 update A22 -= v w^T + w v^T, w = p - K v: threads spread over the
      // columns (NT / L per column while L <= NT), rows strided, four rows of
      // loads issued before the stores
      const int tpr = L <= NT ? NT / L : 1;
      const int jl = L <= NT ? tid % L : lane, r0 = L <= NT ? tid / L : wave;
      const int rstep = L <= NT ? tpr : NW;
      const int jstep = L <= NT ? L : 64;
      if (r0 < rstep)
        for (int j = jl; j < L; j += jstep) {
          const double vj = j == 0 ? v0 : x[j * q];
          const double wj = pw[j] - K * vj;
          int i = r0;
          for (; i + 3 * rstep < L; i += 4 * rstep) {
            double v4[4], w4[4], r4[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int ii = i + u * rstep;
              v4[u] = x[ii * q];
              w4[u] = pw[ii];
              r4[u] = A22[ii * q + j];
            }
            if (i == 0) v4[0] = v0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int ii = i + u * rstep;
              const double nv = r4[u] - (v4[u] * wj + (w4[u] - K * v4[u]) * vj);
              A22[ii * q + j] = nv;
              if (j == 0 && ii >= 1) nxt += nv * nv;
            }
          }
          for (; i < L; i += rstep) {
            const double vi = i == 0 ? v0 : x[i * q];
            const double nv = A22[i * q + j] - (vi * wj + (pw[i] - K * vi) * vj);
            A22[i * q + j] = nv;
            if (j == 0 && i >= 1) nxt += nv * nv;
          }
        }
    } else {
      for (int i = 1 + tid; i < L; i += NT) nxt += A22[i * q] * A22[i * q];
    }
    nxt = wave_sum(nxt);
    if (lane == 0) redN[(k + 1) & 1][wave] = nxt;
    if (tid == 0) {
      d[k] = M[k * q + k];
      e[k] = norm2 > 0.0 ? alpha : x0;
      bet[k] = beta;
    }
    __syncthreads();
    if (tid == 0) M[(k + 1) * q + k] = v0;  // column k is not read again until the back-transform
  }
  __syncthreads();
  if (tid == 0) {
    if (q >= 2) {
      d[q - 2] = M[(q - 2) * q + (q - 2)];
      e[q - 2] = M[(q - 1) * q + (q - 2)];
      if (q >= 3) bet[q - 2] = 0.0;
    }
    d[q - 1] = M[(q - 1) * q + (q - 1)];
  }
  __syncthreads();
  eig_tail<NT>(q, R, d, e, e2, bet, M, y, lu, pivs, sh, lam, V, timers);
}

// ------------------------------------------ small symmetric eigenproblems ----
// Leading R eigenpairs of a symmetric q x q matrix with q <= QM <= 28, in one
// wavefront (no block barriers), same method as k_sym_eig_top:
//   * Householder tridiagonalisation with row `lane` of the matrix in
//     registers; v and w = p - K v are broadcast through LDS, and only the
//     trailing block (rows and columns > j) is updated at step j;
//   * eigenvalues by multisection of the Sturm count: a first round of 256
//     points shared by all, then 64 / R lanes per eigenvalue, four interleaved
//     count chains per lane, until the bracket is below 1e-9 relative (three
//     inverse iterations then converge to working precision unless the gap is
//     under ~1e-4 relative, and those eigenvalues are orthogonalised as a
//     cluster); the returned eigenvalue is the Rayleigh quotient of the
//     computed eigenvector of the tridiagonal;
//   * eigenvectors of the tridiagonal by inverse iteration, one lane each, LU
//     factors in LDS with the lane index fastest (no bank conflicts);
//   * Gram-Schmidt only between vectors whose eigenvalues lie within
//     1e-3 ||T||_1 of each other (elsewhere inverse iteration already gives
//     orthogonal vectors), then back-transformation through the reflectors,
//     four vectors per batched wave reduction.
// order 28 at most (234 VGPRs, SGPR spills into VGPR lanes only); at 32 the
// kernel needs every VGPR
constexpr int kEigSmallMax = 28;

template <int QM>
__device__ inline void sturm4(const double (&d)[QM], const double (&e2)[QM], int q,
                              const double (&x)[4], double pivmin, int (&c)[4]) {
  double t[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    t[k] = d[0] - x[k];
    c[k] = t[k] < 0.0;
  }
  // predicated rather than exited early, so that the loop unrolls and the
  // register arrays keep constant indices
  // each operation is issued for the four chains before the next one, so
  // that the dependent steps of one chain overlap the others
#pragma unroll
  for (int i = 1; i < QM; ++i) {
    if (i < q) {
      double r[4], e[4], dx[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        dx[k] = d[i] - x[k];
        t[k] = fabs(t[k]) <= pivmin ? -pivmin : t[k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) r[k] = __builtin_amdgcn_rcp(t[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) e[k] = fma(-t[k], r[k], 1.0);
#pragma unroll
      for (int k = 0; k < 4; ++k) r[k] = fma(r[k], e[k], r[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) t[k] = fma(-e2[i - 1], r[k], dx[k]);
#pragma unroll
      for (int k = 0; k < 4; ++k) c[k] += t[k] < 0.0;
    }
  }
}

template <int QM>
__global__ __launch_bounds__(64) void k_sym_eig_small(const double* Mg, int q, int R,
                                                      double* lam, double* Vout,
                                                      uint64_t* timers) {
  constexpr int YS = 65;  // row stride of the eigenvector block (odd: no bank conflicts)
  __shared__ double vsh[64], wsh[64];
  __shared__ double dsh[QM], esh[QM], bsh[QM], lsh[QM];
  __shared__ double lu[4][QM][64];  // u0 (reciprocal pivots), u1, u2, multipliers
  __shared__ int8_t pv[QM][64];
  __shared__ double ysh[QM * YS];   // y_t(i) at i * YS + t
  __shared__ int cst[QM];           // first index of the eigenvalue cluster of t
  __shared__ int cnt[256];          // Sturm counts of the first multisection round
  const int lane = threadIdx.x;
  if (timers && lane == 0) timers[0] = wall_clock64();

  // ---- tridiagonalisation ----
  double m[QM], vr[QM];
#pragma unroll
  for (int c = 0; c < QM; ++c) m[c] = (lane < q && c < q) ? Mg[lane * q + c] : 0.0;
  static_for<0, QM>([&](auto JC) {
    constexpr int J = decltype(JC)::value;
    vr[J] = 0.0;
    if (lane == 0) bsh[J] = 0.0;
    if (J + 2 >= q) return;
    const double xl = lane > J ? m[J] : 0.0;
    const double nrm = sqrt(wave_allsum(xl * xl));
    const double x0 = read_lane(m[J], J + 1);
    const double alpha = nrm > 0.0 ? -copysign(nrm, x0) : 0.0;
    const double v0 = x0 - alpha;
    // 2 / v^T v by a true division: |alpha v0| can be tiny for nearly rank-
    // deficient matrices, where the reciprocal-and-Newton form gives NaN
    const double beta = nrm > 0.0 ? -1.0 / (alpha * v0) : 0.0;
    const double vl = lane > J + 1 ? m[J] : (lane == J + 1 ? v0 : 0.0);
    vr[J] = vl;
    if (lane == 0) {
      esh[J] = alpha;
      bsh[J] = beta;
    }
    vsh[lane] = vl;
    __syncthreads();
    double p = 0.0;
#pragma unroll
    for (int c = J + 1; c < QM; ++c) p = fma(m[c], vsh[c], p);
    p *= beta;
    const double K = 0.5 * beta * wave_allsum(vl * p);
    const double wl = fma(-K, vl, p);
    wsh[lane] = wl;
    __syncthreads();
#pragma unroll
    for (int c = J + 1; c < QM; ++c) m[c] = fma(-vl, wsh[c], fma(-wl, vsh[c], m[c]));
    __syncthreads();
  });
  if (timers && lane == 0) timers[1] = wall_clock64();
  // diagonal (never changed after its own step) and the last subdiagonal entry
  static_for<0, QM>([&](auto JC) {
    constexpr int J = decltype(JC)::value;
    const double dj = read_lane(m[J], J);
    const double ej = J + 1 < QM ? read_lane(m[J], (J + 1) % QM) : 0.0;
    if (lane == 0 && J < q) dsh[J] = dj;
    if (lane == 0 && J + 2 == q) esh[J] = ej;
  });
  __syncthreads();

  // ---- eigenvalues ----
  double d[QM], e2[QM];
  double glo = DBL_MAX, ghi = -DBL_MAX, onenrm = 0.0, emax2 = 0.0;
#pragma unroll
  for (int i = 0; i < QM; ++i) {
    d[i] = i < q ? dsh[i] : 0.0;
    const double ei = i + 1 < q ? esh[i] : 0.0;
    e2[i] = ei * ei;
    emax2 = fmax(emax2, e2[i]);
  }
#pragma unroll
  for (int i = 0; i < QM; ++i)
    if (i < q) {
      const double r = (i > 0 ? fabs(esh[i - 1]) : 0.0) + (i + 1 < q ? fabs(esh[i]) : 0.0);
      glo = fmin(glo, d[i] - r);
      ghi = fmax(ghi, d[i] + r);
      onenrm = fmax(onenrm, fabs(d[i]) + r);
    }
  {
    const double pad = 2.0 * DBL_EPSILON * fmax(fabs(glo), fabs(ghi)) + DBL_MIN;
    glo -= pad;
    ghi += pad;
  }
  const double pivmin = DBL_MIN * fmax(1.0, emax2);
  {
    const int G = 64 / R, P = 4 * G;
    const int gi = lane / G, gl = lane - gi * G;
    const bool act = gi < R;
    const int tgt = q - 1 - (act ? gi : 0);
    const uint64_t gmask = (G == 64 ? ~0ull : ((1ull << G) - 1ull)) << (act ? gi * G : 0);
    // first round shared by all eigenvalues: 256 points over the Gershgorin
    // interval, counts (non-decreasing in the point index) through LDS
    double lo = glo, hi = ghi;
    {
      double x[4];
      int c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = glo + (ghi - glo) * double(4 * lane + k + 1) / 257.0;
      sturm4<QM>(d, e2, q, x, pivmin, c);
#pragma unroll
      for (int k = 0; k < 4; ++k) cnt[4 * lane + k] = c[k];
      __syncthreads();
      int a = 0, b = 256;  // first point with count > tgt
      while (a < b) {
        const int mid = (a + b) >> 1;
        if (cnt[mid] > tgt) b = mid;
        else a = mid + 1;
      }
      if (a < 256) hi = glo + (ghi - glo) * double(a + 1) / 257.0;
      if (a > 0) lo = glo + (ghi - glo) * double(a) / 257.0;
    }
    for (int it = 0; it < 64; ++it) {
      const double width = hi - lo;
      const bool conv = !(width > 1e-9 * fmax(fabs(lo), fabs(hi)) + pivmin);
      if (__ballot(act && !conv) == 0ull) break;
      double x[4];
      int c[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[k] = lo + width * double(4 * gl + k + 1) / double(P + 1);
      sturm4<QM>(d, e2, q, x, pivmin, c);
      int f = 4;
#pragma unroll
      for (int k = 3; k >= 0; --k)
        if (c[k] > tgt) f = k;
      const uint64_t hm = __ballot(act && f < 4) & gmask;
      const int L = hm ? __ffsll((unsigned long long)hm) - 1 : lane;
      const int fL = __shfl(f, L);
      if (act && !conv) {
        const int idx = hm ? 4 * (L - gi * G) + fL : P;  // first point above the target
        const double nhi = idx < P ? lo + width * double(idx + 1) / double(P + 1) : hi;
        const double nlo = idx > 0 ? lo + width * double(idx) / double(P + 1) : lo;
        lo = nlo;
        hi = nhi;
      }
    }
    if (act && gl == 0) lsh[gi] = 0.5 * (lo + hi);
  }
  __syncthreads();
  if (timers && lane == 0) timers[2] = wall_clock64();

  // ---- inverse iteration, lane t for eigenvalue t; vectors and factors in
  // LDS with the lane index fastest, loops rolled (q is a run-time bound) ----
  const double tiny = DBL_EPSILON * fmax(onenrm, DBL_MIN);
  if (lane < R) {
    const double mu = lsh[lane];
    double* u0 = &lu[0][0][lane];
    double* u1 = &lu[1][0][lane];
    double* u2 = &lu[2][0][lane];
    double* ml = &lu[3][0][lane];
    int8_t* pl = &pv[0][lane];
    double* y = ysh + lane;
    double p = dsh[0] - mu, qq = q > 1 ? esh[0] : 0.0, rr = 0.0;
    for (int i = 0; i + 1 < q; ++i) {
      const double c = esh[i], a1 = dsh[i + 1] - mu, b1 = i + 2 < q ? esh[i + 1] : 0.0;
      // reciprocals with one Newton step (rcp64) are accurate enough for the
      // factors of inverse iteration and keep the dependent chain short
      if (fabs(p) >= fabs(c)) {
        const double rp = rcp64(p == 0.0 ? tiny : p);
        const double mlt = c * rp;
        u0[i * 64] = rp, u1[i * 64] = qq, u2[i * 64] = rr, pl[i * 64] = 0;
        ml[i * 64] = mlt;
        p = a1 - mlt * qq;
        qq = b1 - mlt * rr;
      } else {
        const double rc = rcp64(c);
        const double mlt = p * rc;
        u0[i * 64] = rc, u1[i * 64] = a1, u2[i * 64] = b1, pl[i * 64] = 1;
        ml[i * 64] = mlt;
        p = qq - mlt * a1;
        qq = rr - mlt * b1;
      }
      rr = 0.0;
    }
    u0[(q - 1) * 64] = rcp64(p == 0.0 ? tiny : p);
    u1[(q - 1) * 64] = 0.0;
    u2[(q - 1) * 64] = 0.0;
    for (int i = 0; i < q; ++i) {
      const uint32_t h = uint32_t(i) * 2654435761u + uint32_t(lane + 1) * 40503u;
      y[i * YS] = 1.0 + double((h >> 8) & 1023u) / 2048.0;
    }
    double scale = 1.0;
    for (int itr = 0; itr < 3; ++itr) {
      // forward: row interchanges and multipliers
      double prev = y[0] * scale;
#pragma unroll 4
      for (int i = 0; i + 1 < q; ++i) {
        double nx = y[(i + 1) * YS] * scale;
        if (pl[i * 64]) {
          const double t = prev;
          prev = nx;
          nx = t;
        }
        y[i * YS] = prev;
        prev = nx - ml[i * 64] * prev;
      }
      y[(q - 1) * YS] = prev;
      // backward: upper triangular with two superdiagonals
      double n2 = 0.0, x1 = 0.0, x2 = 0.0;
#pragma unroll 4
      for (int i = q - 1; i >= 0; --i) {
        const double xi = (y[i * YS] - u1[i * 64] * x1 - u2[i * 64] * x2) * u0[i * 64];
        y[i * YS] = xi;
        n2 += xi * xi;
        x2 = x1;
        x1 = xi;
      }
      scale = 1.0 / sqrt(n2);
    }
    double rq = 0.0;
    for (int i = 0; i < q; ++i) {
      const double yi = y[i * YS] * scale;
      y[i * YS] = yi;
      double ty = dsh[i] * yi;
      if (i > 0) ty = fma(esh[i - 1], y[(i - 1) * YS], ty);
      if (i + 1 < q) ty = fma(esh[i], y[(i + 1) * YS] * scale, ty);
      rq = fma(yi, ty, rq);
    }
    lsh[lane] = rq;
  }
  if (lane == 0) {  // clusters: runs of eigenvalues closer than ortol
    const double ortol = 1e-3 * onenrm;
    int st = 0;
    for (int t = 0; t < R; ++t) {
      if (t > 0 && lsh[t - 1] - lsh[t] > ortol) st = t;
      cst[t] = st;
    }
  }
  __syncthreads();
  if (timers && lane == 0) timers[3] = wall_clock64();

  // ---- lane i holds element i of every vector from here on ----
  double yl[QM];
#pragma unroll
  for (int t = 0; t < QM; ++t) yl[t] = (t < R && lane < q) ? ysh[lane * YS + t] : 0.0;
  static_for<1, QM>([&](auto TC) {
    constexpr int T = decltype(TC)::value;
    if (T >= R) return;
    const int first = cst[T];
    if (first == T) return;
    static_for<0, T>([&](auto UC) {
      constexpr int U = decltype(UC)::value;
      if (U < first) return;
      const double dot = wave_allsum(yl[U] * yl[T]);
      yl[T] = fma(-dot, yl[U], yl[T]);
    });
    yl[T] *= 1.0 / sqrt(wave_allsum(yl[T] * yl[T]));
  });
  if (timers && lane == 0) timers[4] = wall_clock64();
  // back-transform y <- H_0 ... H_{q-3} y
  static_for<0, QM, true>([&](auto JC) {
    constexpr int J = decltype(JC)::value;
    if (J + 2 >= q) return;
    const double beta = bsh[J];
    // chunk of vectors per batched reduction: a multiple of 4 dividing QM
    // (one wide chunk measured slower than several narrow ones)
    constexpr int CH = QM % 12 == 0 ? 12 : (QM % 8 == 0 ? 8 : 4);
    static_assert(QM % CH == 0 && CH % 4 == 0, "back-transform chunks must cover QM");
    static_for<0, QM / CH>([&](auto CC) {
      constexpr int C0 = CH * decltype(CC)::value;
      if (C0 >= R) return;
      double pr[CH], w[CH];
#pragma unroll
      for (int u = 0; u < CH; ++u) pr[u] = vr[J] * yl[C0 + u];
      wave_sums<CH>(pr, w);
#pragma unroll
      for (int u = 0; u < CH; ++u) yl[C0 + u] = fma(-beta * w[u], vr[J], yl[C0 + u]);
    });
  });
  if (lane < q)
#pragma unroll
    for (int t = 0; t < QM; ++t)
      if (t < R) Vout[lane * R + t] = yl[t];
  if (lane < R) lam[lane] = lsh[lane];
  if (timers && lane == 0) timers[5] = wall_clock64();
}

// ----------------------------------------------------- thin Householder QR ----
// Q of the thin QR factorisation of C (r x k, k <= 64), given and returned by
// rows of the transposes: Ct (k x r) with row j = column j of C, Qt (k x r)
// with row j = column j of Q.  One wavefront (column steps are short; no block
// barriers).  Reflector j: I - beta v v^T on indices j.., v_j = c_j - alpha,
// alpha = -sign(c_j) ||c_{j..}||; the dot products of v with the remaining
// columns are accumulated eight at a time and reduced together.  Q is formed
// by applying the reflectors backwards to the first k columns of the identity.
// Work arrays (copy of Ct and Q) live in LDS when they fit, else in gwork.
constexpr int kQrMaxK = 64;

template <bool LDSW>
__global__ __launch_bounds__(64) void k_qr_rows(const double* Ct, int k, int r, double* Qt,
                                                double* gwork, const int* gate) {
  if (gate && *gate == 0) return;  // run only when the Cholesky QR below asked for it
  extern __shared__ double qsm[];
  __shared__ double betas[kQrMaxK];
  double* V = LDSW ? qsm : gwork;          // k x r: reduced columns, reflector j in row j
  double* Q = LDSW ? qsm + k * r : Qt;     // k x r: rows of Q
  const int lane = threadIdx.x;
  for (int t = lane; t < k * r; t += 64) V[t] = Ct[t];
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    double* vj = V + j * r;
    double sig = 0.0;
    for (int i = j + 1 + lane; i < r; i += 64) sig += vj[i] * vj[i];
    sig = wave_sum(sig);
    const double x0 = vj[j];
    const double nrm = sqrt(x0 * x0 + sig);
    const double alpha = nrm > 0.0 ? -copysign(nrm, x0) : 0.0;
    const double v0 = x0 - alpha;
    const double vtv = sig + v0 * v0;
    const double beta = vtv > 0.0 ? 2.0 / vtv : 0.0;
    __syncthreads();
    if (lane == 0) {
      vj[j] = v0;
      betas[j] = beta;
    }
    __syncthreads();
    for (int l0 = j + 1; l0 < k; l0 += 8) {
      double acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = 0.0;
      for (int i = j + lane; i < r; i += 64) {
        const double vi = vj[i];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (l0 + u < k) acc[u] += vi * V[(l0 + u) * r + i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = beta * wave_sum(acc[u]);
      for (int i = j + lane; i < r; i += 64) {
        const double vi = vj[i];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (l0 + u < k) V[(l0 + u) * r + i] -= acc[u] * vi;
      }
    }
    __syncthreads();
  }
  // Q = H_0 ... H_{k-1} [I_k; 0]: rows l < j of Q vanish on indices >= j, so
  // H_j only changes rows l >= j
  for (int t = lane; t < k * r; t += 64) Q[t] = (t % r == t / r) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double* vj = V + j * r;
    const double beta = betas[j];
    for (int l0 = j; l0 < k; l0 += 8) {
      double acc[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = 0.0;
      for (int i = j + lane; i < r; i += 64) {
        const double vi = vj[i];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (l0 + u < k) acc[u] += vi * Q[(l0 + u) * r + i];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] = beta * wave_sum(acc[u]);
      for (int i = j + lane; i < r; i += 64) {
        const double vi = vj[i];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (l0 + u < k) Q[(l0 + u) * r + i] -= acc[u] * vi;
      }
    }
    __syncthreads();
  }
  if (LDSW)
    for (int t = lane; t < k * r; t += 64) Qt[t] = Q[t];
}

// Thin QR by shifted Cholesky QR, three passes (Fukaya, Kannan, Nakatsukasa,
// Zhang & Yamamoto, SIAM J. Sci. Comput. 2020): X_0 = C; pass p forms the
// Gram X_p^T X_p (plus the shift 11 (r k + k (k + 1)) u ||C||_F^2 on the
// diagonal in the first pass), its Cholesky factor R_p and X_{p+1} =
// X_p R_p^{-1}; after three passes Q = X_3 has orthonormal columns to working
// precision whenever C has full numerical column rank.  The kernel first runs
// the first pass unshifted: if its factor is well conditioned (largest over
// smallest diagonal entry of R at most 1e6) and the second pass finds X_1
// nearly orthonormal (every diagonal entry of its R within 0.1 of 1), the two
// plain passes finish (Cholesky QR2, Yamamoto et al., ETNA 2015); otherwise it
// restarts from C with the three shifted passes.  Any orthonormal basis
// of range(C) serves the randomized solve (its SVD of Q^T B Z^T Y fixes A and
// W), so this replaces the Householder QR beyond the register-resident shapes.  A non-positive pivot in
// the unshifted passes (C of numerical rank below k, e.g. an exactly low-rank
// right-hand side) sets *fallback, and the Householder kernel that follows in
// the stream runs only then.
//
// One workgroup of 4 waves, k <= KP (32, 48 or 64).  Grams: FP64 MFMA 16x16x4
// over 64-column blocks of X_p^T (block b to wave b mod 4), wave partials
// summed in LDS in a fixed order.  Cholesky in LDS with every thread in the
// trailing updates; the triangular inverse by wave 0.  X_{p+1}^T = R_p^{-T} X_p^T: MFMA over 16-column pieces of the same
// blocks, so each wave reads back only what it wrote.  The passes write X1, X2
// and Qt, so no buffer is read after it was written within a pass.
template <int KP>
__global__ __launch_bounds__(256) void k_cholqr3(const double* Ct, int k, int r, double* X1,
                                                 double* X2, double* Qt, int* fallback) {
  extern __shared__ double csm[];
  constexpr int SL = KP + 1, SZ = KP * SL, NB = KP / 16;
  __shared__ int bad, restart;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  double* Gs = csm;           // Gram, then R (upper triangle)
  double* Ri = csm + SZ;      // R^{-1} (row-major)
  if (tid == 0) bad = 0, restart = 0;
  // Two unshifted passes (Cholesky QR2) when the first factor is well
  // conditioned, else the three passes of the shifted algorithm from C again
  int npass = 2;
  bool shifted = false;
  for (int pass = 0; pass < npass; ++pass) {
    const double* in = pass == 0 ? Ct : pass == 1 ? X1 : X2;
    double* out = pass == npass - 1 ? Qt : pass == 0 ? X1 : X2;
    // ---- Gram partials over this wave's 64-column blocks ----
    dx4 acc[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[a][b] = dx4{0.0, 0.0, 0.0, 0.0};
    for (int i0 = wave * 64; i0 < r; i0 += 256)
#pragma unroll 2
      for (int ks = 0; ks < 64; ks += 4) {
        const int i = i0 + ks + g;
        double x[NB];
#pragma unroll
        for (int a = 0; a < NB; ++a) {
          const int row = 16 * a + li;
          x[a] = (row < k && i < r) ? in[int64_t(row) * r + i] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < NB; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[a], x[b], acc[a][b], 0, 0, 0);
      }
    __syncthreads();  // the previous pass is done with Gs and Ri
    // partials: waves 0, 1 store to regions 0, 1; waves 2, 3 add theirs; then
    // G = (P0 + P2) + (P1 + P3)
    double* part = csm + size_t(wave & 1) * SZ;
    if (wave < 2) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) part[(16 * a + g + 4 * v) * SL + 16 * b + li] = acc[a][b][v];
    }
    __syncthreads();
    if (wave >= 2) {
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) part[(16 * a + g + 4 * v) * SL + 16 * b + li] += acc[a][b][v];
    }
    __syncthreads();
    for (int e = tid; e < KP * KP; e += 256) {
      const int o = (e / KP) * SL + e % KP;
      Gs[o] = csm[o] + csm[SZ + o];
    }
    __syncthreads();
    if (pass == 0 && shifted && wave == 0) {  // the shift of the first pass
      double tr = 0.0;
      for (int j = 0; j < k; ++j) tr += Gs[j * SL + j];
      const double shift = 11.0 * (double(r) * k + double(k) * (k + 1)) * 0x1.0p-53 * tr;
      if (lane < k) Gs[lane * SL + lane] += shift;
    }
    // ---- Cholesky G = R^T R in LDS, one step per pivot: wave 0 scales row
    // j, every thread takes part in the trailing update ----
    __syncthreads();
    for (int j = 0; j < k; ++j) {
      if (wave == 0) {  // every lane reads the pivot before any lane writes
        const double d = Gs[j * SL + j];
        if (lane == 0 && !(d > 0.0)) bad = 1;
        const double rd = 1.0 / sqrt(d);
        if (lane >= j && lane < k) Gs[j * SL + lane] *= rd;  // R_jj = sqrt(d)
      }
      __syncthreads();
      const int n1 = k - j - 1;  // trailing upper triangle: G_ab -= R_ja R_jb
      for (int e = tid; e < n1 * n1; e += 256) {
        const int a = j + 1 + e / n1, b = j + 1 + e % n1;
        if (a <= b) Gs[a * SL + b] = fma(-Gs[j * SL + a], Gs[j * SL + b], Gs[a * SL + b]);
      }
      __syncthreads();
    }
    if (!shifted) {
      // Cholesky QR2 leaves O(u) orthogonality for kappa(C) well below
      // u^{-1/2} (about 7e7).  First pass: the ratio of the largest to the
      // smallest diagonal entry of R (a lower bound on kappa(C)) at most 1e6.
      // Second pass: X_1 must already be nearly orthonormal, every R_jj within
      // 0.1 of 1 (X_1^T X_1 = R^T R), which also catches a kappa(C) that the
      // ratio underestimates.  Otherwise restart with the shifted passes.
      if (wave == 0) {
        double dmax = lane < k ? Gs[lane * SL + lane] : 0.0;
        double dmin = lane < k ? Gs[lane * SL + lane] : DBL_MAX;
        for (int off = 32; off > 0; off >>= 1) {
          dmax = fmax(dmax, __shfl_xor(dmax, off));
          dmin = fmin(dmin, __shfl_xor(dmin, off));
        }
        const bool ok = pass == 0 ? dmax <= 1e6 * dmin : (dmax <= 1.1 && dmin >= 0.9);
        if (lane == 0 && (bad || !ok)) restart = 1;
      }
      __syncthreads();
      if (restart) {  // workgroup-uniform
        shifted = true;
        npass = 3;
        pass = -1;
        __syncthreads();
        if (tid == 0) bad = 0;
        __syncthreads();
        continue;
      }
    }
    // ---- S = R^{-1} by back substitution (wave 0, lane c holds column c) ----
    if (wave == 0 && !bad) {
      const int c = lane;
      if (c < KP)
        for (int t = 0; t < KP; ++t) Ri[t * SL + c] = 0.0;
      for (int l = k - 1; l >= 0; --l) {
        double sacc = (l == c) ? 1.0 : 0.0;
        int t = l + 1;
        for (; t + 3 < k; t += 4) {
          const double a0 = Gs[l * SL + t] * Ri[t * SL + c];
          const double a1 = Gs[l * SL + t + 1] * Ri[(t + 1) * SL + c];
          const double a2 = Gs[l * SL + t + 2] * Ri[(t + 2) * SL + c];
          const double a3 = Gs[l * SL + t + 3] * Ri[(t + 3) * SL + c];
          sacc -= (a0 + a1) + (a2 + a3);
        }
        for (; t < k; ++t) sacc -= Gs[l * SL + t] * Ri[t * SL + c];
        if (c < k && c >= l) Ri[l * SL + c] = sacc / Gs[l * SL + l];
      }
    }
    __syncthreads();
    if (bad) {
      if (tid == 0) *fallback = 1;
      return;  // workgroup-uniform
    }
    // ---- X_{p+1}^T = R^{-T} X_p^T over the 16-column pieces of this wave's
    // 64-column blocks (the columns its Gram partials read in the next pass) ----
    for (int i0 = wave * 64; i0 < r; i0 += (i0 & 63) == 48 ? 256 - 48 : 16) {
      dx4 o[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) o[cb] = dx4{0.0, 0.0, 0.0, 0.0};
      const int i = i0 + li;
#pragma unroll
      for (int k0 = 0; k0 < KP; k0 += 4) {
        const int l = k0 + g;
        const double xb = (l < k && i < r) ? in[int64_t(l) * r + i] : 0.0;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb)
          o[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(Ri[l * SL + 16 * cb + li], xb, o[cb], 0, 0,
                                                       0);
      }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int c = 16 * cb + g + 4 * v;
          if (c < k && i < r) out[int64_t(c) * r + i] = o[cb][v];
        }
    }
    __syncthreads();  // every wave's columns of X_{p+1} are written
  }
  if (tid == 0) *fallback = 0;
}

// Register-resident variant for r <= 128 and k <= KM <= 24: lane l holds rows
// l and l + 64 of every column and the step loops are unrolled, so the tile
// is indexed by constants.  Reflector j takes a single wave reduction:
// w_c = sum_{i >= j} c_ij c_ic for c >= j gives ||c_{j..}||^2 (c = j) and,
// since v = c_{j..} - alpha e_j, every v^T c_c = w_c - alpha c_jc; with
// alpha = -sign(c_jj) ||c_{j..}||, v^T v = -2 alpha v_j (no cancellation).
constexpr int kQrRegRows = 128, kQrRegMaxK = 24;

__host__ __device__ constexpr int round4(int n) { return (n + 3) / 4 * 4; }

// Q of the thin QR of the k columns held in X (lane l: rows l, l + 64),
// returned in Q with the same layout; one wavefront.
template <int KM>
__device__ __forceinline__ void qr_reg_wave(double (&X)[2][KM], int k, double (&Q)[2][KM]) {
  const int lane = threadIdx.x & 63;
  double beta[KM];
  static_for<0, KM>([&](auto JC) {
    constexpr int J = decltype(JC)::value;
    constexpr int N = round4(KM - J);
    beta[J] = 0.0;
    if (J >= k) return;
    const double xm0 = lane >= J ? X[0][J] : 0.0;  // rows >= 64 are always below J
    double pr[N], w[N];
#pragma unroll
    for (int u = 0; u < N; ++u)
      pr[u] = (J + u < KM) ? fma(xm0, X[0][(J + u) % KM], X[1][J] * X[1][(J + u) % KM]) : 0.0;
    wave_sums<N>(pr, w);
    const double xj = read_lane(X[0][J], J);
    const double nrm = sqrt(w[0]);
    const double alpha = nrm > 0.0 ? -copysign(nrm, xj) : 0.0;
    const double vj = xj - alpha;
    // 2 / v^T v by a true division (tiny |alpha v_j| on nearly dependent columns)
    const double b = nrm > 0.0 ? -1.0 / (alpha * vj) : 0.0;
    beta[J] = b;
    X[0][J] = lane > J ? X[0][J] : (lane == J ? vj : 0.0);
#pragma unroll
    for (int u = 1; u < KM - J; ++u) {
      const double g = b * fma(-alpha, read_lane(X[0][J + u], J), w[u]);
      X[0][J + u] = fma(-g, X[0][J], X[0][J + u]);
      X[1][J + u] = fma(-g, X[1][J], X[1][J + u]);
    }
  });
  // Q = H_0 ... H_{k-1} [I_k; 0]; H_j leaves columns < j of the partial
  // product untouched (they are still unit vectors e_c, c < j)
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int c = 0; c < KM; ++c) Q[p][c] = (lane + 64 * p == c && c < k) ? 1.0 : 0.0;
  static_for<0, KM, true>([&](auto JC) {
    constexpr int J = decltype(JC)::value;
    constexpr int N = round4(KM - J);
    if (J >= k) return;
    double pr[N], w[N];
#pragma unroll
    for (int u = 0; u < N; ++u)
      pr[u] = (J + u < KM) ? fma(X[0][J], Q[0][(J + u) % KM], X[1][J] * Q[1][(J + u) % KM])
                           : 0.0;
    wave_sums<N>(pr, w);
#pragma unroll
    for (int u = 0; u < KM - J; ++u) {
      const double g = beta[J] * w[u];
      Q[0][J + u] = fma(-g, X[0][J], Q[0][J + u]);
      Q[1][J + u] = fma(-g, X[1][J], Q[1][J + u]);
    }
  });
}

template <int KM>
__global__ __launch_bounds__(64) void k_qr_reg(const double* Ct, int k, int r, double* Qt) {
  const int lane = threadIdx.x;
  double X[2][KM], Q[2][KM];
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int c = 0; c < KM; ++c) {
      const int i = lane + 64 * p;
      X[p][c] = (i < r && c < k) ? Ct[c * r + i] : 0.0;
    }
  qr_reg_wave<KM>(X, k, Q);
#pragma unroll
  for (int p = 0; p < 2; ++p)
#pragma unroll
    for (int c = 0; c < KM; ++c) {
      const int i = lane + 64 * p;
      if (i < r && c < k) Qt[c * r + i] = Q[p][c];
    }
}

// Range basis of the randomized solve (Alg. 5), for r <= 128 and k <= KM:
// with B = (Z^T Z)^{-1} and C0 = Z^T Y Omega given, C = B C0, Q = qr(C) and
// P = B Q, all r x k row-major.  256 threads: B, C0/C and Q are staged
// in LDS; the two products use every thread, the QR wave 0 (register
// Householder, as k_qr_reg).
constexpr int kRbT = 256;

template <int KM>
__global__ __launch_bounds__(kRbT) void k_range_basis(const double* C0, const double* B, int r,
                                                      int k, double* Qout, double* Pout) {
  extern __shared__ double rb[];
  const int lb = r + 1;            // odd row stride: rows of B spread over the banks
  double* Bs = rb;                 // r x lb
  double* Cs = rb + r * lb;        // r x KM: C, then Q
  double* Ts = Cs + r * KM;        // r x KM: C0
  const int tid = threadIdx.x;
  // staging: unrolled so that many loads are in flight before the stores
#pragma unroll 8
  for (int t = tid; t < r * r; t += kRbT) Bs[(t / r) * lb + t % r] = B[t];
#pragma unroll 4
  for (int t = tid; t < r * KM; t += kRbT) {
    const int i = t / KM, c = t % KM;
    Ts[t] = c < k ? C0[i * k + c] : 0.0;
  }
  __syncthreads();
  // C = B C0: thread (i, h) forms columns [h KM/2, (h + 1) KM/2) of row i;
  // the C0 values it needs are the same for all lanes of a half (broadcast)
  constexpr int HC = KM / 2;
  const int ri = tid % 128, rh = tid / 128;
  if (ri < r) {
    double acc[HC];
#pragma unroll
    for (int c = 0; c < HC; ++c) acc[c] = 0.0;
    for (int j = 0; j < r; ++j) {
      const double b = Bs[ri * lb + j];
#pragma unroll
      for (int c = 0; c < HC; ++c) acc[c] = fma(b, Ts[j * KM + rh * HC + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < HC; ++c) Cs[ri * KM + rh * HC + c] = acc[c];
  }
  __syncthreads();
  if (tid < 64) {
    double X[2][KM], Q[2][KM];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int c = 0; c < KM; ++c) {
        const int i = tid + 64 * p;
        X[p][c] = i < r ? Cs[i * KM + c] : 0.0;
      }
    qr_reg_wave<KM>(X, k, Q);
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
      for (int c = 0; c < KM; ++c) {
        const int i = tid + 64 * p;
        if (i < r) {
          Cs[i * KM + c] = Q[p][c];
          if (c < k) Qout[i * k + c] = Q[p][c];
        }
      }
  }
  __syncthreads();
  // P = B Q, same split
  if (ri < r) {
    double acc[HC];
#pragma unroll
    for (int c = 0; c < HC; ++c) acc[c] = 0.0;
    for (int j = 0; j < r; ++j) {
      const double b = Bs[ri * lb + j];
#pragma unroll
      for (int c = 0; c < HC; ++c) acc[c] = fma(b, Cs[j * KM + rh * HC + c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < HC; ++c)
      if (rh * HC + c < k) Pout[ri * k + rh * HC + c] = acc[c];
  }
}

// ---------------------------------------------- register-tiled SPD inverse ----
// In-place inverse of an SPD matrix, n <= 128, by the symmetric sweep operator
// (Goodnight 1979): sweeping a pivot set P maps A_PP -> -A_PP^{-1},
// A_iP -> A_iP A_PP^{-1}, A_Pj -> A_PP^{-1} A_Pj and A_ij -> A_ij - A_iP
// A_PP^{-1} A_Pj; sweeps of disjoint sets commute, and after every index has
// been swept the matrix is -G^{-1}.  Pivots are taken two at a time: the 2 x 2
// block is inverted through its Schur complement (the Cholesky pivots of the
// pair, so a non-positive one flags a non-SPD Gram), which halves the number
// of dependent steps and barriers.  256 threads; thread (tr, tc) = (t / 16,
// t % 16) owns rows tr + 16 a and columns tc + 16 b (a, b < NB) in registers.
// Indices >= n are padded with the identity, which the sweep leaves untouched,
// so an odd n needs no special last step.  The two pivot columns of the next
// step are published through LDS (double-buffered: one barrier per step).
//
// Only the pivot rows are fixed up: a swept column is never read again (the
// next pivot columns are unswept, and every entry a later step reads from a
// swept index lies in that index's row), so the rows, hence the lower triangle
// in sweep order, stay exact; the result is mirrored from it through LDS.
constexpr int kPairT = 256, kRegMax = 128;

template <int NB>
constexpr size_t spd_pair_lds() {
  return size_t(16 * NB) * (16 * NB + 1) * 8;
}

// S: NP x (NP + 1) doubles of LDS for the result staging
template <int NB>
__device__ __forceinline__ void spd_inverse_pair_body(double* G, int n, int lda, int* info,
                                                      double* S) {
  constexpr int NP = 16 * NB, SP = NP + 1;
  __shared__ double col[2][2][NP];
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  double A[NB][NB];
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = tr + 16 * a, j = tc + 16 * b;
      A[a][b] = (i < n && j < n) ? G[i * lda + j] : (i == j ? 1.0 : 0.0);
    }
  if (tc < 2)  // columns 0 and 1
#pragma unroll
    for (int a = 0; a < NB; ++a) col[0][tc][tr + 16 * a] = A[a][0];
  __syncthreads();
  int bad = 0;
  const int steps = (n + 1) / 2;
  // the pivot rows and the next pivot columns lie in register block p / 16,
  // a constant of the outer (unrolled) loop, so the tile is never indexed
  // dynamically
  static_for<0, NB>([&](auto KC) {
    constexpr int KB = decltype(KC)::value;
    const int t1 = min(steps, 8 * (KB + 1));
    for (int t = 8 * KB; t < t1; ++t) {
      const int p = 2 * t, kt = p & 15;
      const double* cp = col[t & 1][0];
      const double* cq = col[t & 1][1];
      const double dpp = cp[p], dpq = cp[p + 1], dqq = cq[p + 1];
      const double r1 = rcp64(dpp);
      const double l = dpq * r1;
      const double sch = fma(-l, dpq, dqq);
      const double r2 = rcp64(sch);
      if (bad == 0) bad = !(dpp > 0.0) ? p + 1 : (!(sch > 0.0) ? p + 2 : 0);
      // E = A_PP^{-1}
      const double eqq = r2, epq = -l * r2, epp = fma(l * r2, l, r1);
      double mp[NB], mq[NB], xp[NB], xq[NB];
#pragma unroll
      for (int a = 0; a < NB; ++a) {
        const double ap = cp[tr + 16 * a], aq = cq[tr + 16 * a];
        mp[a] = fma(ap, epp, aq * epq);  // (A_iP E)_p
        mq[a] = fma(ap, epq, aq * eqq);
      }
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        xp[b] = cp[tc + 16 * b];  // A_pj = A_jp
        xq[b] = cq[tc + 16 * b];
      }
#pragma unroll
      for (int a = 0; a < NB; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) A[a][b] = fma(-mp[a], xp[b], fma(-mq[a], xq[b], A[a][b]));
      // rows p, q (lanes tr = kt, kt + 1, which share a wave) -> E A_Pj, and
      // the 2 x 2 block itself -> -E
      if ((tr >> 1) == (kt >> 1)) {
        const bool rowq = tr & 1;
        const double f0 = rowq ? epq : epp, f1 = rowq ? eqq : epq;
#pragma unroll
        for (int b = 0; b < NB; ++b) A[KB][b] = fma(f0, xp[b], f1 * xq[b]);
        if (tc == kt) A[KB][KB] = -f0;
        if (tc == kt + 1) A[KB][KB] = -f1;
      }
      // publish columns p + 2 and p + 3 (block KB, or KB + 1 after the last
      // pair of this block)
      const int nt = (p + 2) & 15;
      if ((tc >> 1) == (nt >> 1)) {
        double* dst = col[(t + 1) & 1][tc & 1];
        if (nt != 0) {
#pragma unroll
          for (int a = 0; a < NB; ++a) dst[tr + 16 * a] = A[a][KB];
        } else if (KB + 1 < NB) {
#pragma unroll
          for (int a = 0; a < NB; ++a) dst[tr + 16 * a] = A[a][(KB + 1) % NB];
        }
      }
      __syncthreads();
    }
  });
  if (tid == 0 && bad) *info = bad;  // sticky: the caller zeroes info once per job
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) S[(tr + 16 * a) * SP + tc + 16 * b] = A[a][b];
  __syncthreads();
#pragma unroll
  for (int a = 0; a < NB; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int i = tr + 16 * a, j = tc + 16 * b;
      if (i < n && j < n) G[i * lda + j] = -(i >= j ? A[a][b] : S[j * SP + i]);
    }
}

template <int NB>
__global__ __launch_bounds__(kPairT) void k_spd_inverse_pair(double* G, int n, int lda,
                                                             int* info) {
  extern __shared__ double S[];
  spd_inverse_pair_body<NB>(G, n, lda, info, S);
}

// C0 = A^T B (A K x M, B K x N, skinny tiles of 4 waves) in blocks [0, tiles)
// and the SPD inverse of G in the last block: the two products of the
// randomized solve that do not depend on each other share one launch, and
// the tiles run on other CUs while the one-workgroup inverse runs.
template <int NB>
__global__ __launch_bounds__(kPairT) void k_c0_inverse(int64_t M, int64_t N, int64_t K,
                                                       const double* A, int64_t lda,
                                                       const double* B, int64_t ldb, double* C,
                                                       int64_t ldc, int tiles_m, int tiles,
                                                       double* G, int n, int ldg, int* info) {
  extern __shared__ double S[];
  if (int(blockIdx.x) < tiles) {
    auto* red = reinterpret_cast<double (*)[16][17]>(S);
    skinny_tile<kPairT / 64, false>(M, N, K, A, lda, M, A, lda, B, ldb, C, ldc,
                                    blockIdx.x % tiles_m, blockIdx.x / tiles_m, red);
  } else {
    spd_inverse_pair_body<NB>(G, n, ldg, info, S);
  }
}

// -------------------------------------------------------------- sign fix ----
__global__ void k_sign_fix(double* A, int64_t rows, int64_t R, double* sgn) {
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
  if (sgn && threadIdx.x == 0) sgn[c] = flip ? -1.0 : 1.0;
  __syncthreads();
  if (flip)
    for (int64_t i = threadIdx.x; i < rows; i += 256) A[i * R + c] = -A[i * R + c];
}

// The same rule for tall A (rows >= kSfSplitRows, R <= 256) in two launches
// over ranges of rpb rows, reading A row-major in order: per range and
// column the first largest magnitude (its index and signed value), then
// every range combines the ranges' results in range order (largest, lowest
// index on ties: the entry k_sign_fix picks) and flips its own rows.  Where
// no entry compares (all NaN) the sign of row 0 decides, as in k_sign_fix.
constexpr int64_t kSfSplitRows = 2048;
constexpr int kSfMaxRanges = 64;

__global__ __launch_bounds__(256) void k_sign_ranges(const double* A, int64_t rows, int R,
                                                     int64_t rpb, double* pv, double* ps,
                                                     int64_t* pix, double* row0) {
  __shared__ double bv[256], bs[256];
  __shared__ int64_t bi[256];
  const int tid = threadIdx.x, RS = 256 / R, c = tid % R, ro = tid / R;
  const int64_t i0 = int64_t(blockIdx.x) * rpb;
  const int64_t i1 = i0 + rpb < rows ? i0 + rpb : rows;
  double best = -1.0, bsig = 0.0;
  int64_t bidx = INT64_MAX;
  if (ro < RS)
    for (int64_t i = i0 + ro; i < i1; i += RS) {
      const double x = A[i * R + c];
      const double a = fabs(x);
      if (a > best) best = a, bidx = i, bsig = x;  // first maximum of this thread's rows
    }
  bv[tid] = best;
  bs[tid] = bsig;
  bi[tid] = bidx;
  __syncthreads();
  if (tid >= R) return;
  for (int o = 1; o < RS; ++o) {
    const int u = o * R + tid;
    if (bv[u] > best || (bv[u] == best && bi[u] < bidx)) best = bv[u], bidx = bi[u], bsig = bs[u];
  }
  const int64_t q = int64_t(blockIdx.x) * R + tid;
  pv[q] = best;
  ps[q] = bsig;
  pix[q] = bidx;
  if (blockIdx.x == 0) row0[tid] = A[tid];
}

__global__ __launch_bounds__(256) void k_sign_apply(double* A, int64_t rows, int R, int64_t rpb,
                                                    int nranges, const double* pv,
                                                    const double* ps, const int64_t* pix,
                                                    const double* row0, double* sgn) {
  __shared__ bool flip[256];
  const int tid = threadIdx.x;
  if (tid < R) {
    double best = -1.0, bsig = 0.0;
    int64_t bidx = INT64_MAX;
    for (int q0 = 0; q0 < nranges; q0 += 8) {  // eight ranges' loads in flight
      double v[8], sg[8];
      int64_t ix[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t e = int64_t(q0 + u < nranges ? q0 + u : nranges - 1) * R + tid;
        v[u] = pv[e];
        sg[u] = ps[e];
        ix[u] = pix[e];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (q0 + u < nranges && (v[u] > best || (v[u] == best && ix[u] < bidx)))
          best = v[u], bidx = ix[u], bsig = sg[u];
    }
    const bool f = (bidx == INT64_MAX ? row0[tid] : bsig) < 0.0;
    flip[tid] = f;
    if (sgn && blockIdx.x == 0) sgn[tid] = f ? -1.0 : 1.0;
  }
  __syncthreads();
  const int64_t i0 = int64_t(blockIdx.x) * rpb;
  const int64_t i1 = i0 + rpb < rows ? i0 + rpb : rows;
  const int64_t n = (i1 - i0) * R;
  double* a = A + i0 * R;
  for (int64_t e = tid; e < n; e += 256)
    if (flip[e % R]) a[e] = -a[e];
}

// W (r x R) = Q U diag(lam * sgn) with Q given by rows of Q^T (k x r) and U
// (k x R) already scaled by lam^{-1/2}: Q times the left singular vectors
// times the singular values, in the column signs chosen for the right ones.
__global__ void k_rsvd_w(const double* Qm, bool q_rows, const double* U, const double* lam,
                         const double* sgn, int k, int r, int R, double* W) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= r * R) return;
  const int i = t / R, c = t % R;
  double s = 0.0;
  for (int j = 0; j < k; ++j) s = fma(q_rows ? Qm[i * k + j] : Qm[j * r + i], U[j * R + c], s);
  W[t] = s * lam[c] * sgn[c];
}

// Last steps of the randomized solve in one launch, one workgroup per column
// c of A: u = U(:, c) lam_c^{-1/2}; A(:, c) = D^T u (each row a dot product
// of length k, the row read in pairs when k is even); the sign that makes the
// largest-magnitude entry positive (lowest index on ties, as k_sign_fix);
// A(:, c) in that sign; and W(:, c) = Q U(:, c) lam_c^{1/2} in the same sign.
// Q is r x k, Dt is s x k; k <= 64.  *bad is set when lam_c is not positive
// (D of rank below R: no division by its square root is meaningful).
constexpr int kFinRegs = 16;  // rows per thread kept in registers by k_rsvd_finish
constexpr int kFinT = 256;

__global__ __launch_bounds__(kFinT) void k_rsvd_finish(const double* Dt, const double* U,
                                                       const double* lam, const double* Q,
                                                       int s, int k, int r, int R, double* A,
                                                       double* W, int* bad) {
  __shared__ double us[64];
  __shared__ double bv[kFinT];
  __shared__ int bi[kFinT];
  __shared__ int bn[kFinT];
  const int c = blockIdx.x, tid = threadIdx.x;
  const double lc = lam[c];
  if (tid == 0 && !(lc > 0.0)) *bad = 1;
  if (tid < k) us[tid] = U[tid * R + c] / sqrt(lc);
  __syncthreads();
  double best = -1.0;
  int bidx = 0, bneg = 0;
  const bool pairs = (k & 1) == 0;
  auto row_value = [&](int i) {
    const double* d = Dt + size_t(i) * k;
    double a0 = 0.0, a1 = 0.0;
    if (pairs) {
      const double2* d2 = reinterpret_cast<const double2*>(d);
      for (int j = 0; j < k / 2; ++j) {
        const double2 v = d2[j];
        a0 = fma(v.x, us[2 * j], a0);
        a1 = fma(v.y, us[2 * j + 1], a1);
      }
    } else {
      for (int j = 0; j < k; ++j) a0 = fma(d[j], us[j], a0);
    }
    const double a = a0 + a1;
    if (fabs(a) > best) best = fabs(a), bidx = i, bneg = a < 0.0;  // first maximum in the stride
    return a;
  };
  // the first kFinRegs rows of this thread stay in registers until the sign
  // is known; rows beyond them (s > kFinRegs kFinT) go through A twice
  double keep[kFinRegs];
#pragma unroll
  for (int t = 0; t < kFinRegs; ++t) {
    const int i = tid + t * kFinT;
    keep[t] = i < s ? row_value(i) : 0.0;
  }
  for (int i = tid + kFinRegs * kFinT; i < s; i += kFinT) A[size_t(i) * R + c] = row_value(i);
  bv[tid] = best;
  bi[tid] = bidx;
  bn[tid] = bneg;
  __syncthreads();
  for (int off = kFinT / 2; off > 0; off >>= 1) {
    if (tid < off) {
      const double o = bv[tid + off];
      const int oi = bi[tid + off];
      if (o > bv[tid] || (o == bv[tid] && oi < bi[tid]))
        bv[tid] = o, bi[tid] = oi, bn[tid] = bn[tid + off];
    }
    __syncthreads();
  }
  const bool flip = bn[0] != 0;
#pragma unroll
  for (int t = 0; t < kFinRegs; ++t) {
    const int i = tid + t * kFinT;
    if (i < s) A[size_t(i) * R + c] = flip ? -keep[t] : keep[t];
  }
  if (flip)
    for (int i = tid + kFinRegs * kFinT; i < s; i += kFinT)
      A[size_t(i) * R + c] = -A[size_t(i) * R + c];
  const double ws = flip ? -sqrt(lc) : sqrt(lc);
  for (int i = tid; i < r; i += kFinT) {
    double w = 0.0;
    for (int j = 0; j < k; ++j) w = fma(Q[i * k + j], U[j * R + c], w);
    W[i * R + c] = w * ws;
  }
}

__global__ void k_scale_inv_sqrt(double* A, int64_t rows, int64_t R, const double* lam, int* bad) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (bad && t < R && !(lam[t] > 0.0)) *bad = 1;
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

// ------------------------------------------------- blocked SPD inverse ----
// Inverse of an SPD matrix of any order by the symmetric sweep operator taken
// one pivot block of TB indices at a time (the block form of the sweeps
// above): sweeping P maps A_PP -> -A_PP^{-1}, A_IP -> A_IP A_PP^{-1},
// A_PJ -> A_PP^{-1} A_PJ and A_IJ -> A_IJ - A_IP A_PP^{-1} A_PJ; after the
// last block the matrix is -G^{-1}.  One launch per block step, one
// workgroup per TB x TB tile of the (full, row-major) matrix; the products
// are FP64 MFMA 16x16x4 tiles from LDS.  The step reads matrix X and writes Y
// (two buffers, so that no tile is overwritten while others still read it).
// The pivot inverse comes from the previous launch: the workgroup of the tile
// that becomes the next pivot block inverts it right after updating it (the
// register-tiled pair sweeps above, on the LDS copy), so each step is one
// launch.  Indices >= n are padded with the identity, which sweeps leave
// untouched.  The pivots of the pair sweeps are those of the Schur complements,
// i.e. the Cholesky pivots of G: the first non-positive one sets *info (global
// index + 1) when *info is still 0.
template <int TB>
constexpr size_t sweep_lds_bytes() {
  return size_t(4) * TB * (TB + 1) * 8;
}

// acc (wave quadrant of a TB x TB tile, (TB/32)^2 MFMA blocks) += A B, both
// TB x TB in LDS with row stride TB + 1
template <int TB>
__device__ __forceinline__ void sweep_tile_mma(const double* A, const double* B,
                                               dx4 (&acc)[TB / 32][TB / 32], int lane, int wave) {
  constexpr int SL = TB + 1, NW = TB / 32;
  const int qi = (wave >> 1) * (TB / 2), qj = (wave & 1) * (TB / 2);
  const int li = lane & 15, g = lane >> 4;
#pragma unroll 4
  for (int k0 = 0; k0 < TB; k0 += 4) {
    double a[NW], b[NW];
#pragma unroll
    for (int x = 0; x < NW; ++x) a[x] = A[(qi + 16 * x + li) * SL + k0 + g];
#pragma unroll
    for (int y = 0; y < NW; ++y) b[y] = B[(k0 + g) * SL + qj + 16 * y + li];
#pragma unroll
    for (int x = 0; x < NW; ++x)
#pragma unroll
      for (int y = 0; y < NW; ++y)
        acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
  }
}

// element (i, j) of the matrix, identity beyond n
__device__ __forceinline__ double sweep_ld(const double* X, int ldx, int n, int i, int j) {
  return (i < n && j < n) ? X[int64_t(i) * ldx + j] : (i == j ? 1.0 : 0.0);
}

// TB x TB tile at (r0, c0) of X into LDS (stride TB + 1), identity-padded
template <int TB>
__device__ __forceinline__ void sweep_stage(double* S, const double* X, int ldx, int n, int r0,
                                            int c0) {
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    const int i = e / TB, j = e % TB;
    S[i * (TB + 1) + j] = sweep_ld(X, ldx, n, r0 + i, c0 + j);
  }
}

// Inverse of the SPD tile held in LDS at T (stride TB + 1, identity-padded
// beyond nb valid indices) into Pout (TB x TB, ld TB); S2 is LDS scratch of
// TB x (TB + 1) doubles.  Pivot failures set *info to base + local pivot + 1.
template <int TB>
__device__ void sweep_pivot_inverse(double* T, int nb, double* S2, double* Pout, int* info,
                                    int base) {
  __shared__ int linfo;
  if (threadIdx.x == 0) linfo = 0;
  __syncthreads();
  spd_inverse_pair_body<TB / 16>(T, nb, TB + 1, &linfo, S2);
  __syncthreads();
  for (int e = threadIdx.x; e < TB * TB; e += 256) {
    const int i = e / TB, j = e % TB;
    Pout[e] = (i < nb && j < nb) ? T[i * (TB + 1) + j] : (i == j ? 1.0 : 0.0);
  }
  if (threadIdx.x == 0 && linfo) atomicCAS(info, 0, base + linfo);
}

template <int TB>
__global__ __launch_bounds__(256) void k_sweep_first(const double* X, int ldx, int n,
                                                     double* Pout, int* info) {
  extern __shared__ double sm[];
  constexpr int SZ = TB * (TB + 1);
  sweep_stage<TB>(sm, X, ldx, n, 0, 0);
  __syncthreads();
  sweep_pivot_inverse<TB>(sm, n < TB ? n : TB, sm + SZ, Pout, info, 0);
}

template <int TB>
__global__ __launch_bounds__(256) void k_sweep_step(const double* X, int ldx, double* Y, int ldy,
                                                    int n, int p, const double* Pin,
                                                    double* Pout, int last, int* info) {
  extern __shared__ double sm[];
  constexpr int SL = TB + 1, SZ = TB * SL, NW = TB / 32;
  double* sIP = sm;
  double* sPin = sm + SZ;
  double* sPJ = sm + 2 * SZ;
  double* sF = sm + 3 * SZ;
  const int I = blockIdx.y, J = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = I * TB, c0 = J * TB, p0 = p * TB;
  const double sg = last ? -1.0 : 1.0;  // the swept matrix is -G^{-1}
  const int qi = (wave >> 1) * (TB / 2), qj = (wave & 1) * (TB / 2);
  const int li = lane & 15, g = lane >> 4;

  dx4 acc[NW][NW];
#pragma unroll
  for (int x = 0; x < NW; ++x)
#pragma unroll
    for (int y = 0; y < NW; ++y) acc[x][y] = dx4{0.0, 0.0, 0.0, 0.0};

  for (int e = tid; e < TB * TB; e += 256) sPin[(e / TB) * SL + e % TB] = Pin[e];
  if (I != p) sweep_stage<TB>(sIP, X, ldx, n, r0, p0);
  if (J != p) sweep_stage<TB>(sPJ, X, ldx, n, p0, c0);
  __syncthreads();
  if (I == p && J == p) {
    // -A_PP^{-1}
#pragma unroll
    for (int x = 0; x < NW; ++x)
#pragma unroll
      for (int y = 0; y < NW; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          acc[x][y][v] = -sPin[(qi + 16 * x + g + 4 * v) * SL + qj + 16 * y + li];
  } else if (J == p) {
    sweep_tile_mma<TB>(sIP, sPin, acc, lane, wave);  // A_IP A_PP^{-1}
  } else if (I == p) {
    sweep_tile_mma<TB>(sPin, sPJ, acc, lane, wave);  // A_PP^{-1} A_PJ
  } else {
    // F = A_IP A_PP^{-1} to LDS, then A_IJ - F A_PJ
    sweep_tile_mma<TB>(sIP, sPin, acc, lane, wave);
#pragma unroll
    for (int x = 0; x < NW; ++x)
#pragma unroll
      for (int y = 0; y < NW; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          sF[(qi + 16 * x + g + 4 * v) * SL + qj + 16 * y + li] = acc[x][y][v];
          acc[x][y][v] = 0.0;
        }
    __syncthreads();
    sweep_tile_mma<TB>(sF, sPJ, acc, lane, wave);
#pragma unroll
    for (int x = 0; x < NW; ++x)
#pragma unroll
      for (int y = 0; y < NW; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = r0 + qi + 16 * x + g + 4 * v, j = c0 + qj + 16 * y + li;
          acc[x][y][v] = sweep_ld(X, ldx, n, i, j) - acc[x][y][v];
        }
  }
  // store (the identity padding beyond n is not stored)
#pragma unroll
  for (int x = 0; x < NW; ++x)
#pragma unroll
    for (int y = 0; y < NW; ++y)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = r0 + qi + 16 * x + g + 4 * v, j = c0 + qj + 16 * y + li;
        if (i < n && j < n) Y[int64_t(i) * ldy + j] = sg * acc[x][y][v];
      }
  if (!last && I == p + 1 && J == p + 1) {
    // this tile is the next pivot block: invert it for the next launch
    __syncthreads();  // every wave is done with sIP, sPJ and sF
#pragma unroll
    for (int x = 0; x < NW; ++x)
#pragma unroll
      for (int y = 0; y < NW; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sPJ[(qi + 16 * x + g + 4 * v) * SL + qj + 16 * y + li] = acc[x][y][v];
    __syncthreads();
    const int nb = n - r0 < TB ? n - r0 : TB;
    sweep_pivot_inverse<TB>(sPJ, nb, sIP, Pout, info, r0);
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
  if (use_lds)
    hipLaunchKernelGGL(k_cholesky<true>, dim3(1), dim3(kCholT), bytes, st, G, int(n), int(lda),
                       info);
  else
    hipLaunchKernelGGL(k_cholesky<false>, dim3(1), dim3(kCholT), 0, st, G, int(n), int(lda), info);
  TSK_LAUNCHED();
  return TSK_OK;
}

bool c0_inverse_fits(int64_t n) {
  return n <= kRegMax &&
         (n <= 64 ? spd_pair_lds<4>() : n <= 112 ? spd_pair_lds<7>() : spd_pair_lds<8>()) + 8192 <=
             size_t(max_lds_bytes());
}

tsk_status c0_and_inverse(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                          const double* B, int64_t ldb, double* C, int64_t ldc, double* G,
                          int64_t n, int64_t ldg, int* info, hipStream_t st) {
  if (!c0_inverse_fits(n)) {
    set_error("fused product and SPD inverse of order %lld is not supported", (long long)n);
    return TSK_EUNSUPPORTED;
  }
  const int tm = int(ceil_div(M, 16)), tiles = tm * int(ceil_div(N, 16));
  const dim3 grid(tiles + 1);
  if (n <= 64)
    hipLaunchKernelGGL(k_c0_inverse<4>, grid, dim3(kPairT), spd_pair_lds<4>(), st, M, N, K, A,
                       lda, B, ldb, C, ldc, tm, tiles, G, int(n), int(ldg), info);
  else if (n <= 112)
    hipLaunchKernelGGL(k_c0_inverse<7>, grid, dim3(kPairT), spd_pair_lds<7>(), st, M, N, K, A,
                       lda, B, ldb, C, ldc, tm, tiles, G, int(n), int(ldg), info);
  else
    hipLaunchKernelGGL(k_c0_inverse<8>, grid, dim3(kPairT), spd_pair_lds<8>(), st, M, N, K, A,
                       lda, B, ldb, C, ldc, tm, tiles, G, int(n), int(ldg), info);
  TSK_LAUNCHED();
  return TSK_OK;
}

bool spd_inverse_fits(int64_t n) { return size_t(n) * n * 8 + 1024 <= size_t(max_lds_bytes()); }

tsk_status spd_inverse(double* G, int64_t n, int64_t lda, int* info, hipStream_t st) {
  const size_t pair_lds = n <= 64 ? spd_pair_lds<4>() : n <= 112 ? spd_pair_lds<7>() : spd_pair_lds<8>();
  if (n <= kRegMax && pair_lds + 8192 <= size_t(max_lds_bytes())) {
    if (n <= 64)
      hipLaunchKernelGGL(k_spd_inverse_pair<4>, dim3(1), dim3(kPairT), spd_pair_lds<4>(), st, G,
                         int(n), int(lda), info);
    else if (n <= 112)
      hipLaunchKernelGGL(k_spd_inverse_pair<7>, dim3(1), dim3(kPairT), spd_pair_lds<7>(), st, G,
                         int(n), int(lda), info);
    else
      hipLaunchKernelGGL(k_spd_inverse_pair<8>, dim3(1), dim3(kPairT), spd_pair_lds<8>(), st, G,
                         int(n), int(lda), info);
    TSK_LAUNCHED();
    return TSK_OK;
  }
  if (!spd_inverse_fits(n)) {
    set_error("SPD inverse of order %lld exceeds the LDS budget", (long long)n);
    return TSK_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(k_spd_inverse, dim3(1), dim3(kGjT), size_t(n) * n * 8, st, G, int(n),
                     int(lda), info);
  TSK_LAUNCHED();
  return TSK_OK;
}

template <int TB>
tsk_status spd_inverse_blocked_t(const double* G, int64_t n, int64_t ldg, double* Ginv,
                                 int64_t ldi, int* info, Ws& ws, hipStream_t st) {
  const int nt = int(ceil_div(n, TB));
  double* T1 = ws.take<double>(size_t(n) * n);
  double* piv = ws.take<double>(size_t(2) * TB * TB);
  if (ws.measuring()) return TSK_OK;
  hipLaunchKernelGGL(k_sweep_first<TB>, dim3(1), dim3(256), sweep_lds_bytes<TB>() / 2, st, G,
                     int(ldg), int(n), piv, info);
  TSK_LAUNCHED();
  const double* src = G;
  int64_t lds = ldg;
  for (int p = 0; p < nt; ++p) {
    // the buffers alternate so that the last step writes Ginv
    const bool to_out = ((nt - 1 - p) & 1) == 0;
    double* dst = to_out ? Ginv : T1;
    const int64_t ldd = to_out ? ldi : n;
    hipLaunchKernelGGL(k_sweep_step<TB>, dim3(nt, nt), dim3(256), sweep_lds_bytes<TB>(), st, src,
                       int(lds), dst, int(ldd), int(n), p, piv + size_t(p & 1) * TB * TB,
                       piv + size_t((p + 1) & 1) * TB * TB, p == nt - 1 ? 1 : 0, info);
    TSK_LAUNCHED();
    src = dst;
    lds = ldd;
  }
  return TSK_OK;
}

tsk_status spd_inverse_blocked(const double* G, int64_t n, int64_t ldg, double* Ginv,
                               int64_t ldi, int* info, Ws& ws, hipStream_t st) {
  if (n <= 0) return TSK_OK;
  if (!ws.measuring() && G == Ginv) {
    set_error("blocked SPD inverse needs distinct input and output");
    return TSK_EINVAL;
  }
  if (n >= 4096) return spd_inverse_blocked_t<64>(G, n, ldg, Ginv, ldi, info, ws, st);
  return spd_inverse_blocked_t<32>(G, n, ldg, Ginv, ldi, info, ws, st);
}

tsk_status chol_solve_rows(const double* L, int64_t n, int64_t ldl, double* X, int64_t rows,
                           int64_t ldx, bool forward_only, hipStream_t st) {
  if (rows == 0 || n == 0) return TSK_OK;
  const size_t budget = size_t(max_lds_bytes()) - 1024;
  const size_t lds_rows = (size_t(n) * n + size_t(kRowT) * (n + 1)) * 8;
  if (lds_rows <= budget) {
    hipLaunchKernelGGL(k_chol_solve_rows_lds, dim3(ceil_div(rows, kRowT)), dim3(kRowT), lds_rows,
                       st, L, int(n), int(ldl), X, int(rows), int(ldx), forward_only ? 1 : 0);
    TSK_LAUNCHED();
    return TSK_OK;
  }
  int64_t rb = int64_t(budget / 8) / n;
  if (rb > 64) rb = 64;
  if (rb < 1) {
    set_error("triangular solve of order %lld exceeds the LDS budget", (long long)n);
    return TSK_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(k_chol_solve_rows, dim3(ceil_div(rows, rb)), dim3(kSolveT),
                     size_t(rb * n * 8), st, L, int(n), int(ldl), X, int(rows), int(ldx), int(rb),
                     forward_only ? 1 : 0);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status sym_eig_top(double* M, int64_t q, int64_t R, double* lam, double* V, Ws& ws,
                       hipStream_t st) {
  auto* nt = static_cast<uint64_t*>(nullptr);
  if (q <= kEigSmallMax && R >= 1 && R <= q) {
    if (ws.measuring()) return TSK_OK;
    ProfScope prof("eig", st);
    if (q <= 16)
      hipLaunchKernelGGL(k_sym_eig_small<16>, dim3(1), dim3(64), 0, st, M, int(q), int(R), lam, V,
                         nt);
    else if (q <= 20)
      hipLaunchKernelGGL(k_sym_eig_small<20>, dim3(1), dim3(64), 0, st, M, int(q), int(R), lam, V,
                         nt);
    else if (q <= 24)
      hipLaunchKernelGGL(k_sym_eig_small<24>, dim3(1), dim3(64), 0, st, M, int(q), int(R), lam, V,
                         nt);
    else
      hipLaunchKernelGGL(k_sym_eig_small<28>, dim3(1), dim3(64), 0, st, M, int(q), int(R), lam, V,
                         nt);
    TSK_LAUNCHED();
    return TSK_OK;
  }
  double* scratch = ws.take<double>(size_t(5) * R * q);
  int8_t* pivs = ws.take<int8_t>(size_t(R) * q);
  if (ws.measuring()) return TSK_OK;
  const size_t budget = size_t(max_lds_bytes()) - 1024;
  const size_t sbytes = size_t(5) * q * 8;
  const size_t vbytes = size_t(5) * R * q * 8 + size_t(R) * q;
  const size_t mbytes = size_t(q) * q * 8;
  if (sbytes > budget) {
    set_error("eigenproblem of order %lld exceeds the LDS budget", (long long)q);
    return TSK_EUNSUPPORTED;
  }
  // everything in LDS when it fits; else the matrix (read and updated in
  // every tridiagonalisation step) before the inverse-iteration vectors
  const bool m_lds = sbytes + mbytes + vbytes <= budget;
  const bool m_only = !m_lds && sbytes + mbytes <= budget;
  const bool v_lds = !m_only && sbytes + (m_lds ? mbytes : 0) + vbytes <= budget;
  const size_t lds = sbytes + (m_lds || m_only ? mbytes : 0) + (v_lds ? vbytes : 0);
  ProfScope prof("eig", st);
  if (m_lds)
    hipLaunchKernelGGL((k_sym_eig_top<kEigT, true, true>), dim3(1), dim3(kEigT), lds, st, M,
                       int(q), int(R), lam, V, scratch, pivs, nt);
  else if (m_only)
    hipLaunchKernelGGL((k_sym_eig_top<kEigT, true, false>), dim3(1), dim3(kEigT), lds, st, M,
                       int(q), int(R), lam, V, scratch, pivs, nt);
  else if (v_lds)
    hipLaunchKernelGGL((k_sym_eig_top<kEigT, false, true>), dim3(1), dim3(kEigT), lds, st, M,
                       int(q), int(R), lam, V, scratch, pivs, nt);
  else
    hipLaunchKernelGGL((k_sym_eig_top<kEigT, false, false>), dim3(1), dim3(kEigT), lds, st, M,
                       int(q), int(R), lam, V, scratch, pivs, nt);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status qr_rows(const double* Ct, int64_t k, int64_t r, double* Qt, Ws& ws, hipStream_t st) {
  if (k > kQrMaxK || k > r) {
    set_error("thin QR of %lld columns of length %lld is not supported", (long long)k,
              (long long)r);
    return TSK_EUNSUPPORTED;
  }
  if (r <= kQrRegRows && k <= kQrRegMaxK) {
    if (ws.measuring()) return TSK_OK;
    if (k <= 8)
      hipLaunchKernelGGL(k_qr_reg<8>, dim3(1), dim3(64), 0, st, Ct, int(k), int(r), Qt);
    else if (k <= 16)
      hipLaunchKernelGGL(k_qr_reg<16>, dim3(1), dim3(64), 0, st, Ct, int(k), int(r), Qt);
    else if (k <= 20)
      hipLaunchKernelGGL(k_qr_reg<20>, dim3(1), dim3(64), 0, st, Ct, int(k), int(r), Qt);
    else
      hipLaunchKernelGGL(k_qr_reg<24>, dim3(1), dim3(64), 0, st, Ct, int(k), int(r), Qt);
    TSK_LAUNCHED();
    return TSK_OK;
  }
  const size_t lds = size_t(2) * k * r * 8;
  const bool fits = lds + 1024 <= size_t(max_lds_bytes());
  double* work = fits ? nullptr : ws.take<double>(size_t(k) * r);
  // shifted Cholesky QR (three passes); the Householder kernel runs only as
  // its fallback
  const bool chol = true;
  double* X1 = chol ? ws.take<double>(size_t(k) * r) : nullptr;
  double* X2 = chol ? ws.take<double>(size_t(k) * r) : nullptr;
  int* flag = chol ? ws.take<int>(1) : nullptr;
  if (ws.measuring()) return TSK_OK;
  if (chol) {
    if (k <= 32)
      hipLaunchKernelGGL(k_cholqr3<32>, dim3(1), dim3(256), size_t(2) * 32 * 33 * 8, st, Ct,
                         int(k), int(r), X1, X2, Qt, flag);
    else if (k <= 48)  // three 16-wide tiles: 44 % less matrix-core work than 64
      hipLaunchKernelGGL(k_cholqr3<48>, dim3(1), dim3(256), size_t(2) * 48 * 49 * 8, st, Ct,
                         int(k), int(r), X1, X2, Qt, flag);
    else
      hipLaunchKernelGGL(k_cholqr3<64>, dim3(1), dim3(256), size_t(2) * 64 * 65 * 8, st, Ct,
                         int(k), int(r), X1, X2, Qt, flag);
    TSK_LAUNCHED();
  }
  if (fits)
    hipLaunchKernelGGL(k_qr_rows<true>, dim3(1), dim3(64), lds, st, Ct, int(k), int(r), Qt, work,
                       flag);
  else
    hipLaunchKernelGGL(k_qr_rows<false>, dim3(1), dim3(64), 0, st, Ct, int(k), int(r), Qt, work,
                       flag);
  TSK_LAUNCHED();
  return TSK_OK;
}

bool range_basis_fits(int64_t r, int64_t k) {
  const size_t lds = (size_t(r) * (r + 1) + 2 * size_t(r) * kQrRegMaxK) * 8;
  return r <= kQrRegRows && k <= kQrRegMaxK && k <= r && lds + 1024 <= size_t(max_lds_bytes());
}

tsk_status range_basis(const double* C0, const double* B, int64_t r, int64_t k, double* Q,
                       double* P, hipStream_t st) {
  if (!range_basis_fits(r, k)) {
    set_error("range basis with r = %lld, k = %lld is not supported", (long long)r,
              (long long)k);
    return TSK_EUNSUPPORTED;
  }
  const int KM = k <= 8 ? 8 : (k <= 16 ? 16 : (k <= 20 ? 20 : 24));
  const size_t lds = (size_t(r) * (r + 1) + 2 * size_t(r) * KM) * 8;
  if (KM == 8)
    hipLaunchKernelGGL(k_range_basis<8>, dim3(1), dim3(kRbT), lds, st, C0, B, int(r), int(k), Q,
                       P);
  else if (KM == 16)
    hipLaunchKernelGGL(k_range_basis<16>, dim3(1), dim3(kRbT), lds, st, C0, B, int(r), int(k),
                       Q, P);
  else if (KM == 20)
    hipLaunchKernelGGL(k_range_basis<20>, dim3(1), dim3(kRbT), lds, st, C0, B, int(r), int(k),
                       Q, P);
  else
    hipLaunchKernelGGL(k_range_basis<24>, dim3(1), dim3(kRbT), lds, st, C0, B, int(r), int(k),
                       Q, P);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status sign_fix_columns(double* A, int64_t rows, int64_t R, hipStream_t st, double* sgn) {
  hipLaunchKernelGGL(k_sign_fix, dim3(R), dim3(256), 0, st, A, rows, R, sgn);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status sign_fix_columns(double* A, int64_t rows, int64_t R, Ws& ws, hipStream_t st,
                            double* sgn) {
  if (rows < kSfSplitRows || R > 256) {
    if (ws.measuring()) return TSK_OK;
    return sign_fix_columns(A, rows, R, st, sgn);
  }
  const int64_t rpb = std::max<int64_t>(256, ceil_div(rows, kSfMaxRanges));
  const int nr = int(ceil_div(rows, rpb));
  double* pv = ws.take<double>(size_t(nr) * R);
  double* ps = ws.take<double>(size_t(nr) * R);
  int64_t* pix = ws.take<int64_t>(size_t(nr) * R);
  double* row0 = ws.take<double>(size_t(R));
  if (ws.measuring()) return TSK_OK;
  hipLaunchKernelGGL(k_sign_ranges, dim3(unsigned(nr)), dim3(256), 0, st, A, rows, int(R), rpb,
                     pv, ps, pix, row0);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_sign_apply, dim3(unsigned(nr)), dim3(256), 0, st, A, rows, int(R), rpb,
                     nr, pv, ps, pix, row0, sgn);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status rsvd_finish(const double* Dt, const double* U, const double* lam, const double* Q,
                       int64_t s, int64_t k, int64_t r, int64_t R, double* A, double* W,
                       int* bad, hipStream_t st) {
  if (k > 64 || s > INT32_MAX / 64) {
    set_error("randomized solve finish supports k <= 64 (k = %lld)", (long long)k);
    return TSK_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(k_rsvd_finish, dim3(R), dim3(kFinT), 0, st, Dt, U, lam, Q, int(s), int(k),
                     int(r), int(R), A, W, bad);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status rsvd_w(const double* Qm, bool q_rows, const double* U, const double* lam,
                  const double* sgn, int64_t k, int64_t r, int64_t R, double* W, hipStream_t st) {
  hipLaunchKernelGGL(k_rsvd_w, dim3(ceil_div(r * R, 256)), dim3(256), 0, st, Qm, q_rows, U, lam,
                     sgn, int(k), int(r), int(R), W);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status scale_columns_inv_sqrt(double* A, int64_t rows, int64_t R, const double* lam,
                                  hipStream_t st, int* bad) {
  hipLaunchKernelGGL(k_scale_inv_sqrt, dim3(ceil_div(rows * R, 256)), dim3(256), 0, st, A, rows,
                     R, lam, bad);
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
