// CP decomposition of the Tucker core (Alg. 6, CP-Sketch-Tucker):
//   init  HOSVD of the core: A_k = leading R_cp left singular vectors of C_(k)
//         (eigenvectors of C_(k) C_(k)^T, sign rule of the factors)
//   CP-ALS (Alg. 2) on the core, subproblem eq. (subproblem) by the normal
//         equations: A_n = MTTKRP(C, n) pinv(hadamard_{k != n} A_k^T A_k);
//         the Hadamard Gram is SPD when the factors have full column rank,
//         so its pseudo-inverse is its inverse, taken by symmetric sweeps (a
//         non-positive pivot is reported as a breakdown)
//   output B^(n) A_n and the CP relative residual against the input tensor.
// All FP64; the core (at most a few 10^4 entries) stays in device memory.

#include <cmath>

#include "common.h"
#include "cp.h"
#include "fit.h"
#include "kernels.h"

namespace tsk {

namespace {

struct CoreDesc {
  int N;
  int64_t R[TSK_MAX_ORDER];
  int64_t csize;
};

// Gram of the mode-k unfolding: G[a][b] = sum_rest C[..a..] C[..b..]
__global__ void k_unfold_gram(const double* C, CoreDesc cd, int k, double* G) {
  const int64_t Rk = cd.R[k];
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= Rk * Rk) return;
  const int64_t a = t / Rk, b = t % Rk;
  int64_t inner = 1;
  for (int l = k + 1; l < cd.N; ++l) inner *= cd.R[l];
  const int64_t outer = cd.csize / (inner * Rk);
  double s = 0.0;
  for (int64_t o = 0; o < outer; ++o)
    for (int64_t in = 0; in < inner; ++in) {
      int64_t base = o * Rk * inner + in;
      s += C[base + a * inner] * C[base + b * inner];
    }
  G[t] = s;
}

struct Facs {
  const double* A[TSK_MAX_ORDER];
};

struct CpFitArgs {
  int N;
  int layout;
  int dtype;
  int64_t dims[TSK_MAX_ORDER];
  const int32_t* idx[TSK_MAX_ORDER];
  const void* vals;
  const double* F[TSK_MAX_ORDER];
  int64_t Rc;
};


// M[i][r] = sum_{rho : rho_n = i} C[rho] prod_{k != n} A_k[rho_k][r]: one
// workgroup per row i; thread (chunk, r) sums every nchunk-th tuple of the
// other modes, the chunks are added in order
constexpr int kMtT = 256;
__global__ __launch_bounds__(kMtT) void k_mttkrp(const double* C, CoreDesc cd, Facs f, int n,
                                                 int64_t Rc, double* M) {
  __shared__ double part[kMtT];
  const int64_t i = blockIdx.x;
  const int nchunk = Rc >= kMtT ? 1 : int(kMtT / Rc);
  const int tid = threadIdx.x, r = int(tid % Rc), chunk = int(tid / Rc);
  const int64_t other = cd.csize / cd.R[n];
  double s = 0.0;
  if (chunk < nchunk)
    for (int64_t u = chunk; u < other; u += nchunk) {
      // u: row-major index of (rho_k)_{k != n}; p: its position in the core
      int64_t x = u, p = 0, stride = 1;
      double w = 1.0;
      for (int k = cd.N - 1; k >= 0; --k) {
        int64_t rk;
        if (k == n) {
          rk = i;
        } else {
          rk = x % cd.R[k];
          x /= cd.R[k];
          w *= f.A[k][rk * Rc + r];
        }
        p += rk * stride;
        stride *= cd.R[k];
      }
      s = fma(C[p], w, s);
    }
  part[tid] = s;
  __syncthreads();
  if (tid < Rc) {
    double t = 0.0;
    for (int c = 0; c < nchunk; ++c) t += part[c * Rc + tid];
    M[i * Rc + tid] = t;
  }
}

// The same sums for order-3 cores with the core slice of row i and the two
// other factors staged in LDS (dynamic: Ra Rb + (Ra + Rb) Rc doubles, a < b
// the other modes): the same tuples u = rho_a Rb + rho_b in the same order per
// thread, the same products (A_b then A_a) and the same chunk sums, so the
// result is that of k_mttkrp bit for bit, without its 64-bit index
// arithmetic and dependent global loads.
//
// With P (Rc x Rc) the row of the updated factor follows in the same launch:
// A[i][c] = sum_r M[i][r] P[r][c], summed as gemm_small does (r in order).
__global__ __launch_bounds__(kMtT) void k_mttkrp3(const double* C, CoreDesc cd, Facs f, int n,
                                                  int Rc, double* M, const double* P,
                                                  double* A) {
  extern __shared__ double ms[];
  __shared__ double part[kMtT];
  const int i = blockIdx.x;
  const int a = n == 0 ? 1 : 0, b = n == 2 ? 1 : 2;
  const int Ra = int(cd.R[a]), Rb = int(cd.R[b]), R1 = int(cd.R[1]), R2 = int(cd.R[2]);
  const int other = Ra * Rb;
  double* S = ms;                    // S[u] = C at (rho_n = i, rho_a, rho_b), u = rho_a Rb + rho_b
  double* Fa = ms + other;           // Ra x Rc
  double* Fb = Fa + Ra * Rc;         // Rb x Rc
  const int tid = threadIdx.x;
  for (int u = tid; u < other; u += kMtT) {
    const int ra = u / Rb, rb = u - ra * Rb;
    const int p = n == 0 ? (i * R1 + ra) * R2 + rb
                  : n == 1 ? (ra * R1 + i) * R2 + rb
                           : (ra * R1 + rb) * R2 + i;
    S[u] = C[p];
  }
  for (int t = tid; t < Ra * Rc; t += kMtT) Fa[t] = f.A[a][t];
  for (int t = tid; t < Rb * Rc; t += kMtT) Fb[t] = f.A[b][t];
  __syncthreads();
  const int nchunk = Rc >= kMtT ? 1 : kMtT / Rc;
  const int r = tid % Rc, chunk = tid / Rc;
  double s = 0.0;
  if (chunk < nchunk)
    for (int u = chunk; u < other; u += nchunk) {
      const int ra = u / Rb, rb = u - ra * Rb;
      const double w = Fb[rb * Rc + r] * Fa[ra * Rc + r];
      s = fma(S[u], w, s);
    }
  part[tid] = s;
  __syncthreads();
  double t = 0.0;
  if (tid < Rc) {
    for (int c = 0; c < nchunk; ++c) t += part[c * Rc + tid];
    if (!P) M[int64_t(i) * Rc + tid] = t;
  }
  if (!P) return;
  __syncthreads();  // every thread has read its chunk sums
  if (tid < Rc) part[tid] = t;
  __syncthreads();
  if (tid < Rc) {
    double acc = 0.0;
    for (int r2 = 0; r2 < Rc; ++r2) acc += part[r2] * P[r2 * Rc + tid];
    A[int64_t(i) * Rc + tid] = 1.0 * acc;
  }
}

constexpr size_t kMttkrp3Lds = 64 * 1024;

// Khatri-Rao product of the factors of modes 1..N-1, transposed:
// KR[r][j] = prod_{k >= 1} F_k[j_k][r], j the row-major index of (j_1, .., j_{N-1})
__global__ void k_khatri_rao_t(CpFitArgs a, int64_t J, double* KR) {
  const int64_t total = a.Rc * J;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = t / J, j = t % J;
    int64_t x = j;
    double w = 1.0;
    for (int k = a.N - 1; k >= 1; --k) {
      w *= a.F[k][(x % a.dims[k]) * a.Rc + r];
      x /= a.dims[k];
    }
    KR[t] = w;
  }
}

// relative residual from the per-block sums of (T - T~)^2 and T^2
__global__ void k_cp_finish_direct(const double* pd, const double* pn, int nb, double* out) {
  if (threadIdx.x != 0) return;
  double d = 0.0, n2 = 0.0;
  for (int b = 0; b < nb; ++b) d += pd[b], n2 += pn[b];
  *out = sqrt(d) / sqrt(n2);
}

// Gam = hadamard_{k != n} A_k^T A_k (Rc x Rc), from precomputed per-mode Grams
__global__ void k_hadamard_grams(const double* grams, int N, int n, int64_t Rc, double* Gam) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= Rc * Rc) return;
  double v = 1.0;
  for (int k = 0; k < N; ++k)
    if (k != n) v *= grams[k * Rc * Rc + t];
  Gam[t] = v;
}

__global__ void k_cp_inner(CpFitArgs a, int64_t nnz, int64_t per, double* pn, double* pi) {
  __shared__ double rn[4], ri[4];
  int64_t lo = int64_t(blockIdx.x) * per, hi = lo + per < nnz ? lo + per : nnz;
  double sn = 0.0, si = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += 256) {
    int64_t ii[TSK_MAX_ORDER];
    if (a.layout == TSK_COO) {
      for (int k = 0; k < a.N; ++k) ii[k] = a.idx[k][e];
    } else {
      int64_t x = e;
      for (int k = a.N - 1; k >= 0; --k) ii[k] = x % a.dims[k], x /= a.dims[k];
    }
    double tv = 0.0;
    for (int64_t r = 0; r < a.Rc; ++r) {
      double p = 1.0;
      for (int k = 0; k < a.N; ++k) p *= a.F[k][ii[k] * a.Rc + r];
      tv += p;
    }
    double v = a.dtype == TSK_F64 ? static_cast<const double*>(a.vals)[e]
                                  : double(static_cast<const float*>(a.vals)[e]);
    sn += v * v;
    si += v * tv;
  }
  for (int off = 32; off > 0; off >>= 1) {
    sn += __shfl_down(sn, off);
    si += __shfl_down(si, off);
  }
  if ((threadIdx.x & 63) == 0) rn[threadIdx.x >> 6] = sn, ri[threadIdx.x >> 6] = si;
  __syncthreads();
  if (threadIdx.x == 0) {
    pn[blockIdx.x] = rn[0] + rn[1] + rn[2] + rn[3];
    pi[blockIdx.x] = ri[0] + ri[1] + ri[2] + ri[3];
  }
}

__global__ void k_cp_finish(const double* pn, const double* pi, int nb, const double* grams,
                            int N, int64_t Rc, double* out) {
  if (threadIdx.x != 0) return;
  double nT2 = 0.0, inner = 0.0, model = 0.0;
  for (int b = 0; b < nb; ++b) nT2 += pn[b], inner += pi[b];
  for (int64_t t = 0; t < Rc * Rc; ++t) {
    double v = 1.0;
    for (int k = 0; k < N; ++k) v *= grams[k * Rc * Rc + t];
    model += v;
  }
  double r2 = nT2 - 2.0 * inner + model;
  *out = sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(nT2);
}

}  // namespace

tsk_status cp_tucker_bufs(const TensorView& T, const int64_t* R, CpTuckerBufs& b, Ws& ws) {
  int64_t cs = 1;
  for (int k = 0; k < T.order; ++k) cs *= R[k];
  b.core = ws.take<double>(cs);
  for (int k = 0; k < T.order; ++k) b.factors[k] = ws.take<double>(T.dims[k] * R[k]);
  return TSK_OK;
}

tsk_status cp_run(const TensorView& T, const int64_t* R, int Rc, int sweeps,
                  const CpTuckerBufs& tb, double* const* cp_factors, double** fit_dev, int* info,
                  Ws& ws, hipStream_t st) {
  const int N = T.order;
  const bool run = !ws.measuring();
  CoreDesc cd{};
  cd.N = N;
  cd.csize = 1;
  int64_t Rmax = 0;
  for (int k = 0; k < N; ++k) {
    cd.R[k] = R[k];
    cd.csize *= R[k];
    Rmax = std::max<int64_t>(Rmax, R[k]);
  }
  double* A[TSK_MAX_ORDER];
  for (int k = 0; k < N; ++k) A[k] = ws.take<double>(R[k] * Rc);
  double* Gu = ws.take<double>(Rmax * Rmax);
  double* lam = ws.take<double>(Rmax);
  double* grams = ws.take<double>(N * Rc * Rc);
  double* Gam = ws.take<double>(Rc * Rc);
  double* P = ws.take<double>(Rc * Rc);
  double* M = ws.take<double>(Rmax * Rc);
  double* fgrams = ws.take<double>(N * Rc * Rc);
  const int nb = 512;
  double* pn = ws.take<double>(nb);
  double* pi = ws.take<double>(nb);
  double* fit = ws.take<double>(1);
  if (fit_dev) *fit_dev = fit;
  const size_t mark = ws.off;
  size_t peak = mark;
  auto release = [&]() {
    peak = std::max(peak, ws.off);
    ws.off = mark;
  };
  ProfScope prof(run ? "cp_core" : "", st);
  // HOSVD of the core
  for (int k = 0; k < N; ++k) {
    if (run) {
      hipLaunchKernelGGL(k_unfold_gram, dim3(ceil_div(R[k] * R[k], 256)), dim3(256), 0, st,
                         tb.core, cd, k, Gu);
      TSK_LAUNCHED();
    }
    TSK_TRY(sym_eig_top(Gu, R[k], Rc, lam, A[k], ws, st));
    if (run) TSK_TRY(sign_fix_columns(A[k], R[k], Rc, st));
    release();
  }
  Facs f{};
  for (int k = 0; k < N; ++k) f.A[k] = A[k];
  for (int sweep = 0; sweep < sweeps; ++sweep)
    for (int n = 0; n < N; ++n) {
      for (int k = 0; k < N; ++k)
        if (k != n && run)
          TSK_TRY(gemm_small(Rc, Rc, R[k], 1.0, A[k], 1, Rc, A[k], Rc, 1, 0.0, grams + k * Rc * Rc,
                             Rc, st));
      if (run) {
        hipLaunchKernelGGL(k_hadamard_grams, dim3(ceil_div(Rc * Rc, 256)), dim3(256), 0, st, grams,
                           N, n, int64_t(Rc), Gam);
        TSK_LAUNCHED();
      }
      // the Hadamard Gram is SPD for factors of full column rank, so its
      // pseudo-inverse is its inverse (sweeps; a non-positive pivot is
      // reported as a breakdown)
      const double* Pinv = P;
      if (spd_inverse_fits(Rc)) {
        if (run) TSK_TRY(spd_inverse(Gam, Rc, Rc, info, st));
        Pinv = Gam;
      } else {
        TSK_TRY(spd_inverse_blocked(Gam, Rc, Rc, P, Rc, info, ws, st));
      }
      if (run) {
        const int a3 = n == 0 ? 1 : 0, b3 = n == 2 ? 1 : 2;
        const size_t lds3 =
            N == 3 ? size_t(R[a3] * R[b3] + (R[a3] + R[b3]) * Rc) * 8 : kMttkrp3Lds + 1;
        if (lds3 <= kMttkrp3Lds && Rc <= kMtT) {  // the factor row in the same launch
          hipLaunchKernelGGL(k_mttkrp3, dim3(unsigned(R[n])), dim3(kMtT), lds3, st, tb.core, cd,
                             f, n, int(Rc), M, Pinv, A[n]);
          TSK_LAUNCHED();
        } else {
          hipLaunchKernelGGL(k_mttkrp, dim3(unsigned(R[n])), dim3(kMtT), 0, st, tb.core, cd, f,
                             n, int64_t(Rc), M);
          TSK_LAUNCHED();
          TSK_TRY(gemm_small(R[n], Rc, Rc, 1.0, M, Rc, 1, Pinv, Rc, 1, 0.0, A[n], Rc, st));
        }
      }
      release();
    }
  // CP factors of the input: B^(n) A_n
  for (int k = 0; k < N; ++k)
    if (run && cp_factors)
      TSK_TRY(gemm_small(T.dims[k], Rc, R[k], 1.0, tb.factors[k], R[k], 1, A[k], Rc, 1, 0.0,
                         cp_factors[k], Rc, st));
  if (fit_dev && (cp_factors || !run)) {  // (the workspace query passes no factors)
    CpFitArgs a{};
    a.N = N;
    a.layout = T.layout;
    a.dtype = T.dtype;
    a.vals = T.values;
    a.Rc = Rc;
    for (int k = 0; k < N; ++k) {
      a.dims[k] = T.dims[k];
      a.idx[k] = T.idx[k];
      a.F[k] = cp_factors ? cp_factors[k] : nullptr;
      if (run)
        TSK_TRY(gemm_small(Rc, Rc, T.dims[k], 1.0, cp_factors[k], 1, Rc, cp_factors[k], Rc, 1, 0.0,
                           fgrams + k * Rc * Rc, Rc, st));
    }
    if (T.layout == TSK_DENSE && Rc <= kDenseFitMaxR) {
      // dense: T~(i, j) = sum_r F_0(i, r) KR(r, j), squared differences summed
      int64_t J = 1;
      for (int k = 1; k < N; ++k) J *= T.dims[k];
      double* KR = ws.take<double>(size_t(Rc) * J);
      double* pd = ws.take<double>(nb);
      if (run) {
        hipLaunchKernelGGL(k_khatri_rao_t,
                           dim3(unsigned(std::min<int64_t>(ceil_div(Rc * J, 256), 8192))),
                           dim3(256), 0, st, a, J, KR);
        TSK_LAUNCHED();
        TSK_TRY(dense_residual_partials(T, KR, cp_factors[0], Rc, nb, pd, pn, pi, st));
        hipLaunchKernelGGL(k_cp_finish_direct, dim3(1), dim3(64), 0, st, pd, pn, nb, fit);
        TSK_LAUNCHED();
      }
    } else if (run) {
      int64_t per = ceil_div(T.nnz, nb);
      hipLaunchKernelGGL(k_cp_inner, dim3(nb), dim3(256), 0, st, a, T.nnz, per, pn, pi);
      TSK_LAUNCHED();
      hipLaunchKernelGGL(k_cp_finish, dim3(1), dim3(64), 0, st, pn, pi, nb, fgrams, N,
                         int64_t(Rc), fit);
      TSK_LAUNCHED();
    }
  }
  ws.off = std::max(peak, ws.off);
  return TSK_OK;
}

}  // namespace tsk
