// Leverage-score sampling of the Kronecker chain kron_{k != n} A^(k)
// (Def. leverage scores; Def. importance sampling; Lemma on Kronecker
// leverage scores: sampling i_k ~ l^(k) / R_k independently per mode samples
// rows of the chain with probability prod_k p^(k)_{i_k}).
//
//   scores  l_i = sum_c A(i,c)^2, columns summed in order, each square rounded
//           before the add (no fused multiply-add), so the scores -- and the
//           sampled indices below -- are a deterministic function of A
//   cdf     sequential FP64 prefix sum (one lane per mode)
//   sample  i_k = first i with cdf[i] > u * cdf[last], u from the keyed stream
//           (seed, 4, sweep, n, k) at counter j; w_j = 1/sqrt(m prod_k l_{i_k}/sum l)
//   rows    Z[j, :] = w_j kron_k A^(k)(i_k, :),  Y[j, :] = w_j T(.., i_k, .., :, ..)

#include "common.h"
#include "kernels.h"
#include "leverage.h"

namespace tsk {

namespace {

struct LevModes {
  int nm;  // N - 1
  int64_t s[TSK_MAX_ORDER];
  int64_t R[TSK_MAX_ORDER];
  const double* A[TSK_MAX_ORDER];
  double* ell[TSK_MAX_ORDER];
  double* cdf[TSK_MAX_ORDER];
  uint64_t key[TSK_MAX_ORDER];
};

__global__ void k_scores(LevModes lm) {
  const int q = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= lm.nm || i >= lm.s[q]) return;
  const double* a = lm.A[q] + i * lm.R[q];
  double acc = 0.0;
  for (int64_t c = 0; c < lm.R[q]; ++c) acc = __dadd_rn(acc, __dmul_rn(a[c], a[c]));
  lm.ell[q][i] = acc;
}

__global__ void k_cdf(LevModes lm) {
  const int q = blockIdx.x;
  if (threadIdx.x != 0 || q >= lm.nm) return;
  const double* e = lm.ell[q];
  double* c = lm.cdf[q];
  double run = 0.0;
  for (int64_t i = 0; i < lm.s[q]; ++i) {
    run = __dadd_rn(run, e[i]);
    c[i] = run;
  }
}

__global__ void k_sample(LevModes lm, int64_t m, int32_t* idx, double* w) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double prob = 1.0;
  for (int q = 0; q < lm.nm; ++q) {
    const double* c = lm.cdf[q];
    const int64_t s = lm.s[q];
    const double total = c[s - 1];
    const double u = uniform_of(draw(lm.key[q], uint64_t(j)));
    const double target = __dmul_rn(u, total);
    int64_t lo = 0, hi = s;  // first i with c[i] > target
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (c[mid] > target)
        hi = mid;
      else
        lo = mid + 1;
    }
    if (lo > s - 1) lo = s - 1;
    idx[j * lm.nm + q] = int32_t(lo);
    prob = __dmul_rn(prob, __ddiv_rn(lm.ell[q][lo], total));
  }
  w[j] = __ddiv_rn(1.0, __dsqrt_rn(__dmul_rn(double(m), prob)));
}

struct LevRows {
  int nm;
  int64_t R[TSK_MAX_ORDER];
  const double* A[TSK_MAX_ORDER];
  int64_t r;
  // dense fibre gather
  int N;
  int n;
  int64_t dims[TSK_MAX_ORDER];
  int dtype;
  const void* vals;
};

__global__ void k_lev_Z(LevRows lr, int64_t m, const int32_t* idx, const double* w, int prec,
                        void* Z) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= m * lr.r) return;
  const int64_t j = t / lr.r;
  int64_t rho = t % lr.r;
  int64_t col[TSK_MAX_ORDER];
  for (int q = lr.nm - 1; q >= 0; --q) col[q] = rho % lr.R[q], rho /= lr.R[q];
  double p = 1.0;
  for (int q = 0; q < lr.nm; ++q)
    p = __dmul_rn(p, lr.A[q][int64_t(idx[j * lr.nm + q]) * lr.R[q] + col[q]]);
  store_prec(Z, size_t(t), __dmul_rn(p, w[j]), prec);
}

__global__ void k_lev_Y(LevRows lr, int64_t m, const int32_t* idx, const double* w, int prec,
                        void* Y) {
  const int64_t sn = lr.dims[lr.n];
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= m * sn) return;
  const int64_t j = t / sn, i = t % sn;
  // row-major offset of (.., i_k, .., i at mode n, ..)
  int64_t off = 0;
  int q = 0;
  for (int k = 0; k < lr.N; ++k) {
    int64_t ik = k == lr.n ? i : int64_t(idx[j * lr.nm + q++]);
    off = off * lr.dims[k] + ik;
  }
  double v = lr.dtype == TSK_F64 ? static_cast<const double*>(lr.vals)[off]
                                 : double(static_cast<const float*>(lr.vals)[off]);
  store_prec(Y, size_t(t), __dmul_rn(w[j], v), prec);
}

}  // namespace

tsk_status leverage_sample(int N, const int64_t* dims, const int64_t* ranks, int n, int64_t m,
                           uint64_t seed, int sweep, const double* const* factors, int32_t* idx,
                           double* w, Ws& ws, hipStream_t st) {
  LevModes lm{};
  int64_t smax = 0;
  for (int k = 0; k < N; ++k) {
    if (k == n) continue;
    int q = lm.nm++;
    lm.s[q] = dims[k];
    lm.R[q] = ranks[k];
    lm.A[q] = factors[k];
    lm.ell[q] = ws.take<double>(dims[k]);
    lm.cdf[q] = ws.take<double>(dims[k]);
    lm.key[q] = stream_key(seed, kLev, sweep, n, k);
    if (dims[k] > smax) smax = dims[k];
  }
  if (ws.measuring()) return TSK_OK;
  ProfScope prof("leverage", st);
  hipLaunchKernelGGL(k_scores, dim3(ceil_div(smax, 256), lm.nm), dim3(256), 0, st, lm);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_cdf, dim3(lm.nm), dim3(64), 0, st, lm);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_sample, dim3(ceil_div(m, 256)), dim3(256), 0, st, lm, m, idx, w);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status leverage_rows(const TensorView& T, const int64_t* ranks, int n, int64_t m,
                         const int32_t* idx, const double* w, const double* const* factors,
                         int prec, void* Z, void* Y, hipStream_t st) {
  LevRows lr{};
  lr.r = 1;
  for (int k = 0; k < T.order; ++k) {
    if (k == n) continue;
    int q = lr.nm++;
    lr.R[q] = ranks[k];
    lr.A[q] = factors[k];
    lr.r *= ranks[k];
  }
  lr.N = T.order;
  lr.n = n;
  for (int k = 0; k < T.order; ++k) lr.dims[k] = T.dims[k];
  lr.dtype = T.dtype;
  lr.vals = T.values;
  ProfScope prof("leverage", st);
  if (Z) {
    hipLaunchKernelGGL(k_lev_Z, dim3(ceil_div(m * lr.r, 256)), dim3(256), 0, st, lr, m, idx, w,
                       prec, Z);
    TSK_LAUNCHED();
  }
  if (Y) {
    hipLaunchKernelGGL(k_lev_Y, dim3(ceil_div(m * T.dims[n], 256)), dim3(256), 0, st, lr, m, idx,
                       w, prec, Y);
    TSK_LAUNCHED();
  }
  return TSK_OK;
}

}  // namespace tsk
