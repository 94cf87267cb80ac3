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
//
// Two launches per subproblem: the scores and the prefix sum of every mode (one
// workgroup per mode; the chain runs out of LDS, not through global memory),
// then the sampler, which stages the cdfs in LDS, searches every (sample, mode)
// pair in parallel and writes its block's Z rows.  Sparse fibres: fibers.hip.

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

constexpr int kLevThreads = 256;
constexpr int kLevChunk = 2048;   // rows of one LDS chunk of the prefix sum
constexpr int kLevSJ = 16;        // samples per workgroup of the sampler
constexpr int kLevLdsCdf = 5120;  // cdf entries (all modes) staged in LDS: 40 KiB
constexpr int kLevLdsRows = 128;  // sum of R_k up to which sampled rows are staged: 16 KiB
constexpr int kLevVec = 16;       // row elements loaded together

// l = sum_c a[c]^2 in column order, squares rounded before the add; the loads
// of a group of kLevVec columns are issued together.
__device__ __forceinline__ double row_score(const double* __restrict__ a, int64_t R) {
  double acc = 0.0;
  for (int64_t c0 = 0; c0 < R; c0 += kLevVec) {
    double v[kLevVec];
#pragma unroll
    for (int u = 0; u < kLevVec; ++u) v[u] = c0 + u < R ? a[c0 + u] : 0.0;
#pragma unroll
    for (int u = 0; u < kLevVec; ++u)
      if (c0 + u < R) acc = __dadd_rn(acc, __dmul_rn(v[u], v[u]));
  }
  return acc;
}

// One workgroup per mode.  Scores one row per thread; the prefix sum is one
// sequential chain (lane 0) read from and written to LDS, chunk by chunk with
// the running sum carried over, so its rounding is that of a plain loop.
__global__ __launch_bounds__(kLevThreads) void k_lev_cdf(LevModes lm) {
  __shared__ double e[kLevChunk];
  __shared__ double c[kLevChunk];
  const int q = blockIdx.x;
  const int64_t s = lm.s[q], R = lm.R[q];
  const double* __restrict__ A = lm.A[q];
  double* __restrict__ ell = lm.ell[q];
  double* __restrict__ cdf = lm.cdf[q];
  double run = 0.0;  // meaningful in lane 0 only
  for (int64_t i0 = 0; i0 < s; i0 += kLevChunk) {
    const int cw = int(min<int64_t>(kLevChunk, s - i0));
    for (int t = threadIdx.x; t < cw; t += kLevThreads) {
      const double l = row_score(A + (i0 + t) * R, R);
      e[t] = l;
      ell[i0 + t] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll 16
      for (int t = 0; t < cw; ++t) {
        run = __dadd_rn(run, e[t]);
        c[t] = run;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cw; t += kLevThreads) cdf[i0 + t] = c[t];
    __syncthreads();
  }
}

// First i in [0, s) with c[i] > target (s - 1 if none).
__device__ __forceinline__ int cdf_search(const double* c, int s, double target) {
  int lo = 0, hi = s;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c[mid] > target)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo > s - 1 ? s - 1 : lo;
}

// kLevSJ samples per workgroup: every (sample, mode) pair searches its mode's
// cdf (staged in LDS when all modes fit), the weight is formed in mode order,
// and, when Z is given, the sampled factor rows are staged in LDS and the
// workgroup's Z rows written (one element per thread, rows contiguous).
// Dynamic LDS: [staged cdfs (stage_cdf)] [kLevSJ x sum_q R_q rows (stage_rows)].
__global__ __launch_bounds__(kLevThreads) void k_lev_sample_rows(LevModes lm, int m,
                                                                 int32_t* idx, double* w, int r,
                                                                 int prec, void* Z,
                                                                 int stage_cdf, int stage_rows) {
  extern __shared__ double dyn[];
  __shared__ int32_t sidx[kLevSJ][TSK_MAX_ORDER];
  __shared__ double sprob[TSK_MAX_ORDER][kLevSJ];
  __shared__ double sw[kLevSJ];
  __shared__ int roff[TSK_MAX_ORDER + 1];
  const int tid = threadIdx.x;
  const int nm = lm.nm;
  const int j0 = blockIdx.x * kLevSJ;
  const int sj = min(kLevSJ, m - j0);
  int scdf = 0;
  if (stage_cdf) {
    for (int q = 0; q < nm; scdf += int(lm.s[q]), ++q)
      for (int i = tid; i < int(lm.s[q]); i += kLevThreads) dyn[scdf + i] = lm.cdf[q][i];
  }
  if (tid == 0) {
    int o = 0;
    for (int q = 0; q < nm; ++q) roff[q] = o, o += int(lm.R[q]);
    roff[nm] = o;
  }
  __syncthreads();
  for (int pq = tid; pq < sj * nm; pq += kLevThreads) {
    const int jj = pq % sj, q = pq / sj;
    const int s = int(lm.s[q]);
    const double* c = lm.cdf[q];
    if (stage_cdf) {
      int off = 0;
      for (int k = 0; k < q; ++k) off += int(lm.s[k]);
      c = dyn + off;
    }
    const double total = c[s - 1];
    const double u = uniform_of(draw(lm.key[q], uint64_t(j0 + jj)));
    const int i = cdf_search(c, s, __dmul_rn(u, total));
    sidx[jj][q] = i;
    sprob[q][jj] = __ddiv_rn(lm.ell[q][i], total);
  }
  __syncthreads();
  if (tid < sj) {
    double prob = 1.0;
    for (int q = 0; q < nm; ++q) {
      prob = __dmul_rn(prob, sprob[q][tid]);
      idx[int64_t(j0 + tid) * nm + q] = sidx[tid][q];
    }
    const double wj = __ddiv_rn(1.0, __dsqrt_rn(__dmul_rn(double(m), prob)));
    sw[tid] = wj;
    w[j0 + tid] = wj;
  }
  if (!Z) return;
  const int RS = roff[nm];
  double* rows = dyn + scdf;  // [jj][roff[q] + col]
  if (stage_rows) {
    for (int t = tid; t < sj * RS; t += kLevThreads) {
      const int jj = t / RS, o = t - jj * RS;
      int q = 0;
      while (o >= roff[q + 1]) ++q;
      rows[t] = lm.A[q][int64_t(sidx[jj][q]) * lm.R[q] + (o - roff[q])];
    }
  }
  __syncthreads();
  const int total = sj * r;
  for (int t = tid; t < total; t += kLevThreads) {
    const int jj = t / r;
    int rho = t - jj * r;
    int col[TSK_MAX_ORDER];
    for (int q = nm - 1; q >= 0; --q) {
      const int Rq = int(lm.R[q]);
      col[q] = rho % Rq;
      rho /= Rq;
    }
    double p = 1.0;
    for (int q = 0; q < nm; ++q) {
      const double a = stage_rows ? rows[jj * RS + roff[q] + col[q]]
                                  : lm.A[q][int64_t(sidx[jj][q]) * lm.R[q] + col[q]];
      p = __dmul_rn(p, a);
    }
    store_prec(Z, size_t(j0) * size_t(r) + size_t(t), __dmul_rn(p, sw[jj]), prec);
  }
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
                           double* w, Ws& ws, hipStream_t st, int prec, void* Z) {
  LevModes lm{};
  int64_t scdf = 0, r = 1;
  for (int k = 0; k < N; ++k) {
    if (k == n) continue;
    int q = lm.nm++;
    lm.s[q] = dims[k];
    lm.R[q] = ranks[k];
    lm.A[q] = factors[k];
    lm.ell[q] = ws.take<double>(dims[k]);
    lm.cdf[q] = ws.take<double>(dims[k]);
    lm.key[q] = stream_key(seed, kLev, sweep, n, k);
    scdf += dims[k];
    r *= ranks[k];
  }
  TSK_REQUIRE(m < (int64_t(1) << 31) && r < (int64_t(1) << 31) && scdf < (int64_t(1) << 31),
              "leverage sampling sizes beyond 32-bit indexing");
  if (ws.measuring() || m == 0) return TSK_OK;
  ProfScope prof("leverage", st);
  hipLaunchKernelGGL(k_lev_cdf, dim3(lm.nm), dim3(kLevThreads), 0, st, lm);
  TSK_LAUNCHED();
  int64_t rsum = 0;
  for (int q = 0; q < lm.nm; ++q) rsum += lm.R[q];
  const int stage_cdf = scdf <= kLevLdsCdf ? 1 : 0;
  const int stage_rows = Z && rsum <= kLevLdsRows ? 1 : 0;
  const size_t lds = ((stage_cdf ? scdf : 0) + (stage_rows ? kLevSJ * rsum : 0)) * sizeof(double);
  hipLaunchKernelGGL(k_lev_sample_rows, dim3(unsigned(ceil_div(m, kLevSJ))), dim3(kLevThreads),
                     lds, st, lm, int(m), idx, w, int(r), prec, Z, stage_cdf, stage_rows);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status leverage_rows(const TensorView& T, const int64_t* ranks, int n, int64_t m,
                         const int32_t* idx, const double* w, const double* const* factors,
                         int prec, void* Z, void* Y, hipStream_t st) {
  TSK_REQUIRE(!Y || T.layout == TSK_DENSE, "dense fibre gather on a COO tensor");
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
