// Relative residual ||T - T~||_F / ||T||_F of a Tucker model (1 - fitness,
// Sec. 7), in FP64 as ||T||^2 - 2 <T, T~> + ||T~||^2:
//   <T, T~>  per stored entry, T~(i) = sum_rho C(rho) prod_k A^(k)(i_k, rho_k)
//   ||T~||^2 = <C x_1 G_1 ... x_N G_N, C>, G_k = A^(k)T A^(k)
// Reductions are two-level with a fixed order (deterministic).

#include "common.h"
#include "kernels.h"
#include "fit.h"

namespace tsk {

namespace {

constexpr int kT = 256;

struct FitArgs {
  int N;
  int layout;
  int dtype;
  int64_t dims[TSK_MAX_ORDER];
  const int32_t* idx[TSK_MAX_ORDER];
  const void* vals;
  int64_t R[TSK_MAX_ORDER];
  const double* A[TSK_MAX_ORDER];
};

__device__ double block_reduce(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kT / 64; ++w) s += red[w];
  return s;
}

__global__ __launch_bounds__(kT) void k_norm2(FitArgs a, int64_t nnz, int64_t per_block,
                                              double* partial) {
  __shared__ double red[kT / 64];
  int64_t lo = int64_t(blockIdx.x) * per_block, hi = lo + per_block < nnz ? lo + per_block : nnz;
  double s = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += kT) {
    double v = a.dtype == TSK_F64 ? static_cast<const double*>(a.vals)[e]
                                  : double(static_cast<const float*>(a.vals)[e]);
    s += v * v;
  }
  s = block_reduce(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kT) void k_inner(FitArgs a, int64_t nnz, int64_t per_block,
                                              const double* core, int64_t csize, int core_lds,
                                              double* partial) {
  extern __shared__ double cs[];
  __shared__ double red[kT / 64];
  const double* C = core;
  if (core_lds) {
    for (int64_t t = threadIdx.x; t < csize; t += kT) cs[t] = core[t];
    __syncthreads();
    C = cs;
  }
  const int N = a.N;
  const int64_t Rl = a.R[N - 1];
  const int64_t outer = csize / Rl;
  int64_t lo = int64_t(blockIdx.x) * per_block, hi = lo + per_block < nnz ? lo + per_block : nnz;
  double s = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += kT) {
    int64_t ii[TSK_MAX_ORDER];
    if (a.layout == TSK_COO) {
      for (int k = 0; k < N; ++k) ii[k] = a.idx[k][e];
    } else {
      int64_t r = e;
      for (int k = N - 1; k >= 0; --k) ii[k] = r % a.dims[k], r /= a.dims[k];
    }
    const double* last = a.A[N - 1] + ii[N - 1] * Rl;
    double tv = 0.0;
    int64_t rho[TSK_MAX_ORDER] = {0};
    for (int64_t p = 0; p < outer; ++p) {
      double pre = 1.0;
      for (int k = 0; k < N - 1; ++k) pre *= a.A[k][ii[k] * a.R[k] + rho[k]];
      const double* crow = C + p * Rl;
      double in = 0.0;
      for (int64_t c = 0; c < Rl; ++c) in += crow[c] * last[c];
      tv += pre * in;
      for (int k = N - 2; k >= 0; --k) {  // odometer over the leading modes
        if (++rho[k] < a.R[k]) break;
        rho[k] = 0;
      }
    }
    double v = a.dtype == TSK_F64 ? static_cast<const double*>(a.vals)[e]
                                  : double(static_cast<const float*>(a.vals)[e]);
    s += v * tv;
  }
  s = block_reduce(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// ||T~||^2 = <C x_k G_k, C>, single block; buf0/buf1 scratch of csize
__global__ __launch_bounds__(kT) void k_model_norm2(FitArgs a, const double* core, int64_t csize,
                                                   const double* grams, double* buf0,
                                                   double* buf1, double* out) {
  __shared__ double red[kT / 64];
  const double* in = core;
  double* bufs[2] = {buf0, buf1};
  int64_t goff = 0;
  for (int k = 0; k < a.N; ++k) {
    const int64_t Rk = a.R[k];
    int64_t inner = 1;
    for (int l = k + 1; l < a.N; ++l) inner *= a.R[l];
    const double* G = grams + goff;
    double* o = bufs[k & 1];
    for (int64_t t = threadIdx.x; t < csize; t += kT) {
      int64_t rk = (t / inner) % Rk, base = t - rk * inner;
      double s = 0.0;
      for (int64_t c = 0; c < Rk; ++c) s += G[rk * Rk + c] * in[base + c * inner];
      o[t] = s;
    }
    __syncthreads();
    in = o;
    goff += Rk * Rk;
  }
  double s = 0.0;
  for (int64_t t = threadIdx.x; t < csize; t += kT) s += in[t] * core[t];
  s = block_reduce(s, red);
  if (threadIdx.x == 0) *out = s;
}

__global__ void k_finish(const double* pn, int nbn, const double* pi, int nbi,
                         const double* model2, double* nT2_out, double* res_out) {
  if (threadIdx.x != 0) return;
  double nT2 = 0.0, inner = 0.0;
  if (pn) {
    for (int b = 0; b < nbn; ++b) nT2 += pn[b];
    *nT2_out = nT2;
  } else {
    nT2 = *nT2_out;
  }
  for (int b = 0; b < nbi; ++b) inner += pi[b];
  double r2 = nT2 - 2.0 * inner + *model2;
  *res_out = sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(nT2);
}

}  // namespace

tsk_status fit_plan(const TensorView& T, const int64_t* R, FitScratch& fs, Ws& ws) {
  int64_t csize = 1, gsz = 0;
  for (int k = 0; k < T.order; ++k) csize *= R[k], gsz += R[k] * R[k];
  fs.nblocks = int(ceil_div(T.nnz, 8192));
  if (fs.nblocks > 1024) fs.nblocks = 1024;
  if (fs.nblocks < 1) fs.nblocks = 1;
  fs.partial_norm = ws.take<double>(fs.nblocks);
  fs.partial_inner = ws.take<double>(fs.nblocks);
  fs.grams = ws.take<double>(gsz);
  fs.buf0 = ws.take<double>(csize);
  fs.buf1 = ws.take<double>(csize);
  fs.model2 = ws.take<double>(1);
  fs.nT2 = ws.take<double>(1);
  return TSK_OK;
}

tsk_status fit_run(const TensorView& T, const int64_t* R, const double* core,
                   const double* const* factors, bool with_norm, FitScratch& fs, double* res,
                   Ws& ws, hipStream_t st) {
  FitArgs a{};
  a.N = T.order;
  a.layout = T.layout;
  a.dtype = T.dtype;
  int64_t csize = 1;
  for (int k = 0; k < T.order; ++k) {
    a.dims[k] = T.dims[k];
    a.idx[k] = T.idx[k];
    a.R[k] = R[k];
    a.A[k] = factors[k];
    csize *= R[k];
  }
  a.vals = T.values;
  int64_t goff = 0;
  for (int k = 0; k < T.order; ++k) {
    TSK_TRY(gemm_tn(TSK_PREC_F64, R[k], R[k], T.dims[k], factors[k], R[k], R[k], nullptr, 0,
                    factors[k], R[k], fs.grams + goff, R[k], ws, st));
    goff += R[k] * R[k];
  }
  if (ws.measuring()) return TSK_OK;
  int64_t per = ceil_div(T.nnz, fs.nblocks);
  if (with_norm) {
    hipLaunchKernelGGL(k_norm2, dim3(fs.nblocks), dim3(kT), 0, st, a, T.nnz, per,
                       fs.partial_norm);
    TSK_LAUNCHED();
  }
  int core_lds = csize * 8 <= 49152 ? 1 : 0;
  hipLaunchKernelGGL(k_inner, dim3(fs.nblocks), dim3(kT), core_lds ? size_t(csize * 8) : 0, st, a,
                     T.nnz, per, core, csize, core_lds, fs.partial_inner);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_model_norm2, dim3(1), dim3(kT), 0, st, a, core, csize, fs.grams, fs.buf0,
                     fs.buf1, fs.model2);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, st, with_norm ? fs.partial_norm : nullptr,
                     fs.nblocks, fs.partial_inner, fs.nblocks, fs.model2, fs.nT2, res);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace tsk
