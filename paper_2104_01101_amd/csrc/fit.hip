// Relative residual ||T - T~||_F / ||T||_F of a Tucker model (1 - fitness,
// Sec. 7), in FP64.  Dense tensors: sum of (T - T~)^2 over all entries, T~
// from the mode products of the core with every factor but the first and one
// R_1-term product per entry.  COO
// tensors (T~ is dense, T is not): ||T||^2 - 2 <T, T~> + ||T~||^2, whose
// cancellation limits the relative residual to ~1e-8 near an exact fit:
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
                                              double* partial, double* partial_direct) {
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
  double s = 0.0, s2 = 0.0;
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
    s2 += (v - tv) * (v - tv);
  }
  s = block_reduce(s, red);
  __syncthreads();
  s2 = block_reduce(s2, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s, partial_direct[blockIdx.x] = s2;
}

// Order-3 and order-4 forms of k_inner: each lane owns one entry, keeps the
// factor rows of its coordinates in registers (RM >= every rank) and reads the
// core from LDS (all lanes read the same core element: broadcast).
template <int RM>
__global__ __launch_bounds__(kT) void k_inner3(FitArgs a, int64_t nnz, int64_t per_block,
                                               const double* core, int core_lds,
                                               double* partial, double* partial_direct) {
  extern __shared__ double cs_lds[];
  __shared__ double red[kT / 64];
  const int R0 = int(a.R[0]), R1 = int(a.R[1]), R2 = int(a.R[2]);
  const double* cs = core;
  if (core_lds) {
    for (int t = threadIdx.x; t < R0 * R1 * R2; t += kT) cs_lds[t] = core[t];
    __syncthreads();
    cs = cs_lds;
  }
  int64_t lo = int64_t(blockIdx.x) * per_block, hi = lo + per_block < nnz ? lo + per_block : nnz;
  double acc = 0.0, acc2 = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += kT) {
    int64_t i0, i1, i2;
    if (a.layout == TSK_COO) {
      i0 = a.idx[0][e], i1 = a.idx[1][e], i2 = a.idx[2][e];
    } else {
      i2 = e % a.dims[2];
      int64_t r = e / a.dims[2];
      i1 = r % a.dims[1];
      i0 = r / a.dims[1];
    }
    double u2[RM], u1[RM];
#pragma unroll
    for (int c = 0; c < RM; ++c) {
      u2[c] = c < R2 ? a.A[2][i2 * R2 + c] : 0.0;
      u1[c] = c < R1 ? a.A[1][i1 * R1 + c] : 0.0;
    }
    const double* a0 = a.A[0] + i0 * R0;
    double tv = 0.0;
    for (int x = 0; x < R0; ++x) {
      double wx = 0.0;
      const double* cx = cs + x * R1 * R2;
#pragma unroll
      for (int y = 0; y < RM; ++y) {
        if (y >= R1) break;
        double s = 0.0;
#pragma unroll
        for (int z = 0; z < RM; ++z) {
          if (z >= R2) break;
          s += cx[y * R2 + z] * u2[z];
        }
        wx += s * u1[y];
      }
      tv += wx * a0[x];
    }
    double v = a.dtype == TSK_F64 ? static_cast<const double*>(a.vals)[e]
                                  : double(static_cast<const float*>(a.vals)[e]);
    acc += v * tv;
    acc2 += (v - tv) * (v - tv);
  }
  acc = block_reduce(acc, red);
  __syncthreads();
  acc2 = block_reduce(acc2, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc, partial_direct[blockIdx.x] = acc2;
}

// Same, all three ranks equal to RR at compile time.  The core is the same
// for every lane, so it is read with scalar loads into SGPRs, which the FP64
// FMAs take as their scalar operand: no LDS traffic for it.  The x and y
// loops stay rolled so that an iteration loads only its RR core values (the
// whole core would not fit the SGPRs), and the multipliers indexed by x and y
// come from a thread-private LDS column rather than a dynamically indexed
// register array.
template <int RR>
__global__ __launch_bounds__(kT) void k_inner3x(FitArgs a, int64_t nnz, int64_t per_block,
                                                const double* __restrict__ core,
                                                double* partial, double* partial_direct) {
  __shared__ double red[kT / 64];
  __shared__ double us[2][RR][kT];  // u0 and u1 of this thread's entry
  const int tid = threadIdx.x;
  int64_t lo = int64_t(blockIdx.x) * per_block, hi = lo + per_block < nnz ? lo + per_block : nnz;
  double acc = 0.0, acc2 = 0.0;
  for (int64_t e = lo + tid; e < hi; e += kT) {
    int64_t i0, i1, i2;
    if (a.layout == TSK_COO) {
      i0 = a.idx[0][e], i1 = a.idx[1][e], i2 = a.idx[2][e];
    } else {
      i2 = e % a.dims[2];
      int64_t r = e / a.dims[2];
      i1 = r % a.dims[1];
      i0 = r / a.dims[1];
    }
    double u2[RR];
#pragma unroll
    for (int c = 0; c < RR; ++c) {
      u2[c] = a.A[2][i2 * RR + c];
      us[0][c][tid] = a.A[0][i0 * RR + c];
      us[1][c][tid] = a.A[1][i1 * RR + c];
    }
    double tv = 0.0;
#pragma unroll 1
    for (int x = 0; x < RR; ++x) {
      const double* gx = core + x * RR * RR;
      double wx = 0.0;
#pragma unroll 2
      for (int y = 0; y < RR; ++y) {
        // even and odd z as two chains (shorter dependent FMA sequences)
        const double* g = gx + y * RR;
        double se = 0.0, so = 0.0;
#pragma unroll
        for (int z = 0; z + 1 < RR; z += 2) {
          se = fma(g[z], u2[z], se);
          so = fma(g[z + 1], u2[z + 1], so);
        }
        if (RR & 1) se = fma(g[RR - 1], u2[RR - 1], se);
        wx = fma(se + so, us[1][y][tid], wx);
      }
      tv = fma(wx, us[0][x][tid], tv);
    }
    double v = a.dtype == TSK_F64 ? static_cast<const double*>(a.vals)[e]
                                  : double(static_cast<const float*>(a.vals)[e]);
    acc += v * tv;
    acc2 += (v - tv) * (v - tv);
  }
  acc = block_reduce(acc, red);
  __syncthreads();
  acc2 = block_reduce(acc2, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc, partial_direct[blockIdx.x] = acc2;
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

// fixed-order sum of n partials by one block: contiguous strides per thread,
// then the block reduction (deterministic)
__device__ double block_sum_of(const double* p, int n, double* red) {
  const int per = (n + kT - 1) / kT;
  const int b0 = threadIdx.x * per, b1 = b0 + per < n ? b0 + per : n;
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += p[b];
  s = block_reduce(s, red);
  __syncthreads();
  return s;
}

// ---- dense tensors: T~ from one mode product per entry ----
// M = C x_2 A^(2) ... x_N A^(N) (R_1 x s_2 x ... x s_N) by mode products
// (k_ttm); then T~(i, j) = sum_a A^(1)(i, a) M(a, j) with j the row-major
// index of the modes 2..N, so each entry costs R_1 multiply-adds and the
// model is never stored.
// out (P x s_k x Q) = in (P x R_k x Q) contracted with A (s_k x R_k) over R_k
__global__ void k_ttm(const double* in, int64_t P, int64_t Rk, int64_t Q, const double* A,
                      int64_t sk, double* out) {
  const int64_t total = P * sk * Q;
  for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += int64_t(gridDim.x) * blockDim.x) {
    const int64_t q = t % Q, pi = t / Q, i = pi % sk, pp = pi / sk;
    const double* a = A + i * Rk;
    const double* x = in + pp * Rk * Q + q;
    double acc = 0.0;
    for (int64_t c = 0; c < Rk; ++c) acc = fma(a[c], x[c * Q], acc);
    out[t] = acc;
  }
}

// per block: sum over its columns j and every i of (T(i, j) - T~(i, j))^2,
// and of T(i, j)^2; one thread per column, the column of M in registers, the
// rows of A^(1) read as wave-uniform (scalar) loads
template <class V, int RM>
__global__ __launch_bounds__(kT) void k_fit_dense(const V* __restrict__ X, const double* __restrict__ M,
                                                  const double* __restrict__ A1, int64_t s1,
                                                  int R1, int64_t J, int64_t per_block,
                                                  double* pdirect, double* pnorm, double* pinner) {
  __shared__ double red[kT / 64];
  const int64_t lo = int64_t(blockIdx.x) * per_block;
  const int64_t hi = lo + per_block < J ? lo + per_block : J;
  double acc = 0.0, nrm = 0.0;
  for (int64_t j = lo + threadIdx.x; j < hi; j += kT) {
    double m[RM];
#pragma unroll
    for (int a = 0; a < RM; ++a) m[a] = a < R1 ? M[a * J + j] : 0.0;
    for (int64_t i = 0; i < s1; ++i) {
      const double* ar = A1 + i * R1;
      double t = 0.0;
#pragma unroll
      for (int a = 0; a < RM; ++a)
        if (a < R1) t = fma(ar[a], m[a], t);
      const double v = double(X[i * J + j]);
      const double d = v - t;
      acc = fma(d, d, acc);
      nrm = fma(v, v, nrm);
    }
  }
  acc = block_reduce(acc, red);
  __syncthreads();
  nrm = block_reduce(nrm, red);
  if (threadIdx.x == 0) {
    pdirect[blockIdx.x] = acc;
    pnorm[blockIdx.x] = nrm;
    pinner[blockIdx.x] = 0.0;
  }
}

// k_model_norm2 and k_finish in one workgroup, the mode products of the
// model norm ping-ponging between two LDS buffers of csize doubles.
__global__ __launch_bounds__(kT) void k_finish_model(FitArgs a, const double* core, int64_t csize,
                                                     const double* grams, const double* pn,
                                                     int nbn, const double* pi, int nbi,
                                                     const double* pd, int dense,
                                                     double* nT2_out, double* res_out) {
  extern __shared__ double lbuf[];  // 2 csize
  __shared__ double red[kT / 64];
  const double* in = core;
  int64_t goff = 0;
  for (int k = 0; k < a.N; ++k) {
    const int64_t Rk = a.R[k];
    int64_t inner = 1;
    for (int l = k + 1; l < a.N; ++l) inner *= a.R[l];
    const double* G = grams + goff;
    double* o = lbuf + (k & 1) * csize;
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
  double m2 = 0.0;
  for (int64_t t = threadIdx.x; t < csize; t += kT) m2 += in[t] * core[t];
  m2 = block_reduce(m2, red);
  __syncthreads();
  double nT2 = 0.0;
  if (pn) {
    nT2 = block_sum_of(pn, nbn, red);
  } else {
    nT2 = *nT2_out;
  }
  const double inner = block_sum_of(pi, nbi, red);
  const double direct = dense ? block_sum_of(pd, nbi, red) : 0.0;
  if (threadIdx.x != 0) return;
  if (pn) *nT2_out = nT2;
  double r2 = nT2 - 2.0 * inner + m2;
  if (dense) r2 = direct;  // every entry stored: sum of squared differences, no cancellation
  *res_out = sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(nT2);
}

__global__ __launch_bounds__(kT) void k_finish(const double* pn, int nbn, const double* pi, int nbi,
                                               const double* pd, int dense, const double* model2,
                                               double* nT2_out, double* res_out) {
  __shared__ double red[kT / 64];
  double nT2 = 0.0;
  if (pn) {
    nT2 = block_sum_of(pn, nbn, red);
  } else {
    nT2 = *nT2_out;
  }
  const double inner = block_sum_of(pi, nbi, red);
  const double direct = dense ? block_sum_of(pd, nbi, red) : 0.0;
  if (threadIdx.x != 0) return;
  if (pn) *nT2_out = nT2;
  double r2 = nT2 - 2.0 * inner + *model2;
  if (dense) r2 = direct;  // every entry stored: sum of squared differences, no cancellation
  *res_out = sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(nT2);
}

}  // namespace

tsk_status dense_residual_partials(const TensorView& T, const double* M, const double* A1,
                                   int64_t R1, int nblocks, double* pdirect, double* pnorm,
                                   double* pinner, hipStream_t st) {
  if (T.layout != TSK_DENSE || R1 < 1 || R1 > kDenseFitMaxR) {
    set_error("dense residual: not a dense tensor or rank %lld outside [1, %d]", (long long)R1,
              kDenseFitMaxR);
    return TSK_EUNSUPPORTED;
  }
  const int64_t s1 = T.dims[0], J = T.nnz / s1;
  const int64_t perj = ceil_div(J, nblocks);
  const int r1 = int(R1);
#define TSK_FITD(V, RM)                                                                       \
  hipLaunchKernelGGL((k_fit_dense<V, RM>), dim3(nblocks), dim3(kT), 0, st,                    \
                     static_cast<const V*>(T.values), M, A1, s1, r1, J, perj, pdirect, pnorm, \
                     pinner)
  if (T.dtype == TSK_F64) {
    if (r1 <= 8) TSK_FITD(double, 8);
    else if (r1 <= 16) TSK_FITD(double, 16);
    else if (r1 <= 32) TSK_FITD(double, 32);
    else TSK_FITD(double, 64);
  } else {
    if (r1 <= 8) TSK_FITD(float, 8);
    else if (r1 <= 16) TSK_FITD(float, 16);
    else if (r1 <= 32) TSK_FITD(float, 32);
    else TSK_FITD(float, 64);
  }
#undef TSK_FITD
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status fit_plan(const TensorView& T, const int64_t* R, FitScratch& fs, Ws& ws) {
  int64_t csize = 1, gsz = 0;
  for (int k = 0; k < T.order; ++k) csize *= R[k], gsz += R[k] * R[k];
  fs.nblocks = int(ceil_div(T.nnz, 1024));
  if (fs.nblocks > 2048) fs.nblocks = 2048;
  if (fs.nblocks < 1) fs.nblocks = 1;
  fs.partial_norm = ws.take<double>(fs.nblocks);
  fs.partial_inner = ws.take<double>(fs.nblocks);
  fs.partial_direct = ws.take<double>(fs.nblocks);
  fs.grams = ws.take<double>(gsz);
  fs.buf0 = ws.take<double>(csize);
  fs.buf1 = ws.take<double>(csize);
  fs.model2 = ws.take<double>(1);
  fs.nT2 = ws.take<double>(1);
  fs.ttm[0] = fs.ttm[1] = nullptr;
  if (T.layout == TSK_DENSE && R[0] <= kDenseFitMaxR) {
    // mode products k = N-1 .. 1 alternate between two buffers, the last
    // (the largest, R_1 x s_2 x ... x s_N) landing in ttm[0]
    int64_t need[2] = {0, 0};
    int64_t size = csize;
    for (int k = T.order - 1, step = 0; k >= 1; --k, ++step) {
      size = size / R[k] * T.dims[k];
      const int buf = ((T.order - 1 - step) & 1) ? 0 : 1;  // the last step (k = 1) -> 0
      need[buf] = std::max(need[buf], size);
    }
    fs.ttm[0] = ws.take<double>(need[0]);
    fs.ttm[1] = ws.take<double>(std::max<int64_t>(need[1], 1));
  }
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
  int64_t goff = 0, rmax_g = 0;
  double* gp[TSK_MAX_ORDER];
  for (int k = 0; k < T.order; ++k) {
    gp[k] = fs.grams + goff;
    goff += R[k] * R[k];
    rmax_g = std::max<int64_t>(rmax_g, R[k]);
  }
  if (rmax_g > 64)
    for (int k = 0; k < T.order; ++k)
      TSK_TRY(gemm_tn(TSK_PREC_F64, R[k], R[k], T.dims[k], factors[k], R[k], R[k], nullptr, 0,
                      factors[k], R[k], gp[k], R[k], ws, st));
  if (ws.measuring()) return TSK_OK;
  ProfScope prof("fit", st);
  if (rmax_g <= 64)  // the factor Grams of every mode in one launch
    TSK_TRY(gram_batch_f64(T.order, R, T.dims, factors, gp, st));
  if (T.layout == TSK_DENSE && fs.ttm[0]) {
    // M = C x_2 A^(2) ... x_N A^(N), then the fused residual over the entries
    const int N = T.order;
    const double* in = core;
    int64_t P = csize, Q = 1;
    for (int k = N - 1, step = 0; k >= 1; --k, ++step) {
      P /= R[k];
      double* out = fs.ttm[((N - 1 - step) & 1) ? 0 : 1];
      const int64_t total = P * T.dims[k] * Q;
      hipLaunchKernelGGL(k_ttm, dim3(unsigned(std::min<int64_t>(ceil_div(total, kT), 8192))),
                         dim3(kT), 0, st, in, P, R[k], Q, factors[k], T.dims[k], out);
      TSK_LAUNCHED();
      in = out;
      Q *= T.dims[k];
    }
    TSK_TRY(dense_residual_partials(T, in, factors[0], R[0], fs.nblocks, fs.partial_direct,
                                    fs.partial_norm, fs.partial_inner, st));
    // with_norm is implied: the fused kernel sums T^2 as well
    if (csize <= 4096) {
      hipLaunchKernelGGL(k_finish_model, dim3(1), dim3(kT), size_t(2 * csize) * 8, st, a, core,
                         csize, fs.grams, fs.partial_norm, fs.nblocks, fs.partial_inner,
                         fs.nblocks, fs.partial_direct, 1, fs.nT2, res);
      TSK_LAUNCHED();
      return TSK_OK;
    }
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(kT), 0, st, fs.partial_norm, fs.nblocks,
                       fs.partial_inner, fs.nblocks, fs.partial_direct, 1, fs.model2, fs.nT2,
                       res);
    TSK_LAUNCHED();
    return TSK_OK;
  }
  int64_t per = ceil_div(T.nnz, fs.nblocks);
  if (with_norm) {
    hipLaunchKernelGGL(k_norm2, dim3(fs.nblocks), dim3(kT), 0, st, a, T.nnz, per,
                       fs.partial_norm);
    TSK_LAUNCHED();
  }
  int64_t rmax = 0;
  for (int k = 0; k < T.order; ++k) rmax = std::max<int64_t>(rmax, R[k]);
  if (T.order == 3 && rmax <= 32) {
    const int core_lds = csize * 8 <= 150000 ? 1 : 0;
    const size_t lds = core_lds ? size_t(csize) * 8 : 0;
    const bool eq = R[0] == R[1] && R[1] == R[2];
    if (eq && R[0] == 5)
      hipLaunchKernelGGL(k_inner3x<5>, dim3(fs.nblocks), dim3(kT), 0, st, a, T.nnz, per, core,
                         fs.partial_inner, fs.partial_direct);
    else if (eq && R[0] == 8)
      hipLaunchKernelGGL(k_inner3x<8>, dim3(fs.nblocks), dim3(kT), 0, st, a, T.nnz, per, core,
                         fs.partial_inner, fs.partial_direct);
    else if (eq && R[0] == 10)
      hipLaunchKernelGGL(k_inner3x<10>, dim3(fs.nblocks), dim3(kT), 0, st, a, T.nnz, per, core,
                         fs.partial_inner, fs.partial_direct);
    else if (eq && R[0] == 16)
      hipLaunchKernelGGL(k_inner3x<16>, dim3(fs.nblocks), dim3(kT), 0, st, a, T.nnz, per, core,
                         fs.partial_inner, fs.partial_direct);
    else if (rmax <= 8)
      hipLaunchKernelGGL(k_inner3<8>, dim3(fs.nblocks), dim3(kT), lds, st, a, T.nnz, per, core,
                         core_lds, fs.partial_inner, fs.partial_direct);
    else if (rmax <= 16)
      hipLaunchKernelGGL(k_inner3<16>, dim3(fs.nblocks), dim3(kT), lds, st, a, T.nnz, per, core,
                         core_lds, fs.partial_inner, fs.partial_direct);
    else
      hipLaunchKernelGGL(k_inner3<32>, dim3(fs.nblocks), dim3(kT), lds, st, a, T.nnz, per, core,
                         core_lds, fs.partial_inner, fs.partial_direct);
  } else {
    int core_lds = csize * 8 <= 49152 ? 1 : 0;
    hipLaunchKernelGGL(k_inner, dim3(fs.nblocks), dim3(kT), core_lds ? size_t(csize * 8) : 0, st,
                       a, T.nnz, per, core, csize, core_lds, fs.partial_inner, fs.partial_direct);
  }
  TSK_LAUNCHED();
  if (csize <= 4096) {  // model norm in LDS inside the final reduction
    hipLaunchKernelGGL(k_finish_model, dim3(1), dim3(kT), size_t(2 * csize) * 8, st, a, core,
                       csize, fs.grams, with_norm ? fs.partial_norm : nullptr, fs.nblocks,
                       fs.partial_inner, fs.nblocks, fs.partial_direct,
                       T.layout == TSK_DENSE ? 1 : 0, fs.nT2, res);
    TSK_LAUNCHED();
    return TSK_OK;
  }
  hipLaunchKernelGGL(k_model_norm2, dim3(1), dim3(kT), 0, st, a, core, csize, fs.grams, fs.buf0,
                     fs.buf1, fs.model2);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(kT), 0, st, with_norm ? fs.partial_norm : nullptr,
                     fs.nblocks, fs.partial_inner, fs.nblocks, fs.partial_direct,
                     T.layout == TSK_DENSE ? 1 : 0, fs.model2, fs.nT2, res);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace tsk
