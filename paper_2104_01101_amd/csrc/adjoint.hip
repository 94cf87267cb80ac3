// Sketched mode-n residual L = ||Z W A^T - Y||_F^2 and its adjoint, with
// Z = S^(n) kron_{k != n} A^(k) (TensorSketch, Sec. 3.1), W = C_(n)^T, A = A^(n)
// and Y = S^(n) T_(n)^T -- the objective of the sketched subproblem of Alg. 4.
//
// E = Z W A^T - Y is never stored: every pass over Y recomputes its entries
// from P = Z W (m x R) and A.
//   forward   L = sum E^2                                   (one pass over Y)
//   backward  EA = E A (m x R), E^T P (s x R)               (two passes over Y)
//             dL/dA  = 2 E^T P,  dL/dW = 2 Z^T (E A) -> dL/dC
//             dL/dZ  = 2 (E A) W^T
//             dL/dCS_k[:, c] = IFFT(sum_{rho_k = c} conj(prod_{l != k} F_l) FFT(dL/dZ[:, rho]))
//             dL/dA^(k)[i, :] = sigma_k(i) dL/dCS_k[h_k(i), :]
// All FP64; reductions in a fixed order (deterministic).

#include "common.h"
#include "kernels.h"

namespace tsk {

namespace {

constexpr int kT = 256;
constexpr int kMaxR = 64;

template <class T>
__device__ inline double ld(const void* p, int64_t i) {
  return double(static_cast<const T*>(p)[i]);
}
__device__ inline double ldy(const void* Y, int dt, int64_t i) {
  return dt == TSK_F64 ? ld<double>(Y, i) : ld<float>(Y, i);
}

__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// partial[row] = sum_i E[row, i]^2
__global__ __launch_bounds__(kT) void k_res_rows(const double* P, const double* A, int64_t R,
                                                 const void* Y, int ydt, int64_t s,
                                                 double* partial) {
  __shared__ double red[kT / 64];
  __shared__ double p[kMaxR];
  const int64_t j = blockIdx.x;
  for (int c = threadIdx.x; c < R; c += kT) p[c] = P[j * R + c];
  __syncthreads();
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < s; i += kT) {
    double e = -ldy(Y, ydt, j * s + i);
    for (int64_t c = 0; c < R; ++c) e += p[c] * A[i * R + c];
    acc += e * e;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) partial[j] = acc;
}

__global__ void k_sum(const double* x, int64_t n, double* out) {
  __shared__ double red[kT / 64];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kT) acc += x[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) *out = acc;
}

// EA[j, :] = sum_i E[j, i] A[i, :]
__global__ __launch_bounds__(kT) void k_EA(const double* P, const double* A, int64_t R,
                                           const void* Y, int ydt, int64_t s, double* EA) {
  __shared__ double red[kT / 64];
  __shared__ double p[kMaxR];
  const int64_t j = blockIdx.x;
  for (int c = threadIdx.x; c < R; c += kT) p[c] = P[j * R + c];
  __syncthreads();
  double acc[kMaxR];
  for (int c = 0; c < R; ++c) acc[c] = 0.0;
  for (int64_t i = threadIdx.x; i < s; i += kT) {
    const double* a = A + i * R;
    double e = -ldy(Y, ydt, j * s + i);
    for (int64_t c = 0; c < R; ++c) e += p[c] * a[c];
    for (int64_t c = 0; c < R; ++c) acc[c] += e * a[c];
  }
  for (int64_t c = 0; c < R; ++c) {
    double v = block_sum(acc[c], red);
    if (threadIdx.x == 0) EA[j * R + c] = v;
  }
}

// EtP[i, :] = sum_j E[j, i] P[j, :]   (thread per column i, rows in order)
__global__ __launch_bounds__(kT) void k_EtP(const double* P, const double* A, int64_t R,
                                            const void* Y, int ydt, int64_t s, int64_t m,
                                            double* EtP) {
  const int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x;
  if (i >= s) return;
  double a[kMaxR], acc[kMaxR];
  for (int64_t c = 0; c < R; ++c) a[c] = A[i * R + c], acc[c] = 0.0;
  for (int64_t j = 0; j < m; ++j) {
    const double* p = P + j * R;
    double e = -ldy(Y, ydt, j * s + i);
    for (int64_t c = 0; c < R; ++c) e += p[c] * a[c];
    for (int64_t c = 0; c < R; ++c) acc[c] += e * p[c];
  }
  for (int64_t c = 0; c < R; ++c) EtP[i * R + c] = 2.0 * acc[c];
}

struct RArr {
  int64_t R[TSK_MAX_ORDER];
};

// gC[rho] = scale * gW[row(rho_{-n}), rho_n]
__global__ void k_w_to_core(const double* gW, int N, int n, RArr r, int64_t csize, double scale,
                            double* gC) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= csize) return;
  int64_t x = t, row = 0, mul = 1, rn = 0;
  for (int k = N - 1; k >= 0; --k) {
    int64_t rk = x % r.R[k];
    x /= r.R[k];
    if (k == n) {
      rn = rk;
    } else {
      row += rk * mul;
      mul *= r.R[k];
    }
  }
  gC[t] = scale * gW[row * r.R[n] + rn];
}

// core (row-major) -> W = C_(n)^T (r x R_n)
__global__ void k_core_to_w(const double* C, int N, int n, RArr r, int64_t csize, double* W) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= csize) return;
  int64_t x = t, row = 0, mul = 1, rn = 0;
  for (int k = N - 1; k >= 0; --k) {
    int64_t rk = x % r.R[k];
    x /= r.R[k];
    if (k == n) {
      rn = rk;
    } else {
      row += rk * mul;
      mul *= r.R[k];
    }
  }
  W[row * r.R[n] + rn] = C[t];
}

// gA_k[i, c] = sigma(i) gCS[h(i), c]
__global__ void k_cs_adjoint(const double* gCS, int64_t R, const int32_t* h, const int8_t* sg,
                             int64_t s, double* gA) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= s * R) return;
  const int64_t i = t / R, c = t % R;
  const double v = gCS[int64_t(h[i]) * R + c];
  gA[t] = sg[i] > 0 ? v : -v;
}

struct AdjCtx {
  int N, n;
  int64_t dims[TSK_MAX_ORDER], R[TSK_MAX_ORDER];
  int64_t m, r, s, Rn, csize;
};

tsk_status adj_common(const AdjCtx& c, const int32_t* const* h, const int8_t* const* sign,
                      const double* const* factors, const double* core, LhsMode* modes,
                      double*& Z, double*& W, double*& P, double*& CS, double*& spec,
                      double*& tw, Ws& ws, hipStream_t st) {
  const bool run = !ws.measuring();
  int64_t totR = 0;
  int q = 0;
  for (int k = 0; k < c.N; ++k) {
    if (k == c.n) continue;
    CsrTable t{ws.take<int32_t>(c.m + 1), ws.take<int32_t>(c.dims[k])};
    TSK_TRY(build_inverse_hash(h[k], c.dims[k], c.m, t, ws, st));
    modes[q++] = LhsMode{factors[k], c.dims[k], c.R[k], sign[k], t};
    totR += c.R[k];
  }
  CS = ws.take<double>(c.m * totR);
  spec = ws.take<double>(2 * c.m * totR);
  tw = ws.take<double>(2 * c.m);
  Z = ws.take<double>(c.m * c.r);
  W = ws.take<double>(c.r * c.Rn);
  P = ws.take<double>(c.m * c.Rn);
  if (!run) return TSK_OK;
  RArr ra{};
  for (int k = 0; k < c.N; ++k) ra.R[k] = c.R[k];
  TSK_TRY(ts_lhs_spectra(modes, c.N - 1, c.m, CS, spec, tw, ws, st));
  TSK_TRY(ts_compose(modes, c.N - 1, c.m, spec, tw, TSK_PREC_F64, Z, st));
  hipLaunchKernelGGL(k_core_to_w, dim3(ceil_div(c.csize, 256)), dim3(256), 0, st, core, c.N, c.n,
                     ra, c.csize, W);
  TSK_LAUNCHED();
  TSK_TRY(gemm_small(c.m, c.Rn, c.r, 1.0, Z, c.r, 1, W, c.Rn, 1, 0.0, P, c.Rn, st));
  return TSK_OK;
}

tsk_status make_ctx(int32_t order, const int64_t* dims, const int32_t* ranks, int32_t n,
                    int64_t m, AdjCtx& c) {
  TSK_REQUIRE(order >= 2 && order <= TSK_MAX_ORDER && dims && ranks, "invalid arguments");
  TSK_REQUIRE(n >= 0 && n < order && m >= 1, "invalid mode or sketch size");
  c.N = order;
  c.n = n;
  c.m = m;
  c.r = 1;
  c.csize = 1;
  for (int k = 0; k < order; ++k) {
    TSK_REQUIRE(dims[k] >= 1 && ranks[k] >= 1, "invalid dims/ranks");
    c.dims[k] = dims[k];
    c.R[k] = ranks[k];
    c.csize *= ranks[k];
    if (k != n) c.r *= ranks[k];
  }
  c.s = dims[n];
  c.Rn = ranks[n];
  TSK_REQUIRE(c.Rn <= kMaxR, "rank R_n = %lld above the adjoint's limit %d", (long long)c.Rn,
              kMaxR);
  return TSK_OK;
}

}  // namespace
}  // namespace tsk

using namespace tsk;

extern "C" {

tsk_status tsk_sketched_residual_fwd(int32_t order, const int64_t* dims, const int32_t* ranks,
                                     int32_t n, int64_t m, const int32_t* const* h,
                                     const int8_t* const* sign, const double* const* factors,
                                     const double* core, const void* Y, int32_t ydtype,
                                     double* L, void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  AdjCtx c{};
  TSK_TRY(make_ctx(order, dims, ranks, n, m, c));
  TSK_REQUIRE(h && sign && factors && core && Y && L, "invalid arguments");
  TSK_REQUIRE(ydtype == TSK_F32 || ydtype == TSK_F64, "unknown Y dtype");
  return with_workspace(ws, ws_bytes, [&](Ws& w) -> tsk_status {
    hipStream_t st = as_stream(stream);
    LhsMode modes[TSK_MAX_ORDER];
    double *Z, *W, *P, *CS, *spec, *tw;
    TSK_TRY(adj_common(c, h, sign, factors, core, modes, Z, W, P, CS, spec, tw, w, st));
    double* part = w.take<double>(c.m);
    if (w.measuring()) return TSK_OK;
    hipLaunchKernelGGL(k_res_rows, dim3(c.m), dim3(kT), 0, st, P, factors[n], c.Rn, Y, ydtype,
                       c.s, part);
    TSK_LAUNCHED();
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, st, part, c.m, L);
    TSK_LAUNCHED();
    return TSK_OK;
  });
}

tsk_status tsk_sketched_residual_bwd(int32_t order, const int64_t* dims, const int32_t* ranks,
                                     int32_t n, int64_t m, const int32_t* const* h,
                                     const int8_t* const* sign, const double* const* factors,
                                     const double* core, const void* Y, int32_t ydtype,
                                     double* const* grads, double* grad_core, void* ws,
                                     size_t* ws_bytes, void* stream) {
  clear_error();
  AdjCtx c{};
  TSK_TRY(make_ctx(order, dims, ranks, n, m, c));
  TSK_REQUIRE(h && sign && factors && core && Y && grads && grad_core, "invalid arguments");
  TSK_REQUIRE(ydtype == TSK_F32 || ydtype == TSK_F64, "unknown Y dtype");
  for (int k = 0; k < order; ++k) TSK_REQUIRE(grads[k], "grads[%d] is NULL", k);
  return with_workspace(ws, ws_bytes, [&](Ws& w) -> tsk_status {
    hipStream_t st = as_stream(stream);
    LhsMode modes[TSK_MAX_ORDER];
    double *Z, *W, *P, *CS, *spec, *tw;
    TSK_TRY(adj_common(c, h, sign, factors, core, modes, Z, W, P, CS, spec, tw, w, st));
    int64_t totR = 0;
    for (int q = 0; q < c.N - 1; ++q) totR += modes[q].R;
    double* EA = w.take<double>(c.m * c.Rn);
    double* gW = w.take<double>(c.r * c.Rn);
    double* gZ = w.take<double>(c.m * c.r);
    double* gspec = w.take<double>(2 * c.m * c.r);
    double* gCS = w.take<double>(c.m * totR);
    if (w.measuring())  // size the Gram launch's split-K scratch
      return gemm_tn(TSK_PREC_F64, c.r, c.Rn, c.m, Z, c.r, c.r, nullptr, 0, EA, c.Rn, gW, c.Rn,
                     w, st);
    hipLaunchKernelGGL(k_EA, dim3(c.m), dim3(kT), 0, st, P, factors[n], c.Rn, Y, ydtype, c.s, EA);
    TSK_LAUNCHED();
    hipLaunchKernelGGL(k_EtP, dim3(ceil_div(c.s, kT)), dim3(kT), 0, st, P, factors[n], c.Rn, Y,
                       ydtype, c.s, c.m, grads[n]);
    TSK_LAUNCHED();
    TSK_TRY(gemm_tn(TSK_PREC_F64, c.r, c.Rn, c.m, Z, c.r, c.r, nullptr, 0, EA, c.Rn, gW, c.Rn, w,
                    st));
    // dL/dW = 2 Z^T EA;  dL/dZ = 2 EA W^T
    RArr ra{};
    for (int k = 0; k < c.N; ++k) ra.R[k] = c.R[k];
    hipLaunchKernelGGL(k_w_to_core, dim3(ceil_div(c.csize, 256)), dim3(256), 0, st, gW, c.N, c.n,
                       ra, c.csize, 2.0, grad_core);
    TSK_LAUNCHED();
    TSK_TRY(gemm_small(c.m, c.r, c.Rn, 2.0, EA, c.Rn, 1, W, 1, c.Rn, 0.0, gZ, c.r, st));
    TSK_TRY(fft_columns(gZ, c.m, c.r, tw, gspec, st));
    TSK_TRY(ts_conv_adjoint(modes, c.N - 1, c.m, spec, gspec, tw, gCS, st));
    double* g = gCS;
    int q = 0;
    for (int k = 0; k < c.N; ++k) {
      if (k == c.n) continue;
      const LhsMode& md = modes[q++];
      hipLaunchKernelGGL(k_cs_adjoint, dim3(ceil_div(md.s * md.R, 256)), dim3(256), 0, st, g,
                         md.R, h[k], sign[k], md.s, grads[k]);
      TSK_LAUNCHED();
      g += c.m * md.R;
    }
    return TSK_OK;
  });
}

}  // extern "C"
