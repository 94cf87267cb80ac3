// Sketched mode-n residual L = ||Z W A^T - Y||_F^2 and its adjoint, with
// Z = S^(n) kron_{k != n} A^(k) (TensorSketch, Sec. 3.1), W = C_(n)^T, A = A^(n)
// and Y = S^(n) T_(n)^T -- the objective of the sketched subproblem of Alg. 4.
//
// E = Z W A^T - Y is never stored: every pass over Y recomputes its entries
// from P = Z W (m x R) and A.
//   forward   L = sum E^2                                   (one pass over Y)
//   backward  EA = E A (m x R), E^T P (s x R)               (one pass over Y)
//             dL/dA  = 2 E^T P,  dL/dW = 2 Z^T (E A) -> dL/dC
//             dL/dZ  = 2 (E A) W^T
//             dL/dCS_k[:, c] = IFFT(sum_{rho_k = c} conj(prod_{l != k} F_l) FFT(dL/dZ[:, rho]))
//             dL/dA^(k)[i, :] = sigma_k(i) dL/dCS_k[h_k(i), :]
// All FP64; reductions in a fixed order (deterministic).

#include <algorithm>

#include "common.h"
#include "kernels.h"

namespace tsk {

namespace {

constexpr int kT = 256;
constexpr int kMaxR = 64;  // largest R_n (the tile pass pads R to 16, 32, 48 or 64)

__device__ double block_sum(double v, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kT / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// One pass over Y for a tile of rows j x columns i, on the FP64 matrix cores
// (16x16x4).  A wave owns RB blocks of 16 rows; the workgroup (4 waves)
// walks a range of 16-column tiles.  Per tile and row block:
//   E     = P A^T - Y            (lane (li, g) holds E[g + 4v][li])
//   L    += sum E^2
//   EtP^T += P^T E               (E is already the B operand: k = rows)
//   EA    += E A                 (E transposed through the wave's LDS tile)
// EtP is summed over the workgroup's waves in LDS (fixed order) and written
// per row block of the grid; EA is written per column range of the grid.
// The next tile's Y and A are loaded into registers during the products.
typedef double dx4 __attribute__((ext_vector_type(4)));

template <int RT>
struct AdjTile {
  static constexpr int NC = RT / 16;  // 16-column blocks of R
  static constexpr int KS = RT / 4;   // k-steps over R
  static constexpr int RB = RT <= 16 ? 4 : RT <= 32 ? 2 : 1;  // row blocks per wave
  static constexpr int RW = 64 * RB;  // rows per workgroup
  static constexpr int AU = 16 * RT / kT;  // A-tile values per thread
};

struct AdjArgs {
  const double* P;  // m x R
  const double* A;  // s x R
  const void* Y;    // m x s
  int64_t m, s, cw; // cw: columns per workgroup (multiple of 16)
  int R;
  double* partL;    // [blocks]
  double* partEA;   // [gridDim.y][m][R]
  double* partEtP;  // [gridDim.x][s][R]
};

template <int RT, bool BWD, class YT>
__global__ __launch_bounds__(kT) void k_adj_tiles(AdjArgs a) {
  typedef AdjTile<RT> S;
  constexpr int NC = S::NC, KS = S::KS, RB = S::RB, RW = S::RW, AU = S::AU, LA = RT + 1;
  __shared__ double sA[16 * LA];            // A[i0 + ii][c]
  __shared__ double sT[BWD ? 4 * 16 * 17 : 1];       // per-wave transpose of E
  __shared__ double sR[BWD ? 4 * 16 * RT : 1];       // per-wave EtP tiles [i][c]
  __shared__ double red[kT / 64];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, li = lane & 15, g = lane >> 4;
  const int64_t jw = int64_t(blockIdx.x) * RW + int64_t(wave) * 16 * RB;
  const int64_t ib = int64_t(blockIdx.y) * a.cw;
  const int64_t ie = ib + a.cw < a.s ? ib + a.cw : a.s;
  const YT* Y = static_cast<const YT*>(a.Y);
  const int R = a.R;

  double pa[RB][KS];  // P[jw + 16 b + li][4 k + g]
#pragma unroll
  for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int64_t j = jw + 16 * b + li;
      const int c = 4 * k + g;
      pa[b][k] = (j < a.m && c < R) ? a.P[j * R + c] : 0.0;
    }
  double pb[BWD ? RB : 1][NC][4];  // P[jw + 16 b + 4 v + g][16 c + li]
  dx4 ea[BWD ? RB : 1][NC];
  if constexpr (BWD) {
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        ea[b][c] = dx4{0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = jw + 16 * b + 4 * v + g;
          const int cc = 16 * c + li;
          pb[b][c][v] = (j < a.m && cc < R) ? a.P[j * R + cc] : 0.0;
        }
      }
  }

  // prefetch registers: Y rows g + 4 v of each row block at column li, and
  // this thread's share of the A tile; loads at clamped indices, out-of-range
  // values zeroed at use
  YT yv[RB][4];
  double av[AU];
  auto fetch = [&](int64_t i0) {
    const int64_t i = min(i0 + li, a.s - 1);
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t j = min(jw + 16 * b + g + 4 * v, a.m - 1);
        yv[b][v] = Y[j * a.s + i];
      }
#pragma unroll
    for (int u = 0; u < AU; ++u) {
      const int t = tid + kT * u, ii = t / RT, c = t % RT;
      av[u] = a.A[min(i0 + ii, a.s - 1) * R + min(c, R - 1)];
    }
  };

  double lsum = 0.0;
  if (ib < ie) fetch(ib);
  for (int64_t i0 = ib; i0 < ie; i0 += 16) {
    __syncthreads();  // the previous tile's readers of sA and sR are done
#pragma unroll
    for (int u = 0; u < AU; ++u) {
      const int t = tid + kT * u, ii = t / RT, c = t % RT;
      sA[ii * LA + c] = (i0 + ii < ie && c < R) ? av[u] : 0.0;
    }
    double ycur[RB][4];
    const bool iv = i0 + li < ie;
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        ycur[b][v] = (iv && jw + 16 * b + g + 4 * v < a.m) ? double(yv[b][v]) : 0.0;
    __syncthreads();
    if (i0 + 16 < ie) fetch(i0 + 16);  // in flight during the products

    double ae[KS];  // A[i0 + li][4 k + g]
#pragma unroll
    for (int k = 0; k < KS; ++k) ae[k] = sA[li * LA + 4 * k + g];
    double aa[BWD ? NC : 1][4];  // A[i0 + 4 v + g][16 c + li]
    dx4 etp[BWD ? NC : 1];
    if constexpr (BWD) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        etp[c] = dx4{0, 0, 0, 0};
#pragma unroll
        for (int v = 0; v < 4; ++v) aa[c][v] = sA[(4 * v + g) * LA + 16 * c + li];
      }
    }
#pragma unroll
    for (int b = 0; b < RB; ++b) {
      dx4 e = {-ycur[b][0], -ycur[b][1], -ycur[b][2], -ycur[b][3]};
#pragma unroll
      for (int k = 0; k < KS; ++k) e = __builtin_amdgcn_mfma_f64_16x16x4f64(pa[b][k], ae[k], e, 0, 0, 0);
      lsum += e[0] * e[0] + e[1] * e[1] + e[2] * e[2] + e[3] * e[3];
      if constexpr (BWD) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            etp[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(pb[b][c][v], e[v], etp[c], 0, 0, 0);
        double* T = sT + wave * 16 * 17;
#pragma unroll
        for (int v = 0; v < 4; ++v) T[(g + 4 * v) * 17 + li] = e[v];
        __builtin_amdgcn_wave_barrier();
        double et[4];  // E[li][4 v + g]
#pragma unroll
        for (int v = 0; v < 4; ++v) et[v] = T[li * 17 + 4 * v + g];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            ea[b][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(et[v], aa[c][v], ea[b][c], 0, 0, 0);
      }
    }
    if constexpr (BWD) {
      // etp[c] lane (li, g): EtP[i0 + li][16 c + g + 4 v]
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) sR[wave * 16 * RT + li * RT + 16 * c + g + 4 * v] = etp[c][v];
      __syncthreads();
      double* out = a.partEtP + int64_t(blockIdx.x) * a.s * R;
      for (int t = tid; t < 16 * RT; t += kT) {
        const int ii = t / RT, c = t % RT;
        const double v = ((sR[t] + sR[16 * RT + t]) + sR[2 * 16 * RT + t]) + sR[3 * 16 * RT + t];
        if (i0 + ii < ie && c < R) out[(i0 + ii) * R + c] = v;
      }
    }
  }
  lsum = block_sum(lsum, red);
  if (tid == 0) a.partL[int64_t(blockIdx.x) * gridDim.y + blockIdx.y] = lsum;
  if constexpr (BWD) {
    // ea[b][c] lane (li, g): EA[jw + 16 b + g + 4 v][16 c + li]
    double* out = a.partEA + int64_t(blockIdx.y) * a.m * R;
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t j = jw + 16 * b + g + 4 * v;
          const int cc = 16 * c + li;
          if (j < a.m && cc < R) out[j * R + cc] = ea[b][c][v];
        }
  }
}

__global__ void k_sum(const double* x, int64_t n, double* out) {
  __shared__ double red[kT / 64];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kT) acc += x[i];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) *out = acc;
}

// out[t] = scale * sum_p part[p n + t], p in order
__global__ void k_sum_parts(const double* part, int nparts, int64_t n, double scale, double* out) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double v = 0.0;
  for (int p = 0; p < nparts; ++p) v += part[int64_t(p) * n + t];
  out[t] = scale * v;
}

// Grid of the tile pass and its partial buffers.
struct AdjPlan {
  int rt;
  int64_t rows_per_block, nrb, ncb, cw;
  double *partL, *partEA, *partEtP;
};

AdjPlan adj_plan(int64_t m, int64_t s, int64_t R, bool bwd, Ws& ws) {
  AdjPlan p{};
  p.rt = int(ceil_div(R, 16) * 16);
  p.rows_per_block = 64 * (p.rt <= 16 ? 4 : p.rt <= 32 ? 2 : 1);
  p.nrb = ceil_div(m, p.rows_per_block);
  // about 512 workgroups, each with at least 4 column tiles
  int64_t ncb = std::max<int64_t>(1, 512 / p.nrb);
  ncb = std::min<int64_t>(ncb, std::max<int64_t>(1, ceil_div(s, 64)));
  p.cw = ceil_div(ceil_div(s, ncb), 16) * 16;
  p.ncb = ceil_div(s, p.cw);
  p.partL = ws.take<double>(size_t(p.nrb * p.ncb));
  p.partEA = bwd ? ws.take<double>(size_t(p.ncb * m * R)) : nullptr;
  p.partEtP = bwd ? ws.take<double>(size_t(p.nrb * s * R)) : nullptr;
  return p;
}

template <int RT, bool BWD>
void launch_adj_t(const AdjPlan& p, const AdjArgs& a, int ydt, hipStream_t st) {
  const dim3 grid{unsigned(p.nrb), unsigned(p.ncb), 1u};
  if (ydt == TSK_F64)
    hipLaunchKernelGGL((k_adj_tiles<RT, BWD, double>), grid, dim3(kT), 0, st, a);
  else
    hipLaunchKernelGGL((k_adj_tiles<RT, BWD, float>), grid, dim3(kT), 0, st, a);
}

template <bool BWD>
tsk_status launch_adj(const AdjPlan& p, const double* P, const double* A, int64_t R,
                      const void* Y, int ydt, int64_t m, int64_t s, hipStream_t st) {
  AdjArgs a{P, A, Y, m, s, p.cw, int(R), p.partL, p.partEA, p.partEtP};
  switch (p.rt) {
    case 16: launch_adj_t<16, BWD>(p, a, ydt, st); break;
    case 32: launch_adj_t<32, BWD>(p, a, ydt, st); break;
    case 48: launch_adj_t<48, BWD>(p, a, ydt, st); break;
    default: launch_adj_t<64, BWD>(p, a, ydt, st); break;
  }
  TSK_LAUNCHED();
  return TSK_OK;
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
    const AdjPlan p = adj_plan(c.m, c.s, c.Rn, false, w);
    if (w.measuring()) return TSK_OK;
    {
      ProfScope prof("adjoint_pass", st);
      TSK_TRY(launch_adj<false>(p, P, factors[n], c.Rn, Y, ydtype, c.m, c.s, st));
    }
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kT), 0, st, p.partL, p.nrb * p.ncb, L);
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
    const AdjPlan p = adj_plan(c.m, c.s, c.Rn, true, w);
    if (w.measuring())  // size the Gram launch's split-K scratch
      return gemm_tn(TSK_PREC_F64, c.r, c.Rn, c.m, Z, c.r, c.r, nullptr, 0, EA, c.Rn, gW, c.Rn,
                     w, st);
    // one pass over Y: EA = E A and dL/dA^(n) = 2 E^T P
    {
      ProfScope prof("adjoint_pass", st);
      TSK_TRY(launch_adj<true>(p, P, factors[n], c.Rn, Y, ydtype, c.m, c.s, st));
    }
    hipLaunchKernelGGL(k_sum_parts, dim3(unsigned(ceil_div(c.m * c.Rn, 256))), dim3(256), 0, st,
                       p.partEA, int(p.ncb), c.m * c.Rn, 1.0, EA);
    TSK_LAUNCHED();
    hipLaunchKernelGGL(k_sum_parts, dim3(unsigned(ceil_div(c.s * c.Rn, 256))), dim3(256), 0, st,
                       p.partEtP, int(p.nrb), c.s * c.Rn, 2.0, grads[n]);
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
