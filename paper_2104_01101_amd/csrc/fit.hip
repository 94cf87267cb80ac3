// Relative residual ||T - T~||_F / ||T||_F of a Tucker model (1 - fitness,
// Sec. 7), in FP64.  Dense tensors: sum of (T - T~)^2 over all entries, T~
// from the mode products of the core with every factor but the first and one
// R_1-term product per entry.  COO
// tensors (T~ is dense, T is not): ||T||^2 - 2 <T, T~> + ||T~||^2, whose
// cancellation limits the relative residual to ~1e-8 near an exact fit:
//   <T, T~>  per stored entry, T~(i) = sum_rho C(rho) prod_k A^(k)(i_k, rho_k)
//   ||T~||^2 = <C x_1 G_1 ... x_N G_N, C>, G_k = A^(k)T A^(k)
// Reductions are two-level with a fixed order (deterministic).
// Order-3 COO tensors of equal ranks 16 take <T, T~> in another order: with
// the entries grouped by their last index k (a stable sort, once per plan),
//   T~(i, j, k) = sum_{x,y} A^(1)(i, x) A^(2)(j, y) W_k(x, y),
//   W_k = sum_z C(:, :, z) A^(3)(k, z),
// R^2 multiply-adds per entry (on the FP64 matrix cores) instead of
// R^3 + R^2 + R, W_k being the same for a whole run of entries.

#include <rocprim/device/device_radix_sort.hpp>

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

// ---- <T, T~> over entries grouped by their last index ----
// the payload that travels with the sort key i_3
template <class V>
struct Ent {
  int32_t i0, i1;
  V v;
};

template <class V>
__global__ __launch_bounds__(kT) void k_last_keys(const int32_t* __restrict__ i0,
                                                  const int32_t* __restrict__ i1,
                                                  const int32_t* __restrict__ i2,
                                                  const V* __restrict__ v, int64_t nnz,
                                                  uint32_t* keys, Ent<V>* ents) {
  for (int64_t e = int64_t(blockIdx.x) * kT + threadIdx.x; e < nnz;
       e += int64_t(gridDim.x) * kT) {
    keys[e] = uint32_t(i2[e]);
    ents[e] = Ent<V>{i0[e], i1[e], v[e]};
  }
}

// Wt[k][y][x] = sum_z C[x][y][z] A3[k][z] (W_k transposed): one thread per
// (y, x) with its row of C in registers, kCoreK values of k per workgroup
// (A3 rows wave-uniform)
constexpr int kCoreK = 16;

template <int RR>
__global__ __launch_bounds__(RR * RR) void k_core_last(const double* __restrict__ C,
                                                       const double* __restrict__ A3, int64_t s3,
                                                       double* Wt) {
  const int t = threadIdx.x, y = t / RR, x = t - y * RR;
  double c[RR];
#pragma unroll
  for (int z = 0; z < RR; ++z) c[z] = C[(x * RR + y) * RR + z];
  const int64_t k0 = int64_t(blockIdx.x) * kCoreK;
  for (int64_t k = k0; k < k0 + kCoreK && k < s3; ++k) {
    const double* a = A3 + k * RR;
    double acc = 0.0;
#pragma unroll
    for (int z = 0; z < RR; ++z) acc = fma(c[z], a[z], acc);
    Wt[k * (RR * RR) + t] = acc;
  }
}

// <T, T~> over the sorted entries, 64 per wave at a time, on
// v_mfma_f64_16x16x4 (lane l = li + 16 g feeds A(li, g) and B(g, li) and holds
// D(g + 4 v, li)).  For each of the four 16-entry tiles m of the group,
// D_m = U0_m W_k (entries x y) over four steps s, with A(li, g) = u0(x = 4 g + s)
// of entry 16 m + li and B(g, li) = W_k(4 g + s, li); then every lane adds
// D(e, y) v_e u1_e(y) for its four entries e = 16 m + g + 4 v and its y = li.
// The group's distinct k (runs of equal k are contiguous) are taken in turn,
// each with its own W_k and only its entries kept (a ballot mask).
template <class V>
__global__ __launch_bounds__(kT) void k_inner3s(const uint32_t* __restrict__ ks,
                                                const Ent<V>* __restrict__ ents,
                                                const double* __restrict__ A0,
                                                const double* __restrict__ A1,
                                                const double* __restrict__ Wt, int64_t nnz,
                                                int64_t per_block, double* partial) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  __shared__ double red[kT / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t lo = int64_t(blockIdx.x) * per_block;
  const int64_t hi = lo + per_block < nnz ? lo + per_block : nnz;
  double acc = 0.0;
  for (int64_t g0 = lo + wave * 64; g0 < hi; g0 += kT) {
    const int64_t e = g0 + lane;
    const bool valid = e < hi;
    const int64_t ec = valid ? e : hi - 1;
    const uint32_t k = ks[ec];
    const Ent<V> en = ents[ec];
    // A operands: u0 of entry 16 m + li, x = 4 g .. 4 g + 3
    double a[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const int64_t r0 = __shfl(en.i0, 16 * m + li);
#pragma unroll
      for (int s = 0; s < 4; ++s) a[m][s] = A0[r0 * 16 + 4 * g + s];
    }
    // v_e u1_e(li) of the entries e = 16 m + g + 4 v whose D rows this lane holds
    double w[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int src = 16 * m + g + 4 * v;
        const int64_t r1 = __shfl(en.i1, src);
        const double val = double(__shfl(en.v, src));
        w[m][v] = val * A1[r1 * 16 + li];
      }
    uint64_t pend = __ballot(valid);
    while (pend) {
      const int first = __ffsll((unsigned long long)pend) - 1;
      const uint32_t kk = uint32_t(__builtin_amdgcn_readlane(int(k), first));
      const uint64_t sel = __ballot(valid && k == kk);
      const double* wk = Wt + size_t(kk) * 256 + li * 16 + 4 * g;
      double b[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) b[s] = wk[s];
      d4 d[4];
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        d[m] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < 4; ++s)
          d[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[m][s], b[s], d[m], 0, 0, 0);
      }
#pragma unroll
      for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const bool mine = (sel >> (16 * m + g + 4 * v)) & 1ull;
          acc = fma(mine ? d[m][v] : 0.0, w[m][v], acc);
        }
      pend &= ~sel;
    }
  }
  acc = block_reduce(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
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
  int b = b0;
  for (; b + 8 <= b1; b += 8) {  // eight loads in flight, summed in index order
    double t[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) t[u] = p[b + u];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += t[u];
  }
  for (; b < b1; ++b) s += p[b];
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
    // rows eight at a time with their loads in flight together; the sums
    // still run over i in order
    int64_t i = 0;
    for (; i + 8 <= s1; i += 8) {
      double v8[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v8[u] = double(X[(i + u) * J + j]);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double* ar = A1 + (i + u) * R1;
        double t = 0.0;
#pragma unroll
        for (int a = 0; a < RM; ++a)
          if (a < R1) t = fma(ar[a], m[a], t);
        const double d = v8[u] - t;
        acc = fma(d, d, acc);
        nrm = fma(v8[u], v8[u], nrm);
      }
    }
    for (; i < s1; ++i) {
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
// model norm ping-ponging between two LDS buffers of csize doubles, read from
// a third holding the core; the factor Grams are staged in LDS too when they
// take at most kGramLds doubles (gl = their total, else 0).  The staging
// keeps eight loads in flight per thread.
constexpr int kGramLds = 2048;

// dst[t] = src[t], t < n, by the workgroup with eight loads in flight per thread
__device__ inline void stage8(const double* __restrict__ src, double* dst, int n) {
  for (int t0 = threadIdx.x; t0 < n; t0 += 8 * kT) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = t0 + u * kT < n ? src[t0 + u * kT] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (t0 + u * kT < n) dst[t0 + u * kT] = v[u];
  }
}

__global__ __launch_bounds__(kT) void k_finish_model(FitArgs a, const double* core, int64_t csize,
                                                     const double* grams, int gl,
                                                     const double* pn, int nbn, const double* pi,
                                                     int nbi, const double* pd, int dense,
                                                     double* nT2_out, double* res_out) {
  extern __shared__ double lbuf[];  // 3 csize + gl
  __shared__ double red[kT / 64];
  const int cs = int(csize);
  double* core_s = lbuf + 2 * cs;
  double* gl_s = lbuf + 3 * cs;
  stage8(core, core_s, cs);
  stage8(grams, gl_s, gl);
  __syncthreads();
  const double* in = core_s;
  int goff = 0;
  for (int k = 0; k < a.N; ++k) {
    const int Rk = int(a.R[k]);
    int inner = 1;
    for (int l = k + 1; l < a.N; ++l) inner *= int(a.R[l]);
    const double* G = (gl ? gl_s : grams) + goff;
    double* o = lbuf + (k & 1) * cs;
    for (int t = threadIdx.x; t < cs; t += kT) {
      const int rk = (t / inner) % Rk, base = t - rk * inner;
      double s = 0.0;
      for (int c = 0; c < Rk; ++c) s += G[rk * Rk + c] * in[base + c * inner];
      o[t] = s;
    }
    __syncthreads();
    in = o;
    goff += Rk * Rk;
  }
  double m2 = 0.0;
  for (int t = threadIdx.x; t < cs; t += kT) m2 += in[t] * core_s[t];
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

// stable radix sort of the entries by i_3 (the temporary size when tmp is NULL)
template <class V>
tsk_status sort_entries(void* tmp, size_t& bytes, const FitScratch& fs, size_t n,
                        hipStream_t st) {
  TSK_HIP(rocprim::radix_sort_pairs(tmp, bytes, fs.keys_in, fs.keys,
                                    static_cast<const Ent<V>*>(fs.ents_in),
                                    static_cast<Ent<V>*>(fs.ents), n, 0u, fs.key_bits, st));
  return TSK_OK;
}

// The grouped order pays where R^3 per entry outweighs the sort: rank 16,
// at least 2^16 entries, indices of the last mode below 2^31.
static bool fit_by_last(const TensorView& T, const int64_t* R) {
  return T.layout == TSK_COO && T.order == 3 && R[0] == 16 && R[1] == 16 && R[2] == 16 &&
         T.nnz >= (int64_t(1) << 16) && T.nnz < (int64_t(1) << 32) &&
         T.dims[2] <= (int64_t(1) << 31);
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
  fs.gram_part = ws.take<double>(size_t(gram_batch_splits(T.order, T.dims)) * gsz);
  fs.buf0 = ws.take<double>(csize);
  fs.buf1 = ws.take<double>(csize);
  fs.model2 = ws.take<double>(1);
  fs.nT2 = ws.take<double>(1);
  fs.ttm[0] = fs.ttm[1] = nullptr;
  fs.by_last = fit_by_last(T, R);
  fs.sorted = false;
  if (fs.by_last) {
    const size_t n = size_t(T.nnz);
    const bool f64 = T.dtype == TSK_F64;
    const size_t eb = f64 ? sizeof(Ent<double>) : sizeof(Ent<float>);
    fs.keys_in = ws.take<uint32_t>(n);
    fs.keys = ws.take<uint32_t>(n);
    fs.ents_in = ws.take<char>(n * eb);
    fs.ents = ws.take<char>(n * eb);
    fs.W = ws.take<double>(size_t(T.dims[2]) * R[0] * R[1]);
    fs.key_bits = 1;
    while (fs.key_bits < 32 && (int64_t(1) << fs.key_bits) < T.dims[2]) ++fs.key_bits;
    fs.sort_bytes = 0;
    if (f64)
      TSK_TRY(sort_entries<double>(nullptr, fs.sort_bytes, fs, n, hipStream_t(nullptr)));
    else
      TSK_TRY(sort_entries<float>(nullptr, fs.sort_bytes, fs, n, hipStream_t(nullptr)));
    fs.sort_tmp = ws.take<char>(fs.sort_bytes);
  }
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

tsk_status fit_presort(const TensorView& T, FitScratch& fs, hipStream_t st) {
  if (!fs.by_last || fs.sorted) return TSK_OK;
  // the entries grouped by their last index, stably (input order within a run)
  ProfScope prof("fit_sort", st);
  const int64_t n = T.nnz;
  const unsigned grid = unsigned(std::min<int64_t>(ceil_div(n, kT), 8192));
  size_t bytes = fs.sort_bytes;
  if (T.dtype == TSK_F64) {
    hipLaunchKernelGGL(k_last_keys<double>, dim3(grid), dim3(kT), 0, st, T.idx[0], T.idx[1],
                       T.idx[2], static_cast<const double*>(T.values), n, fs.keys_in,
                       static_cast<Ent<double>*>(fs.ents_in));
    TSK_LAUNCHED();
    TSK_TRY(sort_entries<double>(fs.sort_tmp, bytes, fs, size_t(n), st));
  } else {
    hipLaunchKernelGGL(k_last_keys<float>, dim3(grid), dim3(kT), 0, st, T.idx[0], T.idx[1],
                       T.idx[2], static_cast<const float*>(T.values), n, fs.keys_in,
                       static_cast<Ent<float>*>(fs.ents_in));
    TSK_LAUNCHED();
    TSK_TRY(sort_entries<float>(fs.sort_tmp, bytes, fs, size_t(n), st));
  }
  fs.sorted = true;
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
  const int gl = goff <= kGramLds ? int(goff) : 0;  // Grams staged in LDS
  if (rmax_g > 64)
    for (int k = 0; k < T.order; ++k)
      TSK_TRY(gemm_tn(TSK_PREC_F64, R[k], R[k], T.dims[k], factors[k], R[k], R[k], nullptr, 0,
                      factors[k], R[k], gp[k], R[k], ws, st));
  if (ws.measuring()) return TSK_OK;
  if (fs.by_last && !fs.sorted) TSK_TRY(fit_presort(T, fs, st));
  ProfScope prof("fit", st);
  if (rmax_g <= 64)  // the factor Grams of every mode in one launch
    TSK_TRY(gram_batch_f64(T.order, R, T.dims, factors, gp, fs.gram_part, st));
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
      hipLaunchKernelGGL(k_finish_model, dim3(1), dim3(kT), size_t(3 * csize + gl) * 8, st, a,
                         core, csize, fs.grams, gl, fs.partial_norm, fs.nblocks,
                         fs.partial_inner, fs.nblocks, fs.partial_direct, 1, fs.nT2, res);
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
  if (fs.by_last) {
    const int64_t s3 = T.dims[2];
    hipLaunchKernelGGL(k_core_last<16>, dim3(unsigned(ceil_div(s3, kCoreK))), dim3(256), 0, st,
                       core, factors[2], s3, fs.W);
    TSK_LAUNCHED();
    if (T.dtype == TSK_F64)
      hipLaunchKernelGGL(k_inner3s<double>, dim3(fs.nblocks), dim3(kT), 0, st, fs.keys,
                         static_cast<const Ent<double>*>(fs.ents), factors[0], factors[1], fs.W,
                         T.nnz, per, fs.partial_inner);
    else
      hipLaunchKernelGGL(k_inner3s<float>, dim3(fs.nblocks), dim3(kT), 0, st, fs.keys,
                         static_cast<const Ent<float>*>(fs.ents), factors[0], factors[1], fs.W,
                         T.nnz, per, fs.partial_inner);
  } else if (T.order == 3 && rmax <= 32) {
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
    hipLaunchKernelGGL(k_finish_model, dim3(1), dim3(kT), size_t(3 * csize + gl) * 8, st, a,
                       core, csize, fs.grams, gl, with_norm ? fs.partial_norm : nullptr,
                       fs.nblocks, fs.partial_inner, fs.nblocks, fs.partial_direct,
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
