// Range-finder sketch of a dense tensor (Alg. 3 with the composite sketch of
// Sec. 5) as one structured GEMM over the tensor:
//
//   B = T_(n) Omega^T G,   B[i, c] = sum_j T_(n)[i, j] tau(j) G[g(j), c]
//
// where (g, tau) is the CountSketch of the other-mode row-major index j (from
// the counter generator, as in the sparse pass) and G (k2 x k1) is Gaussian.
// The rows tau(j) G[g(j), :] are generated from the hash while the GEMM
// consumes them, so neither W = T_(n) Omega^T nor Omega^T G (K x k1) is ever
// stored, and the tensor is read once per mode with no scatter.  In exact
// arithmetic this is (T_(n) Omega^T) G; only the order of the sums differs.
//
// The tensor is viewed as P x s_n x Q (P, Q the products of the dimensions
// before and after mode n), so j = p Q + q.  A workgroup (4 waves) owns 64
// rows i of B and a range of j; per step of KT = 64 values of j it stages the
// tensor tile (64 x KT) and the generated rows (KT x NP, NP = k1 padded) in
// LDS, both with the contraction index contiguous (the next step's values
// are loaded into registers meanwhile), and accumulates on the
// matrix cores: FP64 16x16x4 (FP64 tensors or operands), FP32 16x16x4, or
// BF16 16x16x32 with FP32 accumulation (BF16 operands: the tensor and G
// rounded to BF16).  Each workgroup writes its partial sums (FP64) for its
// range of j; a second kernel adds the ranges in a fixed order
// (deterministic).

#include "common.h"
#include "kernels.h"

namespace tsk {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int kRT = 256;  // threads
constexpr int kBM = 64;   // rows of B per workgroup (16 per wave)
constexpr int kKT = 64;   // contraction values per step
constexpr int kTU = kBM * kKT / kRT;  // tensor values per thread per step

template <class E>
struct Op;
template <>
struct Op<double> {
  typedef d4 Acc;
  static constexpr int LD = kKT + 1;
  __device__ static double cvt(double v) { return v; }
  __device__ static double cvt(float v) { return double(v); }
};
template <>
struct Op<float> {
  typedef f4 Acc;
  static constexpr int LD = kKT + 1;
  __device__ static float cvt(double v) { return float(v); }
  __device__ static float cvt(float v) { return v; }
};
template <>
struct Op<uint16_t> {
  typedef f4 Acc;
  static constexpr int LD = kKT + 8;  // 16-byte aligned rows of 8 bf16 groups
  __device__ static uint16_t cvt(double v) { return f32_to_bf16_bits(float(v)); }
  __device__ static uint16_t cvt(float v) { return f32_to_bf16_bits(v); }
};

struct RrfDenseArgs {
  const void* X;  // tensor values
  int64_t P, s, Q;
  int64_t K;      // P * Q
  int64_t kchunk; // contraction values per split
  int k1, k2;
  uint64_t key;   // CountSketch stream
  const double* G;  // k2 x k1
  double* part;     // splits x s x k1
};

// The next step's tensor values and generated rows are loaded into registers
// while the current step's products run from LDS (one LDS buffer, two
// barriers per step).
template <class V, class E, int NP>
__global__ __launch_bounds__(kRT) void k_rrf_dense(RrfDenseArgs a) {
  constexpr int LD = Op<E>::LD, NB = NP / 16, GU = NP / 4;
  typedef typename Op<E>::Acc Acc;
  __shared__ __attribute__((aligned(16))) E As[kBM * LD];  // [i][j]
  __shared__ __attribute__((aligned(16))) E Bs[NP * LD];   // [c][j]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t i0 = int64_t(blockIdx.x) * kBM;
  const int64_t jbeg = int64_t(blockIdx.y) * a.kchunk;
  const int64_t jend = jbeg + a.kchunk < a.K ? jbeg + a.kchunk : a.K;
  const V* X = static_cast<const V*>(a.X);
  const bool last_mode = a.Q == 1;
  Acc acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = Acc{0, 0, 0, 0};

  // Raw values are held in registers and converted at the stash, after the
  // products of the current step: a conversion right after a load would wait
  // for it.  Loads use clamped (always valid) indices and the values outside
  // the tile are replaced by zero at the stash, so no load sits in a branch.
  V tv[kTU];
  double gv[GU];
  double gsign = 0.0;  // tau(j), or 0 past the end of the range
  // tensor tile T_(n)[i0 + ii, j0 + jj] = X[(p s + i) Q + q]: for the last
  // mode consecutive i are contiguous (thread: one i, every 4th j), else
  // consecutive j within one p (thread: one j, every 4th i)
  auto fetch = [&](int64_t j0) {
    if (last_mode) {
      const int64_t i = min(i0 + (tid & 63), a.s - 1);
#pragma unroll
      for (int u = 0; u < kTU; ++u) {
        const int64_t j = min(j0 + (tid >> 6) + 4 * u, jend - 1);
        tv[u] = X[j * a.s + i];
      }
    } else {
      const int64_t j = min(j0 + (tid & 63), jend - 1);
      const int64_t p = j / a.Q, q = j - p * a.Q;
      const V* base = X + p * a.s * a.Q + q;
#pragma unroll
      for (int u = 0; u < kTU; ++u) {
        const int64_t i = min(i0 + (tid >> 6) + 4 * u, a.s - 1);
        tv[u] = base[i * a.Q];
      }
    }
    // generated row tau(j) G[g(j), :] of j = j0 + tid / 4: columns tid % 4 + 4 t
    const int64_t j = j0 + (tid >> 2);
    const uint64_t x = draw(a.key, uint64_t(j));
    const double* grow = a.G + int64_t(bucket_of(x, uint64_t(a.k2))) * a.k1;
    gsign = j < jend ? (sign_of(x) < 0 ? -1.0 : 1.0) : 0.0;
#pragma unroll
    for (int t = 0; t < GU; ++t) gv[t] = grow[min((tid & 3) + 4 * t, a.k1 - 1)];
  };
  auto stash = [&](int64_t j0) {
    if (last_mode) {
      const bool iv = i0 + (tid & 63) < a.s;
#pragma unroll
      for (int u = 0; u < kTU; ++u) {
        const bool ok = iv && j0 + (tid >> 6) + 4 * u < jend;
        As[(tid & 63) * LD + (tid >> 6) + 4 * u] = Op<E>::cvt(ok ? tv[u] : V(0));
      }
    } else {
      const bool jv = j0 + (tid & 63) < jend;
#pragma unroll
      for (int u = 0; u < kTU; ++u) {
        const bool ok = jv && i0 + (tid >> 6) + 4 * u < a.s;
        As[((tid >> 6) + 4 * u) * LD + (tid & 63)] = Op<E>::cvt(ok ? tv[u] : V(0));
      }
    }
#pragma unroll
    for (int t = 0; t < GU; ++t) {
      const int c = (tid & 3) + 4 * t;
      Bs[c * LD + (tid >> 2)] = Op<E>::cvt(c < a.k1 ? gsign * gv[t] : 0.0);
    }
  };

  if (jbeg < jend) fetch(jbeg);
  for (int64_t j0 = jbeg; j0 < jend; j0 += kKT) {
    stash(j0);
    __syncthreads();
    if (j0 + kKT < jend) fetch(j0 + kKT);  // in flight during the products
    if constexpr (sizeof(E) == 2) {
#pragma unroll
      for (int ks = 0; ks < kKT; ks += 32) {
        bf8 av, bv;
        __builtin_memcpy(&av, &As[(16 * wave + li) * LD + ks + 8 * g], 16);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          __builtin_memcpy(&bv, &Bs[(16 * b + li) * LD + ks + 8 * g], 16);
          acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[b], 0, 0, 0);
        }
      }
    } else {
#pragma unroll 4
      for (int kk = 0; kk < kKT; kk += 4) {
        const E av = As[(16 * wave + li) * LD + kk + g];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const E bv = Bs[(16 * b + li) * LD + kk + g];
          if constexpr (sizeof(E) == 8)
            acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[b], 0, 0, 0);
          else
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane holds column li of each block; rows g + 4 v (FP64) or 4 g + v (FP32)
  double* out = a.part + int64_t(blockIdx.y) * a.s * a.k1;
#pragma unroll
  for (int b = 0; b < NB; ++b)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + 16 * wave + (sizeof(E) == 8 ? g + 4 * v : 4 * g + v);
      const int c = 16 * b + li;
      if (i < a.s && c < a.k1) out[i * a.k1 + c] = double(acc[b][v]);
    }
}

// B[t] = sum over splits, in order
__global__ void k_rrf_reduce(const double* part, int64_t n, int splits, double* B) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[int64_t(z) * n + t];
  B[t] = s;
}

template <class V, class E>
tsk_status launch_rrf(const RrfDenseArgs& a, dim3 grid, int np, hipStream_t st) {
  if (np <= 32)
    hipLaunchKernelGGL((k_rrf_dense<V, E, 32>), grid, dim3(kRT), 0, st, a);
  else if (np <= 64)
    hipLaunchKernelGGL((k_rrf_dense<V, E, 64>), grid, dim3(kRT), 0, st, a);
  else
    hipLaunchKernelGGL((k_rrf_dense<V, E, 128>), grid, dim3(kRT), 0, st, a);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace

bool rrf_dense_supported(const TensorView& T, int64_t k1) {
  return T.layout == TSK_DENSE && k1 >= 1 && k1 <= 128;
}

tsk_status rrf_dense(const TensorView& T, int n, int64_t k1, int64_t k2, uint64_t key,
                     const double* G, int prec, double* B, Ws& ws, hipStream_t st) {
  if (!rrf_dense_supported(T, k1)) {
    set_error("dense range-finder pass: needs a dense tensor and k1 <= 128 (k1 = %lld)",
              (long long)k1);
    return TSK_EUNSUPPORTED;
  }
  RrfDenseArgs a{};
  a.X = T.values;
  a.s = T.dims[n];
  a.P = 1;
  a.Q = 1;
  for (int k = 0; k < n; ++k) a.P *= T.dims[k];
  for (int k = n + 1; k < T.order; ++k) a.Q *= T.dims[k];
  a.K = a.P * a.Q;
  a.k1 = int(k1);
  a.k2 = int(k2);
  a.key = key;
  a.G = G;
  const int64_t mblocks = ceil_div(a.s, kBM);
  // about 1024 workgroups, each with at least 16 steps of the contraction
  int64_t splits = ceil_div(1024, mblocks);
  splits = std::max<int64_t>(1, std::min<int64_t>(splits, ceil_div(a.K, 16 * kKT)));
  a.kchunk = ceil_div(ceil_div(a.K, splits), kKT) * kKT;
  splits = ceil_div(a.K, a.kchunk);
  a.part = ws.take<double>(size_t(splits) * a.s * k1);
  if (ws.measuring() || a.K == 0) return TSK_OK;
  const dim3 grid{unsigned(mblocks), unsigned(splits), 1u};
  const int np = int(ceil_div(k1, 16) * 16);
  if (T.dtype == TSK_F64 || prec == TSK_PREC_F64) {
    if (T.dtype == TSK_F64)
      TSK_TRY((launch_rrf<double, double>(a, grid, np, st)));
    else
      TSK_TRY((launch_rrf<float, double>(a, grid, np, st)));
  } else if (prec == TSK_PREC_BF16) {
    TSK_TRY((launch_rrf<float, uint16_t>(a, grid, np, st)));
  } else {
    TSK_TRY((launch_rrf<float, float>(a, grid, np, st)));
  }
  const int64_t nb = a.s * k1;
  hipLaunchKernelGGL(k_rrf_reduce, dim3(unsigned(ceil_div(nb, 256))), dim3(256), 0, st, a.part,
                     nb, int(splits), B);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace tsk
