// Sampled mode-n fibres of a COO tensor for leverage-score sampling
// (Sec. 3.2: Y[j, :] = w_j T(i_1, .., i_{n-1}, :, i_{n+1}, .., i_N); Sec. 6.1
// prices this right-hand side at O(m s), which presumes that a sampled fibre
// is found without scanning the entries).
//
// Fibre index of mode n, built once per tensor and mode:
//   key(e) = (row-major linear index of (i_k)_{k != n}) * s_n + i_n
//   keys   uint64[nnz], ascending; vals[nnz] the tensor's values in key order.
// A fibre is the key range [b s_n, (b + 1) s_n) of its other-mode index b and
// lies contiguously in the index, ordered by i_n.  The sort is stable, so
// duplicate coordinates stay adjacent and in input order; the gather sums each
// run of equal keys from its first entry on, in FP64.
//
// Gather: one workgroup per sample.  Two waves locate the fibre's two ends
// with a 64-way search (each round probes 64 evenly spaced keys and keeps the
// interval between the last key below the target and the first at or above
// it), the fibre is scattered into an LDS row (one writer per coordinate), and
// the row leaves as one coalesced store of w_j * value in the operand type.

#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"
#include "fibers.h"

namespace tsk {

namespace {

constexpr int kFibThreads = 256;
constexpr int kFibChunk = 4096;  // columns of the LDS row (32 KiB of doubles)

struct KeyJob {
  int N;
  int n;
  int64_t nnz;
  int64_t dims[TSK_MAX_ORDER];
  const int32_t* idx[TSK_MAX_ORDER];
};

__global__ void k_fiber_keys(KeyJob kj, uint64_t* keys) {
  const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= kj.nnz) return;
  uint64_t k = 0;
  for (int q = 0; q < kj.N; ++q)
    if (q != kj.n) k = k * uint64_t(kj.dims[q]) + uint64_t(uint32_t(kj.idx[q][e]));
  keys[e] = k * uint64_t(kj.dims[kj.n]) + uint64_t(uint32_t(kj.idx[kj.n][e]));
}

// First position p in [0, nnz) with keys[p] >= target (nnz if none), found by
// one wave.  Invariant: the answer lies in [a, b].
__device__ int64_t wave_lower_bound(const uint64_t* __restrict__ keys, int64_t nnz,
                                    uint64_t target) {
  const int lane = threadIdx.x & 63;
  int64_t a = 0, b = nnz;
  while (b - a > 64) {
    const int64_t step = (b - a + 63) / 64;
    const int64_t p = a + (lane + 1) * step - 1;
    const bool below = p < b && keys[p] < target;
    const int c = __popcll(__ballot(below));
    const int64_t na = a + c * step;
    b = min(b, na + step - 1);
    a = na;
  }
  const int64_t p = a + lane;
  const bool below = p < b && keys[p] < target;
  return a + __popcll(__ballot(below));
}

template <class V, int PREC>
__global__ __launch_bounds__(kFibThreads) void k_fiber_rows(
    FiberIndexView fx, int64_t m, const int32_t* __restrict__ idx, const double* __restrict__ w,
    void* __restrict__ Y) {
  __shared__ double row[kFibChunk];
  __shared__ int64_t range[2];
  const int64_t j = blockIdx.x;
  const int tid = threadIdx.x;
  const int64_t sn = fx.dims[fx.n];
  const uint64_t* __restrict__ keys = fx.keys;
  const V* __restrict__ vals = static_cast<const V*>(fx.vals);
  uint64_t b = 0;
  for (int q = 0, t = 0; q < fx.N; ++q)
    if (q != fx.n) b = b * uint64_t(fx.dims[q]) + uint64_t(uint32_t(idx[j * (fx.N - 1) + t++]));
  const uint64_t base = b * uint64_t(sn);
  if (tid < 128) {
    const int64_t p = wave_lower_bound(keys, fx.nnz, tid < 64 ? base : base + uint64_t(sn));
    if ((tid & 63) == 0) range[tid >> 6] = p;
  }
  __syncthreads();
  const int64_t lo = range[0], hi = range[1];
  const double wj = w[j];
  for (int64_t c0 = 0; c0 < sn; c0 += kFibChunk) {
    const int cw = int(min<int64_t>(kFibChunk, sn - c0));
    for (int c = tid; c < cw; c += kFibThreads) row[c] = 0.0;
    __syncthreads();
    for (int64_t e = lo + tid; e < hi; e += kFibThreads) {
      const uint64_t key = keys[e];
      const int64_t i = int64_t(key - base) - c0;
      if (i < 0 || i >= cw) continue;
      if (e > lo && keys[e - 1] == key) continue;  // not the first of its run
      double s = double(vals[e]);
      for (int64_t e2 = e + 1; e2 < hi && keys[e2] == key; ++e2) s += double(vals[e2]);
      row[i] = s;
    }
    __syncthreads();
    for (int c = tid; c < cw; c += kFibThreads) {
      const double v = __dmul_rn(wj, row[c]);
      const size_t o = size_t(j) * size_t(sn) + size_t(c0 + c);
      if (PREC == TSK_PREC_F64)
        static_cast<double*>(Y)[o] = v;
      else if (PREC == TSK_PREC_F32)
        static_cast<float*>(Y)[o] = float(v);
      else
        static_cast<uint16_t*>(Y)[o] = f32_to_bf16_bits(float(v));
    }
    __syncthreads();
  }
}

template <class V>
tsk_status launch_rows(const FiberIndexView& fx, int64_t m, const int32_t* idx, const double* w,
                       int prec, void* Y, hipStream_t st) {
  const dim3 grid{unsigned(m)}, block{unsigned(kFibThreads)};
  if (prec == TSK_PREC_F64)
    hipLaunchKernelGGL((k_fiber_rows<V, TSK_PREC_F64>), grid, block, 0, st, fx, m, idx, w, Y);
  else if (prec == TSK_PREC_F32)
    hipLaunchKernelGGL((k_fiber_rows<V, TSK_PREC_F32>), grid, block, 0, st, fx, m, idx, w, Y);
  else
    hipLaunchKernelGGL((k_fiber_rows<V, TSK_PREC_BF16>), grid, block, 0, st, fx, m, idx, w, Y);
  TSK_LAUNCHED();
  return TSK_OK;
}

template <class V>
tsk_status sort_pairs(void* tmp, size_t& bytes, const uint64_t* kin, uint64_t* kout,
                      const void* vin, void* vout, int64_t nnz, unsigned end_bit,
                      hipStream_t st) {
  TSK_HIP(rocprim::radix_sort_pairs(tmp, bytes, kin, kout, static_cast<const V*>(vin),
                                    static_cast<V*>(vout), uint32_t(nnz), 0u, end_bit, st));
  return TSK_OK;
}

}  // namespace

tsk_status fiber_key_bits(const TensorView& T, unsigned* bits) {
  // keys run over [0, prod_k s_k); they must fit 64 bits
  unsigned __int128 total = 1;
  for (int k = 0; k < T.order; ++k) {
    total *= unsigned(T.dims[k]);
    if (total > (unsigned __int128)UINT64_MAX) {
      set_error("fibre index: prod of dims exceeds 2^64");
      return TSK_EUNSUPPORTED;
    }
  }
  const uint64_t top = uint64_t(total) - 1;
  unsigned nb = 0;
  while (nb < 64 && (top >> nb)) ++nb;
  *bits = nb == 0 ? 1 : nb;
  return TSK_OK;
}

tsk_status fiber_index_alloc(const TensorView& T, int n, FiberIndexView& fx, Ws& index) {
  TSK_REQUIRE(T.layout == TSK_COO, "a fibre index is built for COO tensors");
  TSK_REQUIRE(n >= 0 && n < T.order, "invalid mode %d", n);
  unsigned bits = 0;
  TSK_TRY(fiber_key_bits(T, &bits));
  fx.N = T.order;
  fx.n = n;
  fx.nnz = T.nnz;
  fx.dtype = T.dtype;
  for (int k = 0; k < T.order; ++k) fx.dims[k] = T.dims[k];
  fx.keys = index.take<uint64_t>(size_t(std::max<int64_t>(T.nnz, 1)));
  fx.vals = index.take<char>(size_t(std::max<int64_t>(T.nnz, 1)) * (T.dtype == TSK_F64 ? 8 : 4));
  return TSK_OK;
}

tsk_status fiber_index_build(const TensorView& T, const FiberIndexView& fx, Ws& ws,
                             hipStream_t st) {
  unsigned bits = 0;
  TSK_TRY(fiber_key_bits(T, &bits));
  const int64_t nnz = T.nnz;
  uint64_t* kin = ws.take<uint64_t>(size_t(std::max<int64_t>(nnz, 1)));
  size_t tbytes = 0;
  if (nnz > 0) {
    if (T.dtype == TSK_F64)
      TSK_TRY(sort_pairs<double>(nullptr, tbytes, kin, fx.keys, T.values, fx.vals, nnz, bits, st));
    else
      TSK_TRY(sort_pairs<float>(nullptr, tbytes, kin, fx.keys, T.values, fx.vals, nnz, bits, st));
  }
  void* tmp = ws.take<char>(std::max<size_t>(tbytes, 1));
  if (ws.measuring() || nnz == 0) return TSK_OK;
  ProfScope prof("fiber_index", st);
  KeyJob kj{};
  kj.N = T.order;
  kj.n = fx.n;
  kj.nnz = nnz;
  for (int k = 0; k < T.order; ++k) {
    kj.dims[k] = T.dims[k];
    kj.idx[k] = T.idx[k];
  }
  hipLaunchKernelGGL(k_fiber_keys, dim3(unsigned(ceil_div(nnz, 256))), dim3(256), 0, st, kj,
                     kin);
  TSK_LAUNCHED();
  if (T.dtype == TSK_F64)
    TSK_TRY(sort_pairs<double>(tmp, tbytes, kin, fx.keys, T.values, fx.vals, nnz, bits, st));
  else
    TSK_TRY(sort_pairs<float>(tmp, tbytes, kin, fx.keys, T.values, fx.vals, nnz, bits, st));
  return TSK_OK;
}

tsk_status fiber_rows(const FiberIndexView& fx, int64_t m, const int32_t* idx, const double* w,
                      int prec, void* Y, hipStream_t st) {
  if (m == 0) return TSK_OK;
  TSK_REQUIRE(m < (int64_t(1) << 31), "too many samples");
  ProfScope prof("fiber_rows", st);
  return fx.dtype == TSK_F64 ? launch_rows<double>(fx, m, idx, w, prec, Y, st)
                             : launch_rows<float>(fx, m, idx, w, prec, Y, st);
}

}  // namespace tsk
