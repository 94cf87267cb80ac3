// One 16 x 16 tile of an FP64 product C = A^T B (A = [A1 | A2] as K x M, or M
// x K when A_MK) over the whole contraction, by NW waves of the calling
// workgroup: each wave takes a contiguous slice of K with v_mfma_f64_16x16x4
// (lane l feeds A(m0 + l%16, k) and B(k, n0 + l%16), k = k0 + l/16), operands
// loaded straight into registers 64 k at a time so that a wave has 32 loads
// in flight; the NW partial tiles are summed in LDS in wave order
// (deterministic, no split-K launch and no separate reduction).  Used for the
// skinny products (one side of C at most 64) and inside fused launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tsk {

typedef double skinny_doublex4 __attribute__((ext_vector_type(4)));

__device__ inline double skinny_load_a(const double* A1, int64_t lda1, int64_t M1,
                                       const double* A2, int64_t lda2, int64_t k, int64_t i) {
  return i < M1 ? A1[k * lda1 + i] : A2[k * lda2 + (i - M1)];
}

constexpr int kSkChunk = 64;

// red: NW x 16 x 17 doubles of LDS; threads 0 .. 64 NW - 1 of the workgroup;
// CH: k values loaded per round (CH / 2 operand registers in flight per lane)
template <int NW, bool A_MK, int CH = kSkChunk>
__device__ inline void skinny_tile(int64_t M, int64_t N, int64_t K, const double* A1,
                                   int64_t lda1, int64_t M1, const double* A2, int64_t lda2,
                                   const double* B, int64_t ldb, double* C, int64_t ldc,
                                   int64_t mt, int64_t nt, double (*red)[16][17]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t m0 = mt * 16, n0 = nt * 16;
  const int64_t i = m0 + li, j = n0 + li;
  const int64_t kper = ((K + NW * 4 - 1) / (NW * 4)) * 4;
  const int64_t kb = wave * kper, ke = kb + kper < K ? kb + kper : K;
  const bool iv = i < M, jv = j < N;
  const double* arow = A_MK ? A1 + i * lda1 : nullptr;
  skinny_doublex4 acc = {0, 0, 0, 0};
  for (int64_t k0 = kb; k0 < ke; k0 += CH) {
    double a[CH / 4], b[CH / 4];
#pragma unroll
    for (int u = 0; u < CH / 4; ++u) {
      const int64_t k = k0 + 4 * u + g;
      const bool kv = k < ke;
      a[u] = 0.0;
      b[u] = 0.0;
      if (kv && iv) a[u] = A_MK ? arow[k] : skinny_load_a(A1, lda1, M1, A2, lda2, k, i);
      if (kv && jv) b[u] = B[k * ldb + j];
    }
#pragma unroll
    for (int u = 0; u < CH / 4; ++u)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) red[wave][g + 4 * v][li] = acc[v];
  __syncthreads();
  if (threadIdx.x < 256) {
    const int r = threadIdx.x >> 4, c = threadIdx.x & 15;
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NW; ++w) s += red[w][r][c];
    if (m0 + r < M && n0 + c < N) C[(m0 + r) * ldc + n0 + c] = s;
  }
}

}  // namespace tsk
