// Gram products of the sketched operands on the matrix cores:
//
//   C (M x N, FP64) = A^T B,   A = [A1 | A2] (K x M), B (K x N), row-major,
//   (and, FP64 only, C = A B with A given M x K row-major),
//
// i.e. both operands are stored with the contraction index (the sketch row)
// slowest -- the layout in which Z (m x r) and Y (m x s) are produced.  Used
// for [Z^T Z ; Y^T Z] in one launch (A = [Z | Y], B = Z), and for the FP64
// Grams of the solve.  Element types: FP64 (v_mfma_f64_16x16x4f64), FP32
// (v_mfma_f32_16x16x4f32) and BF16 (v_mfma_f32_16x16x32_bf16, FP32
// accumulation).  A 256-thread workgroup computes a 64 x 64 tile (four waves,
// 32 x 32 each as 2 x 2 MFMA blocks); tiles of A and B are staged in LDS with
// the contraction index contiguous, so each lane feeds its MFMA operands
// from one vector read.  Split-K partials are FP64 and are summed by a
// separate kernel in a fixed order (deterministic).

#include <type_traits>

#include "common.h"
#include "skinny.h"
#include "kernels.h"

namespace tsk {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kBM = 64, kBN = 64, kThreads = 256;

template <class E>
struct Cfg;
// Output layout of a 16x16 MFMA block: lane l holds column l % 16; its four
// accumulators are rows 4*(l/16) + v (FP32 accumulation) or l/16 + 4*v (FP64).
template <>
struct Cfg<double> {
  static constexpr int BK = 16;   // 4 MFMA k-steps of 4
  static constexpr int LD = 18;   // row stride in elements (144 B)
  static constexpr bool kRowsInterleaved = true;
  typedef doublex4 Acc;
};
template <>
struct Cfg<float> {
  static constexpr int BK = 32;   // 8 MFMA k-steps of 4
  static constexpr int LD = 36;
  static constexpr bool kRowsInterleaved = false;
  typedef floatx4 Acc;
};
template <>
struct Cfg<uint16_t> {
  static constexpr int BK = 64;   // 2 MFMA k-steps of 32
  static constexpr int LD = 72;
  static constexpr bool kRowsInterleaved = false;
  typedef floatx4 Acc;
};

template <class E>
__device__ inline E zero_e() {
  return E(0);
}

template <class E>
__device__ inline E load_a(const E* A1, int64_t lda1, int64_t M1, const E* A2, int64_t lda2,
                           int64_t k, int64_t i) {
  return i < M1 ? A1[k * lda1 + i] : A2[k * lda2 + (i - M1)];
}

// one 16x16 MFMA block step for lane-local operand runs
__device__ inline void mfma_step(const double* a, const double* b, doublex4& acc) {
#pragma unroll
  for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b[t], acc, 0, 0, 0);
}
__device__ inline void mfma_step(const float* a, const float* b, floatx4& acc) {
#pragma unroll
  for (int t = 0; t < 8; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t], b[t], acc, 0, 0, 0);
}
__device__ inline void mfma_step(const uint16_t* a, const uint16_t* b, floatx4& acc) {
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    bf16x8 av, bv;
    __builtin_memcpy(&av, a + 8 * t, 16);
    __builtin_memcpy(&bv, b + 8 * t, 16);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
}

template <class E, bool A_MK>
__global__ __launch_bounds__(kThreads) void k_gemm_tn(int64_t M, int64_t N, int64_t K,
                                                      const E* A1, int64_t lda1, int64_t M1,
                                                      const E* A2, int64_t lda2, const E* B,
                                                      int64_t ldb, int64_t kchunk, double* C,
                                                      int64_t ldc, int64_t split_stride) {
  constexpr int BK = Cfg<E>::BK, LD = Cfg<E>::LD, RUN = BK / 4;
  typedef typename Cfg<E>::Acc Acc;
  __shared__ __attribute__((aligned(16))) E As[kBM * LD];
  __shared__ __attribute__((aligned(16))) E Bs[kBN * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t i0 = int64_t(blockIdx.x) * kBM, j0 = int64_t(blockIdx.y) * kBN;
  const int64_t kbeg = int64_t(blockIdx.z) * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const int g = lane >> 4, li = lane & 15;

  Acc acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    // stage A and B (K x N slice) as X[row][k]; A is K x M (transposed on
    // the way in) or, for A_MK, M x K (copied)
    for (int e = tid; e < BK * kBM; e += kThreads) {
      int kk = e / kBM, ii = e % kBM;
      int64_t k = k0 + kk, j = j0 + ii;
      E bv = zero_e<E>();
      if (k < kend && j < N) bv = B[k * ldb + j];
      Bs[ii * LD + kk] = bv;
      if (!A_MK) {
        int64_t i = i0 + ii;
        E av = zero_e<E>();
        if (k < kend && i < M) av = load_a(A1, lda1, M1, A2, lda2, k, i);
        As[ii * LD + kk] = av;
      } else {
        int ii2 = e / BK, kk2 = e % BK;
        int64_t i = i0 + ii2, k2 = k0 + kk2;
        E av = zero_e<E>();
        if (k2 < kend && i < M) av = A1[i * lda1 + k2];
        As[ii2 * LD + kk2] = av;
      }
    }
    __syncthreads();
#pragma unroll
    for (int sm = 0; sm < 2; ++sm) {
      E ar[RUN];
      const E* pa = As + (wm * 32 + sm * 16 + li) * LD + g * RUN;
#pragma unroll
      for (int t = 0; t < RUN; ++t) ar[t] = pa[t];
#pragma unroll
      for (int sn = 0; sn < 2; ++sn) {
        E br[RUN];
        const E* pb = Bs + (wn * 32 + sn * 16 + li) * LD + g * RUN;
#pragma unroll
        for (int t = 0; t < RUN; ++t) br[t] = pb[t];
        mfma_step(ar, br, acc[sm][sn]);
      }
    }
    __syncthreads();
  }
  double* Cz = C + int64_t(blockIdx.z) * split_stride;
#pragma unroll
  for (int sm = 0; sm < 2; ++sm)
#pragma unroll
    for (int sn = 0; sn < 2; ++sn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int64_t i = i0 + wm * 32 + sm * 16 + (Cfg<E>::kRowsInterleaved ? g + 4 * v : 4 * g + v);
        int64_t j = j0 + wn * 32 + sn * 16 + li;
        if (i < M && j < N) Cz[i * ldc + j] = double(acc[sm][sn][v]);
      }
}

// Skinny FP64 products: one workgroup of 8 waves per 16 x 16 tile of C
// (skinny_tile in skinny.h).
constexpr int kSkW = 8, kSkT = 64 * kSkW;

template <bool A_MK>
__global__ __launch_bounds__(kSkT) void k_gemm_skinny(int64_t M, int64_t N, int64_t K,
                                                      const double* A1, int64_t lda1, int64_t M1,
                                                      const double* A2, int64_t lda2,
                                                      const double* B, int64_t ldb, double* C,
                                                      int64_t ldc) {
  __shared__ double red[kSkW][16][17];
  skinny_tile<kSkW, A_MK>(M, N, K, A1, lda1, M1, A2, lda2, B, ldb, C, ldc, blockIdx.x, blockIdx.y,
                          red);
}

// One- to four-tile products over a long K: 16 waves per tile, so that each
// wave's share of K (and the chain of operand loads) is half as long.
constexpr int kSkW16 = 16;
template <bool A_MK>
__global__ __launch_bounds__(64 * kSkW16) void k_gemm_skinny16(
    int64_t M, int64_t N, int64_t K, const double* A1, int64_t lda1, int64_t M1, const double* A2,
    int64_t lda2, const double* B, int64_t ldb, double* C, int64_t ldc) {
  __shared__ double red[kSkW16][16][17];
  skinny_tile<kSkW16, A_MK, 32>(M, N, K, A1, lda1, M1, A2, lda2, B, ldb, C, ldc, blockIdx.x,
                                blockIdx.y, red);
}

// Products of one to four tiles over a very long K (K >= 4096): blockIdx.z
// takes a range of K, partial tiles in FP64 are summed in split order by
// k_reduce_splits (deterministic).
__global__ __launch_bounds__(kSkT) void k_gemm_skinny_split(int64_t M, int64_t N, int64_t K,
                                                            int64_t kc, const double* A1,
                                                            int64_t lda1, int64_t M1,
                                                            const double* A2, int64_t lda2,
                                                            const double* B, int64_t ldb,
                                                            double* part) {
  __shared__ double red[kSkW][16][17];
  const int64_t k0 = int64_t(blockIdx.z) * kc;
  const int64_t kn = k0 + kc < K ? kc : K - k0;
  skinny_tile<kSkW, false>(M, N, kn, A1 + k0 * lda1, lda1, M1, A2 ? A2 + k0 * lda2 : nullptr,
                           lda2, B + k0 * ldb, ldb, part + int64_t(blockIdx.z) * M * N, N,
                           blockIdx.x, blockIdx.y, red);
}

// Grams A^T A of several row-major K x R matrices in one launch: blockIdx.z
// picks the matrix and a range of K (splits ranges of kc rows), workgroups
// beyond the matrix's tiles leave at once.  With one range the tile goes to
// C; with more, each range's partial tile goes to part (matrix p, range q at
// part[p] + q R^2) and k_gram_sum adds them in range order (deterministic).
struct GramBatch {
  int n, splits;
  int64_t R[TSK_MAX_ORDER];
  int64_t K[TSK_MAX_ORDER];
  int64_t kc[TSK_MAX_ORDER];
  const double* A[TSK_MAX_ORDER];
  double* C[TSK_MAX_ORDER];
  double* part[TSK_MAX_ORDER];
};
__global__ __launch_bounds__(kSkT) void k_gram_batch(GramBatch gb) {
  __shared__ double red[kSkW][16][17];
  const int p = blockIdx.z / gb.splits, q = blockIdx.z - p * gb.splits;
  const int64_t R = gb.R[p];
  if (int64_t(blockIdx.x) * 16 >= R || int64_t(blockIdx.y) * 16 >= R) return;  // uniform
  const int64_t k0 = q * gb.kc[p];
  const int64_t kn = k0 >= gb.K[p] ? 0 : (k0 + gb.kc[p] < gb.K[p] ? gb.kc[p] : gb.K[p] - k0);
  const double* A = gb.A[p] + (kn > 0 ? k0 * R : 0);
  double* out = gb.splits == 1 ? gb.C[p] : gb.part[p] + q * R * R;
  skinny_tile<kSkW, false>(R, R, kn, A, R, R, nullptr, 0, A, R, out, R, blockIdx.x, blockIdx.y,
                           red);
}

__global__ __launch_bounds__(256) void k_gram_sum(GramBatch gb) {
  const int p = blockIdx.x;
  const int64_t rr = gb.R[p] * gb.R[p];
  for (int64_t t = threadIdx.x; t < rr; t += 256) {
    double s = 0.0;
    for (int q = 0; q < gb.splits; ++q) s += gb.part[p][q * rr + t];
    gb.C[p][t] = s;
  }
}

// FP32 operands, both K-major (A = [A1 | A2] as K x M, B as K x N), 64 x 64
// tiles, 4 waves (2 x 2, 32 x 32 each), K slabs of 64 double-buffered in LDS
// in [k][m] layout (row stride 80 floats: the four k rows that one MFMA
// operand read touches fall in different bank halves), float4 global loads;
// the next slab is fetched into registers while the current one feeds the
// MFMAs.  Requires M1, lda1, lda2, ldb multiples of 4 and 16-byte aligned
// bases (k_gemm_tn covers the rest).
constexpr int kF4K = 64, kF4LD = 80, kF4LDA = 68;

__device__ inline float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

template <bool A_MK>
__global__ __launch_bounds__(kThreads) void k_gemm_tn_f32v(int64_t M, int64_t N, int64_t K,
                                                          const float* A1, int64_t lda1,
                                                          int64_t M1, const float* A2,
                                                          int64_t lda2, const float* B,
                                                          int64_t ldb, int64_t kchunk, double* C,
                                                          int64_t ldc, int64_t split_stride) {
  __shared__ __attribute__((aligned(16))) float As[2][kF4K * kF4LD];
  __shared__ __attribute__((aligned(16))) float Bs[2][kF4K * kF4LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t i0 = int64_t(blockIdx.x) * kBM, j0 = int64_t(blockIdx.y) * kBN;
  const int64_t kbeg = int64_t(blockIdx.z) * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const int g = lane >> 4, li = lane & 15;
  // loader: thread covers column quad cq (4 consecutive m or n) of rows
  // kr + 16 u, u < 4
  const int cq = (tid & 15) * 4, kr = tid >> 4;
  const int64_t ia = i0 + cq, jb = j0 + cq;
  const bool a_in = ia + 3 < M, b_in = jb + 3 < N;
  const float* abase = ia < M1 ? A1 + ia : A2 + (ia - M1);
  const int64_t alda = ia < M1 ? lda1 : lda2;
  // A_MK (A given M x K, row-major): thread covers k quad cq of rows
  // mr + 16 u, staged as [m][k] (row stride kF4LDA: the 16 rows one operand
  // read touches fall in different banks)
  const int mr = tid >> 4;
  float4 ra[4], rb[4];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t k = k0 + kr + 16 * u;
      const bool kv = k < kend;
      if constexpr (A_MK) {
        const int64_t i = i0 + mr + 16 * u, kq = k0 + cq;
        if (i < M && kq + 3 < kend) {
          ra[u] = ld4(A1 + i * lda1 + kq);
        } else {
          float t[4];
#pragma unroll
          for (int e = 0; e < 4; ++e) t[e] = (i < M && kq + e < kend) ? A1[i * lda1 + kq + e] : 0.f;
          ra[u] = make_float4(t[0], t[1], t[2], t[3]);
        }
      } else if (kv && a_in) {
        ra[u] = ld4(abase + k * alda);
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t i = ia + e;
          t[e] = (kv && i < M) ? (i < M1 ? A1[k * lda1 + i] : A2[k * lda2 + (i - M1)]) : 0.f;
        }
        ra[u] = make_float4(t[0], t[1], t[2], t[3]);
      }
      if (kv && b_in) {
        rb[u] = ld4(B + k * ldb + jb);
      } else {
        float t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (kv && jb + e < N) ? B[k * ldb + jb + e] : 0.f;
        rb[u] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if constexpr (A_MK)
        *reinterpret_cast<float4*>(&As[buf][(mr + 16 * u) * kF4LDA + cq]) = ra[u];
      else
        *reinterpret_cast<float4*>(&As[buf][(kr + 16 * u) * kF4LD + cq]) = ra[u];
      *reinterpret_cast<float4*>(&Bs[buf][(kr + 16 * u) * kF4LD + cq]) = rb[u];
    }
  };
  floatx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
  int buf = 0;
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += kF4K) {
    const bool more = k0 + kF4K < kend;
    if (more) fetch(k0 + kF4K);
    const float* as = As[buf];
    const float* bs = Bs[buf];
#pragma unroll
    for (int t = 0; t < kF4K / 4; ++t) {
      const int kk = 4 * t + g;
      float av[2], bv[2];
#pragma unroll
      for (int sm = 0; sm < 2; ++sm)
        av[sm] = A_MK ? as[(wm * 32 + sm * 16 + li) * kF4LDA + kk]
                      : as[kk * kF4LD + wm * 32 + sm * 16 + li];
#pragma unroll
      for (int sn = 0; sn < 2; ++sn) bv[sn] = bs[kk * kF4LD + wn * 32 + sn * 16 + li];
#pragma unroll
      for (int sm = 0; sm < 2; ++sm)
#pragma unroll
        for (int sn = 0; sn < 2; ++sn)
          acc[sm][sn] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[sm], bv[sn], acc[sm][sn], 0, 0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* Cz = C + int64_t(blockIdx.z) * split_stride;
#pragma unroll
  for (int sm = 0; sm < 2; ++sm)
#pragma unroll
    for (int sn = 0; sn < 2; ++sn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wm * 32 + sm * 16 + 4 * g + v;
        const int64_t j = j0 + wn * 32 + sn * 16 + li;
        if (i < M && j < N) Cz[i * ldc + j] = double(acc[sm][sn][v]);
      }
}

// BF16 operands, both K-major (A = [A1 | A2] as K x M, B as K x N), 64 x 64
// tiles, 4 waves (2 x 2, 32 x 32 each), K slabs of 128 double-buffered in LDS
// in [m][k] layout (row stride 136 elements: the 16 rows of one operand read
// start in different banks), so that a lane feeds its 16x16x32 MFMA from one
// 16-byte read.  Each thread loads one task of A and one of B per slab: 8 k
// rows x 4 consecutive columns (eight 8-byte global loads), transposed in
// registers into 4 columns x 8 k and stored with four 16-byte LDS writes; the
// next slab is fetched into registers while the current one feeds the MFMAs.
// Requires M1, lda1, lda2, ldb multiples of 4 and 8-byte aligned bases
// (k_gemm_tn covers the rest).
constexpr int kB8K = 128, kB8LD = 136;

__global__ __launch_bounds__(kThreads) void k_gemm_tn_bf16v(int64_t M, int64_t N, int64_t K,
                                                           const uint16_t* A1, int64_t lda1,
                                                           int64_t M1, const uint16_t* A2,
                                                           int64_t lda2, const uint16_t* B,
                                                           int64_t ldb, int64_t kchunk,
                                                           double* C, int64_t ldc,
                                                           int64_t split_stride) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][kBM * kB8LD];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][kBN * kB8LD];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t i0 = int64_t(blockIdx.x) * kBM, j0 = int64_t(blockIdx.y) * kBN;
  const int64_t kbeg = int64_t(blockIdx.z) * kchunk;
  const int64_t kend = kbeg + kchunk < K ? kbeg + kchunk : K;
  const int g = lane >> 4, li = lane & 15;
  // loader task of this thread (the same for A and B): k group kg (8 rows),
  // column quad cq
  const int kg = tid >> 4, cq = (tid & 15) * 4;
  const int64_t ca = i0 + cq, cb = j0 + cq;
  const bool fa = ca + 3 < M, fb = cb + 3 < N;
  const uint16_t* abase = ca < M1 ? A1 + ca : A2 + (ca - M1);
  const int64_t alda = ca < M1 ? lda1 : lda2;
  uint2 ra[8], rb[8];
  auto pack4 = [](const uint16_t (&t)[4]) {
    return make_uint2(t[0] | (uint32_t(t[1]) << 16), t[2] | (uint32_t(t[3]) << 16));
  };
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int64_t k = k0 + 8 * kg + r;
      const bool kv = k < kend;
      if (kv && fa) {
        ra[r] = *reinterpret_cast<const uint2*>(abase + k * alda);
      } else {
        uint16_t t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int64_t c = ca + e;
          t[e] = (kv && c < M) ? (c < M1 ? A1[k * lda1 + c] : A2[k * lda2 + (c - M1)]) : 0;
        }
        ra[r] = pack4(t);
      }
      if (kv && fb) {
        rb[r] = *reinterpret_cast<const uint2*>(B + k * ldb + cb);
      } else {
        uint16_t t[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) t[e] = (kv && cb + e < N) ? B[k * ldb + cb + e] : 0;
        rb[r] = pack4(t);
      }
    }
  };
  // column c (0..3) of 8 rows as 8 consecutive k: one 16-byte word
  auto column = [](const uint2 (&v)[8], int c) {
    auto h = [&](int r) -> uint32_t {
      const uint32_t w = c < 2 ? v[r].x : v[r].y;
      return (c & 1) ? (w >> 16) : (w & 0xffffu);
    };
    return make_uint4(h(0) | (h(1) << 16), h(2) | (h(3) << 16), h(4) | (h(5) << 16),
                      h(6) | (h(7) << 16));
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      *reinterpret_cast<uint4*>(&As[buf][(cq + c) * kB8LD + 8 * kg]) = column(ra, c);
      *reinterpret_cast<uint4*>(&Bs[buf][(cq + c) * kB8LD + 8 * kg]) = column(rb, c);
    }
  };
  floatx4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = floatx4{0, 0, 0, 0};
  int buf = 0;
  if (kbeg < kend) {
    fetch(kbeg);
    stash(0);
  }
  __syncthreads();
  for (int64_t k0 = kbeg; k0 < kend; k0 += kB8K) {
    const bool more = k0 + kB8K < kend;
    if (more) fetch(k0 + kB8K);
    const uint16_t* as = As[buf];
    const uint16_t* bs = Bs[buf];
#pragma unroll
    for (int ks = 0; ks < kB8K / 32; ++ks) {
      bf16x8 av[2], bv[2];
#pragma unroll
      for (int sm = 0; sm < 2; ++sm)
        av[sm] = *reinterpret_cast<const bf16x8*>(as + (wm * 32 + sm * 16 + li) * kB8LD +
                                                  32 * ks + 8 * g);
#pragma unroll
      for (int sn = 0; sn < 2; ++sn)
        bv[sn] = *reinterpret_cast<const bf16x8*>(bs + (wn * 32 + sn * 16 + li) * kB8LD +
                                                  32 * ks + 8 * g);
#pragma unroll
      for (int sm = 0; sm < 2; ++sm)
#pragma unroll
        for (int sn = 0; sn < 2; ++sn)
          acc[sm][sn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[sm], bv[sn], acc[sm][sn], 0,
                                                                0, 0);
    }
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  double* Cz = C + int64_t(blockIdx.z) * split_stride;
#pragma unroll
  for (int sm = 0; sm < 2; ++sm)
#pragma unroll
    for (int sn = 0; sn < 2; ++sn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + wm * 32 + sm * 16 + 4 * g + v;
        const int64_t j = j0 + wn * 32 + sn * 16 + li;
        if (i < M && j < N) Cz[i * ldc + j] = double(acc[sm][sn][v]);
      }
}

__global__ void k_reduce_splits(const double* part, int64_t M, int64_t N, int splits,
                                double* C, int64_t ldc) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= M * N) return;
  int64_t i = t / N, j = t % N;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[int64_t(z) * M * N + t];
  C[i * ldc + j] = s;
}

// Skinny products with FP32 operands and at most 32 output columns, the
// products with Y of the randomized solve: C (M x N, FP64) = A B with A given
// as M x K (A_MK: rows along the contraction, Y Omega) or K x M (Y^T (Z P)),
// and B given transposed (Bt: N x K, rows zero beyond K up to ldbt).  One
// workgroup per 64 rows of C and range of 4 kcw contraction indices, one wave
// per kcw of them, on v_mfma_f32_16x16x4 (lane l = li + 16 g feeds A(li, g),
// B(g, li) and holds D(4 g + v, li)): for four contraction steps t the lane's
// k is k0 + 4 g + t, so that the B values (and A's when A_MK) of one lane are
// four consecutive floats, one vector load.  FP32 accumulation within a wave;
// the four waves' tiles summed in FP64 in wave order through LDS; the ranges'
// tiles summed in range order by k_reduce_splits.  No operands are staged:
// A is streamed once from HBM, Bt (small) comes from L2.
constexpr int kYsT = 256;

template <bool A_MK>
__global__ __launch_bounds__(kYsT) void k_gemm_yskinny(int64_t M, int N, int64_t K,
                                                       const float* __restrict__ A, int64_t lda,
                                                       const float* __restrict__ Bt,
                                                       int64_t ldbt, int64_t kcw, double* out,
                                                       int64_t ldo, int64_t split_stride) {
  __shared__ float red[3][64][33];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 15, g = lane >> 4;
  const int64_t i0 = int64_t(blockIdx.x) * 64;
  const int64_t kb = (int64_t(blockIdx.y) * 4 + wave) * kcw;
  const int64_t ke = kb + kcw < K ? kb + kcw : K;
  floatx4 acc[4][2];
#pragma unroll
  for (int sm = 0; sm < 4; ++sm)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[sm][nt] = floatx4{0, 0, 0, 0};
  // rows of A (A_MK) or columns (K x M) this lane reads, clamped into range
  int64_t ia[4];
  bool iv[4];
#pragma unroll
  for (int sm = 0; sm < 4; ++sm) {
    const int64_t i = i0 + 16 * sm + li;
    iv[sm] = i < M;
    ia[sm] = iv[sm] ? i : M - 1;
  }
  const float* brow[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int n = 16 * nt + li;
    brow[nt] = Bt + int64_t(n < N ? n : N - 1) * ldbt;
  }
  const bool bv0 = li < N, bv1 = 16 + li < N;
  // one 16-index step: B (and A when A_MK) as float4 loads, masked past ke
  auto load = [&](int64_t k0, float (&a)[4][4], float (&b)[2][4]) {
    const int64_t k = k0 + 4 * g;
    const bool kin = k0 < ke;
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      float4 v = float4{0.f, 0.f, 0.f, 0.f};
      if (kin) v = *reinterpret_cast<const float4*>(brow[nt] + k);  // k < ceil16(K) <= ldbt
      b[nt][0] = v.x, b[nt][1] = v.y, b[nt][2] = v.z, b[nt][3] = v.w;
    }
    if (!bv0)
#pragma unroll
      for (int t = 0; t < 4; ++t) b[0][t] = 0.f;
    if (!bv1)
#pragma unroll
      for (int t = 0; t < 4; ++t) b[1][t] = 0.f;
#pragma unroll
    for (int sm = 0; sm < 4; ++sm) {
      if (A_MK) {  // K % 4 == 0 and ranges of multiples of 16: all four in or out
        float4 v = float4{0.f, 0.f, 0.f, 0.f};
        if (k < ke) v = *reinterpret_cast<const float4*>(A + ia[sm] * lda + k);
        a[sm][0] = v.x, a[sm][1] = v.y, a[sm][2] = v.z, a[sm][3] = v.w;
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int64_t kt = k + t < ke ? k + t : ke - 1;
          const float x = kin ? A[kt * lda + ia[sm]] : 0.f;
          a[sm][t] = k + t < ke ? x : 0.f;
        }
      }
      if (!iv[sm])
#pragma unroll
        for (int t = 0; t < 4; ++t) a[sm][t] = 0.f;
    }
  };
  auto mma = [&](const float (&a)[4][4], const float (&b)[2][4]) {
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int sm = 0; sm < 4; ++sm)
#pragma unroll
        for (int nt = 0; nt < 2; ++nt)
          acc[sm][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[sm][t], b[nt][t], acc[sm][nt], 0,
                                                              0, 0);
  };
  if (A_MK) {  // two steps' loads in flight before their products
    for (int64_t k0 = kb; k0 < ke; k0 += 32) {
      float a0[4][4], b0[2][4], a1[4][4], b1[2][4];
      load(k0, a0, b0);
      load(k0 + 16, a1, b1);
      mma(a0, b0);
      mma(a1, b1);
    }
  } else {
    for (int64_t k0 = kb; k0 < ke; k0 += 16) {
      float a0[4][4], b0[2][4];
      load(k0, a0, b0);
      mma(a0, b0);
    }
  }
  if (wave > 0)
#pragma unroll
    for (int sm = 0; sm < 4; ++sm)
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wave - 1][16 * sm + 4 * g + v][16 * nt + li] = acc[sm][nt][v];
  __syncthreads();
  if (wave > 0) return;
  double* o = out + int64_t(blockIdx.y) * split_stride;
#pragma unroll
  for (int sm = 0; sm < 4; ++sm)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * sm + 4 * g + v, c = 16 * nt + li;
        const int64_t i = i0 + r;
        if (i >= M || c >= N) continue;
        double x = double(acc[sm][nt][v]);
#pragma unroll
        for (int w = 0; w < 3; ++w) x += double(red[w][r][c]);
        o[i * ldo + c] = x;
      }
}

__global__ void k_gemm_small(int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                             int64_t sai, int64_t sak, const double* B, int64_t sbk, int64_t sbj,
                             double beta, double* C, int64_t ldc) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= M * N) return;
  int64_t i = t / N, j = t % N;
  double s = 0.0;
  for (int64_t k = 0; k < K; ++k) s += A[i * sai + k * sak] * B[k * sbk + j * sbj];
  double* c = C + i * ldc + j;
  *c = beta == 0.0 ? alpha * s : alpha * s + beta * *c;
}

__global__ void k_to_f64(const void* src, int bytes, int64_t n, double* dst) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (bytes == 8)
    dst[t] = static_cast<const double*>(src)[t];
  else if (bytes == 4)
    dst[t] = double(static_cast<const float*>(src)[t]);
  else
    dst[t] = double(bf16_bits_to_f32(static_cast<const uint16_t*>(src)[t]));
}

// Split-K plan: at least ~512 workgroups when the output has few tiles, at
// least four BK blocks of the contraction per split.
template <class E>
void split_plan(int64_t M, int64_t N, int64_t K, int64_t& splits, int64_t& kchunk) {
  constexpr int BK = Cfg<E>::BK;
  const int64_t tm = ceil_div(M, kBM), tn = ceil_div(N, kBN);
  const int64_t kblocks = ceil_div(K, BK);
  splits = ceil_div(512, tm * tn);
  const int64_t maxs = kblocks / 4;
  if (splits > maxs) splits = maxs;
  if (splits < 1) splits = 1;
  kchunk = ceil_div(kblocks, splits) * BK;
  splits = K > 0 ? ceil_div(K, kchunk) : 1;
}

template <class E, bool A_MK>
tsk_status gemm_tn_t(int64_t M, int64_t N, int64_t K, const void* A1, int64_t lda1, int64_t M1,
                     const void* A2, int64_t lda2, const void* B, int64_t ldb, double* C,
                     int64_t ldc, Ws& ws, hipStream_t st) {
  if (std::is_same<E, double>::value && (M <= 64 || N <= 64) && K > 0) {
    if (!A_MK && ceil_div(M, 16) * ceil_div(N, 16) <= 4 && K >= 4096) {
      const int64_t kc = ceil_div(ceil_div(K, std::min<int64_t>(32, K / 256)), 4) * 4;
      const int64_t spl = ceil_div(K, kc);
      double* part = ws.take<double>(size_t(spl * M * N));
      if (ws.measuring() || M == 0 || N == 0) return TSK_OK;
      hipLaunchKernelGGL(k_gemm_skinny_split, dim3(ceil_div(M, 16), ceil_div(N, 16), spl),
                         dim3(kSkT), 0, st, M, N, K, kc, static_cast<const double*>(A1), lda1, M1,
                         static_cast<const double*>(A2), lda2, static_cast<const double*>(B), ldb,
                         part);
      TSK_LAUNCHED();
      hipLaunchKernelGGL(k_reduce_splits, dim3(ceil_div(M * N, 256)), dim3(256), 0, st, part, M, N,
                         int(spl), C, ldc);
      TSK_LAUNCHED();
      return TSK_OK;
    }
    if (ws.measuring() || M == 0 || N == 0) return TSK_OK;
    if (ceil_div(M, 16) * ceil_div(N, 16) <= 4 && K >= 1024) {
      hipLaunchKernelGGL((k_gemm_skinny16<A_MK>), dim3(ceil_div(M, 16), ceil_div(N, 16)),
                         dim3(64 * kSkW16), 0, st, M, N, K, static_cast<const double*>(A1), lda1,
                         M1, static_cast<const double*>(A2), lda2,
                         static_cast<const double*>(B), ldb, C, ldc);
      TSK_LAUNCHED();
      return TSK_OK;
    }
    hipLaunchKernelGGL((k_gemm_skinny<A_MK>), dim3(ceil_div(M, 16), ceil_div(N, 16)), dim3(kSkT),
                       0, st, M, N, K, static_cast<const double*>(A1), lda1, M1,
                       static_cast<const double*>(A2), lda2, static_cast<const double*>(B), ldb,
                       C, ldc);
    TSK_LAUNCHED();
    return TSK_OK;
  }
  int64_t tm = ceil_div(M, kBM), tn = ceil_div(N, kBN);
  int64_t splits, kchunk;
  split_plan<E>(M, N, K, splits, kchunk);
  double* part = splits > 1 ? ws.take<double>(splits * M * N) : nullptr;
  if (ws.measuring()) return TSK_OK;
  if (M == 0 || N == 0) return TSK_OK;
  if (K == 0) {
    for (int64_t i = 0; i < M; ++i) TSK_HIP(hipMemsetAsync(C + i * ldc, 0, N * 8, st));
    return TSK_OK;
  }
  dim3 grid(tm, tn, splits);
  if (std::is_same<E, float>::value) {
    const bool vec = M1 % 4 == 0 && lda1 % 4 == 0 && lda2 % 4 == 0 && ldb % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(A1) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(A2) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(B) % 16 == 0;
    if (vec) {
      const int64_t kch = ceil_div(kchunk, kF4K) * kF4K;
      const int64_t spl = ceil_div(K, kch);
      double* dst = spl > 1 ? part : C;
      hipLaunchKernelGGL(k_gemm_tn_f32v<A_MK>, dim3(tm, tn, spl), dim3(kThreads), 0, st, M, N, K,
                         static_cast<const float*>(A1), lda1, M1,
                         static_cast<const float*>(A2), lda2, static_cast<const float*>(B), ldb,
                         kch, dst, spl > 1 ? N : ldc, spl > 1 ? M * N : int64_t(0));
      TSK_LAUNCHED();
      if (spl > 1) {
        hipLaunchKernelGGL(k_reduce_splits, dim3(ceil_div(M * N, 256)), dim3(256), 0, st, part, M,
                           N, int(spl), C, ldc);
        TSK_LAUNCHED();
      }
      return TSK_OK;
    }
  }
  if constexpr (std::is_same<E, uint16_t>::value && !A_MK) {
    const bool vec = M1 % 4 == 0 && lda1 % 4 == 0 && lda2 % 4 == 0 && ldb % 4 == 0 &&
                     reinterpret_cast<uintptr_t>(A1) % 8 == 0 &&
                     reinterpret_cast<uintptr_t>(A2) % 8 == 0 &&
                     reinterpret_cast<uintptr_t>(B) % 8 == 0;
    if (vec) {
      const int64_t kch = ceil_div(kchunk, kB8K) * kB8K;
      const int64_t spl = ceil_div(K, kch);
      double* dst = spl > 1 ? part : C;
      hipLaunchKernelGGL(k_gemm_tn_bf16v, dim3(tm, tn, spl), dim3(kThreads), 0, st, M, N, K,
                         static_cast<const uint16_t*>(A1), lda1, M1,
                         static_cast<const uint16_t*>(A2), lda2,
                         static_cast<const uint16_t*>(B), ldb, kch, dst, spl > 1 ? N : ldc,
                         spl > 1 ? M * N : int64_t(0));
      TSK_LAUNCHED();
      if (spl > 1) {
        hipLaunchKernelGGL(k_reduce_splits, dim3(ceil_div(M * N, 256)), dim3(256), 0, st, part, M,
                           N, int(spl), C, ldc);
        TSK_LAUNCHED();
      }
      return TSK_OK;
    }
  }
  if (splits == 1) {
    hipLaunchKernelGGL((k_gemm_tn<E, A_MK>), grid, dim3(kThreads), 0, st, M, N, K,
                       static_cast<const E*>(A1), lda1, M1, static_cast<const E*>(A2), lda2,
                       static_cast<const E*>(B), ldb, kchunk, C, ldc, int64_t(0));
    TSK_LAUNCHED();
  } else {
    hipLaunchKernelGGL((k_gemm_tn<E, A_MK>), grid, dim3(kThreads), 0, st, M, N, K,
                       static_cast<const E*>(A1), lda1, M1, static_cast<const E*>(A2), lda2,
                       static_cast<const E*>(B), ldb, kchunk, part, N, M * N);
    TSK_LAUNCHED();
    hipLaunchKernelGGL(k_reduce_splits, dim3(ceil_div(M * N, 256)), dim3(256), 0, st, part, M, N,
                       int(splits), C, ldc);
    TSK_LAUNCHED();
  }
  return TSK_OK;
}

}  // namespace

int gram_batch_splits(int n, const int64_t* K) {
  int64_t kmax = 0;
  for (int p = 0; p < n; ++p) kmax = K[p] > kmax ? K[p] : kmax;
  const int64_t s = kmax / 1024;  // at least 1024 rows per range
  return int(s < 1 ? 1 : s > kGramSplitsMax ? kGramSplitsMax : s);
}

tsk_status gram_batch_f64(int n, const int64_t* R, const int64_t* K, const double* const* A,
                          double* const* C, double* part, hipStream_t st) {
  TSK_REQUIRE(n >= 1 && n <= TSK_MAX_ORDER, "gram batch of %d matrices", n);
  GramBatch gb{};
  gb.n = n;
  gb.splits = part ? gram_batch_splits(n, K) : 1;
  int64_t rmax = 0, off = 0;
  for (int p = 0; p < n; ++p) {
    TSK_REQUIRE(R[p] >= 1 && R[p] <= 64 && K[p] >= 1, "gram batch shapes");
    gb.R[p] = R[p];
    gb.K[p] = K[p];
    gb.kc[p] = ceil_div(ceil_div(K[p], gb.splits), 4) * 4;
    gb.A[p] = A[p];
    gb.C[p] = C[p];
    gb.part[p] = part ? part + off : nullptr;
    off += int64_t(gb.splits) * R[p] * R[p];
    rmax = R[p] > rmax ? R[p] : rmax;
  }
  const unsigned t = unsigned(ceil_div(rmax, 16));
  hipLaunchKernelGGL(k_gram_batch, dim3(t, t, unsigned(n * gb.splits)), dim3(kSkT), 0, st, gb);
  TSK_LAUNCHED();
  if (gb.splits > 1) {
    hipLaunchKernelGGL(k_gram_sum, dim3(unsigned(n)), dim3(256), 0, st, gb);
    TSK_LAUNCHED();
  }
  return TSK_OK;
}

bool yskinny_fits(bool a_mk, int64_t N, int64_t K, const void* A, int64_t lda, const void* Bt,
                  int64_t ldbt) {
  const bool vec_b = ldbt % 4 == 0 && ldbt >= ceil_div(K, 16) * 16 &&
                     reinterpret_cast<uintptr_t>(Bt) % 16 == 0;
  const bool vec_a = !a_mk || (K % 4 == 0 && lda % 4 == 0 &&
                               reinterpret_cast<uintptr_t>(A) % 16 == 0);
  return N >= 1 && N <= 32 && K >= 1 && vec_b && vec_a;
}

tsk_status gemm_yskinny_f32(bool a_mk, int64_t M, int64_t N, int64_t K, const float* A,
                            int64_t lda, const float* Bt, int64_t ldbt, double* C, int64_t ldc,
                            Ws& ws, hipStream_t st) {
  // ranges of 4 kcw indices (kcw a multiple of 16) so that there are about 512
  // workgroups (A_MK, two steps in flight per wave) or 1024 (K x M, one step)
  const int64_t tm = ceil_div(M, 64);
  const int64_t target = a_mk ? 512 : 1024;
  int64_t nr = std::max<int64_t>(1, std::min<int64_t>(ceil_div(target, tm), ceil_div(K, 64)));
  const int64_t kcw = ceil_div(ceil_div(K, 4 * nr), 16) * 16;
  nr = ceil_div(K, 4 * kcw);
  double* part = nr > 1 ? ws.take<double>(size_t(nr) * M * N) : nullptr;
  if (ws.measuring() || M == 0) return TSK_OK;
  TSK_REQUIRE(yskinny_fits(a_mk, N, K, A, lda, Bt, ldbt), "skinny FP32 product: shapes");
  double* dst = nr > 1 ? part : C;
  const dim3 grid{unsigned(tm), unsigned(nr)};
  if (a_mk)
    hipLaunchKernelGGL(k_gemm_yskinny<true>, grid, dim3(kYsT), 0, st, M, int(N), K, A, lda, Bt,
                       ldbt, kcw, dst, nr > 1 ? N : ldc, nr > 1 ? M * N : int64_t(0));
  else
    hipLaunchKernelGGL(k_gemm_yskinny<false>, grid, dim3(kYsT), 0, st, M, int(N), K, A, lda, Bt,
                       ldbt, kcw, dst, nr > 1 ? N : ldc, nr > 1 ? M * N : int64_t(0));
  TSK_LAUNCHED();
  if (nr > 1) {
    hipLaunchKernelGGL(k_reduce_splits, dim3(ceil_div(M * N, 256)), dim3(256), 0, st, part, M, N,
                       int(nr), C, ldc);
    TSK_LAUNCHED();
  }
  return TSK_OK;
}

tsk_status gemm_tn(int prec, int64_t M, int64_t N, int64_t K, const void* A1, int64_t lda1,
                   int64_t M1, const void* A2, int64_t lda2, const void* B, int64_t ldb,
                   double* C, int64_t ldc, Ws& ws, hipStream_t st) {
  if (!A2) {
    A2 = A1;
    lda2 = lda1;
    M1 = M;
  }
  switch (prec) {
    case TSK_PREC_F64:
      return gemm_tn_t<double, false>(M, N, K, A1, lda1, M1, A2, lda2, B, ldb, C, ldc, ws, st);
    case TSK_PREC_F32:
      return gemm_tn_t<float, false>(M, N, K, A1, lda1, M1, A2, lda2, B, ldb, C, ldc, ws, st);
    default:
      return gemm_tn_t<uint16_t, false>(M, N, K, A1, lda1, M1, A2, lda2, B, ldb, C, ldc, ws, st);
  }
}

tsk_status gemm_nn_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t lda,
                       const double* B, int64_t ldb, double* C, int64_t ldc, Ws& ws,
                       hipStream_t st) {
  return gemm_tn_t<double, true>(M, N, K, A, lda, M, A, lda, B, ldb, C, ldc, ws, st);
}

tsk_status gemm_nn(int prec, int64_t M, int64_t N, int64_t K, const void* A, int64_t lda,
                   const void* B, int64_t ldb, double* C, int64_t ldc, Ws& ws, hipStream_t st) {
  switch (prec) {
    case TSK_PREC_F64:
      return gemm_tn_t<double, true>(M, N, K, A, lda, M, A, lda, B, ldb, C, ldc, ws, st);
    case TSK_PREC_F32:
      return gemm_tn_t<float, true>(M, N, K, A, lda, M, A, lda, B, ldb, C, ldc, ws, st);
    default:
      return gemm_tn_t<uint16_t, true>(M, N, K, A, lda, M, A, lda, B, ldb, C, ldc, ws, st);
  }
}

tsk_status gemm_small(int64_t M, int64_t N, int64_t K, double alpha, const double* A,
                      int64_t sai, int64_t sak, const double* B, int64_t sbk, int64_t sbj,
                      double beta, double* C, int64_t ldc, hipStream_t st) {
  if (M * N == 0) return TSK_OK;
  hipLaunchKernelGGL(k_gemm_small, dim3(ceil_div(M * N, 256)), dim3(256), 0, st, M, N, K, alpha,
                     A, sai, sak, B, sbk, sbj, beta, C, ldc);
  TSK_LAUNCHED();
  return TSK_OK;
}

__global__ void k_from_f64(const double* src, int64_t rows, int64_t cols, void* dst,
                           int64_t ldd, int prec) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= rows * ldd) return;
  const int64_t i = t / ldd, j = t % ldd;  // padding columns are zeroed
  store_prec(dst, size_t(t), j < cols ? src[i * cols + j] : 0.0, prec);
}

tsk_status convert_from_f64(const double* src, int64_t rows, int64_t cols, void* dst,
                            int64_t ldd, int prec, hipStream_t st) {
  if (rows * ldd <= 0) return TSK_OK;
  hipLaunchKernelGGL(k_from_f64, dim3(ceil_div(rows * ldd, 256)), dim3(256), 0, st, src, rows,
                     cols, dst, ldd, prec);
  TSK_LAUNCHED();
  return TSK_OK;
}

// dst (cols x ldd, FP32) = src^T for src rows x cols (FP64, row-major); the
// columns rows .. ldd - 1 of dst are zeroed
__global__ void k_from_f64_t(const double* src, int64_t rows, int64_t cols, float* dst,
                             int64_t ldd) {
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= cols * ldd) return;
  const int64_t c = t / ldd, r = t % ldd;
  dst[t] = r < rows ? float(src[r * cols + c]) : 0.f;
}

tsk_status convert_from_f64_t(const double* src, int64_t rows, int64_t cols, float* dst,
                              int64_t ldd, hipStream_t st) {
  if (cols * ldd <= 0) return TSK_OK;
  hipLaunchKernelGGL(k_from_f64_t, dim3(ceil_div(cols * ldd, 256)), dim3(256), 0, st, src, rows,
                     cols, dst, ldd);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status convert_to_f64(const void* src, int bytes, int64_t count, double* dst,
                          hipStream_t st) {
  if (count <= 0) return TSK_OK;
  hipLaunchKernelGGL(k_to_f64, dim3(ceil_div(count, 256)), dim3(256), 0, st, src, bytes, count,
                     dst);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace tsk
