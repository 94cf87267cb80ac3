// Cross-lane sums inside one 64-lane wavefront of gfx950, on the vector ALU
// only (DPP row patterns and the lane-swap instructions), with no LDS round
// trip.  Every lane of a group ends with the same bits: each step adds a value
// and its partner's, and the two lanes of a pair add the same two numbers.
#pragma once

#include <hip/hip_runtime.h>

namespace tsk {

// DPP controls: quad_perm [1,0,3,2] (lane ^ 1), quad_perm [2,3,0,1] (lane ^ 2),
// row_half_mirror (i <-> 7 - i in each 8 lanes), row_mirror (i <-> 15 - i in
// each 16 lanes).
constexpr int kDppXor1 = 0xb1, kDppXor2 = 0x4e, kDppHalfMirror = 0x141, kDppMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp(int(b), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}

__device__ __forceinline__ double join64(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)lo | ((long long)hi << 32));
}

// Sum of a 16-lane row, in every lane of the row.
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp_mov<kDppXor1>(v);
  v += dpp_mov<kDppXor2>(v);
  v += dpp_mov<kDppHalfMirror>(v);
  v += dpp_mov<kDppMirror>(v);
  return v;
}

// Pairwise lane-half folds of two values a (kept by lanes 0-31) and b (kept by
// lanes 32-63): v_permlane32_swap exchanges the upper half of its first operand
// with the lower half of its second, so after the swap the sum of the two
// registers is a[l] + a[l+32] in the lower lanes and b[l-32] + b[l] in the upper.
__device__ __forceinline__ double fold32(double a, double b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap(unsigned(x), unsigned(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(unsigned(x >> 32), unsigned(y >> 32), false,
                                                  false);
  return join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
}

// Same for 16-lane rows: v_permlane16_swap exchanges the odd rows of the first
// operand with the even rows of the second, so rows 0 and 2 end with a's pair
// sums (row 0 + row 1, row 2 + row 3) and rows 1 and 3 with b's.
__device__ __forceinline__ double fold16(double a, double b) {
  const long long x = __double_as_longlong(a), y = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap(unsigned(x), unsigned(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(unsigned(x >> 32), unsigned(y >> 32), false,
                                                  false);
  return join64(lo[0], hi[0]) + join64(lo[1], hi[1]);
}

// Sum over the 64 lanes, in every lane.
__device__ __forceinline__ double wave_allsum(double v) {
  v = row_sum16(v);
  v = fold16(v, v);
  return fold32(v, v);
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane(unsigned(b), lane);
  const unsigned hi = __builtin_amdgcn_readlane(unsigned(b >> 32), lane);
  return join64(lo, hi);
}

// Wave sums of N values per lane (N a multiple of 4), returned as wave-uniform
// values: out[c] = sum over lanes of p[c].  Two folds halve the count each
// (lanes 0-31 keep p[0, N/2), and within each half the even rows keep the
// first half of what that half kept), a row sum finishes, and each value is
// read from the first lane of the row that holds it.
template <int N>
__device__ __forceinline__ void wave_sums(const double (&p)[N], double (&out)[N]) {
  static_assert(N % 4 == 0, "wave_sums needs a multiple of 4 values");
  constexpr int H = N / 2, Q = N / 4;
  double s[H], t[Q];
#pragma unroll
  for (int u = 0; u < H; ++u) s[u] = fold32(p[u], p[u + H]);
#pragma unroll
  for (int u = 0; u < Q; ++u) t[u] = row_sum16(fold16(s[u], s[u + Q]));
  // lane 32 h + 16 q holds value u + q Q + h H
#pragma unroll
  for (int u = 0; u < Q; ++u) {
    out[u] = read_lane(t[u], 0);
    out[u + Q] = read_lane(t[u], 16);
    out[u + H] = read_lane(t[u], 32);
    out[u + H + Q] = read_lane(t[u], 48);
  }
}

}  // namespace tsk
