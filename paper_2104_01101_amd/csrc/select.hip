// Deterministic leverage selection (Sec. 3.2: keep the rows of largest
// leverage score instead of drawing them; no rescaling, every weight 1).
//
// Rows of kron_{k != n} A^(k) are multi-indices (i_k); by the Lemma on
// Kronecker leverage scores a row's score is pi = prod_k l^(k)_{i_k}, the
// product taken in increasing k.  Order: pi descending, then the per-mode
// ranks (position in score-descending, index-ascending order) compared
// lexicographically; the first m rows are kept, in that order.
//
// Candidates.  pi is monotone in every factor, and equal pi falls back to the
// rank order, so every row whose ranks are componentwise <= those of a row t
// comes before t.  A kept row therefore has prod_k (rank_k + 1) <= m: only the
// rank tuples under that bound (with rank_k < min(s_k, m)) are candidates,
// about m ln m of them for three modes instead of prod_k s_k.  The candidate
// set depends only on m and the dimensions, so it is enumerated once per job,
// in lexicographic order of the rank tuples.
//
// Per subproblem: scores of every mode; ranks by counting (each row counts
// the rows before it in the rank order, no sort); candidate products from the
// rank-sorted scores; a stable descending radix sort of (pi bits, candidate
// id) -- stability keeps the lexicographic order among equal pi; the first m
// candidates are mapped back to row indices.

#include <rocprim/device/device_radix_sort.hpp>

#include "common.h"
#include "select.h"

namespace tsk {

namespace {

constexpr int kSelThreads = 256;
constexpr int kSelTile = 2048;  // scores staged per LDS tile of the rank count

// Candidates of levels q0..nm-1 under the product bound M0: rank tuples with
// r_q < cap[q] and prod (r_q + 1) <= M0, counted by walking them in the same
// lexicographic order as the enumeration below (whole last-level ranges at once).
__host__ __device__ int64_t count_from(const int64_t* cap, int nm, int q0, int64_t M0) {
  if (q0 == nm - 1) return cap[q0] < M0 ? cap[q0] : M0;
  int64_t r[TSK_MAX_ORDER], bound[TSK_MAX_ORDER + 1];
  int q = q0;
  bound[q0] = M0;
  r[q0] = 0;
  int64_t total = 0;
  while (true) {
    if (q < nm - 1) {
      const int64_t top = cap[q] < bound[q] ? cap[q] : bound[q];
      if (r[q] < top) {
        bound[q + 1] = bound[q] / (r[q] + 1);
        ++q;
        r[q] = 0;
        continue;
      }
      if (q == q0) break;
      --q;
      ++r[q];
      continue;
    }
    total += cap[q] < bound[q] ? cap[q] : bound[q];
    --q;
    ++r[q];
  }
  return total;
}

struct SelModes {
  int nm;
  int64_t s[TSK_MAX_ORDER];
  int64_t R[TSK_MAX_ORDER];
  int64_t cap[TSK_MAX_ORDER];  // min(s_k, m)
  const double* A[TSK_MAX_ORDER];
  double* ell[TSK_MAX_ORDER];    // scores
  double* sorted[TSK_MAX_ORDER];  // scores in rank order
  int32_t* order[TSK_MAX_ORDER];  // row index of every rank
};

// Block sizes of the first level: cnt[r1] candidates start with rank r1.
__global__ void k_sel_count(SelModes sm, int64_t m, int64_t* cnt) {
  const int64_t r1 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t n1 = sm.cap[0] < m ? sm.cap[0] : m;
  if (r1 >= n1) return;
  cnt[r1] = sm.nm == 1 ? 1 : count_from(sm.cap, sm.nm, 1, m / (r1 + 1));
}

// Exclusive prefix sum of cnt[0, n) into off[0, n] by one workgroup (each
// thread sums a contiguous stretch; the stretch totals are scanned in LDS).
__global__ __launch_bounds__(kSelThreads) void k_sel_scan(const int64_t* cnt, int64_t n,
                                                          int64_t* off) {
  __shared__ int64_t part[kSelThreads];
  const int t = threadIdx.x;
  const int64_t per = (n + kSelThreads - 1) / kSelThreads;
  const int64_t b = t * per, e = b + per < n ? b + per : n;
  int64_t s = 0;
  for (int64_t i = b; i < e; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int u = 0; u < kSelThreads; ++u) {
      const int64_t v = part[u];
      part[u] = run;
      run += v;
    }
    off[n] = run;
  }
  __syncthreads();
  int64_t run = part[t];
  for (int64_t i = b; i < e; ++i) {
    off[i] = run;
    run += cnt[i];
  }
}

// One workgroup per first-level rank r1: the prefixes of the middle levels are
// walked in lexicographic order (uniformly by the whole workgroup) and the
// last level's contiguous rank range is written in parallel.
__global__ __launch_bounds__(kSelThreads) void k_sel_enumerate(SelModes sm, int64_t m,
                                                               const int64_t* off,
                                                               int32_t* tup) {
  const int64_t r1 = blockIdx.x;
  const int nm = sm.nm;
  int64_t pos = off[r1];
  if (nm == 1) {
    if (threadIdx.x == 0) tup[pos] = int32_t(r1);
    return;
  }
  // prefix ranks of levels 1..nm-2 and the bound left for the next level
  int64_t r[TSK_MAX_ORDER], bound[TSK_MAX_ORDER + 1];
  bound[1] = m / (r1 + 1);
  int q = 1;
  for (int k = 1; k < nm; ++k) r[k] = 0;
  while (true) {
    if (q < nm - 1) {
      // descend: level q takes rank r[q] if it fits, else back up
      const int64_t top = sm.cap[q] < bound[q] ? sm.cap[q] : bound[q];
      if (r[q] < top) {
        bound[q + 1] = bound[q] / (r[q] + 1);
        ++q;
        r[q] = 0;
        continue;
      }
      if (q == 1) break;
      --q;
      ++r[q];
      continue;
    }
    // last level: ranks [0, L) after the prefix (r1, r[1..nm-2])
    const int64_t L = sm.cap[q] < bound[q] ? sm.cap[q] : bound[q];
    for (int64_t t = threadIdx.x; t < L; t += kSelThreads) {
      int32_t* row = tup + (pos + t) * nm;
      row[0] = int32_t(r1);
      for (int k = 1; k < nm - 1; ++k) row[k] = int32_t(r[k]);
      row[nm - 1] = int32_t(t);
    }
    pos += L;
    if (q == 1) break;
    --q;
    ++r[q];
  }
}

__global__ void k_sel_scores(SelModes sm) {
  const int q = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= sm.nm || i >= sm.s[q]) return;
  const double* a = sm.A[q] + i * sm.R[q];
  double acc = 0.0;
  for (int64_t c = 0; c < sm.R[q]; ++c) acc = __dadd_rn(acc, __dmul_rn(a[c], a[c]));
  sm.ell[q][i] = acc;
}

// rank(i) = #{j : l_j > l_i} + #{j < i : l_j == l_i}.  A workgroup takes 64
// rows; its four waves count over interleaved quarters of the j range, and the
// partial counts are added in LDS.  Scores are >= 0, so their bit patterns
// compare as unsigned integers.
constexpr int kSelRows = 64;
__global__ __launch_bounds__(kSelThreads) void k_sel_rank(SelModes sm) {
  __shared__ uint64_t tile[kSelTile];
  __shared__ int32_t part[kSelThreads / 64][kSelRows];
  const int q = blockIdx.y;
  const int64_t s = sm.s[q];
  if (int64_t(blockIdx.x) * kSelRows >= s) return;  // uniform per workgroup
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = int64_t(blockIdx.x) * kSelRows + lane;
  const uint64_t* ell = reinterpret_cast<const uint64_t*>(sm.ell[q]);
  const uint64_t li = i < s ? ell[i] : 0;
  int32_t rank = 0;
  for (int64_t j0 = 0; j0 < s; j0 += kSelTile) {
    const int tw = int(s - j0 < kSelTile ? s - j0 : kSelTile);
    __syncthreads();
    for (int t = threadIdx.x; t < tw; t += kSelThreads) tile[t] = ell[j0 + t];
    __syncthreads();
    const int64_t ir = i - j0;  // rows j < i in this tile: t < ir
#pragma unroll 8
    for (int t = wave; t < tw; t += kSelThreads / 64) {
      const uint64_t lj = tile[t];
      rank += (lj > li) | ((lj == li) & (t < ir));
    }
  }
  part[wave][lane] = rank;
  __syncthreads();
  if (wave == 0 && i < s) {
    const int32_t r = part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane];
    sm.order[q][r] = int32_t(i);
    sm.sorted[q][r] = __longlong_as_double(static_cast<long long>(li));
  }
}

__global__ void k_sel_products(SelModes sm, int64_t ncand, const int32_t* tup, uint64_t* key,
                               int32_t* val) {
  const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncand) return;
  const int32_t* t = tup + c * sm.nm;
  double pi = sm.sorted[0][t[0]];
  for (int q = 1; q < sm.nm; ++q) pi = __dmul_rn(pi, sm.sorted[q][t[q]]);
  key[c] = uint64_t(__double_as_longlong(pi));
  val[c] = int32_t(c);
}

__global__ void k_sel_emit(SelModes sm, int64_t m, const int32_t* tup, const int32_t* best,
                           int32_t* idx, double* w) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int32_t* t = tup + int64_t(best[j]) * sm.nm;
  for (int q = 0; q < sm.nm; ++q) idx[j * sm.nm + q] = sm.order[q][t[q]];
  if (w) w[j] = 1.0;
}

SelModes modes_of(int N, const int64_t* dims, const int64_t* ranks, int n, int64_t m,
                  const double* const* factors) {
  SelModes sm{};
  for (int k = 0; k < N; ++k) {
    if (k == n) continue;
    const int q = sm.nm++;
    sm.s[q] = dims[k];
    sm.R[q] = ranks ? ranks[k] : 0;
    sm.cap[q] = dims[k] < m ? dims[k] : m;
    sm.A[q] = factors ? factors[k] : nullptr;
  }
  return sm;
}

}  // namespace

tsk_status select_plan(int N, const int64_t* dims, int n, int64_t m, SelectPlan& p, Ws& ws,
                       hipStream_t st) {
  SelModes sm = modes_of(N, dims, nullptr, n, m, nullptr);
  double rows = 1.0;
  for (int q = 0; q < sm.nm; ++q) rows *= double(sm.s[q]);
  TSK_REQUIRE(m >= 1 && double(m) <= rows,
              "deterministic selection of m = %lld rows from %.0f rows of the Kronecker chain",
              (long long)m, rows);
  p.nm = sm.nm;
  p.m = m;
  p.ncand = count_from(sm.cap, sm.nm, 0, m);
  TSK_REQUIRE(p.ncand >= m && p.ncand < (int64_t(1) << 31),
              "selection candidates %lld outside [m, 2^31)", (long long)p.ncand);
  p.tup = ws.take<int32_t>(size_t(p.ncand) * sm.nm);
  const int64_t n1 = sm.cap[0] < m ? sm.cap[0] : m;
  int64_t* cnt = ws.take<int64_t>(n1);
  int64_t* off = ws.take<int64_t>(n1 + 1);
  if (ws.measuring()) return TSK_OK;
  hipLaunchKernelGGL(k_sel_count, dim3(unsigned(ceil_div(n1, 256))), dim3(256), 0, st, sm, m,
                     cnt);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_sel_scan, dim3(1), dim3(kSelThreads), 0, st, cnt, n1, off);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_sel_enumerate, dim3(unsigned(n1)), dim3(kSelThreads), 0, st, sm, m, off,
                     p.tup);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status select_rows(int N, const int64_t* dims, const int64_t* ranks, int n,
                       const SelectPlan& p, const double* const* factors, int32_t* idx,
                       double* w, Ws& ws, hipStream_t st) {
  SelModes sm = modes_of(N, dims, ranks, n, p.m, factors);
  int64_t smax = 0;
  for (int q = 0; q < sm.nm; ++q) {
    sm.ell[q] = ws.take<double>(sm.s[q]);
    sm.sorted[q] = ws.take<double>(sm.s[q]);
    sm.order[q] = ws.take<int32_t>(sm.s[q]);
    smax = sm.s[q] > smax ? sm.s[q] : smax;
  }
  uint64_t* kin = ws.take<uint64_t>(p.ncand);
  uint64_t* kout = ws.take<uint64_t>(p.ncand);
  int32_t* vin = ws.take<int32_t>(p.ncand);
  int32_t* vout = ws.take<int32_t>(p.ncand);
  size_t tbytes = 0;
  TSK_HIP(rocprim::radix_sort_pairs_desc(nullptr, tbytes, kin, kout, vin, vout,
                                         uint32_t(p.ncand), 0u, 63u, st));
  void* tmp = ws.take<char>(tbytes);
  if (ws.measuring()) return TSK_OK;
  ProfScope prof("select", st);
  hipLaunchKernelGGL(k_sel_scores, dim3(unsigned(ceil_div(smax, 256)), sm.nm), dim3(256), 0, st,
                     sm);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_sel_rank, dim3(unsigned(ceil_div(smax, kSelRows)), sm.nm),
                     dim3(kSelThreads), 0, st, sm);
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_sel_products, dim3(unsigned(ceil_div(p.ncand, 256))), dim3(256), 0, st,
                     sm, p.ncand, p.tup, kin, vin);
  TSK_LAUNCHED();
  TSK_HIP(rocprim::radix_sort_pairs_desc(tmp, tbytes, kin, kout, vin, vout, uint32_t(p.ncand),
                                         0u, 63u, st));
  hipLaunchKernelGGL(k_sel_emit, dim3(unsigned(ceil_div(p.m, 256))), dim3(256), 0, st, sm, p.m,
                     p.tup, vout, idx, w);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace tsk
