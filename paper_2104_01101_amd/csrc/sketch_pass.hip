// Deterministic hash-and-sign scatter-add of a tensor unfolding:
//
//   Y_job[row(i), i_n] += sign(i) * T(i)      for every entry i of T,
//
// where (row, sign) is either the TensorSketch hash/sign of the other-mode
// indices, H = (sum_{k != n} h_k(i_k)) mod m and S = prod_{k != n} sigma_k(i_k)
// (Def. TensorSketch, eq. h_ts / s_ts) -- giving Y = S^(n) T_(n)^T -- or the
// CountSketch hash g and sign tau of the other-mode linear index (the first
// factor of the composite range-finder sketch, Sec. 5) -- giving
// (T_(n) Omega^T)^T.
//
// No floating-point atomics.  The output Y_job (rows x ncols, row-major) is cut
// into tiles of <= TC consecutive cells that fit in LDS.  Four kernels:
//   count    per chunk of entries, per tile: number of entries (LDS integer
//            histogram, exact)
//   scan     exclusive prefix over (tile, chunk) -> where each chunk's entries
//            of each tile go
//   scatter  stable partition of (16-bit fine cell, signed value) by tile;
//            inside a wavefront the lanes that hit the same tile are matched
//            with ballots over the tile id bits, and the four waves of a
//            workgroup claim their ranges in wave order once per batch, so the
//            partition keeps input order
//   accum    one single-wave workgroup per tile: zero the tile in LDS, add the
//            tile's entries in input order (lanes hitting the same cell are
//            matched by ballots over the cell bits and applied rank by rank),
//            write the whole tile (zeros included) once, coalesced.
// Every cell is therefore the left-to-right sum of its contributions in input
// order, independent of scheduling.

#include "common.h"
#include "kernels.h"

namespace tsk {

namespace {

constexpr int kBlock = 256;

struct Coords {
  int N;
  int layout;
  int dtype;
  int64_t dims[TSK_MAX_ORDER];
  const int32_t* idx[TSK_MAX_ORDER];
  const void* vals;
};

struct Job {
  int type;  // 0 TensorSketch, 1 range-finder CountSketch
  int col_mode;
  int tile_bits;
  int pad_;
  int64_t rows, ncols;
  const int32_t* h[TSK_MAX_ORDER];
  const int8_t* sg[TSK_MAX_ORDER];
  uint64_t key;
  int64_t rpt;   // rows per tile (ncols <= TC), else 0
  int64_t cbpr;  // column blocks per row (ncols > TC)
  int64_t ntiles;
  int64_t tile0;
  void* out;
  uint16_t* part_fine;
  void* part_val;
};

constexpr int kMaxJobs = 4;  // jobs per pass; more run as further passes

struct JobSet {
  int njobs;
  int fine_bits;
  int64_t tc;
  Job job[kMaxJobs];
};

__device__ inline void coords_of(const Coords& c, int64_t e, int32_t* i) {
  if (c.layout == TSK_COO) {
#pragma unroll
    for (int k = 0; k < TSK_MAX_ORDER; ++k)
      if (k < c.N) i[k] = c.idx[k][e];
  } else {
    int64_t r = e;
#pragma unroll
    for (int k = TSK_MAX_ORDER - 1; k >= 0; --k)
      if (k < c.N) {
        i[k] = int32_t(r % c.dims[k]);
        r /= c.dims[k];
      }
  }
}

__device__ inline int32_t pick(const int32_t* i, int k) {
  int32_t r = 0;
#pragma unroll
  for (int t = 0; t < TSK_MAX_ORDER; ++t)
    if (t == k) r = i[t];
  return r;
}

template <class T>
__device__ inline T value_of(const Coords& c, int64_t e) {
  return static_cast<const T*>(c.vals)[e];
}

// row and sign of an entry for a job
__device__ inline void row_sign(const Job& j, const Coords& c, const int32_t* i, int64_t& row,
                                int& sg) {
  if (j.type == 0) {
    int64_t H = 0;
    int s = 1;
#pragma unroll
    for (int k = 0; k < TSK_MAX_ORDER; ++k) {
      if (k >= c.N || k == j.col_mode) continue;
      H += j.h[k][i[k]];
      s *= j.sg[k][i[k]];
    }
    row = H % j.rows;
    sg = s;
  } else {
    int64_t lin = 0;
#pragma unroll
    for (int k = 0; k < TSK_MAX_ORDER; ++k) {
      if (k >= c.N || k == j.col_mode) continue;
      lin = lin * c.dims[k] + i[k];
    }
    uint64_t x = draw(j.key, uint64_t(lin));
    row = bucket_of(x, uint64_t(j.rows));
    sg = sign_of(x);
  }
}

__device__ inline void tile_of(const Job& j, int64_t tc, int64_t row, int64_t col, int& tile,
                               uint32_t& fine) {
  if (j.rpt > 0) {
    tile = int(row / j.rpt);
    fine = uint32_t((row % j.rpt) * j.ncols + col);
  } else {
    tile = int(row * j.cbpr + col / tc);
    fine = uint32_t(col % tc);
  }
}

__device__ inline void tile_range(const Job& j, int64_t tc, int64_t t, int64_t& start,
                                  int64_t& len) {
  if (j.rpt > 0) {
    start = t * j.rpt * j.ncols;
    int64_t r = j.rows - t * j.rpt;
    len = (r < j.rpt ? r : j.rpt) * j.ncols;
  } else {
    int64_t row = t / j.cbpr, cb = t % j.cbpr;
    start = row * j.ncols + cb * tc;
    int64_t l = j.ncols - cb * tc;
    len = l < tc ? l : tc;
  }
}

// lanes of this wave whose `key` equals mine, restricted to `active`
__device__ inline uint64_t match_lanes(uint32_t key, int bits, uint64_t active) {
  uint64_t m = active;
  for (int b = 0; b < bits; ++b) {
    bool bit = (key >> b) & 1u;
    uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

__device__ inline uint64_t lanemask_lt() {
  int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// --------------------------------------------------------------- count ----
// Per chunk, per tile: number of entries.  Each thread keeps four entries in
// flight; counting uses LDS integer atomics (exact, order-independent).
template <class T>
__global__ __launch_bounds__(kBlock) void k_count(Coords c, JobSet js, int64_t nnz,
                                                  int64_t chunk, int32_t* counts, int ttot) {
  extern __shared__ int hist[];
  for (int t = threadIdx.x; t < ttot; t += kBlock) hist[t] = 0;
  __syncthreads();
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < nnz ? lo + chunk : nnz;
  for (int64_t e0 = lo + threadIdx.x; e0 < hi; e0 += 4 * kBlock) {
    int32_t ii[4][TSK_MAX_ORDER];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (e0 + u * kBlock < hi) coords_of(c, e0 + u * kBlock, ii[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (e0 + u * kBlock >= hi) continue;
#pragma unroll
      for (int q = 0; q < kMaxJobs; ++q) {
        if (q >= js.njobs) continue;
        const Job& j = js.job[q];
        int64_t row;
        int sg;
        row_sign(j, c, ii[u], row, sg);
        int tile;
        uint32_t fine;
        tile_of(j, js.tc, row, pick(ii[u], j.col_mode), tile, fine);
        atomicAdd(&hist[j.tile0 + tile], 1);  // integer count: exact
      }
    }
  }
  __syncthreads();
  int32_t* out = counts + size_t(blockIdx.x) * ttot;
  for (int t = threadIdx.x; t < ttot; t += kBlock) out[t] = hist[t];
}

// ---------------------------------------------------------------- scan ----
// counts[c][t] -> exclusive prefix over chunks (in place); totals[t].  Eight
// threads per tile, each owning a contiguous range of chunks.
constexpr int kScanSeg = 8;
__global__ __launch_bounds__(256) void k_scan_chunks(int32_t* counts, int32_t* totals,
                                                     int nchunks, int ttot) {
  __shared__ int32_t segsum[256];
  const int tl = threadIdx.x / kScanSeg, sg = threadIdx.x % kScanSeg;
  const int t = blockIdx.x * (256 / kScanSeg) + tl;
  const int per = (nchunks + kScanSeg - 1) / kScanSeg;
  const int c0 = sg * per, c1 = c0 + per < nchunks ? c0 + per : nchunks;
  int32_t sum = 0;
  if (t < ttot)
    for (int cc = c0; cc < c1; ++cc) sum += counts[size_t(cc) * ttot + t];
  segsum[threadIdx.x] = sum;
  __syncthreads();
  int32_t run = 0;
  for (int q = 0; q < sg; ++q) run += segsum[tl * kScanSeg + q];
  if (t < ttot) {
    for (int cc = c0; cc < c1; ++cc) {
      const int32_t v = counts[size_t(cc) * ttot + t];
      counts[size_t(cc) * ttot + t] = run;
      run += v;
    }
    if (sg == kScanSeg - 1) totals[t] = run;
  }
}

// exclusive prefix of tile totals inside each job -> begin[t]; single block
__global__ void k_scan_tiles(const int32_t* totals, int32_t* begin, JobSet js) {
  __shared__ int32_t part[1024];
  for (int q = 0; q < js.njobs; ++q) {
    int64_t t0 = js.job[q].tile0, nt = js.job[q].ntiles;
    int32_t carry = 0;
    for (int64_t base = 0; base < nt; base += 1024) {
      int64_t t = base + threadIdx.x;
      int32_t v = t < nt ? totals[t0 + t] : 0;
      part[threadIdx.x] = v;
      __syncthreads();
      for (int off = 1; off < 1024; off <<= 1) {
        int32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
      }
      if (t < nt) begin[t0 + t] = carry + part[threadIdx.x] - v;
      int32_t blocksum = part[1023];
      __syncthreads();
      carry += blocksum;
    }
  }
}

// ------------------------------------------------------------- scatter ----
// Stable partition of (fine cell, signed value) by tile.  A batch is
// kBlock * kRounds consecutive entries; wave w owns the w-th quarter of the
// batch and hashes and ranks its kRounds rounds of 64 entries in parallel with
// the other waves; the ranges in the tiles are then claimed wave by wave (one
// barrier per wave per batch), which keeps input order inside every tile.
constexpr int kRounds = 4;
template <class T>
__global__ __launch_bounds__(kBlock) void k_scatter(Coords c, JobSet js, int64_t nnz,
                                                    int64_t chunk, const int32_t* offs,
                                                    const int32_t* begin, int ttot) {
  extern __shared__ int cursor[];
  const int32_t* my = offs + size_t(blockIdx.x) * ttot;
  for (int t = threadIdx.x; t < ttot; t += kBlock) cursor[t] = begin[t] + my[t];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t lo = blockIdx.x * chunk, hi = lo + chunk < nnz ? lo + chunk : nnz;
  for (int64_t b0 = lo; b0 < hi; b0 += kBlock * kRounds) {
    int gt[kRounds][kMaxJobs], rank[kRounds][kMaxJobs], cnt[kRounds][kMaxJobs],
        leader[kRounds][kMaxJobs];
    uint32_t fine[kRounds][kMaxJobs];
    bool neg[kRounds][kMaxJobs];
    bool valid[kRounds];
    T v[kRounds];
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int64_t e = b0 + (wave * kRounds + u) * 64 + lane;
      valid[u] = e < hi;
      int32_t ii[TSK_MAX_ORDER];
      v[u] = T(0);
      if (valid[u]) {
        coords_of(c, e, ii);
        v[u] = value_of<T>(c, e);
      }
      const uint64_t active = __ballot(valid[u]);
#pragma unroll
      for (int q = 0; q < kMaxJobs; ++q) {
        if (q >= js.njobs) continue;
        const Job& j = js.job[q];
        int tile = 0, sgn = 1;
        uint32_t f = 0;
        if (valid[u]) {
          int64_t row;
          row_sign(j, c, ii, row, sgn);
          tile_of(j, js.tc, row, pick(ii, j.col_mode), tile, f);
        }
        const uint64_t mt = match_lanes(uint32_t(tile), j.tile_bits, active);
        gt[u][q] = int(j.tile0) + tile;
        fine[u][q] = f;
        neg[u][q] = sgn < 0;
        rank[u][q] = __popcll(mt & lanemask_lt());
        cnt[u][q] = __popcll(mt);
        leader[u][q] = valid[u] ? __ffsll((unsigned long long)mt) - 1 : lane;
      }
    }
    __syncthreads();  // cursors initialised / previous batch claimed
    for (int w = 0; w < kBlock / 64; ++w) {
      if (wave == w) {
#pragma unroll
        for (int u = 0; u < kRounds; ++u)
#pragma unroll
          for (int q = 0; q < kMaxJobs; ++q) {
            if (q >= js.njobs) continue;
            const Job& j = js.job[q];
            int base = 0;
            if (valid[u] && rank[u][q] == 0) {
              base = cursor[gt[u][q]];
              cursor[gt[u][q]] = base + cnt[u][q];
            }
            base = __shfl(base, leader[u][q]);
            if (valid[u]) {
              const int pos = base + rank[u][q];
              j.part_fine[pos] = uint16_t(fine[u][q]);
              static_cast<T*>(j.part_val)[pos] = neg[u][q] ? -v[u] : v[u];
            }
          }
      }
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------- accum ----
// One single-wave workgroup per tile: no barriers.  Rounds of 64 consecutive
// entries of the tile (input order); lanes that hit the same cell are matched
// with ballots over the cell bits and applied rank by rank, so every cell is
// the in-order sum of its entries.  The tile is then written once, coalesced.
template <class T>
__global__ __launch_bounds__(64) void k_accum(JobSet js, const int32_t* begin,
                                              const int32_t* totals, int ttot) {
  extern __shared__ unsigned char smem_raw[];
  T* tile = reinterpret_cast<T*>(smem_raw);
  const int gt = blockIdx.x;
  int q = 0;
  while (q + 1 < js.njobs && gt >= js.job[q + 1].tile0) ++q;
  const Job& j = js.job[q];
  const int64_t t = gt - j.tile0;
  int64_t start, len;
  tile_range(j, js.tc, t, start, len);
  const int lane = threadIdx.x;
  for (int i = lane; i < len; i += 64) tile[i] = T(0);
  const int32_t b = begin[gt], n = totals[gt];
  const uint16_t* pf = j.part_fine + b;
  const T* pv = static_cast<const T*>(j.part_val) + b;
  for (int32_t r0 = 0; r0 < n; r0 += 64 * kRounds) {
    uint32_t f[kRounds];
    T v[kRounds];
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {  // loads first
      const int32_t e = r0 + u * 64 + lane;
      f[u] = e < n ? uint32_t(pf[e]) : 0u;
      v[u] = e < n ? pv[e] : T(0);
    }
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int32_t e = r0 + u * 64 + lane;
      const bool valid = e < n;
      const uint64_t active = __ballot(valid);
      if (active == 0ull) break;
      const uint64_t mt = match_lanes(f[u], js.fine_bits, active);
      const int rank = valid ? __popcll(mt & lanemask_lt()) : 64;
      for (int k = 0; __ballot(rank == k) != 0ull; ++k)
        if (rank == k) tile[f[u]] += v[u];
    }
  }
  T* out = static_cast<T*>(j.out) + start;
  for (int i = lane; i < len; i += 64) out[i] = tile[i];
}

int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

}  // namespace

// One pass over the entries for a group of jobs whose tiles fit the LDS
// histogram.  `specs` describe the jobs; outputs are overwritten.
tsk_status sketch_pass(const TensorView& T, const PassJob* specs, int njobs, Ws& ws,
                       hipStream_t st) {
  const int64_t nnz = T.nnz;
  const bool f64 = T.dtype == TSK_F64;
  const int64_t tc = f64 ? 4096 : 8192;  // 32 KiB of LDS per tile; cell index fits 16 bits
  const int kMaxTiles = 16384;            // 64 KiB LDS histogram / cursors

  Coords c{};
  c.N = T.order;
  c.layout = T.layout;
  c.dtype = T.dtype;
  for (int k = 0; k < T.order; ++k) {
    c.dims[k] = T.dims[k];
    c.idx[k] = T.idx[k];
  }
  c.vals = T.values;

  // group jobs so that each group's tiles fit; groups run one after the other
  // on the stream and reuse the same scratch
  const size_t mark = ws.off;
  size_t peak = mark;
  int g0 = 0;
  while (g0 < njobs) {
    ws.off = mark;
    JobSet js{};
    js.tc = tc;
    js.fine_bits = bits_for(tc);
    int64_t ttot = 0;
    int q = g0;
    for (; q < njobs; ++q) {
      const PassJob& p = specs[q];
      Job j{};
      j.type = p.type;
      j.col_mode = p.col_mode;
      j.rows = p.rows;
      j.ncols = T.dims[p.col_mode];
      for (int k = 0; k < T.order; ++k) {
        j.h[k] = p.h ? p.h[k] : nullptr;
        j.sg[k] = p.sg ? p.sg[k] : nullptr;
      }
      j.key = p.key;
      if (j.ncols <= tc) {
        j.rpt = tc / j.ncols;
        j.cbpr = 0;
        j.ntiles = ceil_div(j.rows, j.rpt);
      } else {
        j.rpt = 0;
        j.cbpr = ceil_div(j.ncols, tc);
        j.ntiles = j.rows * j.cbpr;
      }
      if (j.ntiles > kMaxTiles) {
        set_error("sketch output of %lld x %lld cells exceeds the tile budget",
                  (long long)j.rows, (long long)j.ncols);
        return TSK_EUNSUPPORTED;
      }
      if (ttot + j.ntiles > kMaxTiles || js.njobs == kMaxJobs) break;
      j.tile_bits = bits_for(j.ntiles);
      j.tile0 = ttot;
      j.out = p.out;
      ttot += j.ntiles;
      js.job[js.njobs++] = j;
    }
    // chunks of the entry stream: about two per compute unit, whole batches
    int64_t nchunks = ceil_div(nnz, kBlock * kRounds);
    if (nchunks > 512) nchunks = 512;
    if (nchunks < 1) nchunks = 1;
    int64_t chunk = ceil_div(nnz, nchunks);
    chunk = ceil_div(chunk, kBlock * kRounds) * kBlock * kRounds;
    nchunks = nnz > 0 ? ceil_div(nnz, chunk) : 1;

    int32_t* counts = ws.take<int32_t>(size_t(nchunks) * ttot);
    int32_t* totals = ws.take<int32_t>(ttot);
    int32_t* begin = ws.take<int32_t>(ttot);
    for (int k = 0; k < js.njobs; ++k) {
      js.job[k].part_fine = ws.take<uint16_t>(nnz);
      js.job[k].part_val = f64 ? (void*)ws.take<double>(nnz) : (void*)ws.take<float>(nnz);
    }
    if (!ws.measuring()) {
      size_t hist_bytes = size_t(ttot) * sizeof(int32_t);
      size_t tile_bytes = size_t(tc) * (f64 ? 8 : 4);
      if (nnz > 0) {
        if (f64)
          hipLaunchKernelGGL(k_count<double>, dim3(nchunks), dim3(kBlock), hist_bytes, st, c, js,
                             nnz, chunk, counts, int(ttot));
        else
          hipLaunchKernelGGL(k_count<float>, dim3(nchunks), dim3(kBlock), hist_bytes, st, c, js,
                             nnz, chunk, counts, int(ttot));
        TSK_LAUNCHED();
        hipLaunchKernelGGL(k_scan_chunks, dim3(ceil_div(ttot, 256 / kScanSeg)), dim3(256), 0, st,
                           counts, totals, int(nchunks), int(ttot));
        TSK_LAUNCHED();
      } else {
        TSK_HIP(hipMemsetAsync(totals, 0, size_t(ttot) * 4, st));
      }
      hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, st, totals, begin, js);
      TSK_LAUNCHED();
      if (nnz > 0) {
        if (f64)
          hipLaunchKernelGGL(k_scatter<double>, dim3(nchunks), dim3(kBlock), hist_bytes, st, c,
                             js, nnz, chunk, counts, begin, int(ttot));
        else
          hipLaunchKernelGGL(k_scatter<float>, dim3(nchunks), dim3(kBlock), hist_bytes, st, c,
                             js, nnz, chunk, counts, begin, int(ttot));
        TSK_LAUNCHED();
      }
      if (f64)
        hipLaunchKernelGGL(k_accum<double>, dim3(ttot), dim3(64), tile_bytes, st, js, begin,
                           totals, int(ttot));
      else
        hipLaunchKernelGGL(k_accum<float>, dim3(ttot), dim3(64), tile_bytes, st, js, begin,
                           totals, int(ttot));
      TSK_LAUNCHED();
    }
    g0 = q;
    peak = std::max(peak, ws.off);
  }
  ws.off = peak;
  return TSK_OK;
}

}  // namespace tsk
