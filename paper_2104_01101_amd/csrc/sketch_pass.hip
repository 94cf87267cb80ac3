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
// No atomics on values.  The output Y_job (rows x ncols, row-major) is cut
// into bins of TC consecutive cells (8, 16 or 32 KiB, one LDS tile).  Three kernels:
//
//   partition  one workgroup per chunk of E consecutive entries.  The chunk is
//              read once (coalesced) and kept in registers; for every job the
//              workgroup hashes it (hash tables staged in LDS), stable-sorts
//              the (cell-in-bin, signed value) records by bin in LDS -- wave w
//              owns a contiguous E/8 slice, counts per (wave, bin), one block
//              scan, then every wave places its slice in order -- and writes
//              the sorted chunk contiguously, plus the bin offsets inside the
//              chunk.
//   transpose  the [chunk][bin] offset table becomes [bin][chunk], so a bin
//              reads the start of its run in every chunk contiguously.
//   tiles      four consecutive bins per workgroup (one wave each, so the
//              four waves share L1 lines of neighbouring runs), consecutive
//              workgroups of one XCD on consecutive bins.  A wave walks its
//              bin's runs in chunk order, 64 chunks per window (lane -> run by
//              binary search over the window's prefix), adds each record to
//              its LDS tile in sequence (lanes hitting the same cell are
//              matched with ballots and applied rank by rank), then writes the
//              whole tile once, zeros included.
//
// Every cell is therefore the left-to-right sum of its contributions in input
// order, independent of scheduling.

#include "common.h"
#include "kernels.h"

#include <algorithm>
#include <vector>

namespace tsk {

namespace {

constexpr int kWaves = 8;              // partition: 512 threads
constexpr int kMaxJobs = 4;            // jobs per pass; more run as further passes
constexpr int kLds = 160 * 1024;       // LDS per workgroup
constexpr int kTileMax = 32 * 1024;  // largest bin (one LDS tile); 8 and 16 KiB also built

struct Coords {
  int N;
  int layout;
  int64_t dims[TSK_MAX_ORDER];
  const int32_t* idx[TSK_MAX_ORDER];
  const void* vals;
};

struct Job {
  int type;      // 0 TensorSketch, 1 range-finder CountSketch
  int col_mode;
  int bin_bits;  // bits of a bin index inside the slab
  int tab_lds;   // TensorSketch tables staged in LDS (packed 15-bit hash + sign)
  int64_t rows, ncols, cells;
  const int32_t* h[TSK_MAX_ORDER];
  const int8_t* sg[TSK_MAX_ORDER];
  int32_t tab_off[TSK_MAX_ORDER];  // LDS offset of mode k's packed table
  int32_t tab_len;                 // packed table entries in LDS
  int32_t pad_;
  uint16_t* ptab;                  // packed tables in global memory (16-byte padded)
  uint64_t key;
  int64_t bin_lo;  // first bin of this slab of the output
  int32_t nbins;   // bins of this slab
  int32_t bin0;    // first bin of this job among the group's bins
  void* out;
  uint16_t* rec_fine;  // [nchunks * E] cell inside the bin
  void* rec_val;       // [nchunks * E] signed value
  uint16_t* meta;      // [nchunks][nbins + 1] run starts inside each chunk
  uint16_t* meta_t;    // [nbins + 1][nchp]
};

struct JobSet {
  int njobs;
  int tc_bits;
  int bmax;     // LDS cursor rows are bmax wide
  int tab_max;  // packed table entries reserved in LDS
  int nchunks;
  int nchp;     // row stride of meta_t: nchunks rounded up to 8
  int btot;     // bins over all jobs
  Job job[kMaxJobs];
};

template <int NC>
__device__ inline void coords_of(const Coords& c, int64_t e, int32_t* i) {
  if (c.layout == TSK_COO) {
#pragma unroll
    for (int k = 0; k < NC; ++k)
      if (k < c.N) i[k] = c.idx[k][e];
  } else {
    int64_t r = e;
#pragma unroll
    for (int k = NC - 1; k >= 0; --k)
      if (k < c.N) {
        i[k] = int32_t(r % c.dims[k]);
        r /= c.dims[k];
      }
  }
}

template <int NC>
__device__ inline int32_t pick(const int32_t* i, int k) {
  int32_t r = 0;
#pragma unroll
  for (int t = 0; t < NC; ++t)
    if (t == k) r = i[t];
  return r;
}

// A job's fields held in registers for the partition loops.
template <int NC>
struct JobRegs {
  int col_mode;
  int bin_bits;
  int nbins;
  int64_t rows, ncols, bin_lo;
  uint64_t key;
  int32_t tab_off[NC];
  const int32_t* h[NC];
  const int8_t* sg[NC];
};

template <int NC>
__device__ inline JobRegs<NC> job_regs(const Job& j) {
  JobRegs<NC> r;
  r.col_mode = j.col_mode;
  r.bin_bits = j.bin_bits;
  r.nbins = j.nbins;
  r.rows = j.rows;
  r.ncols = j.ncols;
  r.bin_lo = j.bin_lo;
  r.key = j.key;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    r.tab_off[k] = j.tab_off[k];
    r.h[k] = j.h[k];
    r.sg[k] = j.sg[k];
  }
  return r;
}

// row and sign of an entry for a job: PATH 0 TensorSketch with LDS tables,
// 1 TensorSketch with global tables, 2 range-finder CountSketch
template <int NC, int PATH>
__device__ inline void row_sign(const JobRegs<NC>& j, int N, const int64_t* dims,
                                const int32_t* i, const uint16_t* tab, int64_t& row, bool& neg) {
  if (PATH != 2) {
    int64_t H = 0;
    bool ng = false;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (k >= N || k == j.col_mode) continue;
      if (PATH == 0) {
        const uint32_t p = tab[j.tab_off[k] + i[k]];
        H += p & 0x7fffu;
        ng ^= (p >> 15) != 0;
      } else {
        H += j.h[k][i[k]];
        ng ^= j.sg[k][i[k]] < 0;
      }
    }
#pragma unroll
    for (int k = 0; k < NC - 1; ++k)
      if (H >= j.rows) H -= j.rows;  // H < (N-1) m
    row = H;
    neg = ng;
  } else {
    int64_t lin = 0;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
      if (k >= N || k == j.col_mode) continue;
      lin = lin * dims[k] + i[k];
    }
    const uint64_t x = draw(j.key, uint64_t(lin));
    row = int64_t(bucket_of(x, uint64_t(j.rows)));
    neg = sign_of(x) < 0;
  }
}

// lanes of this wave whose `key` equals mine, restricted to `active`
__device__ inline uint64_t match_lanes(uint32_t key, int bits, uint64_t active) {
  uint64_t m = active;
  for (int b = 0; b < bits; ++b) {
    const bool bit = (key >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

// same, with at most MAXB key bits (unrolled; bits beyond `bits` skipped)
template <int MAXB>
__device__ inline uint64_t match_lanes_n(uint32_t key, int bits, uint64_t active) {
  uint64_t m = active;
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    if (b >= bits) break;
    const bool bit = (key >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

__device__ inline uint64_t lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

constexpr uint32_t kSkip = 0xffffffffu;

// packed bin / sign / cell-in-bin of every round's entry for one job
template <int NC, int RW, int PATH>
__device__ inline void hash_rounds(const JobRegs<NC>& j, int N, const int64_t* dims,
                                   const int32_t (*ii)[NC], const uint16_t* tab, int tc_bits,
                                   uint32_t* pk) {
  const uint32_t cmask = (1u << tc_bits) - 1u;
#pragma unroll
  for (int u = 0; u < RW; ++u) {
    pk[u] = kSkip;
    if (ii[u][0] < 0) continue;
    int64_t row;
    bool neg;
    row_sign<NC, PATH>(j, N, dims, ii[u], tab, row, neg);
    const int64_t cell = row * j.ncols + pick<NC>(ii[u], j.col_mode);
    const int64_t bin = (cell >> tc_bits) - j.bin_lo;
    if (bin >= 0 && bin < j.nbins)
      pk[u] = (uint32_t(bin) << 16) | (neg ? 0x8000u : 0u) | (uint32_t(cell) & cmask);
  }
}

// ----------------------------------------------------------- partition ----
// Cursors are 16-bit counters packed in pairs into 32-bit LDS words, so that
// integer LDS atomics can update them: counts use atomic adds (exact, order
// independent); placement uses one atomic add with return per (round, bin) by
// the round's first lane of that bin -- a wave owns its cursor row and LDS
// executes one wave's operations in order, so the claimed ranges follow the
// input order.
__device__ inline uint32_t cursor_add(uint32_t* row, uint32_t bin, uint32_t n) {
  const uint32_t sh = (bin & 1u) * 16u;
  return (atomicAdd(row + (bin >> 1), n << sh) >> sh) & 0xffffu;
}

template <class T, int NC, int RW, int PATH>
__global__ __launch_bounds__(512) void k_partition(Coords c, JobSet js, int64_t nnz) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int E = 512 * RW;
  T* s_val = reinterpret_cast<T*>(lds);
  uint16_t* s_fine = reinterpret_cast<uint16_t*>(lds + size_t(E) * sizeof(T));
  const int bw = (js.bmax + 1) >> 1;  // 32-bit words per cursor row
  uint32_t* cur = reinterpret_cast<uint32_t*>(s_fine + E);
  uint16_t* tab = reinterpret_cast<uint16_t*>(cur + kWaves * bw);
  int32_t* scr = reinterpret_cast<int32_t*>(tab + ((js.tab_max + 7) & ~7));
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t chunk = blockIdx.x;
  const int64_t ebase = chunk * E + wave * (RW * 64) + lane;
  const int N = c.N;
  int64_t dims[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) dims[k] = k < N ? c.dims[k] : 1;

  int32_t ii[RW][NC];
  T v[RW];
#pragma unroll
  for (int u = 0; u < RW; ++u) {  // all loads issued before any use
    const int64_t e = ebase + u * 64;
    v[u] = T(0);
    ii[u][0] = -1;
    if (e < nnz) {
      coords_of<NC>(c, e, ii[u]);
      v[u] = static_cast<const T*>(c.vals)[e];
    }
  }
  const int njobs = js.njobs, tc_bits = js.tc_bits;
  for (int q = 0; q < njobs; ++q) {
    const JobRegs<NC> j = job_regs<NC>(js.job[q]);
    if (PATH == 0) {  // packed tables: 16-byte copies
      const uint4* src = reinterpret_cast<const uint4*>(js.job[q].ptab);
      uint4* dst = reinterpret_cast<uint4*>(tab);
      const int n16 = (js.job[q].tab_len + 7) >> 3;
#pragma unroll 4
      for (int i = tid; i < n16; i += 512) dst[i] = src[i];
    }
    uint32_t* mycur = cur + wave * bw;
    const int nw = (j.nbins + 1) >> 1;
    for (int b = lane; b < nw; b += 64) mycur[b] = 0;
    __syncthreads();

    // hash and count per (wave, bin)
    uint32_t pk[RW];  // bin << 16 | negative << 15 | cell in bin
    hash_rounds<NC, RW, PATH>(j, N, dims, ii, tab, tc_bits, pk);
#pragma unroll
    for (int u = 0; u < RW; ++u)
      if (pk[u] != kSkip) {
        const uint32_t bin = pk[u] >> 16;
        atomicAdd(mycur + (bin >> 1), 1u << ((bin & 1u) * 16u));
      }
    __syncthreads();

    // scan: cursor(w, b) = start of bin b + entries of bin b in waves < w
    {
      const uint16_t* c16 = reinterpret_cast<const uint16_t*>(cur);
      uint16_t* w16 = reinterpret_cast<uint16_t*>(cur);
      const int rs = 2 * bw;  // u16 row stride
      const int G = (j.nbins + 511) / 512;
      const int b0 = tid * G;
      int32_t tsum = 0;
      for (int g = 0; g < G; ++g) {
        const int b = b0 + g;
        if (b < j.nbins)
#pragma unroll
          for (int w = 0; w < kWaves; ++w) tsum += c16[w * rs + b];
      }
      int32_t incl = tsum;
      for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
      }
      if (lane == 63) scr[wave] = incl;
      __syncthreads();
      int32_t run = incl - tsum;
      for (int w = 0; w < wave; ++w) run += scr[w];
      uint16_t* meta = js.job[q].meta + chunk * (j.nbins + 1);
      for (int g = 0; g < G; ++g) {
        const int b = b0 + g;
        if (b >= j.nbins) break;
        meta[b] = uint16_t(run);
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
          const int32_t t = c16[w * rs + b];
          w16[w * rs + b] = uint16_t(run);
          run += t;
        }
      }
      if (b0 < j.nbins && b0 + G >= j.nbins) {
        meta[j.nbins] = uint16_t(run);
        scr[kWaves] = run;
      }
    }
    __syncthreads();

    // stable placement: claims for all rounds first, then the stores
    uint32_t rk[RW];  // rank | leader << 8, or kSkip
#pragma unroll
    for (int u = 0; u < RW; ++u) {
      const bool valid = pk[u] != kSkip;
      const uint64_t act = __ballot(valid);
      const uint64_t mt = match_lanes_n<16>(pk[u] >> 16, j.bin_bits, act);
      const uint32_t rank = __popcll(mt & lanemask_lt(lane));
      const uint32_t lead = valid ? uint32_t(__ffsll((unsigned long long)mt) - 1) : uint32_t(lane);
      uint32_t base = 0;
      if (valid && rank == 0) base = cursor_add(mycur, pk[u] >> 16, uint32_t(__popcll(mt)));
      rk[u] = valid ? (rank | (lead << 8) | (base << 16)) : kSkip;
    }
#pragma unroll
    for (int u = 0; u < RW; ++u) {
      const uint32_t base = uint32_t(__shfl(int(rk[u] >> 16), int((rk[u] >> 8) & 0xffu)));
      if (rk[u] != kSkip) {
        const uint32_t pos = base + (rk[u] & 0xffu);
        s_fine[pos] = uint16_t(pk[u] & 0x7fffu);
        s_val[pos] = (pk[u] & 0x8000u) ? -v[u] : v[u];
      }
    }
    __syncthreads();

    const int32_t total = scr[kWaves];
    uint16_t* rf = js.job[q].rec_fine + chunk * E;
    T* rv = static_cast<T*>(js.job[q].rec_val) + chunk * E;
    for (int i = tid; i < total; i += 512) {
      rf[i] = s_fine[i];
      rv[i] = s_val[i];
    }
    __syncthreads();  // LDS is reused by the next job
  }
}

// packed 15-bit hash | sign << 15 of the other modes of a TensorSketch job,
// concatenated in mode order; one job per blockIdx.y
__global__ __launch_bounds__(256) void k_pack_tables(JobSet js, Coords c) {
  const Job& j = js.job[blockIdx.y];
  if (j.type != 0 || !j.tab_lds) return;
  const int t = blockIdx.x * 256 + threadIdx.x;
  for (int k = 0; k < c.N; ++k) {
    if (k == j.col_mode) continue;
    const int i = t - j.tab_off[k];
    if (i >= 0 && i < c.dims[k]) j.ptab[t] = uint16_t(j.h[k][i] | (j.sg[k][i] < 0 ? 0x8000 : 0));
  }
}

// [chunk][bin] -> [bin][chunk], one job per blockIdx.z
__global__ __launch_bounds__(256) void k_meta_transpose(JobSet js) {
  __shared__ uint16_t t[64][65];
  const Job& j = js.job[blockIdx.z];
  const int nb1 = j.nbins + 1, nch = js.nchunks;
  const int b0 = blockIdx.x * 64, c0 = blockIdx.y * 64;
  if (b0 >= nb1 || c0 >= nch) return;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4)
    if (c0 + r < nch && b0 + tx < nb1) t[r][tx] = j.meta[size_t(c0 + r) * nb1 + b0 + tx];
  __syncthreads();
  for (int r = ty; r < 64; r += 4)
    if (b0 + r < nb1 && c0 + tx < nch) j.meta_t[size_t(b0 + r) * js.nchp + c0 + tx] = t[tx][r];
}

// ---------------------------------------------------------------- tiles ----
constexpr int kWin = 256;   // chunks per window: 4 per lane
constexpr int kSub = 1024;  // records per sub-window (record -> run map in LDS)
constexpr int kWaveScratch = kSub * 2 + kWin * 8;

template <class T, int K, int TB>
__global__ __launch_bounds__(256) void k_tiles(JobSet js, int E, int ngroups_pad) {
  extern __shared__ __align__(16) unsigned char lds[];
  constexpr int TC = TB / sizeof(T);
  constexpr int FB = TC == 8192 ? 13 : TC == 4096 ? 12 : TC == 2048 ? 11 : TC == 1024 ? 10 : 0;
  static_assert((1 << FB) == TC, "tile cells must be a power of two");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // XCD-aware: workgroups g, g + 8, g + 16, ... run on one XCD and take
  // consecutive groups of bins
  const int g = blockIdx.x;
  const int grp = (g % 8) * (ngroups_pad / 8) + g / 8;
  const int bt = grp * 4 + wave;
  if (bt >= js.btot) return;  // waves are independent: no barriers below
  int q = 0;
  while (q + 1 < js.njobs && bt >= js.job[q + 1].bin0) ++q;
  const Job& j = js.job[q];
  const int b = bt - j.bin0;
  T* tile = reinterpret_cast<T*>(lds) + wave * TC;
  unsigned char* wsc = lds + 4 * TB + wave * kWaveScratch;
  uint16_t* map = reinterpret_cast<uint16_t*>(wsc);      // run index + 1 per record
  uint32_t* wex = reinterpret_cast<uint32_t*>(wsc + kSub * 2);  // run start in the window
  uint32_t* wad = wex + kWin;                                 // run start address
  for (int i = lane; i < TC; i += 64) tile[i] = T(0);

  const int nch = js.nchunks;
  const uint16_t* St = j.meta_t + size_t(b) * js.nchp;
  const uint16_t* Sn = St + js.nchp;
  const uint16_t* rf = j.rec_fine;
  const T* rv = static_cast<const T*>(j.rec_val);
  for (int c0 = 0; c0 < nch; c0 += kWin) {
    // runs of chunks c0 + 4 lane .. + 3 (rows are padded to 8 entries)
    const int cl = c0 + 4 * lane;
    uint32_t s4[4] = {0, 0, 0, 0}, n4[4] = {0, 0, 0, 0};
    if (cl < nch) {
      const uint2 a = *reinterpret_cast<const uint2*>(St + cl);
      const uint2 z = *reinterpret_cast<const uint2*>(Sn + cl);
      s4[0] = a.x & 0xffffu;
      s4[1] = a.x >> 16;
      s4[2] = a.y & 0xffffu;
      s4[3] = a.y >> 16;
      const uint32_t e4[4] = {z.x & 0xffffu, z.x >> 16, z.y & 0xffffu, z.y >> 16};
#pragma unroll
      for (int h = 0; h < 4; ++h) n4[h] = cl + h < nch ? e4[h] - s4[h] : 0u;
    }
    const uint32_t lsum = n4[0] + n4[1] + n4[2] + n4[3];
    uint32_t incl = lsum;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t y = __shfl_up(incl, off);
      if (lane >= off) incl += y;
    }
    const int32_t total = int32_t(__shfl(incl, 63));
    uint32_t ex4[4];
    {
      uint32_t run = incl - lsum;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        ex4[h] = run;
        wex[4 * lane + h] = run;
        wad[4 * lane + h] = uint32_t(cl + h) * uint32_t(E) + s4[h];
        run += n4[h];
      }
    }
    for (int32_t x0 = 0; x0 < total; x0 += kSub) {
      const int n = total - x0 < kSub ? total - x0 : kSub;
      uint32_t* map32 = reinterpret_cast<uint32_t*>(map);
      for (int w = lane; w < (n + 1) >> 1; w += 64) map32[w] = 0;
      // every run of this sub-window marks its first record in it
#pragma unroll
      for (int h = 0; h < 4; ++h)
        if (n4[h] > 0 && ex4[h] < uint32_t(x0 + n) && ex4[h] + n4[h] > uint32_t(x0)) {
          const uint32_t p = ex4[h] > uint32_t(x0) ? ex4[h] - uint32_t(x0) : 0u;
          map[p] = uint16_t(4 * lane + h + 1);
        }
      // inclusive max-scan of the marks: each record gets its run
      {
        const int P = (n + 63) >> 6;
        const int p0 = lane * P, p1 = p0 + P < n ? p0 + P : n;
        uint32_t mx = 0;
        for (int p = p0; p < p1; ++p) mx = mx > map[p] ? mx : map[p];
        uint32_t carry = mx;
        for (int off = 1; off < 64; off <<= 1) {
          const uint32_t y = __shfl_up(carry, off);
          if (lane >= off) carry = carry > y ? carry : y;
        }
        uint32_t run = __shfl_up(carry, 1);
        if (lane == 0) run = 0;
        for (int p = p0; p < p1; ++p) {
          const uint32_t v = map[p];
          run = run > v ? run : v;
          map[p] = uint16_t(run);
        }
      }
      for (int r0 = 0; r0 < n; r0 += 64 * K) {
        uint32_t f[K];
        T val[K];
#pragma unroll
        for (int u = 0; u < K; ++u) {  // branch-free: out-of-range lanes reload the last record
          const int x = r0 + u * 64 + lane;
          const int xc = x < n ? x : n - 1;
          const int ci = int(map[xc]) - 1;
          const uint32_t a = wad[ci] + (uint32_t(x0 + xc) - wex[ci]);
          f[u] = rf[a];
          val[u] = rv[a];
        }
#pragma unroll
        for (int u = 0; u < K; ++u) {
          const bool valid = r0 + u * 64 + lane < n;
          const uint64_t act = __ballot(valid);
          if (act == 0ull) break;
          const uint64_t mt = match_lanes_n<FB>(f[u], FB, act);
          const int rank = valid ? __popcll(mt & lanemask_lt(lane)) : 64;
          for (int k = 0; __ballot(rank == k) != 0ull; ++k)
            if (rank == k) tile[f[u]] += val[u];
        }
      }
    }
  }
  const int64_t first = (j.bin_lo + b) * int64_t(TC);
  const int64_t rem = j.cells - first;
  const int len = rem < TC ? int(rem) : TC;
  T* out = static_cast<T*>(j.out) + first;
  for (int i = lane; i < len; i += 64) out[i] = tile[i];
}

int bits_for(int64_t n) {
  int b = 1;
  while ((int64_t(1) << b) < n) ++b;
  return b;
}

int path_of(const Job& j) { return j.type == 1 ? 2 : j.tab_lds ? 0 : 1; }

template <class T, int NC, int RW>
void launch_partition(int path, int nchunks, size_t lds, hipStream_t st, const Coords& c,
                      const JobSet& js, int64_t nnz) {
  if (path == 0)
    hipLaunchKernelGGL((k_partition<T, NC, RW, 0>), dim3(nchunks), dim3(512), lds, st, c, js, nnz);
  else if (path == 1)
    hipLaunchKernelGGL((k_partition<T, NC, RW, 1>), dim3(nchunks), dim3(512), lds, st, c, js, nnz);
  else
    hipLaunchKernelGGL((k_partition<T, NC, RW, 2>), dim3(nchunks), dim3(512), lds, st, c, js, nnz);
}

}  // namespace

// Jobs are expanded into slabs of bins whose LDS cursors fit; up to four slabs
// share one read of the entries.  Groups run one after the other on the
// stream and reuse the same scratch.
tsk_status sketch_pass(const TensorView& T, const PassJob* specs, int njobs, Ws& ws,
                       hipStream_t st) {
  const int64_t nnz = T.nnz;
  const bool f64 = T.dtype == TSK_F64;
  const int vb = f64 ? 8 : 4;
  const bool wide = T.order > 4;  // coordinates kept per round: 3, 4 or 8
  // order 3: 16 rounds (8192-entry chunks), or 8 (4096) when that still leaves
  // fewer than two chunks per CU, so that small tensors fill the chip
  const bool small3 = T.order == 3 && nnz < int64_t(512) * 8192;
  const int RW = wide ? 8 : T.order == 4 ? 12 : small3 ? 8 : 16;
  const int E = 512 * RW;
  const int64_t nchunks = nnz > 0 ? ceil_div(nnz, E) : 0;
  // Tile (bin) size: halved from 32 KiB while the pass has fewer than 2048
  // bins (too few waves for the accumulation) and the smaller bins still get
  // enough records per (chunk, bin) run on average, else the per-run
  // bookkeeping dominates: 8, or 4 with the small chunks (both measured on
  // MI355X: sparse 2000^3 with 10^6 entries, 10000^3 with 10^7).
  const double min_run = small3 ? 4.0 : 8.0;
  int64_t cells_all = 0;
  for (int q = 0; q < njobs; ++q) cells_all += specs[q].rows * T.dims[specs[q].col_mode];
  int tile_bytes = kTileMax;
  while (tile_bytes > 8 * 1024) {
    const int64_t bins = ceil_div(cells_all, tile_bytes / vb);
    const double per_run =
        double(tile_bytes / 2 / vb) * double(std::min<int64_t>(E, std::max<int64_t>(nnz, 1))) *
        double(njobs) / double(std::max<int64_t>(cells_all, 1));
    if (bins >= 2048 || per_run < min_run) break;
    tile_bytes /= 2;
  }
  const int64_t tc = tile_bytes / vb;
  if ((nchunks + 1) * int64_t(E) >= (int64_t(1) << 31)) {
    set_error("the sketch pass supports fewer than 2^31 - %d entries", E);
    return TSK_EUNSUPPORTED;
  }
  const int64_t fixed = int64_t(E) * (vb + 2) + 128;  // staging + scan scratch

  Coords c{};
  c.N = T.order;
  c.layout = T.layout;
  for (int k = 0; k < T.order; ++k) {
    c.dims[k] = T.dims[k];
    c.idx[k] = T.idx[k];
  }
  c.vals = T.values;

  std::vector<Job> all;
  for (int q = 0; q < njobs; ++q) {
    const PassJob& p = specs[q];
    Job j{};
    j.type = p.type;
    j.col_mode = p.col_mode;
    j.rows = p.rows;
    j.ncols = T.dims[p.col_mode];
    j.cells = j.rows * j.ncols;
    for (int k = 0; k < T.order; ++k) {
      j.h[k] = p.h ? p.h[k] : nullptr;
      j.sg[k] = p.sg ? p.sg[k] : nullptr;
    }
    j.key = p.key;
    j.out = p.out;
    int64_t tab = 0;
    if (p.type == 0)
      for (int k = 0; k < T.order; ++k)
        if (k != p.col_mode) {
          j.tab_off[k] = int32_t(tab);
          tab += T.dims[k];
        }
    j.tab_lds = p.type == 0 && p.rows <= 32768 && fixed + 2 * (tab + 8) + 16 * 64 <= kLds;
    j.tab_len = j.tab_lds ? int32_t(tab) : 0;
    const int64_t room = (kLds - fixed - 2 * (int64_t(j.tab_len) + 8)) / (2 * kWaves);
    const int64_t bmax = std::min<int64_t>(room, 32768);
    const int64_t nb = ceil_div(j.cells, tc);
    for (int64_t lo = 0; lo < nb; lo += bmax) {
      Job s = j;
      s.bin_lo = lo;
      s.nbins = int32_t(std::min(bmax, nb - lo));
      s.bin_bits = bits_for(s.nbins);
      all.push_back(s);
    }
  }

  const size_t mark = ws.off;
  size_t peak = mark;
  for (size_t g0 = 0; g0 < all.size();) {  // groups of up to four slabs of one hash path
    ws.off = mark;
    JobSet js{};
    js.tc_bits = bits_for(tc);
    js.nchunks = int(nchunks);
    js.nchp = int(ceil_div(nchunks, 8) * 8);
    const int path = path_of(all[g0]);
    int bins = 0;
    size_t q = g0;
    for (; q < all.size() && js.njobs < kMaxJobs && path_of(all[q]) == path; ++q) {
      Job j = all[q];
      // the partition's LDS holds one cursor row of the largest slab and the
      // longest packed table of the group: close the group before a slab that
      // would overflow it (every slab fits alone by construction)
      const int64_t need = fixed + 2 * int64_t(kWaves) * std::max(js.bmax, j.nbins) +
                           2 * ceil_div(std::max(js.tab_max, j.tab_len), 8) * 8;
      if (js.njobs > 0 && need > kLds) break;
      j.bin0 = bins;
      bins += j.nbins;
      js.bmax = std::max(js.bmax, j.nbins);
      js.tab_max = std::max(js.tab_max, j.tab_len);
      j.rec_fine = ws.take<uint16_t>(size_t(nchunks) * E);
      j.rec_val = ws.take<char>(size_t(nchunks) * E * vb);
      j.meta = ws.take<uint16_t>(size_t(nchunks) * (j.nbins + 1));
      j.meta_t = ws.take<uint16_t>(size_t(js.nchp) * (j.nbins + 2));
      j.ptab = j.tab_lds ? ws.take<uint16_t>(size_t(ceil_div(j.tab_len, 8) * 8)) : nullptr;
      js.job[js.njobs++] = j;
    }
    g0 = q;
    js.btot = bins;
    peak = std::max(peak, ws.off);
    if (ws.measuring()) continue;

    if (nchunks > 0) {
      if (js.tab_max > 0) {
        hipLaunchKernelGGL(k_pack_tables, dim3(unsigned(ceil_div(js.tab_max, 256)), unsigned(js.njobs)),
                           dim3(256), 0, st, js, c);
        TSK_LAUNCHED();
      }
      const size_t lds =
          size_t(fixed + 2 * int64_t(kWaves) * js.bmax + 2 * int64_t(ceil_div(js.tab_max, 8) * 8));
      if (lds > size_t(kLds)) {
        set_error("sketch pass: partition needs %zu bytes of LDS (limit %d)", lds, kLds);
        return TSK_EUNSUPPORTED;
      }
      if (f64) {
        if (wide)
          launch_partition<double, 8, 8>(path, int(nchunks), lds, st, c, js, nnz);
        else if (T.order == 4)
          launch_partition<double, 4, 12>(path, int(nchunks), lds, st, c, js, nnz);
        else if (RW == 8)
          launch_partition<double, 3, 8>(path, int(nchunks), lds, st, c, js, nnz);
        else
          launch_partition<double, 3, 16>(path, int(nchunks), lds, st, c, js, nnz);
      } else {
        if (wide)
          launch_partition<float, 8, 8>(path, int(nchunks), lds, st, c, js, nnz);
        else if (T.order == 4)
          launch_partition<float, 4, 12>(path, int(nchunks), lds, st, c, js, nnz);
        else if (RW == 8)
          launch_partition<float, 3, 8>(path, int(nchunks), lds, st, c, js, nnz);
        else
          launch_partition<float, 3, 16>(path, int(nchunks), lds, st, c, js, nnz);
      }
      TSK_LAUNCHED();
      int maxb1 = 0;
      for (int q = 0; q < js.njobs; ++q) maxb1 = std::max(maxb1, js.job[q].nbins + 1);
      hipLaunchKernelGGL(k_meta_transpose,
                         dim3(unsigned(ceil_div(maxb1, 64)), unsigned(ceil_div(nchunks, 64)),
                              unsigned(js.njobs)),
                         dim3(256), 0, st, js);
      TSK_LAUNCHED();
    }
    const size_t tiles_lds = 4 * size_t(tile_bytes) + 4 * kWaveScratch;
    const int ngroups = int(ceil_div(js.btot, 4));
    const int ngroups_pad = int(ceil_div(ngroups, 8) * 8);
    const dim3 tg(ngroups_pad), tb(256);
#define TSK_TILES(TY, B)                                                                   \
  hipLaunchKernelGGL((k_tiles<TY, 8, B>), tg, tb, tiles_lds, st, js, E, ngroups_pad)
    if (f64) {
      if (tile_bytes == 8 * 1024) TSK_TILES(double, 8 * 1024);
      else if (tile_bytes == 16 * 1024) TSK_TILES(double, 16 * 1024);
      else TSK_TILES(double, 32 * 1024);
    } else {
      if (tile_bytes == 8 * 1024) TSK_TILES(float, 8 * 1024);
      else if (tile_bytes == 16 * 1024) TSK_TILES(float, 16 * 1024);
      else TSK_TILES(float, 32 * 1024);
    }
#undef TSK_TILES
    TSK_LAUNCHED();
  }
  ws.off = peak;
  return TSK_OK;
}

}  // namespace tsk
