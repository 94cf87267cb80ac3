// TensorSketch of a Kronecker chain, Z = S^(n) kron_{k != n} A^(k) (Sec. 3.1):
//
//   CS_k  = S^(k) A^(k)                 CountSketch of every factor (m x R_k)
//   Z(:, rho) = IFFT( prod_k FFT(CS_k(:, rho_k)) )   length-m circular convolution
//
// CountSketch is a gather over the inverse hash (bucket -> increasing row
// indices), so each CS entry is the in-order sum of its rows.  The FFTs are
// exact-length mixed-radix Stockham transforms (radix 4, 2, 3, 5, direct DFT
// for other primes) staged in LDS, in FP64; the inverse transform of two
// output columns is done at once by packing them as real and imaginary parts.

#include "common.h"
#include "kernels.h"

namespace tsk {

namespace {

constexpr int64_t kTableLdsBytes = 160 * 1024;  // LDS of one workgroup on gfx950
constexpr int kFftBlock = 512;
constexpr int kMaxRadices = 48;

struct Radices {
  int n;
  int r[kMaxRadices];
};

Radices factor_length(int64_t m) {
  Radices rd{};
  int64_t x = m;
  while (x % 4 == 0) rd.r[rd.n++] = 4, x /= 4;
  while (x % 2 == 0) rd.r[rd.n++] = 2, x /= 2;
  for (int p = 3; p <= 5; p += 2)
    while (x % p == 0) rd.r[rd.n++] = p, x /= p;
  for (int64_t q = 7; x > 1; q += 2)
    while (x % q == 0) rd.r[rd.n++] = int(q), x /= q;
  return rd;
}

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 conj_if(double2 a, bool c) { return c ? make_double2(a.x, -a.y) : a; }
// multiply by -i (forward) or +i (inverse)
__device__ inline double2 rot(double2 a, bool inv) {
  return inv ? make_double2(-a.y, a.x) : make_double2(a.y, -a.x);
}

// One radix-RR butterfly of a Stockham stage (RR known at compile time, so the
// operands stay in registers).
template <int RR>
__device__ inline void butterfly(const double2* a, double2* b, int j, int k, int nb, int Ns,
                                 int idxD, int tstep, int wstep, const double2* tw, bool inv) {
  double2 v[RR];
#pragma unroll
  for (int r = 0; r < RR; ++r) {
    const double2 x = a[j + r * nb];
    v[r] = r == 0 ? x : cmul(x, conj_if(tw[r * k * tstep], inv));
  }
  if (RR == 2) {
    b[idxD] = cadd(v[0], v[1]);
    b[idxD + Ns] = csub(v[0], v[1]);
  } else if (RR == 4) {
    const double2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const double2 s13 = cadd(v[1], v[3]), d13 = rot(csub(v[1], v[3]), inv);
    b[idxD] = cadd(s02, s13);
    b[idxD + Ns] = cadd(d02, d13);
    b[idxD + 2 * Ns] = csub(s02, s13);
    b[idxD + 3 * Ns] = csub(d02, d13);
  } else {
#pragma unroll
    for (int o = 0; o < RR; ++o) {
      double2 acc = v[0];
#pragma unroll
      for (int r = 1; r < RR; ++r)
        acc = cadd(acc, cmul(v[r], conj_if(tw[((o * r) % RR) * wstep], inv)));
      b[idxD + o * Ns] = acc;
    }
  }
}

// In-place-by-ping-pong FFT of a[0..m) in LDS (b is scratch of the same size).
// Returns the buffer holding the result.  tw[t] = exp(-2 pi i t / m).
__device__ double2* fft_lds(double2* a, double2* b, int m, const Radices& rd, const double2* tw,
                            bool inv) {
  int Ns = 1;
  for (int p = 0; p < rd.n; ++p) {
    const int R = rd.r[p];
    const int nb = m / R;
    const int tstep = m / (Ns * R);
    const int wstep = m / R;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) {
      const int k = j % Ns;
      const int idxD = (j / Ns) * Ns * R + k;
      if (R == 4)
        butterfly<4>(a, b, j, k, nb, Ns, idxD, tstep, wstep, tw, inv);
      else if (R == 2)
        butterfly<2>(a, b, j, k, nb, Ns, idxD, tstep, wstep, tw, inv);
      else if (R == 3)
        butterfly<3>(a, b, j, k, nb, Ns, idxD, tstep, wstep, tw, inv);
      else if (R == 5)
        butterfly<5>(a, b, j, k, nb, Ns, idxD, tstep, wstep, tw, inv);
      else  // prime radix > 5: direct DFT from LDS
        for (int o = 0; o < R; ++o) {
          double2 acc = make_double2(0.0, 0.0);
          for (int r = 0; r < R; ++r) {
            double2 x = a[j + r * nb];
            if (r) x = cmul(x, conj_if(tw[r * k * tstep], inv));
            acc = cadd(acc, cmul(x, conj_if(tw[((o * r) % R) * wstep], inv)));
          }
          b[idxD + o * Ns] = acc;
        }
    }
    __syncthreads();
    double2* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

__global__ void k_twiddles(int64_t m, double2* tw) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= m) return;
  double s, c;
  sincospi(-2.0 * double(t) / double(m), &s, &c);
  tw[t] = make_double2(c, s);
}

// ---- inverse hash (bucket -> rows), stable: rows increasing in a bucket ----
// One wave; bucket counters in LDS (m + 1 ints).  Counting uses LDS integer
// atomics (exact); placement is stable: lanes of a round are ranked within
// their bucket by ballots over the bucket bits, rounds go in row order.
__global__ __launch_bounds__(64) void k_inverse_hash(const int32_t* h, int s, int m, int32_t* ptr,
                                                     int32_t* items) {
  extern __shared__ int32_t cur[];  // m + 1
  const int lane = threadIdx.x;
  for (int b = lane; b <= m; b += 64) cur[b] = 0;
  __syncthreads();
  for (int i = lane; i < s; i += 64) atomicAdd(&cur[h[i] + 1], 1);
  __syncthreads();
  // inclusive scan of cur[0..m] (shifted counts) = bucket starts; lane owns a chunk
  const int chunk = (m + 1 + 63) / 64;
  const int b0 = lane * chunk, b1 = b0 + chunk < m + 1 ? b0 + chunk : m + 1;
  int32_t run = 0;
  for (int b = b0; b < b1; ++b) run += cur[b];
  int32_t incl = run;
  for (int off = 1; off < 64; off <<= 1) {
    int32_t o = __shfl_up(incl, off);
    if (lane >= off) incl += o;
  }
  int32_t base = incl - run;
  for (int b = b0; b < b1; ++b) {
    base += cur[b];
    cur[b] = base;
    ptr[b] = base;
  }
  __syncthreads();
  int bits = 1;
  while ((1 << bits) < m) ++bits;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int i0 = 0; i0 < s; i0 += 64) {
    const int i = i0 + lane;
    const bool valid = i < s;
    const uint32_t key = valid ? uint32_t(h[i]) : 0u;
    uint64_t mt = __ballot(valid);
    for (int bt = 0; bt < bits; ++bt) {
      const bool bit = (key >> bt) & 1u;
      const uint64_t bal = __ballot(bit);
      mt &= bit ? bal : ~bal;
    }
    const int rank = __popcll(mt & lt);
    int bs = 0;
    if (valid && rank == 0) {
      bs = cur[key];
      cur[key] = bs + __popcll(mt);
    }
    const int leader = valid ? __ffsll((unsigned long long)mt) - 1 : lane;
    bs = __shfl(bs, leader);
    if (valid) items[bs + rank] = i;
  }
}

// The same table by a 256-thread workgroup with h staged in LDS (all loads in
// flight): the items are cut into four contiguous quarters, one per wave;
// each wave counts its quarter per bucket, wave 0 scans the bucket totals,
// every bucket's start is split between the waves in wave order, and the
// waves place their quarters at once, each as the one-wave kernel does (rows
// still increase within a bucket).  For (5 (m + 1) + s) * 4 bytes of LDS
// within kTableLdsBytes.  One workgroup per table of the batch; the hash
// tables themselves come from k_hash_table_batch.
__global__ void k_hash_table_batch(TableBatch b, uint64_t m) {
  const int q = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= b.n || i >= b.s[q]) return;
  const uint64_t x = draw(b.key[q], uint64_t(i));
  b.h[q][i] = int32_t(bucket_of(x, m));
  b.sg[q][i] = int8_t(sign_of(x));
}

__global__ __launch_bounds__(256) void k_inverse_hash_lds(TableBatch tb, int m) {
  extern __shared__ int32_t sh[];
  const int q = blockIdx.x;
  const int32_t* h = tb.h[q];
  const int s = int(tb.s[q]);
  int32_t* ptr = tb.csr[q].ptr;
  int32_t* items = tb.csr[q].items;
  int32_t* cur = sh;                // m + 1: bucket starts
  int32_t* wc = sh + (m + 1);       // 4 x (m + 1): per-wave counts, then cursors
  int32_t* hs = sh + 5 * (m + 1);   // s
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int b = tid; b < 5 * (m + 1); b += 256) sh[b] = 0;
#pragma unroll 4
  for (int i = tid; i < s; i += 256) hs[i] = h[i];
  __syncthreads();
  const int quarter = (s + 255) / 256 * 64;  // multiple of 64
  const int i_lo = wave * quarter, i_hi = min(s, i_lo + quarter);
  int32_t* mine = wc + wave * (m + 1);
  for (int i = i_lo + lane; i < i_hi; i += 64) atomicAdd(&mine[hs[i]], 1);
  __syncthreads();
  if (wave == 0) {
    // totals of bucket b - 1 at b, inclusive scan = bucket starts
    const int chunk = (m + 1 + 63) / 64;
    const int b0 = lane * chunk, b1 = b0 + chunk < m + 1 ? b0 + chunk : m + 1;
    int32_t run = 0;
    for (int b = b0; b < b1; ++b) {
      const int32_t t = b == 0 ? 0
                               : wc[b - 1] + wc[(m + 1) + b - 1] + wc[2 * (m + 1) + b - 1] +
                                     wc[3 * (m + 1) + b - 1];
      cur[b] = t;
      run += t;
    }
    int32_t incl = run;
    for (int off = 1; off < 64; off <<= 1) {
      int32_t o = __shfl_up(incl, off);
      if (lane >= off) incl += o;
    }
    int32_t base = incl - run;
    for (int b = b0; b < b1; ++b) {
      base += cur[b];
      cur[b] = base;
      ptr[b] = base;
    }
  }
  __syncthreads();
  // wave w's cursor of bucket b (over its count): the bucket's start plus
  // the counts of the waves before w
  for (int b = tid; b < m; b += 256) {
    int32_t c = cur[b];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      int32_t* ww = wc + w * (m + 1);
      const int32_t n = ww[b];
      ww[b] = c;
      c += n;
    }
  }
  __syncthreads();
  int bits = 1;
  while ((1 << bits) < m) ++bits;
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  for (int i0 = i_lo; i0 < i_hi; i0 += 64) {
    const int i = i0 + lane;
    const bool valid = i < i_hi;
    const uint32_t key = valid ? uint32_t(hs[i]) : 0u;
    uint64_t mt = __ballot(valid);
    for (int bt = 0; bt < bits; ++bt) {
      const bool bit = (key >> bt) & 1u;
      const uint64_t bal = __ballot(bit);
      mt &= bit ? bal : ~bal;
    }
    const int rank = __popcll(mt & lt);
    int bs = 0;
    if (valid && rank == 0) {
      bs = mine[key];
      mine[key] = bs + __popcll(mt);
    }
    const int leader = valid ? __ffsll((unsigned long long)mt) - 1 : lane;
    bs = __shfl(bs, leader);
    if (valid) items[bs + rank] = i;
  }
}

// ---- CountSketch by gather: CS[b, c] = sum_{i in bucket b} sg[i] A[i, c] ----
__global__ void k_cs_gather(const double* A, int64_t R, const int8_t* sg, const int32_t* ptr,
                            const int32_t* items, int64_t m, double* CS) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= m * R) return;
  int64_t b = t / R, c = t % R;
  double acc = 0.0;
  for (int32_t q = ptr[b]; q < ptr[b + 1]; ++q) {
    int32_t i = items[q];
    double v = A[int64_t(i) * R + c];
    acc += sg[i] > 0 ? v : -v;
  }
  CS[t] = acc;
}

// ---- forward FFT of every CountSketch column ----
struct SpecJob {
  int nmodes;
  int64_t s[TSK_MAX_ORDER];  // rows of A (items of the inverse hash), for the staged gather
  int64_t R[TSK_MAX_ORDER];
  int64_t coloff[TSK_MAX_ORDER];  // first column index of mode q in the spectra array
  const double* CS[TSK_MAX_ORDER];
  // gathered in the spectra kernel itself (CS not materialised)
  const double* A[TSK_MAX_ORDER];
  const int8_t* sg[TSK_MAX_ORDER];
  const int32_t* ptr[TSK_MAX_ORDER];
  const int32_t* items[TSK_MAX_ORDER];
};

// TWL: the twiddle table lives in LDS after the two work buffers and is
// computed there (the same expression as k_twiddles, so the same values);
// otherwise the global table is read
template <bool TWL>
__device__ inline const double2* stage_twiddles(double2* buf, int64_t m, const double2* tw) {
  if (!TWL) return tw;
  double2* t = buf + 2 * m;
  for (int64_t f = threadIdx.x; f < m; f += blockDim.x) {
    double sn, cs;
    sincospi(-2.0 * double(f) / double(m), &sn, &cs);
    t[f] = make_double2(cs, sn);
  }
  return t;  // visible after the caller's next barrier
}

// GATHER: CountSketch column c of mode q formed here, bucket by bucket in the
// order of k_cs_gather (same sums), instead of being read from sj.CS
template <bool TWL, bool GATHER>
__global__ __launch_bounds__(kFftBlock) void k_spectra(SpecJob sj, int64_t m, Radices rd,
                                                       const double2* twg, double2* spec) {
  extern __shared__ double2 buf[];
  double2* a = buf;
  double2* b = buf + m;
  const double2* tw = stage_twiddles<TWL>(buf, m, twg);
  int col = blockIdx.x;
  int q = 0;
  while (q + 1 < sj.nmodes && col >= sj.coloff[q + 1]) ++q;
  int64_t c = col - sj.coloff[q];
  int64_t R = sj.R[q];
  if (GATHER) {
    const double* A = sj.A[q];
    const int8_t* sg = sj.sg[q];
    const int32_t* ptr = sj.ptr[q];
    const int32_t* items = sj.items[q];
    const int64_t sq = sj.s[q];
    // the signed entries of the items staged into the (still unused) FFT work
    // buffer b, 2m at a time with all loads in flight, and the bucket starts
    // into LDS after the twiddles; each bucket is summed in item order across
    // the chunks (the in-order sums of k_cs_gather, bit for bit)
    double* val = reinterpret_cast<double*>(b);
    int32_t* ps = reinterpret_cast<int32_t*>(buf + 3 * m);
    for (int64_t f = threadIdx.x; f <= m; f += blockDim.x) ps[f] = ptr[f];
    for (int64_t f = threadIdx.x; f < m; f += blockDim.x) a[f] = make_double2(0.0, 0.0);
    const int64_t CH = 2 * m;
    for (int64_t c0 = 0; c0 < sq; c0 += CH) {
      const int64_t c1 = c0 + CH < sq ? c0 + CH : sq;
      __syncthreads();  // the previous chunk is summed
#pragma unroll 4
      for (int64_t p = c0 + threadIdx.x; p < c1; p += blockDim.x) {
        const int32_t i = items[p];
        const double v = A[int64_t(i) * R + c];
        val[p - c0] = sg[i] > 0 ? v : -v;
      }
      __syncthreads();
      for (int64_t f = threadIdx.x; f < m; f += blockDim.x) {
        const int64_t lo = ps[f] > c0 ? ps[f] : c0, hi = ps[f + 1] < c1 ? ps[f + 1] : c1;
        if (lo < hi) {
          double acc = a[f].x;
          for (int64_t p = lo; p < hi; ++p) acc += val[p - c0];
          a[f].x = acc;
        }
      }
    }
  } else {
    const double* CS = sj.CS[q];
    for (int64_t f = threadIdx.x; f < m; f += blockDim.x) a[f] = make_double2(CS[f * R + c], 0.0);
  }
  __syncthreads();
  double2* out = fft_lds(a, b, int(m), rd, tw, false);
  double2* dst = spec + int64_t(col) * m;
  for (int64_t f = threadIdx.x; f < m; f += blockDim.x) dst[f] = out[f];
}

// ---- Hadamard product of spectra and inverse FFT of two columns at once ----
template <bool TWL>
__global__ __launch_bounds__(kFftBlock) void k_compose(SpecJob sj, int64_t m, int64_t r,
                                                       Radices rd, const double2* twg,
                                                       const double2* spec, int prec, void* Z) {
  extern __shared__ double2 buf[];
  double2* a = buf;
  double2* b = buf + m;
  const double2* tw = stage_twiddles<TWL>(buf, m, twg);
  int64_t ra = 2 * int64_t(blockIdx.x), rb = ra + 1;
  bool has_b = rb < r;
  // column indices of each mode for rho_a, rho_b (row-major over modes)
  int64_t ca[TSK_MAX_ORDER], cb[TSK_MAX_ORDER];
  {
    int64_t xa = ra, xb = has_b ? rb : 0;
    for (int q = sj.nmodes - 1; q >= 0; --q) {
      ca[q] = xa % sj.R[q];
      xa /= sj.R[q];
      cb[q] = xb % sj.R[q];
      xb /= sj.R[q];
    }
  }
  for (int64_t f = threadIdx.x; f < m; f += blockDim.x) {
    double2 pa = make_double2(1.0, 0.0), pb = make_double2(has_b ? 1.0 : 0.0, 0.0);
    for (int q = 0; q < sj.nmodes; ++q) {
      pa = cmul(pa, spec[(sj.coloff[q] + ca[q]) * m + f]);
      if (has_b) pb = cmul(pb, spec[(sj.coloff[q] + cb[q]) * m + f]);
    }
    a[f] = make_double2(pa.x - pb.y, pa.y + pb.x);  // pa + i pb
  }
  __syncthreads();
  double2* out = fft_lds(a, b, int(m), rd, tw, true);
  const double inv_m = 1.0 / double(m);
  for (int64_t f = threadIdx.x; f < m; f += blockDim.x) {
    store_prec(Z, size_t(f * r + ra), out[f].x * inv_m, prec);
    if (has_b) store_prec(Z, size_t(f * r + rb), out[f].y * inv_m, prec);
  }
}

// one workgroup per (mode q, column c) of the CountSketches; output gCS in
// the CS layout (mode q block: m x R_q row-major, blocks in mode order)
__global__ void k_conv_adjoint(SpecJob sj, int64_t m, int64_t r, Radices rd, const double2* tw,
                               const double2* spec, const double2* gspec, double* gCS) {
  extern __shared__ double2 buf[];
  double2* a = buf;
  double2* b = buf + m;
  const int col = blockIdx.x;
  int q = 0;
  while (q + 1 < sj.nmodes && col >= sj.coloff[q + 1]) ++q;
  const int64_t c = col - sj.coloff[q];
  int64_t inner = 1;
  for (int l = q + 1; l < sj.nmodes; ++l) inner *= sj.R[l];
  const int64_t outer = r / (inner * sj.R[q]);
  for (int64_t f = threadIdx.x; f < m; f += blockDim.x) {
    double2 acc = make_double2(0.0, 0.0);
    for (int64_t o = 0; o < outer; ++o)
      for (int64_t in = 0; in < inner; ++in) {
        const int64_t rho = (o * sj.R[q] + c) * inner + in;
        double2 prod = make_double2(1.0, 0.0);
        int64_t x = rho;
        for (int l = sj.nmodes - 1; l >= 0; --l) {
          const int64_t cl = x % sj.R[l];
          x /= sj.R[l];
          if (l != q) prod = cmul(prod, spec[(sj.coloff[l] + cl) * m + f]);
        }
        acc = cadd(acc, cmul(conj_if(prod, true), gspec[rho * m + f]));
      }
    a[f] = acc;
  }
  __syncthreads();
  double2* out = fft_lds(a, b, int(m), rd, tw, true);
  double* dst = gCS;
  for (int l = 0; l < q; ++l) dst += m * sj.R[l];
  const double inv_m = 1.0 / double(m);
  for (int64_t f = threadIdx.x; f < m; f += blockDim.x) dst[f * sj.R[q] + c] = out[f].x * inv_m;
}

}  // namespace

tsk_status build_inverse_hash(const int32_t* h, int64_t s, int64_t m, CsrTable csr, Ws& ws,
                              hipStream_t st) {
  (void)ws;
  if (ws.measuring()) return TSK_OK;
  if (m + 1 > 40000) {
    set_error("TensorSketch size m = %lld above the inverse-hash LDS limit", (long long)m);
    return TSK_EUNSUPPORTED;
  }
  if (table_batch_fits(s, m)) {
    TableBatch tb{};
    tb.n = 1;
    tb.s[0] = s;
    tb.h[0] = const_cast<int32_t*>(h);
    tb.csr[0] = csr;
    hipLaunchKernelGGL(k_inverse_hash_lds, dim3(1), dim3(256), size_t(5 * (m + 1) + s) * 4, st,
                       tb, int(m));
  } else {
    hipLaunchKernelGGL(k_inverse_hash, dim3(1), dim3(64), size_t(m + 1) * 4, st, h, int(s),
                       int(m), csr.ptr, csr.items);
  }
  TSK_LAUNCHED();
  return TSK_OK;
}

static int fft_max_lds();

bool table_batch_fits(int64_t s, int64_t m) {
  return (5 * (m + 1) + s) * 4 <= std::min<int64_t>(kTableLdsBytes, fft_max_lds());
}

tsk_status hash_tables_batch(const TableBatch& b, int64_t m, hipStream_t st) {
  if (b.n <= 0) return TSK_OK;
  int64_t smax = 0;
  for (int q = 0; q < b.n; ++q) {
    TSK_REQUIRE(table_batch_fits(b.s[q], m), "inverse-hash table beyond the LDS budget");
    smax = b.s[q] > smax ? b.s[q] : smax;
  }
  hipLaunchKernelGGL(k_hash_table_batch, dim3(unsigned(ceil_div(smax, 256)), unsigned(b.n)),
                     dim3(256), 0, st, b, uint64_t(m));
  TSK_LAUNCHED();
  hipLaunchKernelGGL(k_inverse_hash_lds, dim3(unsigned(b.n)), dim3(256),
                     size_t(5 * (m + 1) + smax) * 4, st, b, int(m));
  TSK_LAUNCHED();
  return TSK_OK;
}

static int fft_max_lds() {
  static int v = -1;
  if (v < 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      v = 65536;
  }
  return v;
}

// a, b and the twiddles in LDS, plus the bucket starts of the staged gather
static bool twiddles_fit(int64_t m) { return int64_t(3) * m * 16 + (m + 1) * 4 <= fft_max_lds(); }

static void launch_spectra(int64_t cols, int64_t m, const Radices& rd, const SpecJob& sj, const double* tw,
                    double* spec, hipStream_t st) {
  if (twiddles_fit(m))
    hipLaunchKernelGGL((k_spectra<true, false>), dim3(cols), dim3(kFftBlock), size_t(3 * m * 16),
                       st, sj, m, rd, reinterpret_cast<const double2*>(tw),
                       reinterpret_cast<double2*>(spec));
  else
    hipLaunchKernelGGL((k_spectra<false, false>), dim3(cols), dim3(kFftBlock),
                       size_t(2 * m * 16), st, sj, m, rd, reinterpret_cast<const double2*>(tw),
                       reinterpret_cast<double2*>(spec));
}

static tsk_status check_fft_lds(int64_t m) {
  static int max_lds = -1;
  if (max_lds < 0) {
    int dev = 0;
    TSK_HIP(hipGetDevice(&dev));
    TSK_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  }
  if (int64_t(2) * m * 16 > max_lds) {
    set_error("TensorSketch length m = %lld exceeds the LDS-resident FFT limit (%d bytes)",
              (long long)m, max_lds);
    return TSK_EUNSUPPORTED;
  }
  return TSK_OK;
}

tsk_status ts_lhs_spectra(const LhsMode* modes, int nmodes, int64_t m, double* CS, double* spec,
                          double* tw, Ws& ws, hipStream_t st) {
  (void)ws;
  Radices rd = factor_length(m);
  SpecJob sj{};
  sj.nmodes = nmodes;
  int64_t off = 0, csoff = 0;
  for (int q = 0; q < nmodes; ++q) {
    sj.R[q] = modes[q].R;
    sj.coloff[q] = off;
    sj.CS[q] = CS + csoff;
    off += modes[q].R;
    csoff += m * modes[q].R;
  }
  TSK_TRY(check_fft_lds(m));
  hipLaunchKernelGGL(k_twiddles, dim3(ceil_div(m, 256)), dim3(256), 0, st, m,
                     reinterpret_cast<double2*>(tw));
  TSK_LAUNCHED();
  for (int q = 0; q < nmodes; ++q) {
    const LhsMode& md = modes[q];
    int64_t n = m * md.R;
    hipLaunchKernelGGL(k_cs_gather, dim3(ceil_div(n, 256)), dim3(256), 0, st, md.A, md.R, md.sg,
                       md.csr.ptr, md.csr.items, m, const_cast<double*>(sj.CS[q]));
    TSK_LAUNCHED();
  }
  launch_spectra(off, m, rd, sj, tw, spec, st);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status ts_compose(const LhsMode* modes, int nmodes, int64_t m, const double* spec,
                      const double* tw, int prec, void* Z, hipStream_t st) {
  int64_t r = 1;
  for (int q = 0; q < nmodes; ++q) r *= modes[q].R;
  Radices rd = factor_length(m);
  SpecJob sj{};
  sj.nmodes = nmodes;
  int64_t off = 0;
  for (int q = 0; q < nmodes; ++q) {
    sj.R[q] = modes[q].R;
    sj.coloff[q] = off;
    off += modes[q].R;
  }
  if (twiddles_fit(m))
    hipLaunchKernelGGL(k_compose<true>, dim3(ceil_div(r, 2)), dim3(kFftBlock),
                       size_t(3 * m * 16), st, sj, m, r, rd, reinterpret_cast<const double2*>(tw),
                       reinterpret_cast<const double2*>(spec), prec, Z);
  else
    hipLaunchKernelGGL(k_compose<false>, dim3(ceil_div(r, 2)), dim3(kFftBlock),
                       size_t(2 * m * 16), st, sj, m, r, rd, reinterpret_cast<const double2*>(tw),
                       reinterpret_cast<const double2*>(spec), prec, Z);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status ts_lhs(const LhsMode* modes, int nmodes, int64_t m, int prec, void* Z, Ws& ws,
                  hipStream_t st) {
  int64_t totR = 0;
  for (int q = 0; q < nmodes; ++q) totR += modes[q].R;
  double* CS = ws.take<double>(m * totR);
  double* spec = ws.take<double>(2 * m * totR);
  double* tw = ws.take<double>(2 * m);
  if (ws.measuring()) return TSK_OK;
  ProfScope prof("ts_lhs", st);
  TSK_TRY(check_fft_lds(m));
  if (!twiddles_fit(m)) {
    TSK_TRY(ts_lhs_spectra(modes, nmodes, m, CS, spec, tw, ws, st));
    return ts_compose(modes, nmodes, m, spec, tw, prec, Z, st);
  }
  // two launches: spectra with the CountSketch gather and the twiddles in
  // the kernel, then the composition (twiddles in the kernel)
  Radices rd = factor_length(m);
  SpecJob sj{};
  sj.nmodes = nmodes;
  int64_t off = 0;
  for (int q = 0; q < nmodes; ++q) {
    sj.R[q] = modes[q].R;
    sj.coloff[q] = off;
    sj.A[q] = modes[q].A;
    sj.sg[q] = modes[q].sg;
    sj.ptr[q] = modes[q].csr.ptr;
    sj.items[q] = modes[q].csr.items;
    sj.s[q] = modes[q].s;
    off += modes[q].R;
  }
  // a, b and the twiddles (3 m double2), then the bucket starts (m + 1 int32)
  const size_t spec_lds = size_t(3 * m * 16) + size_t(m + 1) * 4;
  hipLaunchKernelGGL((k_spectra<true, true>), dim3(off), dim3(kFftBlock), spec_lds, st,
                     sj, m, rd, static_cast<const double2*>(nullptr),
                     reinterpret_cast<double2*>(spec));
  TSK_LAUNCHED();
  return ts_compose(modes, nmodes, m, spec, nullptr, prec, Z, st);
}

// FFT of the columns of a real m x cols row-major matrix (twiddles already set)
tsk_status fft_columns(const double* X, int64_t m, int64_t cols, const double* tw, double* spec,
                       hipStream_t st) {
  TSK_TRY(check_fft_lds(m));
  Radices rd = factor_length(m);
  SpecJob sj{};
  sj.nmodes = 1;
  sj.R[0] = cols;
  sj.coloff[0] = 0;
  sj.CS[0] = X;
  launch_spectra(cols, m, rd, sj, tw, spec, st);
  TSK_LAUNCHED();
  return TSK_OK;
}

// Adjoint of the convolution: for mode q (of the modes list) and column c,
// gCS_q[:, c] = IFFT( sum_{rho : rho_q = c} conj(prod_{l != q} F_l[:, rho_l]) * G[:, rho] )
tsk_status ts_conv_adjoint(const LhsMode* modes, int nmodes, int64_t m, const double* spec,
                           const double* gspec, const double* tw, double* gCS, hipStream_t st) {
  Radices rd = factor_length(m);
  SpecJob sj{};
  sj.nmodes = nmodes;
  int64_t off = 0, r = 1;
  for (int q = 0; q < nmodes; ++q) {
    sj.R[q] = modes[q].R;
    sj.coloff[q] = off;
    off += modes[q].R;
    r *= modes[q].R;
  }
  hipLaunchKernelGGL(k_conv_adjoint, dim3(off), dim3(kFftBlock), size_t(2 * m * 16), st, sj, m, r,
                     rd, reinterpret_cast<const double2*>(tw),
                     reinterpret_cast<const double2*>(spec),
                     reinterpret_cast<const double2*>(gspec), gCS);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace tsk
