// C ABI of libtsk: argument validation, workspace planning and the host-side
// sequencing of Sketch-Tucker-ALS (Alg. 4) and CP-Sketch-Tucker (Alg. 6).
// Every arithmetic step runs in the kernels of the other translation units;
// this file only orders launches on the caller's stream.

#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "cp.h"
#include "fibers.h"
#include "fit.h"
#include "kernels.h"
#include "leverage.h"
#include "select.h"

namespace tsk {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
}
void clear_error() { g_err.clear(); }
hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

namespace {

__global__ void k_convert(const void* src, int src_dtype, int64_t n, void* dst, int prec) {
  int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n) return;
  double v = src_dtype == TSK_F64 ? static_cast<const double*>(src)[t]
                                  : double(static_cast<const float*>(src)[t]);
  store_prec(dst, size_t(t), v, prec);
}

tsk_status convert_tensor_to_prec(const void* src, int dtype, int64_t n, void* dst, int prec,
                                  hipStream_t st) {
  if (n <= 0) return TSK_OK;
  hipLaunchKernelGGL(k_convert, dim3(ceil_div(n, 256)), dim3(256), 0, st, src, dtype, n, dst,
                     prec);
  TSK_LAUNCHED();
  return TSK_OK;
}

bool prec_matches_dtype(int prec, int dtype) {
  return (prec == TSK_PREC_F64 && dtype == TSK_F64) || (prec == TSK_PREC_F32 && dtype == TSK_F32);
}

tsk_status view_tensor(const tsk_tensor* T, TensorView& tv) {
  TSK_REQUIRE(T, "tensor is NULL");
  TSK_REQUIRE(T->order >= 2 && T->order <= TSK_MAX_ORDER, "tensor order %d not in [2, %d]",
              T->order, TSK_MAX_ORDER);
  TSK_REQUIRE(T->dtype == TSK_F32 || T->dtype == TSK_F64, "unknown dtype %d", T->dtype);
  TSK_REQUIRE(T->layout == TSK_DENSE || T->layout == TSK_COO, "unknown layout %d", T->layout);
  std::memset(&tv, 0, sizeof(tv));
  tv.order = T->order;
  tv.dtype = T->dtype;
  tv.layout = T->layout;
  tv.values = T->values;
  int64_t total = 1;
  for (int k = 0; k < T->order; ++k) {
    TSK_REQUIRE(T->dims[k] >= 1 && T->dims[k] < (int64_t(1) << 31), "dims[%d] = %lld invalid", k,
                (long long)T->dims[k]);
    tv.dims[k] = T->dims[k];
    total *= T->dims[k];
  }
  if (T->layout == TSK_DENSE) {
    tv.nnz = total;
  } else {
    TSK_REQUIRE(T->nnz >= 0 && T->nnz < (int64_t(1) << 31), "nnz = %lld invalid",
                (long long)T->nnz);
    tv.nnz = T->nnz;
    for (int k = 0; k < T->order; ++k) {
      TSK_REQUIRE(T->nnz == 0 || T->idx[k], "COO index array %d is NULL", k);
      tv.idx[k] = T->idx[k];
    }
  }
  TSK_REQUIRE(tv.nnz == 0 || T->values, "tensor values are NULL");
  return TSK_OK;
}

tsk_status check_ranks(const TensorView& tv, const int32_t* ranks, int64_t* R) {
  TSK_REQUIRE(ranks, "ranks is NULL");
  for (int k = 0; k < tv.order; ++k) {
    TSK_REQUIRE(ranks[k] >= 1 && ranks[k] <= tv.dims[k],
                "rank R_%d = %d must satisfy 1 <= R <= s = %lld", k, ranks[k],
                (long long)tv.dims[k]);
    R[k] = ranks[k];
  }
  for (int k = 0; k < tv.order; ++k) {
    int64_t r = prod_except(R, tv.order, k);
    TSK_REQUIRE(R[k] <= r, "rank R_%d = %lld exceeds the product of the other ranks (%lld)", k,
                (long long)R[k], (long long)r);
  }
  return TSK_OK;
}

void rrf_sizes(int64_t m, const int64_t* R, int N, int n, int32_t k1o, int32_t k2o, int64_t& k1,
               int64_t& k2) {
  double K = double(m) / double(prod_except(R, N, n));
  k1 = int64_t(std::ceil(std::sqrt(K) * double(R[n]) - 1e-9));
  if (k1 < R[n]) k1 = R[n];
  k2 = R[n] * R[n] + k1;
  if (k1o > 0) k1 = k1o;
  if (k2o > 0) k2 = k2o;
}

// ---------------------------------------------------------------- RRF ----
struct RrfBufs {
  int64_t k1, k2;
  bool dense;     // B from the dense structured-GEMM pass (no W)
  void* Wt;       // k2 x s_n, tensor dtype (sketch-pass output)
  double* Wt64;   // k2 x s_n
  double* G;      // k2 x k1
  double* B;      // s_n x k1
  double* Mq;     // k1 x k1
  double* lam;    // R
  double* V;      // k1 x R
};

// Dense tensors take the structured-GEMM pass (rrf_dense.hip), which forms
// B = T_(n) Omega^T G directly; other tensors the CountSketch pass into W.
bool rrf_uses_dense_pass(const TensorView& T, int64_t k1) { return rrf_dense_supported(T, k1); }

tsk_status rrf_plan(const TensorView& T, int n, int64_t R, int64_t k1, int64_t k2, RrfBufs& b,
                    Ws& ws) {
  const int64_t s = T.dims[n];
  b.k1 = k1;
  b.k2 = k2;
  b.dense = rrf_uses_dense_pass(T, k1);
  b.Wt = b.dense ? nullptr
                 : T.dtype == TSK_F64 ? (void*)ws.take<double>(k2 * s)
                                      : (void*)ws.take<float>(k2 * s);
  b.Wt64 = b.dense ? nullptr : ws.take<double>(k2 * s);
  b.G = ws.take<double>(k2 * k1);
  b.B = ws.take<double>(s * k1);
  b.Mq = ws.take<double>(k1 * k1);
  b.lam = ws.take<double>(R);
  b.V = ws.take<double>(k1 * R);
  return TSK_OK;
}

// G (k2 x k1), i.i.d. N(0, 1/k1), stream (seed, RRF Gaussian, n)
tsk_status rrf_gaussian(int n, uint64_t seed, const RrfBufs& b, hipStream_t st) {
  return launch_gauss(stream_key(seed, kRRFGauss, n), b.k2 * b.k1, 1.0 / std::sqrt(double(b.k1)),
                      b.G, st);
}

// Range-finder passes of the modes `modes`: dense tensors one structured GEMM
// per mode into b.B (G drawn first), others one CountSketch pass over the
// entries for all modes into b.Wt
tsk_status rrf_passes(const TensorView& T, const int* modes, int nm, uint64_t seed, int prec,
                      RrfBufs* bufs, Ws& ws, hipStream_t st) {
  const bool run = !ws.measuring();
  ProfScope prof(run ? "rrf_pass" : "", st);
  std::vector<PassJob> jobs;
  for (int t = 0; t < nm; ++t) {
    const int n = modes[t];
    RrfBufs& b = bufs[t];
    if (b.dense) {
      if (run) TSK_TRY(rrf_gaussian(n, seed, b, st));
      const size_t mark = ws.off;
      TSK_TRY(rrf_dense(T, n, b.k1, b.k2, stream_key(seed, kRRF, n), b.G, prec, b.B, ws, st));
      ws.off = std::max(ws.off, mark);
    } else {
      jobs.push_back(PassJob{1, n, b.k2, nullptr, nullptr, stream_key(seed, kRRF, n), b.Wt});
    }
  }
  if (!jobs.empty()) TSK_TRY(sketch_pass(T, jobs.data(), int(jobs.size()), ws, st));
  return TSK_OK;
}

// after the range-finder pass: B = W G unless the dense pass formed B, then
// A = leading left singular vectors of B
tsk_status rrf_finish(const TensorView& T, int n, int64_t R, uint64_t seed, RrfBufs& b,
                      double* A, int* info, Ws& ws, hipStream_t st) {
  const int64_t s = T.dims[n];
  const bool run = !ws.measuring();
  ProfScope prof(run ? "rrf" : "", st);
  if (!b.dense) {  // B = W G from the CountSketch pass's W (k2 x s_n, transposed)
    if (run) {
      TSK_TRY(convert_to_f64(b.Wt, T.dtype == TSK_F64 ? 8 : 4, b.k2 * s, b.Wt64, st));
      TSK_TRY(rrf_gaussian(n, seed, b, st));
    }
    TSK_TRY(gemm_tn(TSK_PREC_F64, s, b.k1, b.k2, b.Wt64, s, s, nullptr, 0, b.G, b.k1, b.B, b.k1,
                    ws, st));
  }
  TSK_TRY(gemm_tn(TSK_PREC_F64, b.k1, b.k1, s, b.B, b.k1, b.k1, nullptr, 0, b.B, b.k1, b.Mq, b.k1,
                  ws, st));
  TSK_TRY(sym_eig_top(b.Mq, b.k1, R, b.lam, b.V, ws, st));
  if (run) {
    TSK_TRY(gemm_small(s, R, b.k1, 1.0, b.B, b.k1, 1, b.V, R, 1, 0.0, A, R, st));
    TSK_TRY(scale_columns_inv_sqrt(A, s, R, b.lam, st, info));
  }
  TSK_TRY(cholqr(A, s, R, info, ws, st));
  TSK_TRY(sign_fix_columns(A, s, R, ws, st));
  return TSK_OK;
}

// ------------------------------------------------------------ driver ----
// device breakdown flags of a driver run (see finish_sync)
constexpr int kInfoSlots = 5;

struct TuckerArgs {
  TensorView T;
  int64_t R[TSK_MAX_ORDER];
  tsk_options opt;
  double* core;             // device, prod R
  double* factors[TSK_MAX_ORDER];
  // results of the run (device pointers into the workspace)
  double* fit_dev = nullptr;
  int* info_dev = nullptr;
  int sweeps_done = 0;
};

// columns of the RSVD-LRLS test matrix: O(R) in Alg. 5, R + 10 by default
int64_t rsvd_width(int32_t rsvd_k, int64_t R, int64_t r) {
  return rsvd_k > 0 ? rsvd_k : std::min<int64_t>(R + 10, r);
}

tsk_status validate_options(const TensorView& T, const int64_t* R, const tsk_options* opt) {
  TSK_REQUIRE(opt, "options are NULL");
  TSK_REQUIRE(opt->sketch >= TSK_SKETCH_TS && opt->sketch <= TSK_SKETCH_LEV_DET,
              "unknown sketch %d", opt->sketch);
  TSK_REQUIRE(opt->init >= TSK_INIT_RRF && opt->init <= TSK_INIT_USER, "unknown init %d",
              opt->init);
  TSK_REQUIRE(opt->prec >= TSK_PREC_F64 && opt->prec <= TSK_PREC_BF16, "unknown precision %d",
              opt->prec);
  TSK_REQUIRE(opt->sweeps >= 0, "sweeps = %d < 0", opt->sweeps);
  TSK_REQUIRE(opt->first_sweep >= 0, "first_sweep = %d < 0", opt->first_sweep);
  TSK_REQUIRE(opt->tol >= 0.0, "tol = %g < 0", opt->tol);
  TSK_REQUIRE(opt->tol == 0.0 || ((opt->flags & TSK_FLAG_RECORD_FIT) &&
                                  !(opt->flags & TSK_FLAG_FINAL_FIT)),
              "tol > 0 needs the residual of every sweep (TSK_FLAG_RECORD_FIT without "
              "TSK_FLAG_FINAL_FIT)");
  TSK_REQUIRE(opt->solve == TSK_SOLVE_EXACT || opt->solve == TSK_SOLVE_RSVD, "unknown solve %d",
              opt->solve);
  TSK_REQUIRE(opt->rsvd_k >= 0, "rsvd_k = %d < 0", opt->rsvd_k);
  for (int n = 0; n < T.order; ++n) {
    int64_t r = prod_except(R, T.order, n);
    if (opt->solve == TSK_SOLVE_RSVD) {
      const int64_t k = rsvd_width(opt->rsvd_k, R[n], r);
      TSK_REQUIRE(k >= R[n] && k <= r && k <= 64,
                  "RSVD-LRLS test matrix of %lld columns for mode %d needs R_n <= k <= "
                  "min(prod_{k != n} R_k, 64)",
                  (long long)k, n);
    }
    TSK_REQUIRE(opt->m >= r,
                "sketch size m = %lld is smaller than prod_{k != %d} R_k = %lld (the sketched "
                "problem would not have a unique solution)",
                (long long)opt->m, n, (long long)r);
    if (opt->sketch == TSK_SKETCH_LEV_DET) {
      double rows = 1.0;
      for (int k = 0; k < T.order; ++k)
        if (k != n) rows *= double(T.dims[k]);
      TSK_REQUIRE(double(opt->m) <= rows,
                  "deterministic selection of m = %lld rows exceeds the %.0f rows of mode %d",
                  (long long)opt->m, rows, n);
    }
  }
  TSK_REQUIRE(opt->m < (int64_t(1) << 31), "sketch size too large");
  if (opt->sketch != TSK_SKETCH_TS && T.layout == TSK_COO) {
    unsigned bits = 0;
    TSK_TRY(fiber_key_bits(T, &bits));
  }
  return TSK_OK;
}

tsk_status run_tucker(TuckerArgs& a, Ws& ws) {
  const TensorView& T = a.T;
  const tsk_options& o = a.opt;
  const int N = T.order;
  const int64_t m = o.m;
  const int prec = o.prec;
  const bool run = !ws.measuring();
  const bool ts = o.sketch == TSK_SKETCH_TS;
  const bool record = (o.flags & (TSK_FLAG_RECORD_FIT | TSK_FLAG_FINAL_FIT)) != 0;
  const bool final_only = (o.flags & TSK_FLAG_FINAL_FIT) != 0;
  const int sw0 = o.first_sweep;  // absolute index of the first sweep (per-sweep streams)
  hipStream_t st = as_stream(o.stream);

  int64_t rmax = 0, smax = 0, Rmax = 0;
  for (int n = 0; n < N; ++n) {
    rmax = std::max<int64_t>(rmax, prod_except(a.R, N, n));
    smax = std::max<int64_t>(smax, T.dims[n]);
    Rmax = std::max<int64_t>(Rmax, a.R[n]);
  }
  // ---- persistent allocations ----
  a.info_dev = ws.take<int>(kInfoSlots);
  a.fit_dev = ws.take<double>(std::max(1, o.sweeps));
  std::vector<int32_t*> h(N * N, nullptr);
  std::vector<int8_t*> sg(N * N, nullptr);
  std::vector<CsrTable> csr(N * N);
  std::vector<void*> Yt(N, nullptr), Yp(N, nullptr);
  const size_t tbytes = T.dtype == TSK_F64 ? 8 : 4;
  if (ts) {
    for (int n = 0; n < N; ++n)
      for (int k = 0; k < N; ++k) {
        if (k == n) continue;
        h[n * N + k] = ws.take<int32_t>(T.dims[k]);
        sg[n * N + k] = ws.take<int8_t>(T.dims[k]);
        csr[n * N + k].ptr = ws.take<int32_t>(m + 1);
        csr[n * N + k].items = ws.take<int32_t>(T.dims[k]);
      }
    for (int n = 0; n < N; ++n) {
      Yt[n] = ws.take<char>(size_t(m) * T.dims[n] * tbytes);
      Yp[n] = prec_matches_dtype(prec, T.dtype) ? Yt[n]
                                                  : ws.take<char>(size_t(m) * T.dims[n] *
                                                                  prec_bytes(prec));
    }
  }
  std::vector<RrfBufs> rrf(N);
  if (o.init == TSK_INIT_RRF)
    for (int n = 1; n < N; ++n) {
      int64_t k1, k2;
      rrf_sizes(m, a.R, N, n, o.rrf_k1, o.rrf_k2, k1, k2);
      TSK_REQUIRE(k1 >= a.R[n], "range-finder size k1 = %lld < R_%d", (long long)k1, n);
      TSK_TRY(rrf_plan(T, n, a.R[n], k1, k2, rrf[n], ws));
    }
  void* Z = ws.take<char>(size_t(m) * rmax * prec_bytes(prec));
  double* W = ws.take<double>(rmax * Rmax);
  const bool rsvd = o.solve == TSK_SOLVE_RSVD;
  double* Om = nullptr;
  std::vector<double*> Om_all;  // every sweep's test matrices, drawn at once when they fit
  if (rsvd) {
    int64_t kmax = 0, per_sweep = 0;
    for (int n = 0; n < N; ++n) {
      const int64_t k = rsvd_width(o.rsvd_k, a.R[n], prod_except(a.R, N, n));
      kmax = std::max(kmax, k);
      per_sweep += T.dims[n] * k;
    }
    if (int64_t(o.sweeps) * per_sweep <= (int64_t(8) << 20)) {
      Om_all.resize(size_t(o.sweeps) * N);
      for (int sw = 0; sw < o.sweeps; ++sw)
        for (int n = 0; n < N; ++n)
          Om_all[size_t(sw) * N + n] = ws.take<double>(
              size_t(T.dims[n]) * rsvd_width(o.rsvd_k, a.R[n], prod_except(a.R, N, n)));
    } else {
      Om = ws.take<double>(size_t(smax) * kmax);
    }
  }
  int32_t* lev_idx = nullptr;
  double* lev_w = nullptr;
  void* Ylev = nullptr;
  const bool fibres = !ts && T.layout == TSK_COO;
  const bool det = o.sketch == TSK_SKETCH_LEV_DET;
  std::vector<FiberIndexView> fib(N);
  std::vector<SelectPlan> sel(N);
  if (!ts) {
    lev_idx = ws.take<int32_t>(size_t(m) * (N - 1));
    lev_w = ws.take<double>(m);
    Ylev = ws.take<char>(size_t(m) * smax * prec_bytes(prec));
    if (fibres)
      for (int n = 0; n < N; ++n) TSK_TRY(fiber_index_alloc(T, n, fib[n], ws));
    if (det)  // candidate rank tuples of every mode (independent of the data)
      for (int n = 0; n < N; ++n) TSK_TRY(select_plan(N, T.dims, n, m, sel[n], ws, st));
  }
  FitScratch fs{};
  if (record) TSK_TRY(fit_plan(T, a.R, fs, ws));
  // The residual's sorted copy of the entries depends on the tensor alone: it
  // is built on a side stream beside the sweeps (chains of small launches
  // that leave most of the chip idle; the passes over the entries before them
  // do not), and joined before the first residual.
  SideJob presort(st);

  const size_t mark = ws.off;
  size_t peak = mark;
  auto release = [&]() {
    peak = std::max(peak, ws.off);
    ws.off = mark;
  };

  // ---- preparation: maps, sketched right-hand sides (Sec. 6.1) ----
  if (run) TSK_HIP(hipMemsetAsync(a.info_dev, 0, kInfoSlots * sizeof(int), st));
  {
  ProfScope phase(run ? "phase_prep" : "", st);
  if (ts) {  // maps and their inverse tables, batched when every table fits in LDS
    bool batch = true;
    for (int k = 0; k < N; ++k) batch = batch && table_batch_fits(T.dims[k], m);
    TableBatch tb{};
    for (int n = 0; n < N; ++n)
      for (int k = 0; k < N; ++k) {
        if (k == n) continue;
        if (batch) {
          tb.key[tb.n] = stream_key(o.seed, kTS, n, k);
          tb.s[tb.n] = T.dims[k];
          tb.h[tb.n] = h[n * N + k];
          tb.sg[tb.n] = sg[n * N + k];
          tb.csr[tb.n] = csr[n * N + k];
          if (++tb.n == kTableBatch) {
            if (run) TSK_TRY(hash_tables_batch(tb, m, st));
            tb.n = 0;
          }
          continue;
        }
        if (run)
          TSK_TRY(launch_hash_table(stream_key(o.seed, kTS, n, k), T.dims[k], m, h[n * N + k],
                                    sg[n * N + k], st));
        TSK_TRY(build_inverse_hash(h[n * N + k], T.dims[k], m, csr[n * N + k], ws, st));
        release();
      }
    if (run && batch) TSK_TRY(hash_tables_batch(tb, m, st));
  }
  if (fibres)  // mode-n fibre indices of a COO tensor for the sampled right-hand sides
    for (int n = 0; n < N; ++n) {
      TSK_TRY(fiber_index_build(T, fib[n], ws, st));
      release();
    }
  if (ts) {  // sketched right-hand sides of every mode: one pass over the entries
    std::vector<PassJob> jobs;
    for (int n = 0; n < N; ++n) jobs.push_back(PassJob{0, n, m, &h[n * N], &sg[n * N], 0, Yt[n]});
    ProfScope prof(run ? "sketch_pass" : "", st);
    TSK_TRY(sketch_pass(T, jobs.data(), int(jobs.size()), ws, st));
    release();
  }
  if (ts && run)
    for (int n = 0; n < N; ++n)
      if (Yp[n] != Yt[n])
        TSK_TRY(convert_tensor_to_prec(Yt[n], T.dtype, m * T.dims[n], Yp[n], prec, st));
  }
  // ---- initialisation of modes 2..N (Alg. 3, or a random orthonormal start) ----
  {
  ProfScope phase(run ? "phase_init" : "", st);
  if (o.init == TSK_INIT_RRF) {  // range-finder sketches of modes 2..N: one more pass
    std::vector<int> modes;
    for (int n = 1; n < N; ++n) modes.push_back(n);
    TSK_TRY(rrf_passes(T, modes.data(), int(modes.size()), o.seed, prec, rrf.data() + 1, ws, st));
    release();
  }
  if (o.init == TSK_INIT_RRF) {
    for (int n = 1; n < N; ++n) {
      TSK_TRY(rrf_finish(T, n, a.R[n], o.seed, rrf[n], a.factors[n], a.info_dev + 2, ws, st));
      release();
    }
  } else if (o.init == TSK_INIT_RANDOM) {
    for (int n = 1; n < N; ++n) {
      if (run)
        TSK_TRY(launch_gauss(stream_key(o.seed, kInit, n), T.dims[n] * a.R[n], 1.0,
                             a.factors[n], st));
      TSK_TRY(cholqr(a.factors[n], T.dims[n], a.R[n], a.info_dev + 2, ws, st));
      TSK_TRY(sign_fix_columns(a.factors[n], T.dims[n], a.R[n], ws, st));
      release();
    }
  }
  }

  if (run && !Om_all.empty()) {  // Gaussian test matrices of every (sweep, n), batched
    GaussBatch gb{};
    for (int sw = 0; sw < o.sweeps; ++sw)
      for (int n = 0; n < N; ++n) {
        gb.key[gb.n] = stream_key(o.seed, kRSVD, sw0 + sw, n);
        gb.count[gb.n] =
            T.dims[n] * rsvd_width(o.rsvd_k, a.R[n], prod_except(a.R, N, n));
        gb.out[gb.n] = Om_all[size_t(sw) * N + n];
        if (++gb.n == kGaussBatch) {
          TSK_TRY(launch_gauss_batch(gb, st));
          gb.n = 0;
        }
      }
    TSK_TRY(launch_gauss_batch(gb, st));
  }

  if (run && record && fs.by_last && !ws.serial) {
    hipStream_t side = nullptr;
    TSK_TRY(side_stream(&side));
    if (side) {
      TSK_TRY(presort.fork(side));
      TSK_TRY(fit_presort(T, fs, side));
      TSK_TRY(presort.done());
    }
  }

  // ---- sweeps (Alg. 4) ----
  const int64_t csize = [&] {
    int64_t p = 1;
    for (int k = 0; k < N; ++k) p *= a.R[k];
    return p;
  }();
  for (int sweep = 0; sweep < o.sweeps; ++sweep) {
    ProfScope phase(run ? "phase_sweeps" : "", st);
    for (int n = 0; n < N; ++n) {
      const int64_t r = prod_except(a.R, N, n);
      const void* Y = nullptr;
      if (ts) {
        LhsMode modes[TSK_MAX_ORDER];
        int q = 0;
        for (int k = 0; k < N; ++k) {
          if (k == n) continue;
          modes[q++] = LhsMode{a.factors[k], T.dims[k], a.R[k], sg[n * N + k], csr[n * N + k]};
        }
        TSK_TRY(ts_lhs(modes, N - 1, m, prec, Z, ws, st));
        Y = Yp[n];
      } else {
        if (det) {
          TSK_TRY(select_rows(N, T.dims, a.R, n, sel[n], a.factors, lev_idx, lev_w, ws, st));
        } else {
          TSK_TRY(leverage_sample(N, T.dims, a.R, n, m, o.seed, sw0 + sweep, a.factors, lev_idx,
                                  lev_w, ws, st, prec, Z));
        }
        if (run) {
          if (det)
            TSK_TRY(leverage_rows(T, a.R, n, m, lev_idx, lev_w, a.factors, prec, Z, nullptr, st));
          if (fibres)
            TSK_TRY(fiber_rows(fib[n], m, lev_idx, lev_w, prec, Ylev, st));
          else
            TSK_TRY(leverage_rows(T, a.R, n, m, lev_idx, lev_w, a.factors, prec, nullptr, Ylev,
                                  st));
        }
        Y = Ylev;
      }
      if (rsvd) {  // RSVD-LRLS (Alg. 5) with the test matrix of stream (seed, RSVD, sweep, n)
        const int64_t k = rsvd_width(o.rsvd_k, a.R[n], r);
        double* Om_n = Om_all.empty() ? Om : Om_all[size_t(sweep) * N + n];
        if (run && Om_all.empty())
          TSK_TRY(launch_gauss(stream_key(o.seed, kRSVD, sw0 + sweep, n), T.dims[n] * k, 1.0, Om,
                               st));
        TSK_TRY(rsvd_solve(Z, Y, m, r, T.dims[n], int(a.R[n]), prec, Om_n, k, a.factors[n], W,
                           a.info_dev, ws, st));
      } else {
        TSK_TRY(rc_solve(Z, Y, m, r, T.dims[n], int(a.R[n]), prec, a.factors[n], W, a.info_dev,
                         ws, st));
      }
      release();
    }
    if (run && a.core)
      TSK_HIP(hipMemcpyAsync(a.core, W, csize * sizeof(double), hipMemcpyDeviceToDevice, st));
    phase.end();
    if (record && (!final_only || sweep == o.sweeps - 1)) {
      ProfScope prof(run ? "phase_fit" : "", st);
      TSK_TRY(presort.join());
      TSK_TRY(fit_run(T, a.R, a.core, a.factors, sweep == 0 || final_only, fs,
                      a.fit_dev + sweep, ws, st));
      release();
    }
    a.sweeps_done = sweep + 1;
    if (run && o.tol > 0.0 && sweep >= 1) {  // optional stop: |fit_i - fit_{i-1}| < tol
      double f[2];
      TSK_HIP(hipMemcpyAsync(f, a.fit_dev + sweep - 1, sizeof(f), hipMemcpyDeviceToHost, st));
      TSK_HIP(hipStreamSynchronize(st));
      if (std::fabs(f[1] - f[0]) < o.tol) break;
    }
  }
  ws.off = peak;
  return TSK_OK;
}

tsk_status make_args(const tsk_tensor* T, const int32_t* ranks, const tsk_options* opt,
                     TuckerArgs& a) {
  TSK_TRY(view_tensor(T, a.T));
  TSK_TRY(check_ranks(a.T, ranks, a.R));
  TSK_TRY(validate_options(a.T, a.R, opt));
  a.opt = *opt;
  return TSK_OK;
}

tsk_status finish_sync(TuckerArgs& a, double* fit_history, int32_t* sweeps_done) {
  hipStream_t st = as_stream(a.opt.stream);
  TSK_HIP(hipStreamSynchronize(st));
  int info[kInfoSlots] = {0, 0, 0, 0, 0};
  TSK_HIP(hipMemcpy(info, a.info_dev, sizeof(info), hipMemcpyDeviceToHost));
  if (fit_history && a.sweeps_done > 0) {
    if (a.opt.flags & TSK_FLAG_FINAL_FIT) {  // only the last sweep was evaluated
      for (int i = 0; i < a.opt.sweeps; ++i) fit_history[i] = NAN;
      TSK_HIP(hipMemcpy(fit_history + a.sweeps_done - 1, a.fit_dev + a.sweeps_done - 1,
                        sizeof(double), hipMemcpyDeviceToHost));
    } else if (a.opt.flags & TSK_FLAG_RECORD_FIT) {
      TSK_HIP(hipMemcpy(fit_history, a.fit_dev, a.sweeps_done * sizeof(double),
                        hipMemcpyDeviceToHost));
    }
  }
  if (sweeps_done) *sweeps_done = a.sweeps_done;
  // info: [0] a sketched Gram's pivot, [1] the QR of a solve's factor, [2] the
  // initialisation (range finder or QR of the random start), [3] a zero
  // singular value of a subproblem, [4] a Hadamard Gram of CP-ALS
  if (info[0] || info[1] || info[2] || info[3] || info[4]) {
    set_error("numerical breakdown: %s%s%s%s%s",
              info[0] ? "sketched Gram not positive definite; " : "",
              info[1] ? "factor QR of a solve failed; " : "",
              info[2] ? "initialisation failed (zero or rank-deficient range); " : "",
              info[3] ? "sketched right-hand side of rank below R; " : "",
              info[4] ? "CP-ALS Gram of the core factors not positive definite; " : "");
    return TSK_ENUMERIC;
  }
  return TSK_OK;
}

// Alg. 6: sketched Tucker into workspace buffers, then CP-ALS on the core
tsk_status run_cp(TuckerArgs& a, int Rc, int cp_sweeps, double* const* cp_factors,
                  double** fit_dev, Ws& ws) {
  CpTuckerBufs tb{};
  TSK_TRY(cp_tucker_bufs(a.T, a.R, tb, ws));
  a.core = tb.core;
  for (int k = 0; k < a.T.order; ++k) a.factors[k] = tb.factors[k];
  TSK_TRY(run_tucker(a, ws));
  double* fd = nullptr;
  TSK_TRY(cp_run(a.T, a.R, Rc, cp_sweeps, tb, cp_factors, &fd, a.info_dev + 4, ws,
                 as_stream(a.opt.stream)));
  if (fit_dev) *fit_dev = fd;
  return TSK_OK;
}

}  // namespace
}  // namespace tsk

using namespace tsk;

extern "C" {

int32_t tsk_abi_version(void) { return TSK_ABI_VERSION; }
const char* tsk_last_error(void) { return g_err.c_str(); }

uint64_t tsk_stream_key(uint64_t seed, int32_t purpose, int64_t a, int64_t b, int64_t c) {
  return stream_key(seed, purpose, a, b, c);
}
uint64_t tsk_draw(uint64_t key, uint64_t counter) { return draw(key, counter); }

tsk_status tsk_workspace_size(const tsk_tensor* T, const int32_t* ranks, const tsk_options* opt,
                              size_t* bytes) {
  clear_error();
  TSK_REQUIRE(bytes, "bytes is NULL");
  TuckerArgs a{};
  TSK_TRY(make_args(T, ranks, opt, a));
  Ws probe;
  TSK_TRY(run_tucker(a, probe));
  *bytes = probe.off + 256;
  return TSK_OK;
}

tsk_status tsk_tucker_sketch_als(const tsk_tensor* T, const int32_t* ranks,
                                 const tsk_options* opt, double* core, double* const* factors,
                                 double* fit_history, int32_t* sweeps_done) {
  clear_error();
  TuckerArgs a{};
  TSK_TRY(make_args(T, ranks, opt, a));
  TSK_REQUIRE(core, "core is NULL");
  TSK_REQUIRE(factors, "factors is NULL");
  for (int k = 0; k < a.T.order; ++k) {
    TSK_REQUIRE(factors[k], "factors[%d] is NULL", k);
    a.factors[k] = factors[k];
  }
  a.core = core;
  size_t need = 0;
  {
    Ws probe;
    TuckerArgs b = a;
    TSK_TRY(run_tucker(b, probe));
    need = probe.off + 256;
  }
  TSK_REQUIRE(opt->workspace, "workspace is NULL (query tsk_workspace_size)");
  TSK_REQUIRE((reinterpret_cast<uintptr_t>(opt->workspace) & 255) == 0,
              "workspace must be 256-byte aligned");
  if (opt->workspace_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", opt->workspace_bytes, need);
    return TSK_ENOMEM;
  }
  Ws w;
  w.base = static_cast<char*>(opt->workspace);
  w.cap = opt->workspace_bytes;
  TSK_TRY(run_tucker(a, w));
  return finish_sync(a, fit_history, sweeps_done);
}

tsk_status tsk_hash_tables(int32_t order, const int64_t* dims, int32_t n, int64_t m,
                           uint64_t seed, int32_t* const* h, int8_t* const* sign, void* stream) {
  clear_error();
  TSK_REQUIRE(order >= 2 && order <= TSK_MAX_ORDER && dims && h && sign, "invalid arguments");
  TSK_REQUIRE(n >= 0 && n < order && m >= 1, "invalid mode or sketch size");
  for (int k = 0; k < order; ++k) {
    if (k == n) continue;
    TSK_REQUIRE(h[k] && sign[k], "table pointers of mode %d are NULL", k);
    TSK_TRY(launch_hash_table(stream_key(seed, kTS, n, k), dims[k], m, h[k], sign[k],
                              as_stream(stream)));
  }
  return TSK_OK;
}

tsk_status tsk_sketch_rhs_ts(const tsk_tensor* T, int32_t n, int64_t m, const int32_t* const* h,
                             const int8_t* const* sign, void* Y, void* ws, size_t* ws_bytes,
                             void* stream) {
  clear_error();
  TensorView tv;
  TSK_TRY(view_tensor(T, tv));
  TSK_REQUIRE(n >= 0 && n < tv.order && m >= 1 && h && sign, "invalid arguments");
  for (int k = 0; k < tv.order; ++k)
    TSK_REQUIRE(k == n || (h[k] && sign[k]), "table pointers of mode %d are NULL", k);
  TSK_REQUIRE(ws == nullptr || Y, "Y is NULL");
  PassJob job{0, n, m, h, sign, 0, Y};
  return with_workspace(ws, ws_bytes, [&](Ws& w) {
    return sketch_pass(tv, &job, 1, w, as_stream(stream));
  });
}

tsk_status tsk_sketch_lhs_ts(int32_t order, const int64_t* dims, const int32_t* ranks, int32_t n,
                             int64_t m, const int32_t* const* h, const int8_t* const* sign,
                             const double* const* factors, int32_t prec, void* Z, void* ws,
                             size_t* ws_bytes, void* stream) {
  clear_error();
  TSK_REQUIRE(order >= 2 && order <= TSK_MAX_ORDER && dims && ranks && h && sign && factors,
              "invalid arguments");
  TSK_REQUIRE(n >= 0 && n < order && m >= 1, "invalid mode or sketch size");
  TSK_REQUIRE(prec >= TSK_PREC_F64 && prec <= TSK_PREC_BF16, "unknown precision");
  return with_workspace(ws, ws_bytes, [&](Ws& w) -> tsk_status {
    hipStream_t st = as_stream(stream);
    LhsMode modes[TSK_MAX_ORDER];
    int q = 0;
    for (int k = 0; k < order; ++k) {
      if (k == n) continue;
      CsrTable c{w.take<int32_t>(m + 1), w.take<int32_t>(dims[k])};
      TSK_TRY(build_inverse_hash(h[k], dims[k], m, c, w, st));
      modes[q++] = LhsMode{factors[k], dims[k], ranks[k], sign[k], c};
    }
    return ts_lhs(modes, q, m, prec, Z, w, st);
  });
}

tsk_status tsk_rc_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s, int32_t R,
                        int32_t prec, double* A, double* W, void* ws, size_t* ws_bytes,
                        void* stream) {
  clear_error();
  TSK_REQUIRE(m >= r && r >= 1 && s >= 1 && R >= 1 && R <= r && R <= s,
              "shapes violate m >= r, 1 <= R <= min(r, s)");
  TSK_REQUIRE(prec >= TSK_PREC_F64 && prec <= TSK_PREC_BF16, "unknown precision");
  int* info = nullptr;
  tsk_status stt = with_workspace(ws, ws_bytes, [&](Ws& w) -> tsk_status {
    info = w.take<int>(4);
    if (!w.measuring()) TSK_HIP(hipMemsetAsync(info, 0, 4 * sizeof(int), as_stream(stream)));
    return rc_solve(Z, Y, m, r, s, R, prec, A, W, info, w, as_stream(stream));
  });
  if (stt != TSK_OK || ws == nullptr) return stt;
  TSK_HIP(hipStreamSynchronize(as_stream(stream)));
  int hinfo[4];
  TSK_HIP(hipMemcpy(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost));
  if (hinfo[0] || hinfo[1] || hinfo[3]) {
    set_error("numerical breakdown in the sketched solve (info %d %d %d)", hinfo[0], hinfo[1],
              hinfo[3]);
    return TSK_ENUMERIC;
  }
  return TSK_OK;
}

tsk_status tsk_rsvd_solve(const void* Z, const void* Y, int64_t m, int64_t r, int64_t s,
                          int32_t R, int32_t prec, const double* Omega, int32_t k, double* A,
                          double* W, void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  TSK_REQUIRE(Z && Y && Omega && (ws == nullptr || (A && W)), "NULL argument");
  TSK_REQUIRE(m >= r && r >= 1 && s >= 1 && R >= 1 && R <= r && R <= s,
              "invalid sizes m=%lld r=%lld s=%lld R=%d", (long long)m, (long long)r,
              (long long)s, R);
  TSK_REQUIRE(k >= R && k <= r && k <= 64, "test matrix width k = %d needs R <= k <= min(r, 64)",
              k);
  TSK_REQUIRE(prec >= TSK_PREC_F64 && prec <= TSK_PREC_BF16, "unknown precision");
  int* info = nullptr;
  TSK_TRY(with_workspace(ws, ws_bytes, [&](Ws& w) -> tsk_status {
    info = w.take<int>(4);
    if (!w.measuring()) TSK_HIP(hipMemsetAsync(info, 0, 4 * sizeof(int), as_stream(stream)));
    return rsvd_solve(Z, Y, m, r, s, R, prec, Omega, k, A, W, info, w, as_stream(stream));
  }));
  if (!ws) return TSK_OK;
  TSK_HIP(hipStreamSynchronize(as_stream(stream)));
  int hinfo[4];
  TSK_HIP(hipMemcpy(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost));
  if (hinfo[0] || hinfo[1] || hinfo[3]) {
    set_error("numerical breakdown in the randomized solve (info %d %d %d)", hinfo[0], hinfo[1],
              hinfo[3]);
    return TSK_ENUMERIC;
  }
  return TSK_OK;
}


tsk_status tsk_rrf_init(const tsk_tensor* T, int32_t n, int32_t R, int32_t k1, int32_t k2,
                        uint64_t seed, double* A, void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  TensorView tv;
  TSK_TRY(view_tensor(T, tv));
  TSK_REQUIRE(n >= 0 && n < tv.order, "invalid mode");
  TSK_REQUIRE(R >= 1 && R <= k1 && k1 >= 1 && k2 >= 1 && R <= tv.dims[n],
              "range finder needs 1 <= R <= k1 and R <= s_n");
  int* info = nullptr;
  tsk_status stt = with_workspace(ws, ws_bytes, [&](Ws& w) -> tsk_status {
    hipStream_t st = as_stream(stream);
    info = w.take<int>(4);
    RrfBufs b{};
    TSK_TRY(rrf_plan(tv, n, R, k1, k2, b, w));
    if (!w.measuring()) TSK_HIP(hipMemsetAsync(info, 0, 4 * sizeof(int), st));
    const int modes[1] = {n};
    TSK_TRY(rrf_passes(tv, modes, 1, seed, tv.dtype == TSK_F64 ? TSK_PREC_F64 : TSK_PREC_F32, &b,
                       w, st));
    return rrf_finish(tv, n, R, seed, b, A, info, w, st);
  });
  if (stt != TSK_OK || ws == nullptr) return stt;
  TSK_HIP(hipStreamSynchronize(as_stream(stream)));
  int hinfo[1];
  TSK_HIP(hipMemcpy(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost));
  if (hinfo[0]) {
    set_error("numerical breakdown in the range finder (info %d)", hinfo[0]);
    return TSK_ENUMERIC;
  }
  return TSK_OK;
}

tsk_status tsk_leverage_sample(int32_t order, const int64_t* dims, const int32_t* ranks,
                               int32_t n, int64_t m, uint64_t seed, int32_t sweep,
                               const double* const* factors, int32_t* idx, double* w, void* ws,
                               size_t* ws_bytes, void* stream) {
  clear_error();
  TSK_REQUIRE(order >= 2 && order <= TSK_MAX_ORDER && dims && ranks && factors,
              "invalid arguments");
  TSK_REQUIRE(n >= 0 && n < order && m >= 1, "invalid mode or sample count");
  int64_t R[TSK_MAX_ORDER];
  for (int k = 0; k < order; ++k) R[k] = ranks[k];
  return with_workspace(ws, ws_bytes, [&](Ws& wk) {
    return leverage_sample(order, dims, R, n, m, seed, sweep, factors, idx, w, wk,
                           as_stream(stream));
  });
}

tsk_status tsk_leverage_select(int32_t order, const int64_t* dims, const int32_t* ranks,
                               int32_t n, int64_t m, const double* const* factors, int32_t* idx,
                               void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  TSK_REQUIRE(order >= 2 && order <= TSK_MAX_ORDER && dims && ranks && factors,
              "invalid arguments");
  TSK_REQUIRE(n >= 0 && n < order && m >= 1, "invalid mode or row count");
  int64_t R[TSK_MAX_ORDER];
  for (int k = 0; k < order; ++k) {
    TSK_REQUIRE(dims[k] >= 1 && dims[k] < (int64_t(1) << 31) && ranks[k] >= 1,
                "invalid dims or ranks");
    R[k] = ranks[k];
  }
  hipStream_t st = as_stream(stream);
  return with_workspace(ws, ws_bytes, [&](Ws& wk) -> tsk_status {
    SelectPlan p{};
    TSK_TRY(select_plan(order, dims, n, m, p, wk, st));
    return select_rows(order, dims, R, n, p, factors, idx, nullptr, wk, st);
  });
}

tsk_status tsk_sketch_lev(const tsk_tensor* T, const int32_t* ranks, int32_t n, int64_t m,
                          const int32_t* idx, const double* w, const double* const* factors,
                          int32_t prec, void* Z, void* Y, void* stream) {
  clear_error();
  TensorView tv;
  TSK_TRY(view_tensor(T, tv));
  TSK_REQUIRE(ranks && idx && w && factors && n >= 0 && n < tv.order && m >= 1,
              "invalid arguments");
  if (tv.layout == TSK_COO && Y) {
    set_error("sampled fibres of a COO tensor come from tsk_sketch_lev_coo (fibre index)");
    return TSK_EUNSUPPORTED;
  }
  int64_t R[TSK_MAX_ORDER];
  for (int k = 0; k < tv.order; ++k) R[k] = ranks[k];
  return leverage_rows(tv, R, n, m, idx, w, factors, prec, Z, Y, as_stream(stream));
}

tsk_status tsk_fiber_index(const tsk_tensor* T, int32_t n, void* index, size_t* index_bytes,
                           void* ws, size_t* ws_bytes, void* stream) {
  clear_error();
  TensorView tv;
  TSK_TRY(view_tensor(T, tv));
  TSK_REQUIRE(tv.layout == TSK_COO, "a fibre index is built for COO tensors");
  TSK_REQUIRE(n >= 0 && n < tv.order, "invalid mode %d", n);
  TSK_REQUIRE(index_bytes && ws_bytes, "index_bytes and ws_bytes must not be NULL");
  hipStream_t st = as_stream(stream);
  FiberIndexView fx{};
  Ws ix_probe, ws_probe;
  TSK_TRY(fiber_index_alloc(tv, n, fx, ix_probe));
  TSK_TRY(fiber_index_build(tv, fx, ws_probe, st));
  const size_t need_ix = ix_probe.off + 256, need_ws = ws_probe.off + 256;
  if (!index || !ws) {
    *index_bytes = need_ix;
    *ws_bytes = need_ws;
    return TSK_OK;
  }
  TSK_REQUIRE(!(reinterpret_cast<uintptr_t>(index) & 255) &&
                  !(reinterpret_cast<uintptr_t>(ws) & 255),
              "index and workspace must be 256-byte aligned");
  TSK_REQUIRE(*index_bytes >= need_ix && *ws_bytes >= need_ws,
              "buffers too small: index %zu < %zu or workspace %zu < %zu", *index_bytes, need_ix,
              *ws_bytes, need_ws);
  Ws ix, w;
  ix.base = static_cast<char*>(index);
  ix.cap = *index_bytes;
  w.base = static_cast<char*>(ws);
  w.cap = *ws_bytes;
  TSK_TRY(fiber_index_alloc(tv, n, fx, ix));
  return fiber_index_build(tv, fx, w, st);
}

tsk_status tsk_sketch_lev_coo(const tsk_tensor* T, int32_t n, const void* index, int64_t m,
                              const int32_t* idx, const double* w, int32_t prec, void* Y,
                              void* stream) {
  clear_error();
  TensorView tv;
  TSK_TRY(view_tensor(T, tv));
  TSK_REQUIRE(tv.layout == TSK_COO, "tsk_sketch_lev_coo takes a COO tensor");
  TSK_REQUIRE(n >= 0 && n < tv.order, "invalid mode %d", n);
  TSK_REQUIRE(index && !(reinterpret_cast<uintptr_t>(index) & 255), "index NULL or misaligned");
  TSK_REQUIRE(m >= 0 && m < (int64_t(1) << 31), "invalid sample count");
  TSK_REQUIRE(m == 0 || (idx && w && Y), "invalid arguments");
  TSK_REQUIRE(prec >= TSK_PREC_F64 && prec <= TSK_PREC_BF16, "unknown precision %d", prec);
  FiberIndexView fx{};
  Ws ix;
  ix.base = static_cast<char*>(const_cast<void*>(index));
  ix.cap = ~size_t(0);
  TSK_TRY(fiber_index_alloc(tv, n, fx, ix));
  return fiber_rows(fx, m, idx, w, prec, Y, as_stream(stream));
}

tsk_status tsk_fit(const tsk_tensor* T, const int32_t* ranks, const double* core,
                   const double* const* factors, double* rel_residual, void* ws,
                   size_t* ws_bytes, void* stream) {
  clear_error();
  TensorView tv;
  TSK_TRY(view_tensor(T, tv));
  int64_t R[TSK_MAX_ORDER];
  TSK_TRY(check_ranks(tv, ranks, R));
  TSK_REQUIRE(core && factors && rel_residual, "invalid arguments");
  double* res = nullptr;
  tsk_status stt = with_workspace(ws, ws_bytes, [&](Ws& w) -> tsk_status {
    FitScratch fs{};
    TSK_TRY(fit_plan(tv, R, fs, w));
    res = w.take<double>(1);
    return fit_run(tv, R, core, factors, true, fs, res, w, as_stream(stream));
  });
  if (stt != TSK_OK || ws == nullptr) return stt;
  TSK_HIP(hipStreamSynchronize(as_stream(stream)));
  TSK_HIP(hipMemcpy(rel_residual, res, sizeof(double), hipMemcpyDeviceToHost));
  return TSK_OK;
}

tsk_status tsk_cp_workspace_size(const tsk_tensor* T, int32_t cp_rank, const int32_t* tucker_ranks,
                                 const tsk_options* opt, size_t* bytes) {
  clear_error();
  TSK_REQUIRE(bytes, "bytes is NULL");
  TuckerArgs a{};
  TSK_TRY(make_args(T, tucker_ranks, opt, a));
  Ws probe;
  TSK_TRY(run_cp(a, cp_rank, 1, nullptr, nullptr, probe));
  *bytes = probe.off + 256;
  return TSK_OK;
}

tsk_status tsk_cp_via_tucker(const tsk_tensor* T, int32_t cp_rank, const int32_t* tucker_ranks,
                             int32_t cp_sweeps, const tsk_options* opt, double* const* cp_factors,
                             double* cp_fit) {
  clear_error();
  TuckerArgs a{};
  TSK_TRY(make_args(T, tucker_ranks, opt, a));
  TSK_REQUIRE(cp_factors, "cp_factors is NULL");
  TSK_REQUIRE(cp_sweeps >= 0, "cp_sweeps < 0");
  for (int k = 0; k < a.T.order; ++k) {
    TSK_REQUIRE(cp_factors[k], "cp_factors[%d] is NULL", k);
    TSK_REQUIRE(cp_rank >= 1 && cp_rank <= a.R[k],
                "CP rank %d must be in [1, Tucker rank R_%d = %lld]", cp_rank, k,
                (long long)a.R[k]);
  }
  size_t need = 0;
  {
    Ws probe;
    TuckerArgs b = a;
    TSK_TRY(run_cp(b, cp_rank, cp_sweeps, cp_factors, nullptr, probe));
    need = probe.off + 256;
  }
  TSK_REQUIRE(opt->workspace, "workspace is NULL (query tsk_cp_workspace_size)");
  TSK_REQUIRE((reinterpret_cast<uintptr_t>(opt->workspace) & 255) == 0,
              "workspace must be 256-byte aligned");
  if (opt->workspace_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", opt->workspace_bytes, need);
    return TSK_ENOMEM;
  }
  Ws w;
  w.base = static_cast<char*>(opt->workspace);
  w.cap = opt->workspace_bytes;
  double* fit_dev = nullptr;
  TSK_TRY(run_cp(a, cp_rank, cp_sweeps, cp_factors, &fit_dev, w));
  TSK_TRY(finish_sync(a, nullptr, nullptr));
  if (cp_fit) TSK_HIP(hipMemcpy(cp_fit, fit_dev, sizeof(double), hipMemcpyDeviceToHost));
  return TSK_OK;
}

}  // extern "C"
