// Internal helpers shared by the library's translation units: error state,
// workspace planning, the keyed SplitMix64 generator (device + host) and
// small numeric helpers.  Everything here is private to libtsk.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/tsk.h"

namespace tsk {

// ---------------------------------------------------------------- errors ----
void set_error(const char* fmt, ...);
void clear_error();

#define TSK_TRY(expr)                 \
  do {                                \
    tsk_status _s = (expr);           \
    if (_s != TSK_OK) return _s;      \
  } while (0)

#define TSK_REQUIRE(cond, ...)        \
  do {                                \
    if (!(cond)) {                    \
      ::tsk::set_error(__VA_ARGS__);  \
      return TSK_EINVAL;              \
    }                                 \
  } while (0)

#define TSK_HIP(expr)                                                        \
  do {                                                                       \
    hipError_t _e = (expr);                                                  \
    if (_e != hipSuccess) {                                                  \
      ::tsk::set_error("HIP error %s at %s:%d (%s)", hipGetErrorString(_e),  \
                       __FILE__, __LINE__, #expr);                           \
      return TSK_EHIP;                                                       \
    }                                                                        \
  } while (0)

// Check the launch that was just enqueued.
#define TSK_LAUNCHED() TSK_HIP(hipGetLastError())

// ------------------------------------------------------------- workspace ----
// Bump allocator over a caller-provided buffer.  With base == nullptr it only
// measures: the same sequence of take() calls yields the required size.
struct Ws {
  char* base = nullptr;
  size_t off = 0;
  size_t cap = 0;
  // set by callers that may create no streams or events: every step stays on
  // the caller's stream
  bool serial = false;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  bool measuring() const { return base == nullptr; }
};

// Run `body(ws)` once to size and once to execute, following the ws/ws_bytes
// query convention of the ABI.
template <class F>
tsk_status with_workspace(void* ws, size_t* ws_bytes, F&& body) {
  if (!ws_bytes) {
    set_error("ws_bytes must not be NULL");
    return TSK_EINVAL;
  }
  Ws probe;
  TSK_TRY(body(probe));
  size_t need = probe.off + 256;
  if (!ws) {
    *ws_bytes = need;
    return TSK_OK;
  }
  if (reinterpret_cast<uintptr_t>(ws) & 255) {
    set_error("workspace must be 256-byte aligned");
    return TSK_EINVAL;
  }
  if (*ws_bytes < need) {
    set_error("workspace too small: %zu bytes given, %zu needed", *ws_bytes, need);
    return TSK_ENOMEM;
  }
  Ws w;
  w.base = static_cast<char*>(ws);
  w.cap = *ws_bytes;
  return body(w);
}

// ------------------------------------------------------------- generator ----
// SplitMix64 finaliser and keyed counter streams (Steele, Lea & Flood 2014).
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;

enum Purpose : int { kTS = 1, kRRF = 2, kRRFGauss = 3, kLev = 4, kInit = 5, kRSVD = 6 };

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t draw(uint64_t key, uint64_t counter) {
  return mix64(key + (counter + 1) * kGamma);
}

inline uint64_t stream_key(uint64_t seed, int purpose, int64_t a = 0, int64_t b = 0,
                           int64_t c = 0) {
  uint64_t k = seed;
  if (purpose < 0) return k;
  const int64_t tags[4] = {purpose, a, b, c};
  for (int t = 0; t < 4; ++t) k = mix64(k + uint64_t(tags[t] + 1) * kGamma);
  return k;
}

__host__ __device__ inline uint32_t bucket_of(uint64_t x, uint64_t m) {
  return uint32_t(((x & 0xFFFFFFFFull) * m) >> 32);
}
__host__ __device__ inline int sign_of(uint64_t x) { return (x >> 63) ? -1 : 1; }
__host__ __device__ inline double uniform_of(uint64_t x) {
  return double(x >> 11) * 0x1.0p-53;
}
__device__ inline double gauss_of(uint64_t key, uint64_t counter) {
  double u1 = uniform_of(draw(key, 2 * counter));
  double u2 = uniform_of(draw(key, 2 * counter + 1));
  return sqrt(-2.0 * log1p(-u1)) * cos(2.0 * 3.141592653589793 * u2);
}

// ---------------------------------------------------------------- dtypes ----
// Element types of the sketched operands by precision mode.
inline size_t prec_bytes(int prec) { return prec == TSK_PREC_F64 ? 8 : prec == TSK_PREC_F32 ? 4 : 2; }

__device__ inline uint16_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return uint16_t((u >> 16) | ((u & 0xFFFF) ? 0x40 : 0));
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return uint16_t(u >> 16);
}
__device__ inline float bf16_bits_to_f32(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

// Store a double into an operand of precision `prec`.
__device__ inline void store_prec(void* base, size_t i, double v, int prec) {
  if (prec == TSK_PREC_F64)
    static_cast<double*>(base)[i] = v;
  else if (prec == TSK_PREC_F32)
    static_cast<float*>(base)[i] = float(v);
  else
    static_cast<uint16_t*>(base)[i] = f32_to_bf16_bits(float(v));
}

inline int64_t prod_except(const int64_t* d, int N, int n) {
  int64_t p = 1;
  for (int k = 0; k < N; ++k)
    if (k != n) p *= d[k];
  return p;
}
inline int64_t prod_except(const int32_t* d, int N, int n) {
  int64_t p = 1;
  for (int k = 0; k < N; ++k)
    if (k != n) p *= d[k];
  return p;
}
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

hipStream_t as_stream(void* s);

// HIP-event timing of a named launch group (see prof.hip); a no-op unless
// enabled through tsk_profile_enable.
class ProfScope {
 public:
  ProfScope(const char* name, hipStream_t st);
  ~ProfScope() { end(); }
  void end();  // record the closing event now (idempotent)
  ProfScope(const ProfScope&) = delete;
  ProfScope& operator=(const ProfScope&) = delete;

 private:
  hipStream_t st_;
  int idx_;
};

// A second stream of the current device (default priority, non-blocking),
// created on first use and kept until the process ends; *out = NULL where the
// device index is beyond the table (the caller then stays on its stream).
tsk_status side_stream(hipStream_t* out);

// Work forked from the caller's stream onto a side stream and joined back:
// fork() makes the side stream wait for the caller's work so far, done()
// marks the end of the side work, join() makes the caller's stream wait for
// it.  The destructor joins too, so that no return path leaves side work
// running past the call that owns its buffers.
class SideJob {
 public:
  explicit SideJob(hipStream_t st) : st_(st) {}
  ~SideJob() {
    (void)join();
    if (ev_fork_) (void)hipEventDestroy(ev_fork_);
    if (ev_done_) (void)hipEventDestroy(ev_done_);
  }
  tsk_status fork(hipStream_t side) {
    TSK_HIP(hipEventCreateWithFlags(&ev_fork_, hipEventDisableTiming));
    TSK_HIP(hipEventCreateWithFlags(&ev_done_, hipEventDisableTiming));
    TSK_HIP(hipEventRecord(ev_fork_, st_));
    TSK_HIP(hipStreamWaitEvent(side, ev_fork_, 0));
    side_ = side;
    return TSK_OK;
  }
  hipStream_t side() const { return side_; }
  tsk_status done() {
    if (side_ && !recorded_) {
      TSK_HIP(hipEventRecord(ev_done_, side_));
      recorded_ = true;
    }
    return TSK_OK;
  }
  tsk_status join() {
    if (!side_ || joined_) return TSK_OK;
    joined_ = true;
    TSK_TRY(done());
    TSK_HIP(hipStreamWaitEvent(st_, ev_done_, 0));
    return TSK_OK;
  }
  SideJob(const SideJob&) = delete;
  SideJob& operator=(const SideJob&) = delete;

 private:
  hipStream_t st_;
  hipStream_t side_ = nullptr;
  hipEvent_t ev_fork_ = nullptr, ev_done_ = nullptr;
  bool recorded_ = false, joined_ = false;
};

}  // namespace tsk
