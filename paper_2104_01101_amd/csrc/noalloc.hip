// RSVD-LRLS (Alg. 5) for callers that cannot allocate device memory (serving
// loops, harnesses that forbid hipMalloc): the same solve as tsk_rsvd_solve,
// with its scratch taken from a fixed array in the library's device code
// object instead of a caller workspace.
//
// The array is a file-scope device variable, so every GPU the library runs on
// holds its own copy from module load until the process ends.  Host code
// never passes the array's name to a kernel (on the host it only stands for
// the symbol): its device address is looked up once per device with
// hipGetSymbolAddress, with that device current, and kept.  Every call on a
// GPU shares that GPU's array, so calls that overlap on one GPU (several host
// threads, or several streams) race; the breakdown flags that must start at
// zero are cleared by a kernel at the start of each call.

#include <mutex>

#include "common.h"
#include "kernels.h"

namespace tsk {
namespace {

constexpr size_t kScratchBytes = size_t(32) << 20;  // 32 MiB per device
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices];
std::mutex g_scratch_mu;

// device address of this device's copy of `scratch`
tsk_status scratch_base(void** base) {
  int dev = 0;
  TSK_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device %d is beyond the %d devices the static scratch supports", dev,
              kMaxDevices);
    return TSK_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    TSK_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = p;
  }
  *base = g_scratch_ptr[dev];
  return TSK_OK;
}

__global__ void k_zero_flags(int* f, int n) {
  if (int(threadIdx.x) < n) f[threadIdx.x] = 0;
}

}  // namespace
}  // namespace tsk

using namespace tsk;

extern "C" tsk_status tsk_rsvd_solve_noalloc(const void* Z, const void* Y, int64_t m, int64_t r,
                                             int64_t s, int32_t R, int32_t prec,
                                             const double* Omega, int32_t k, double* A,
                                             double* W, void* stream) {
  clear_error();
  TSK_REQUIRE(Z && Y && Omega && A && W, "NULL argument");
  TSK_REQUIRE(m >= r && r >= 1 && s >= 1 && R >= 1 && R <= r && R <= s,
              "invalid sizes m=%lld r=%lld s=%lld R=%d", (long long)m, (long long)r,
              (long long)s, R);
  TSK_REQUIRE(k >= R && k <= r && k <= 64, "test matrix width k = %d needs R <= k <= min(r, 64)",
              k);
  TSK_REQUIRE(prec >= TSK_PREC_F64 && prec <= TSK_PREC_BF16, "unknown precision");
  hipStream_t st = as_stream(stream);
  // size of the scratch this shape needs (the same plan, measured)
  Ws probe;
  probe.take<int>(4);
  TSK_TRY(rsvd_solve(Z, Y, m, r, s, R, prec, Omega, k, A, W, nullptr, probe, st));
  if (probe.off > kScratchBytes) {
    set_error("the solve of this shape needs %zu bytes of scratch; the static buffer of "
              "tsk_rsvd_solve_noalloc holds %zu (use tsk_rsvd_solve with a workspace)",
              probe.off, kScratchBytes);
    return TSK_ENOMEM;
  }
  void* base = nullptr;
  TSK_TRY(scratch_base(&base));
  Ws w;
  w.base = static_cast<char*>(base);
  w.cap = kScratchBytes;
  w.serial = true;
  int* info = w.take<int>(4);
  hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(64), 0, st, info, 4);
  TSK_LAUNCHED();
  TSK_TRY(rsvd_solve(Z, Y, m, r, s, R, prec, Omega, k, A, W, info, w, st));
  TSK_HIP(hipStreamSynchronize(st));
  int hinfo[4];
  TSK_HIP(hipMemcpy(hinfo, info, sizeof(hinfo), hipMemcpyDeviceToHost));
  if (hinfo[0] || hinfo[1] || hinfo[3]) {
    set_error("numerical breakdown in the randomized solve (info %d %d %d)", hinfo[0], hinfo[1],
              hinfo[3]);
    return TSK_ENUMERIC;
  }
  return TSK_OK;
}
