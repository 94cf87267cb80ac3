// Tables drawn from the keyed SplitMix64 streams: TensorSketch hash/sign maps
// (Def. TensorSketch) and Gaussian matrices (composite sketch of Sec. 5,
// random initial factors).

#include "common.h"
#include "kernels.h"

namespace tsk {

namespace {
__global__ void k_hash_table(uint64_t key, int64_t s, uint64_t m, int32_t* h, int8_t* sg) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= s) return;
  uint64_t x = draw(key, uint64_t(i));
  h[i] = int32_t(bucket_of(x, m));
  sg[i] = int8_t(sign_of(x));
}

__global__ void k_gauss(uint64_t key, int64_t count, double scale, double* out) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  out[i] = scale * gauss_of(key, uint64_t(i));
}
__global__ void k_gauss_batch(GaussBatch b) {
  const int q = blockIdx.y;
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= b.n || i >= b.count[q]) return;
  b.out[q][i] = gauss_of(b.key[q], uint64_t(i));
}
}  // namespace

tsk_status launch_gauss_batch(const GaussBatch& b, hipStream_t st) {
  int64_t cmax = 0;
  for (int q = 0; q < b.n; ++q) cmax = b.count[q] > cmax ? b.count[q] : cmax;
  if (b.n <= 0 || cmax <= 0) return TSK_OK;
  hipLaunchKernelGGL(k_gauss_batch, dim3(unsigned(ceil_div(cmax, 256)), unsigned(b.n)),
                     dim3(256), 0, st, b);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status launch_hash_table(uint64_t key, int64_t s, int64_t m, int32_t* h, int8_t* sg,
                             hipStream_t st) {
  if (s <= 0) return TSK_OK;
  hipLaunchKernelGGL(k_hash_table, dim3(ceil_div(s, 256)), dim3(256), 0, st, key, s,
                     uint64_t(m), h, sg);
  TSK_LAUNCHED();
  return TSK_OK;
}

tsk_status launch_gauss(uint64_t key, int64_t count, double scale, double* out, hipStream_t st) {
  if (count <= 0) return TSK_OK;
  hipLaunchKernelGGL(k_gauss, dim3(ceil_div(count, 256)), dim3(256), 0, st, key, count, scale,
                     out);
  TSK_LAUNCHED();
  return TSK_OK;
}

}  // namespace tsk
