// Fibre index of a COO tensor and the sampled-fibre gather of leverage-score
// sampling.
#pragma once
#include "kernels.h"

namespace tsk {

struct FiberIndexView {
  int N;
  int n;
  int dtype;  // of vals (the tensor's)
  int64_t nnz;
  int64_t dims[TSK_MAX_ORDER];
  uint64_t* keys;  // nnz, ascending: other-mode linear index * s_n + i_n
  void* vals;      // nnz, the tensor's values in key order
};

// Bits of the largest key (prod_k s_k - 1); EUNSUPPORTED if prod_k s_k > 2^64.
tsk_status fiber_key_bits(const TensorView& T, unsigned* bits);
// Carve the index arrays for mode n out of `index` (sizes only when measuring).
tsk_status fiber_index_alloc(const TensorView& T, int n, FiberIndexView& fx, Ws& index);
// Fill the index (keys, stable radix sort of (key, value) pairs); sort scratch from ws.
tsk_status fiber_index_build(const TensorView& T, const FiberIndexView& fx, Ws& ws,
                             hipStream_t st);
// Y[j, :] = w_j * (fibre of sample j), Y m x s_n in the operand type of prec.
tsk_status fiber_rows(const FiberIndexView& fx, int64_t m, const int32_t* idx, const double* w,
                      int prec, void* Y, hipStream_t st);

}  // namespace tsk
