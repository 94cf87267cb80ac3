// CP-ALS on the Tucker core (CP-Sketch-Tucker, Alg. 6).
#pragma once
#include "kernels.h"

namespace tsk {
struct CpTuckerBufs {
  double* core;
  double* factors[TSK_MAX_ORDER];
};
// Tucker core and factors of the compression step, in the workspace
tsk_status cp_tucker_bufs(const TensorView& T, const int64_t* R, CpTuckerBufs& b, Ws& ws);
// HOSVD-of-core init, cp_sweeps CP-ALS sweeps on the core, cp_factors[n] = B^(n) A^(n);
// *fit_dev (if fit_dev) <- device pointer of the CP relative residual; *info
// (device int) <- 1 + pivot when a Hadamard Gram is not positive definite
tsk_status cp_run(const TensorView& T, const int64_t* R, int Rc, int sweeps,
                  const CpTuckerBufs& tb, double* const* cp_factors, double** fit_dev, int* info,
                  Ws& ws, hipStream_t st);
}  // namespace tsk
