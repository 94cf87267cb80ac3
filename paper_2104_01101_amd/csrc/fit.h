// Fit (relative residual) scratch and launchers.
#pragma once
#include "kernels.h"

namespace tsk {
struct FitScratch {
  int nblocks;
  double *partial_norm, *partial_inner, *partial_direct, *grams, *buf0, *buf1, *model2, *nT2;
};
tsk_status fit_plan(const TensorView& T, const int64_t* R, FitScratch& fs, Ws& ws);
// res (device double) <- relative residual; with_norm recomputes ||T||^2 into fs.nT2
tsk_status fit_run(const TensorView& T, const int64_t* R, const double* core,
                   const double* const* factors, bool with_norm, FitScratch& fs, double* res,
                   Ws& ws, hipStream_t st);
}  // namespace tsk
