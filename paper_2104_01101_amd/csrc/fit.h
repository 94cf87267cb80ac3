// Fit (relative residual) scratch and launchers.
#pragma once
#include "kernels.h"

namespace tsk {
// largest R_1 of the dense residual path (the column of M kept in registers)
constexpr int kDenseFitMaxR = 64;
struct FitScratch {
  int nblocks;
  double *partial_norm, *partial_inner, *partial_direct, *grams, *buf0, *buf1, *model2, *nT2;
  double* gram_part;  // partial factor Grams over ranges of rows (R_k <= 64)
  double* ttm[2];  // dense tensors: mode products of the core (R_1 x s_2 x ... x s_N)
  // order-3 COO tensors of rank 16: the entries sorted by their last index
  // (once per plan), W = C x_3 A^(3) (s_3 x R x R), <T, T~> at R^2 per entry
  bool by_last = false;  // this path is planned
  bool sorted = false;   // the sorted copy is in place
  uint32_t *keys_in, *keys;  // i_3, then i_3 sorted
  void *ents_in, *ents;       // (i_1, i_2, value) of every entry, then sorted with the keys
  double* W;
  void* sort_tmp;
  size_t sort_bytes;
  unsigned key_bits;
};
tsk_status fit_plan(const TensorView& T, const int64_t* R, FitScratch& fs, Ws& ws);
// Dense T (s_1 x J, row-major) against T~ = A1 M, A1 s_1 x R1 (R1 <= kDenseFitMaxR),
// M R1 x J: per-block sums of (T - T~)^2 into pdirect and of T^2 into pnorm
// (nblocks blocks; pinner set to 0), fixed order.
tsk_status dense_residual_partials(const TensorView& T, const double* M, const double* A1,
                                   int64_t R1, int nblocks, double* pdirect, double* pnorm,
                                   double* pinner, hipStream_t st);
// The sorted copy of the entries that the rank-16 COO path reads (a no-op
// unless fs.by_last and not yet built): enqueued on st, which may be a side
// stream joined into the residual's stream before fit_run.
tsk_status fit_presort(const TensorView& T, FitScratch& fs, hipStream_t st);
// res (device double) <- relative residual; with_norm recomputes ||T||^2 into fs.nT2
tsk_status fit_run(const TensorView& T, const int64_t* R, const double* core,
                   const double* const* factors, bool with_norm, FitScratch& fs, double* res,
                   Ws& ws, hipStream_t st);
}  // namespace tsk
