// Leverage-score sampling launchers.
#pragma once
#include "kernels.h"

namespace tsk {
// idx (m x (N-1)) and w (m); with Z also the sampled Kronecker rows (m x r, prec)
tsk_status leverage_sample(int N, const int64_t* dims, const int64_t* ranks, int n, int64_t m,
                           uint64_t seed, int sweep, const double* const* factors, int32_t* idx,
                           double* w, Ws& ws, hipStream_t st, int prec = 0,
                           void* Z = nullptr);
// Z (m x r) and/or Y (m x dims[n], dense T only; COO fibres: fibers.h), precision prec
tsk_status leverage_rows(const TensorView& T, const int64_t* ranks, int n, int64_t m,
                         const int32_t* idx, const double* w, const double* const* factors,
                         int prec, void* Z, void* Y, hipStream_t st);
}  // namespace tsk
