// Deterministic leverage selection (the m rows of largest Kronecker leverage
// score, weights 1).
#pragma once
#include "kernels.h"

namespace tsk {

// Candidate rank tuples of mode n (data-independent): ncand x nm int32 in
// lexicographic order, every tuple with prod (rank + 1) <= m.
struct SelectPlan {
  int nm;
  int64_t m;
  int64_t ncand;
  int32_t* tup;
};

// Enumerate the candidates into ws (persistent for as long as the plan is used).
tsk_status select_plan(int N, const int64_t* dims, int n, int64_t m, SelectPlan& p, Ws& ws,
                       hipStream_t st);
// idx (m x (N-1), modes k != n increasing) of the kept rows in order; w[j] = 1
// when w is given.  Scratch from ws.
tsk_status select_rows(int N, const int64_t* dims, const int64_t* ranks, int n,
                       const SelectPlan& p, const double* const* factors, int32_t* idx,
                       double* w, Ws& ws, hipStream_t st);

}  // namespace tsk
