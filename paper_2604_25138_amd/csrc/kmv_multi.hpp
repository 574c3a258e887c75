// Kernel product for several right-hand sides sharing one map (kmv_multi.hip).
#pragma once

#include "internal.hpp"

namespace lk {

constexpr int kMaxRhs = 8;   // columns of one multi-right-hand-side product

struct KmvMultiArgs {
  const void* Q;        // prepared query rows (m x dp)
  int64_t m;
  const void* K;        // prepared key rows (n x dp)
  int64_t n;
  const double* P;      // k columns over the key rows, column q at P + q n
  double* part;         // partials: column q, range s, row i at part[(q nsplit + s) m + i]
  int k;
  int64_t cps;          // filled by kmv_multi_run
  int nsplit;           // filled by kmv_multi_run
  PcgScalars* S;        // k run states of a multi-column PCG (null: a plain product)
  int pcg_step;         // 1: the launch starts a PCG iteration of every running column
  int finish;           // 1: a second pass writes out = lam pself + the partials
  double lam;
  const double* pself;  // k columns over the output rows (null: no lam term)
  double* out;          // k output columns of m rows
};

struct KmvMultiPlan {
  int rowblocks;        // blocks of 64 rows
  int nsplit;           // column ranges
  int64_t cols_per_split;
};

KmvMultiPlan kmv_multi_plan(int64_t m, int64_t n);
size_t kmv_multi_part_elems(int64_t m, int64_t n, int k);
hipError_t kmv_multi_run(int prec, int dp, KmvMultiArgs A, hipStream_t st);

}  // namespace lk
