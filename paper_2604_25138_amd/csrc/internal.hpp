// Host-side launchers shared between the translation units of the library.
#pragma once

#include "common.hpp"

namespace lk {

// ---- embeddings and the fused kernel product (kmv.hip) ----

// Bytes of a prepared embedding copy of `rows` rows in precision `prec`.
size_t embed_bytes(int64_t rows, int dp, int prec);

// Writes the prepared copy of E (rows x d, float64) padded to dp columns:
//   F64:  sqrt(s) * e                      (kernel uses exp)
//   F32:  fp32(sqrt(s log2 e) * e)         (kernel uses exp2)
//   BF16: bf16(fp32(sqrt(s log2 e) * e))   (kernel uses exp2)
hipError_t prep_embed(const double* E, int64_t rows, int d, int dp, double scale, int prec,
                      void* out, hipStream_t st);

constexpr int kMaxSplit = 64;   // largest number of column ranges of one product

// Row blocks x column ranges of one product.
struct KmvPlan {
  int nsplit;
  int64_t cols_per_split;
  int rowblocks;
};
KmvPlan kmv_plan(int64_t m, int64_t n, int prec);
int kmv_rows_per_block(int prec);

// One fused product  out_i = lam * pself_i + sum_j exp(<q_i, k_j>) p_j  (exp2 for
// the float32 / bfloat16 prepared copies).  All vectors are float64.  The
// float64 kernel accumulates in float64; the float32 / bfloat16 kernels sum the
// products of one LDS stage (4 per lane and row) in float32 and add each stage
// sum into a float64 accumulator, so the rounding of the sums does not grow
// with n.
struct KmvArgs {
  const void* Q;        // prepared query rows (m x dp)
  int64_t m;
  const void* K;        // prepared key rows (n x dp)
  int64_t n;
  const double* p;      // vector over the key rows
  double* part;         // nsplit x m column-range partials
  int64_t cps;          // filled by kmv_run
  int nsplit;           // filled by kmv_run
  int mode;             // 0: partials only; 1: finished output
  double lam;           // lambda (0 for the rectangular product)
  const double* pself;  // vector over the output rows for lam * pself; null: none
  double* out;          // output vector (mode 1)
  PcgScalars* S;        // when set, the launch is skipped once S->done
  int pcg_step;         // 1: this product starts a PCG iteration (advances S->kcur)
};
hipError_t kmv_run(int prec, int dp, const KmvPlan& pl, KmvArgs A, hipStream_t st);

// Products of several problems in one launch: block b computes tile
// (problem, row block, column range) = tiles_dev[3 b .. 3 b + 2] with the
// problem's arguments As_dev[problem] (cps and nsplit filled in).  With
// `finish`, a second launch writes out = lam pself + the partials for every
// problem whose mode is 1 (max_m: the largest row count).
hipError_t kmv_run_batch(int prec, int dp, int count, const KmvArgs* As_dev, const int* tiles_dev, int ntiles,
                         bool finish, int64_t max_m, hipStream_t st);

// ---- multi right-hand-side product and the fit (fit.hip) ----

}  // namespace lk
