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

// Column split of the fused product: how many column ranges, and their width.
struct KmvPlan {
  int nsplit;
  int64_t cols_per_split;
};
KmvPlan kmv_plan(int64_t m, int64_t n, int prec);

// part[s * m + i] = sum_{j in split s} exp(<q_i, k_j>) * p_j   (F64)
//                 = sum_{j in split s} exp2(<q_i, k_j>) * p_j  (F32/BF16)
// p and part are in the vector type of the precision (double for F64, float otherwise).
hipError_t kmv_partials(int prec, int dp, const void* Q, int64_t m, const void* K, int64_t n,
                        const void* p, void* part, const KmvPlan& plan, const int* done,
                        hipStream_t st);

// w_i = lam * p_i + sum_s part[s * m + i]   (vector type of the precision; w may be double)
hipError_t kmv_finish(int prec, int64_t m, double lam, const void* p, const void* part, int nsplit,
                      void* w, bool w_double, hipStream_t st);

// float64 <-> vector-type conversions
hipError_t convert_vec(const void* src, int src_prec, void* dst, int dst_prec, int64_t n,
                       hipStream_t st);

// ---- multi right-hand-side product and the fit (fit.hip) ----

}  // namespace lk
