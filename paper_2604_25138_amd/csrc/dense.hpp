// Dense float64 helpers of the preconditioner fit (dense.hip).
#pragma once

#include "common.hpp"

namespace lk {

// Number of K-splits for an M x N x K product, limited so that the partial
// buffer holds at most max_elems doubles.
int gemm_pick_split(int64_t M, int64_t N, int64_t K, int64_t max_elems);
size_t gemm_partials_elems(int64_t M, int64_t N, int nsplit);

// C = alpha * (*alpha_dev) * op(A) op(B) + beta * C with
//   op(A)(i, k) = A[i * sai + k * sak]  (M x K),  op(B)(k, j) = B[k * sbk + j * sbj]  (K x N),
//   C row-major with leading dimension ldc.  `partials` holds nsplit * M * N doubles.
hipError_t gemm_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t sai, int64_t sak, const double* B,
                    int64_t sbk, int64_t sbj, double* C, int64_t ldc, double alpha, const double* alpha_dev,
                    double beta, double* partials, int nsplit, hipStream_t st);

// Doubles of side storage spd_inverse_inplace needs for an N x N matrix.
size_t gj_side_elems(int64_t N);

// In-place inverse of an SPD N x N row-major matrix by blocked Gauss-Jordan;
// logdet[0] receives log det A; flag[0] is set to 1 on a non-positive pivot
// (and later launches of the same inverse do nothing).
hipError_t spd_inverse_inplace(double* A, int64_t N, double* side, double* logdet, int* flag, hipStream_t st);

}  // namespace lk
