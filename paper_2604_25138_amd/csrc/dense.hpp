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

// Doubles of the partner buffer spd_inverse_sweep needs per N x N matrix.
size_t gj_side_elems(int64_t N);

// Grid-barrier arrivals one spd_inverse_sweep of `count` N x N matrices adds to
// its counter.
unsigned gj_barriers(int64_t N, int count);

// In-place inverses of `count` (1 or 2) SPD N x N row-major matrices A[z] by a
// blocked Gauss-Jordan sweep in one cooperative launch; side[z] is an N x N
// partner buffer, logdet[z][0] receives log det A[z].  flag[0] is set to 1 on a
// non-positive pivot (later sweeps then do nothing).  `bar` is the barrier
// counter, whose value at launch must be `base`; the sweep adds
// gj_barriers(N, count) to it.  The launch needs (ceil(N/64))^2 * count blocks
// resident at once.
hipError_t spd_inverse_sweep(int count, double* const* A, double* const* side, double* const* logdet, int64_t N,
                             int* flag, unsigned* bar, unsigned base, hipStream_t st);

}  // namespace lk
