// Small dense float64 linear algebra on the device, used by the preconditioner
// fit: a tiled GEMM with column/row strides and split-K partials, and an
// in-place blocked Gauss-Jordan inverse of an SPD matrix (no pivoting: the
// Schur complements of an SPD matrix stay SPD) that also returns log det.
#include "dense.hpp"

namespace lk {

namespace {

constexpr int TB = 64;   // output tile
constexpr int TK = 16;   // depth slice

__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K, const double* __restrict__ A,
                                                       int64_t sai, int64_t sak, const double* __restrict__ B,
                                                       int64_t sbk, int64_t sbj, double* __restrict__ P,
                                                       int64_t kps) {
  __shared__ double As[TK][TB + 1];
  __shared__ double Bs[TK][TB + 1];
  const int tid = threadIdx.x;
  const int ty = tid >> 4, tx = tid & 15;
  const int64_t i0 = (int64_t)blockIdx.y * TB, j0 = (int64_t)blockIdx.x * TB;
  const int64_t k0 = (int64_t)blockIdx.z * kps;
  const int64_t k1 = k0 + kps < K ? k0 + kps : K;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
  const bool a_row_contig = (sak == 1);
  const bool b_row_contig = (sbj == 1);
  for (int64_t kk = k0; kk < k1; kk += TK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      int idx = tid + 256 * q;
      int ii, k_;
      if (a_row_contig) { ii = idx / TK; k_ = idx % TK; } else { k_ = idx / TB; ii = idx % TB; }
      int64_t gi = i0 + ii, gk = kk + k_;
      As[k_][ii] = (gi < M && gk < k1) ? A[gi * sai + gk * sak] : 0.0;
      int jj, kb;
      if (b_row_contig) { kb = idx / TB; jj = idx % TB; } else { jj = idx / TK; kb = idx % TK; }
      int64_t gj = j0 + jj, gkb = kk + kb;
      Bs[kb][jj] = (gj < N && gkb < k1) ? B[gkb * sbk + gj * sbj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k_ = 0; k_ < TK; ++k_) {
      double av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = As[k_][ty * 4 + a];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = Bs[k_][tx * 4 + b];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = fma(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();
  }
  double* out = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int64_t gi = i0 + ty * 4 + a;
    if (gi >= M) continue;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int64_t gj = j0 + tx * 4 + b;
      if (gj < N) out[gi * N + gj] = acc[a][b];
    }
  }
}

// C[i*ldc + j] = alpha * (*alpha_dev) * sum_s P[s] + beta * C   (alpha_dev may be null)
__global__ void gemm_reduce_kernel(int64_t M, int64_t N, const double* __restrict__ P, int nsplit, double alpha,
                                   const double* __restrict__ alpha_dev, double beta, double* __restrict__ C,
                                   int64_t ldc) {
  const double al = alpha * (alpha_dev != nullptr ? alpha_dev[0] : 1.0);
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < M * N;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t i = idx / N, j = idx - i * N;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += P[(int64_t)k * M * N + idx];
    double* c = C + i * ldc + j;
    *c = beta != 0.0 ? fma(al, s, beta * *c) : al * s;
  }
}

constexpr int NB = 32;   // Gauss-Jordan pivot block

// Pivot step of blocked Gauss-Jordan on block column K = [k0, k0 + nb):
//   Pinv = A_KK^{-1} (scalar GJ in LDS; log det accumulated),
//   Rh[r][j] = (Pinv A_K,:)[r][j] for j outside K, Pinv[r][j - k0] inside K,
//   Cp[i][r] = A[i][k0 + r] (old column panel).
// Every block inverts the small pivot block itself (identically) and then
// produces its own 64 columns of Rh and 64 rows of Cp; block 0 records log det.
__global__ __launch_bounds__(256) void gj_pivot_kernel(const double* __restrict__ A, int64_t N, int64_t lda,
                                                       int64_t k0, int nb, double* __restrict__ Rh,
                                                       double* __restrict__ Cp, double* __restrict__ logdet,
                                                       int* __restrict__ flag, int first) {
  __shared__ double Ps[2][NB][NB + 1];
  __shared__ double pivs[NB];
  __shared__ double lsum;
  const int tid = threadIdx.x;
  if (flag != nullptr && *flag) return;
  for (int idx = tid; idx < nb * nb; idx += 256) {
    int r = idx / nb, c = idx % nb;
    Ps[0][r][c] = A[(k0 + r) * lda + k0 + c];
  }
  __syncthreads();
  // scalar in-place Gauss-Jordan on the nb x nb block, one barrier per step:
  // step k reads buffer k & 1 and writes the other.  Row k is scaled by the
  // pivot (its column-k entry becoming 1/piv); every other row loses its
  // multiple of row k (its column-k entry becoming -f/piv).
  for (int k = 0; k < nb; ++k) {
    const int cur = k & 1;
    const double piv = Ps[cur][k][k];
    const double ip = 1.0 / piv;
    if (tid == 0) pivs[k] = piv;
    for (int idx = tid; idx < nb * nb; idx += 256) {
      const int r = idx / nb, c = idx % nb;
      const double rk = (c == k ? 1.0 : Ps[cur][k][c]) * ip;
      double v;
      if (r == k) v = rk;
      else v = (c == k ? 0.0 : Ps[cur][r][c]) - Ps[cur][r][k] * rk;
      Ps[cur ^ 1][r][c] = v;
    }
    __syncthreads();
  }
  const int fin = nb & 1;   // buffer holding the inverse
  // log det = sum of the logs of the pivots (one per thread, summed in order)
  if (blockIdx.x == 0) {
    if (tid < nb) pivs[tid] = (pivs[tid] > 0.0 && isfinite(pivs[tid])) ? log(pivs[tid]) : NAN;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int k = 0; k < nb; ++k) s += pivs[k];
      lsum = s;
      logdet[0] = (first ? 0.0 : logdet[0]) + s;
      if (!isfinite(s) && flag != nullptr) *flag = 1;
    }
  }
  // this block's 64 columns of Rh = Pinv * A[K, :] (outside K), Pinv (inside K);
  // the nb x 64 slab of A[K, :] is staged in LDS first
  __shared__ double As[NB][64 + 1];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  for (int idx = tid; idx < nb * 64; idx += 256) {
    const int r = idx / 64;
    const int64_t j = c0 + (idx % 64);
    As[r][idx % 64] = j < N ? A[(k0 + r) * lda + j] : 0.0;
  }
  __syncthreads();
  for (int idx = tid; idx < nb * 64; idx += 256) {
    const int r = idx / 64;
    const int jl = idx % 64;
    const int64_t j = c0 + jl;
    if (j >= N) continue;
    double v;
    if (j >= k0 && j < k0 + nb) {
      v = Ps[fin][r][j - k0];
    } else {
      v = 0.0;
      for (int c = 0; c < nb; ++c) v = fma(Ps[fin][r][c], As[c][jl], v);
    }
    Rh[(int64_t)r * N + j] = v;
  }
  // and its 64 rows of the old column panel
  for (int idx = tid; idx < 64 * nb; idx += 256) {
    const int64_t i = c0 + idx / nb;
    const int c = idx % nb;
    if (i < N) Cp[i * NB + c] = A[i * lda + k0 + c];
  }
}

// Update of all entries for pivot block K:
//   rows in K:      A[i][j] = Rh[i - k0][j]
//   rows outside K: A[i][j] = [j outside K] A[i][j] - sum_r Cp[i][r] Rh[r][j]
__global__ __launch_bounds__(256) void gj_update_kernel(double* __restrict__ A, int64_t N, int64_t lda, int64_t k0,
                                                        int nb, const double* __restrict__ Rh,
                                                        const double* __restrict__ Cp, const int* __restrict__ flag) {
  if (flag != nullptr && *flag) return;
  __shared__ double Rs[NB][TB + 1];
  __shared__ double Cs[TB][NB + 1];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * TB, j0 = (int64_t)blockIdx.x * TB;
  for (int idx = tid; idx < NB * TB; idx += 256) {
    int r = idx / TB, c = idx % TB;
    int64_t j = j0 + c;
    Rs[r][c] = (r < nb && j < N) ? Rh[(int64_t)r * N + j] : 0.0;
    int ii = idx / NB, rr = idx % NB;
    int64_t i = i0 + ii;
    Cs[ii][rr] = (rr < nb && i < N) ? Cp[i * NB + rr] : 0.0;
  }
  __syncthreads();
  const int ty = tid >> 4, tx = tid & 15;
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    int64_t i = i0 + ty * 4 + a;
    if (i >= N) continue;
    const bool in_k_row = (i >= k0 && i < k0 + nb);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      int64_t j = j0 + tx * 4 + b;
      if (j >= N) continue;
      double* aij = A + i * lda + j;
      if (in_k_row) {
        *aij = Rs[i - k0][tx * 4 + b];
      } else {
        double s = 0.0;
        for (int r = 0; r < nb; ++r) s = fma(Cs[ty * 4 + a][r], Rs[r][tx * 4 + b], s);
        const bool in_k_col = (j >= k0 && j < k0 + nb);
        *aij = (in_k_col ? 0.0 : *aij) - s;
      }
    }
  }
}

inline int ew_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

size_t gemm_partials_elems(int64_t M, int64_t N, int nsplit) { return (size_t)M * N * nsplit; }

int gemm_pick_split(int64_t M, int64_t N, int64_t K, int64_t max_elems) {
  int64_t tiles = ((M + TB - 1) / TB) * ((N + TB - 1) / TB);
  int64_t s = (1024 + tiles - 1) / tiles;
  int64_t kt = (K + TK - 1) / TK;
  if (s > kt) s = kt;
  if (s > 64) s = 64;
  while (s > 1 && s * M * N > max_elems) --s;
  return (int)(s < 1 ? 1 : s);
}

hipError_t gemm_f64(int64_t M, int64_t N, int64_t K, const double* A, int64_t sai, int64_t sak, const double* B,
                    int64_t sbk, int64_t sbj, double* C, int64_t ldc, double alpha, const double* alpha_dev,
                    double beta, double* partials, int nsplit, hipStream_t st) {
  int64_t kps = (K + nsplit - 1) / nsplit;
  kps = ((kps + TK - 1) / TK) * TK;
  int ns = (int)((K + kps - 1) / kps);
  if (ns < 1) ns = 1;
  dim3 grid((unsigned)((N + TB - 1) / TB), (unsigned)((M + TB - 1) / TB), (unsigned)ns);
  gemm_f64_kernel<<<grid, 256, 0, st>>>(M, N, K, A, sai, sak, B, sbk, sbj, partials, kps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  gemm_reduce_kernel<<<ew_grid(M * N), 256, 0, st>>>(M, N, partials, ns, alpha, alpha_dev, beta, C, ldc);
  return hipGetLastError();
}

size_t gj_side_elems(int64_t N) { return (size_t)N * NB * 2; }

hipError_t spd_inverse_inplace(double* A, int64_t N, double* side, double* logdet, int* flag, hipStream_t st) {
  double* Rh = side;
  double* Cp = side + (size_t)N * NB;
  dim3 grid((unsigned)((N + TB - 1) / TB), (unsigned)((N + TB - 1) / TB));
  for (int64_t k0 = 0; k0 < N; k0 += NB) {
    int nb = (int)(N - k0 < NB ? N - k0 : NB);
    gj_pivot_kernel<<<(unsigned)((N + 63) / 64), 256, 0, st>>>(A, N, N, k0, nb, Rh, Cp, logdet, flag,
                                                               k0 == 0 ? 1 : 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    gj_update_kernel<<<grid, 256, 0, st>>>(A, N, N, k0, nb, Rh, Cp, flag);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace lk
