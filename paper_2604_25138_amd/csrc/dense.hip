// Small dense float64 linear algebra on the device, used by the preconditioner
// fit: a tiled GEMM on the f64 MFMA with column/row strides and split-K
// partials, and an
// in-place blocked Gauss-Jordan inverse of an SPD matrix (no pivoting: the
// Schur complements of an SPD matrix stay SPD) that also returns log det.
#include "dense.hpp"

namespace lk {

namespace {

constexpr int TB = 64;   // output tile
constexpr int TK = 16;   // depth slice

// One split-K part of C = A B on the 16x16x4 f64 MFMA: a block forms a 64 x 64
// output tile from 16-deep slices of A and B staged in LDS (any strides); wave w
// owns rows 32 (w / 2) .. + 31 and columns 32 (w % 2) .. + 31 as 2 x 2 MFMA
// tiles.  In MFMA step q of a slice a lane supplies A[row l % 16][k = 4 q + l / 16]
// and B[k = 4 q + l / 16][column l % 16]; register r of its result holds row
// 4 r + l / 16, column l % 16 of the tile.
typedef double v4d_ __attribute__((ext_vector_type(4)));
__global__ __launch_bounds__(256) void gemm_f64_kernel(int64_t M, int64_t N, int64_t K, const double* __restrict__ A,
                                                       int64_t sai, int64_t sak, const double* __restrict__ B,
                                                       int64_t sbk, int64_t sbj, double* __restrict__ P,
                                                       int64_t kps) {
  __shared__ double As[TK][TB + 1];
  __shared__ double Bs[TK][TB + 1];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int c = lane & 15, h = lane >> 4;
  const int wr = (wv >> 1) * 32, wc = (wv & 1) * 32;
  const int64_t i0 = (int64_t)blockIdx.y * TB, j0 = (int64_t)blockIdx.x * TB;
  const int64_t k0 = (int64_t)blockIdx.z * kps;
  const int64_t k1 = k0 + kps < K ? k0 + kps : K;
  v4d_ acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = v4d_{0.0, 0.0, 0.0, 0.0};
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
    for (int q = 0; q < TK / 4; ++q) {
      const int kr = 4 * q + h;
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kr][wr + 16 * a + c];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Bs[kr][wc + 16 * b + c];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = P + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int64_t gj = j0 + wc + 16 * b + c;
      if (gj >= N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gi = i0 + wr + 16 * a + 4 * r + h;
        if (gi < M) out[gi * N + gj] = acc[a][b][r];
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
constexpr int GT = 64;   // output tile of one block of the sweep

// Arrival barrier over all blocks of a cooperative launch: every block adds one
// to *bar once its writes are done, and waits until the counter reaches
// `target`.  The wait is bounded (about 0.1 s); a block that gives up sets
// *flag, so a stuck launch still drains.
__device__ bool grid_barrier(unsigned* bar, unsigned target, int* flag) {
  __shared__ int ok;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int good = 1;
    unsigned spins = 0;
    while ((int)(__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) - target) < 0) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (1u << 21)) {
        good = 0;
        break;
      }
    }
    __threadfence();
    if (!good) __hip_atomic_store(flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

struct GjArgs {
  double* A[2];       // matrices inverted in place (blockIdx.z selects one)
  double* T[2];       // N x N partner buffer of each: the sweep alternates between the two
  double* logdet[2];  // log det of each input
  int* flag;          // set to 1 on a non-positive or non-finite pivot (or a stalled barrier)
  unsigned* bar;      // arrival counter of the grid barrier
  unsigned base;      // its value when the launch starts
  int64_t N;
};

// Blocked Gauss-Jordan inverse of SPD matrices (no pivoting: every Schur
// complement of an SPD matrix is SPD) in one cooperative launch.  Step k takes
// the pivot block K = [k0, k0 + nb) of the current matrix S and writes the next
// matrix D:
//   P = S_KK^{-1};  x_j = P S_Kj for j outside K,  x_j = P e_(j - k0) inside K;
//   D_ij = x_j[i - k0]                        for i in K,
//   D_ij = [j outside K] S_ij - S_iK x_j      for i outside K,
// which is the usual in-place sweep written with one update formula.  Every block
// owns one 64 x 64 tile of D and computes P itself from the same data (so all
// blocks take the same pivots and the same exits); one grid barrier per step
// publishes the tiles.  log det is the sum of the logs of the scalar pivots.
__global__ __launch_bounds__(256) void gj_sweep_kernel(GjArgs g) {
  __shared__ double Ps[2][NB][NB + 1];
  __shared__ double Sik[GT][NB + 1];
  __shared__ double Skj[NB][GT + 1];
  __shared__ double X[NB][GT + 1];
  __shared__ double pivs[NB];
  __shared__ double lds_ld;
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int z = blockIdx.z;
  const int64_t N = g.N;
  const int64_t i0 = (int64_t)blockIdx.y * GT, j0 = (int64_t)blockIdx.x * GT;
  const unsigned nblk = gridDim.x * gridDim.y * gridDim.z;
  double* const bufs[2] = {g.A[z], g.T[z]};
  if (__hip_atomic_load(g.flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
  if (tid == 0) {
    lds_ld = 0.0;
    bad = 0;
  }
  const int ty = tid >> 4, tx = tid & 15;
  int step = 0;
  for (int64_t k0 = 0; k0 < N; k0 += NB, ++step) {
    const int nb = (int)(N - k0 < NB ? N - k0 : NB);
    const double* __restrict__ S = bufs[step & 1];
    double* __restrict__ D = bufs[(step & 1) ^ 1];
    for (int idx = tid; idx < NB * NB; idx += 256) {
      const int r = idx / NB, c = idx % NB;
      Ps[0][r][c] = (r < nb && c < nb) ? S[(k0 + r) * N + k0 + c] : 0.0;
    }
    for (int idx = tid; idx < GT * NB; idx += 256) {
      const int r = idx / NB, c = idx % NB;
      const int64_t i = i0 + r;
      Sik[r][c] = (i < N && c < nb) ? S[i * N + k0 + c] : 0.0;
    }
    for (int idx = tid; idx < NB * GT; idx += 256) {
      const int r = idx / GT, c = idx % GT;
      const int64_t j = j0 + c;
      Skj[r][c] = (r < nb && j < N) ? S[(k0 + r) * N + j] : 0.0;
    }
    __syncthreads();
    // Gauss-Jordan of the pivot block by the first wave, rows in registers:
    // lane l holds row l / 2, columns 16 (l % 2) .. 16 (l % 2) + 15; pivot rows
    // and multipliers travel by lane shuffles.  Rows and columns past nb are
    // zero and stay zero.  The inverse lands in Ps[1].
    if (tid < 64) {
      const int r = tid >> 1, h = tid & 1;
      double v[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) v[q] = Ps[0][r][16 * h + q];
#pragma unroll
      for (int k = 0; k < NB; ++k) {
        if (k < nb) {
          const int kq = k & 15, kh = k >> 4;
          const double piv = __shfl(v[kq], 2 * k + kh, 64);
          const double m = __shfl(v[kq], 2 * r + kh, 64);
          const double ip = 1.0 / piv;
          if (tid == 0) pivs[k] = piv;
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            const double rowk = __shfl(v[q], 2 * k + h, 64);
            const int c = 16 * h + q;
            const double rk = (c == k ? 1.0 : rowk) * ip;
            v[q] = (r == k) ? rk : (c == k ? 0.0 : v[q]) - m * rk;
          }
        }
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) Ps[1][r][16 * h + q] = v[q];
    }
    __syncthreads();
    // log det: the logs of the pivots, summed in order by one thread
    if (tid < nb) {
      const double pv = pivs[tid];
      pivs[tid] = (pv > 0.0 && isfinite(pv)) ? log(pv) : NAN;
    }
    __syncthreads();
    if (tid == 0) {
      double sl = 0.0;
      for (int k = 0; k < nb; ++k) sl += pivs[k];
      if (isfinite(sl)) lds_ld += sl;
      else bad = 1;
    }
    __syncthreads();
    if (bad) {
      if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0)
        __hip_atomic_store(g.flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;   // every block saw the same pivots and leaves at the same step
    }
    // X = P S_KJ (2 x 4 outputs per thread), then the columns inside K
    {
      const int r0 = (tid >> 4) * 2, cx = tid & 15;
      double xa[2][4];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) xa[a][b] = 0.0;
      for (int q = 0; q < nb; ++q) {
        const double p0 = Ps[1][r0][q], p1 = Ps[1][r0 + 1][q];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const double sk = Skj[q][cx + 16 * b];
          xa[0][b] = fma(p0, sk, xa[0][b]);
          xa[1][b] = fma(p1, sk, xa[1][b]);
        }
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int rr = r0 + a, c = cx + 16 * b;
          const int64_t j = j0 + c;
          double v = xa[a][b];
          if (j >= k0 && j < k0 + nb) v = Ps[1][rr][j - k0];
          X[rr][c] = (rr < nb && j < N) ? v : 0.0;
        }
    }
    __syncthreads();
    // the tile of D (4 x 4 outputs per thread)
    {
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int q = 0; q < nb; ++q) {
        double sa[4], xb[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) sa[a] = Sik[ty + 16 * a][q];
#pragma unroll
        for (int b = 0; b < 4; ++b) xb[b] = X[q][tx + 16 * b];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(sa[a], xb[b], acc[a][b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int il = ty + 16 * a;
        const int64_t i = i0 + il;
        if (i >= N) continue;
        const bool in_k = (i >= k0 && i < k0 + nb);
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int jl = tx + 16 * b;
          const int64_t j = j0 + jl;
          if (j >= N) continue;
          const bool k_col = (j >= k0 && j < k0 + nb);
          D[i * N + j] = in_k ? X[i - k0][jl] : (k_col ? 0.0 : S[i * N + j]) - acc[a][b];
        }
      }
    }
    if (k0 + NB < N) {
      if (!grid_barrier(g.bar, g.base + (unsigned)(step + 1) * nblk, g.flag)) return;
    }
  }
  // the result sits in the buffer written last; bring it home (each block
  // copies the tile it wrote itself)
  if (step & 1) {
    const double* __restrict__ R = bufs[1];
    double* __restrict__ A = bufs[0];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int64_t i = i0 + ty + 16 * a;
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int64_t j = j0 + tx + 16 * b;
        if (i < N && j < N) A[i * N + j] = R[i * N + j];
      }
    }
  }
  if (blockIdx.x == 0 && blockIdx.y == 0 && tid == 0) g.logdet[z][0] = lds_ld;
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

size_t gj_side_elems(int64_t N) { return (size_t)N * N; }

unsigned gj_barriers(int64_t N, int count) {
  const unsigned t = (unsigned)((N + GT - 1) / GT);
  const unsigned steps = (unsigned)((N + NB - 1) / NB);
  return (steps > 0 ? steps - 1 : 0) * t * t * (unsigned)count;
}

hipError_t spd_inverse_sweep(int count, double* const* A, double* const* side, double* const* logdet, int64_t N,
                             int* flag, unsigned* bar, unsigned base, hipStream_t st) {
  if (count < 1 || count > 2) return hipErrorInvalidValue;
  GjArgs g{};
  for (int z = 0; z < count; ++z) {
    g.A[z] = A[z];
    g.T[z] = side[z];
    g.logdet[z] = logdet[z];
  }
  g.flag = flag;
  g.bar = bar;
  g.base = base;
  g.N = N;
  const unsigned t = (unsigned)((N + GT - 1) / GT);
  dim3 grid(t, t, (unsigned)count);
  void* args[] = {&g};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(gj_sweep_kernel), grid, dim3(256), args, 0, st);
}

}  // namespace lk
