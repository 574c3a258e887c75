// Kernels of the learned preconditioner's network: a bfloat16 MFMA matrix
// product (32x32x16 tiles, float32 accumulation, split-K partials) whose
// epilogue adds the bias and applies SiLU or its derivative, the per-point
// feature construction, and the Adam update of the float32 master weights.
#include "mlp.hpp"

#include <math.h>

namespace lk {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kT = 256;
constexpr int MT = 64;        // block tile (rows and columns)
constexpr int KC = 32;        // depth staged per pass
constexpr int KP = KC + 8;    // LDS pitch in bfloat16 elements (80 bytes: 16-byte aligned rows)

__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);   // round to nearest even (finite inputs)
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// Block tile 64 x 64 of partial `blockIdx.z` (depth range [k0, k1)); four waves
// each own a 32 x 32 sub-tile.  Lane l of a wave feeds row (or column) l % 32
// and the 8 consecutive depth indices 8 (l / 32) .. of each 16-deep step to
// both operands, so the MFMA pairs equal depth indices; the 16 accumulators of
// lane l hold rows 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.
__global__ __launch_bounds__(kT) void mm_bf16_kernel(int64_t M, int64_t N, int64_t K, const float* __restrict__ A,
                                                     int64_t sai, int64_t sak, const float* __restrict__ B,
                                                     int64_t sbk, int64_t sbj, float* __restrict__ part,
                                                     int64_t kps) {
  __shared__ __attribute__((aligned(16))) uint16_t As[MT][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[MT][KP];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  const int64_t i0 = (int64_t)blockIdx.y * MT, j0 = (int64_t)blockIdx.x * MT;
  const int64_t k0 = (int64_t)blockIdx.z * kps;
  const int64_t k1 = k0 + kps < K ? k0 + kps : K;
  const bool a_kc = (sak == 1);   // depth contiguous in A: threads walk depth first
  const bool b_kc = (sbk == 1);
  v16f acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.f;
  for (int64_t kk = k0; kk < k1; kk += KC) {
#pragma unroll
    for (int q = 0; q < MT * KC / kT; ++q) {
      const int idx = tid + kT * q;
      int r, k;
      if (a_kc) {
        r = idx / KC;
        k = idx % KC;
      } else {
        r = idx % MT;
        k = idx / MT;
      }
      const int64_t gi = i0 + r, gk = kk + k;
      As[r][k] = to_bf16((gi < M && gk < k1) ? A[gi * sai + gk * sak] : 0.f);
      int c, kb;
      if (b_kc) {
        c = idx / KC;
        kb = idx % KC;
      } else {
        c = idx % MT;
        kb = idx / MT;
      }
      const int64_t gj = j0 + c, gkb = kk + kb;
      Bs[c][kb] = to_bf16((gj < N && gkb < k1) ? B[gkb * sbk + gj * sbj] : 0.f);
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC; ks += 16) {
      const int h = lane >> 5;
      const v8bf a = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4*>(&As[wr * 32 + (lane & 31)][ks + 8 * h]));
      const v8bf b = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4*>(&Bs[wc * 32 + (lane & 31)][ks + 8 * h]));
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  float* __restrict__ P = part + (int64_t)blockIdx.z * M * N;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t gi = i0 + wr * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
    const int64_t gj = j0 + wc * 32 + (lane & 31);
    if (gi < M && gj < N) P[gi * N + gj] = acc[r];
  }
}

__global__ void mm_epilogue_kernel(const float* __restrict__ part, int nsplit, int64_t M, int64_t N, int epi,
                                   const float* __restrict__ bias, const float* __restrict__ zpre,
                                   float* __restrict__ out, float* __restrict__ out2) {
  const int64_t total = M * N;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    float s = 0.f;
    for (int z = 0; z < nsplit; ++z) s += part[(int64_t)z * total + idx];
    const int64_t j = idx % N;
    if (epi == kEpiLinear) {
      out[idx] = bias != nullptr ? s + bias[j] : s;
    } else if (epi == kEpiSilu) {
      const float zz = bias != nullptr ? s + bias[j] : s;
      out2[idx] = zz;
      out[idx] = silu(zz);
    } else {
      out[idx] = s * silu_grad(zpre[idx]);
    }
  }
}

// column sums of E and E*E over a range of rows per block
__global__ __launch_bounds__(kT) void colstat_kernel(const double* __restrict__ E, int64_t n, int d,
                                                     double* __restrict__ colpart, double* __restrict__ stats,
                                                     unsigned* cnt) {
  __shared__ double s1[kT], s2[kT];
  const int64_t rows = (n + gridDim.x - 1) / gridDim.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows;
  const int64_t r1 = r0 + rows < n ? r0 + rows : n;
  for (int c0 = 0; c0 < d; c0 += kT / 4) {
    // four row groups per column, 64 columns per pass
    const int c = c0 + (threadIdx.x & 63);
    const int g = threadIdx.x >> 6;
    double a = 0.0, b = 0.0;
    if (c < d)
      for (int64_t i = r0 + g; i < r1; i += 4) {
        const double e = E[i * d + c];
        a += e;
        b += e * e;
      }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    if (threadIdx.x < 64 && c < d) {
      const int t = threadIdx.x;
      colpart[(int64_t)blockIdx.x * 2 * d + c] = s1[t] + s1[t + 64] + s1[t + 128] + s1[t + 192];
      colpart[(int64_t)blockIdx.x * 2 * d + d + c] = s2[t] + s2[t + 64] + s2[t + 128] + s2[t + 192];
    }
    __syncthreads();
  }
  if (last_block_arrived(cnt)) {
    for (int c = threadIdx.x; c < 2 * d; c += kT) {
      double s = 0.0;
      for (unsigned b = 0; b < gridDim.x; ++b) s += colpart[(int64_t)b * 2 * d + c];
      stats[c] = s / (double)n;
    }
    if (threadIdx.x == 0) *cnt = 0;
  }
}

__global__ void features_kernel(const double* __restrict__ E, int64_t n, int d, double lambda,
                                const double* __restrict__ stats, float* __restrict__ X) {
  const int in = 3 * d + 2;
  const int64_t total = n * in;
  const double ll = log(lambda), ln = log((double)n) / 10.0;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t i = idx / in;
    const int c = (int)(idx - i * in);
    double v;
    if (c < d) v = E[i * d + c];
    else if (c == d) v = ll;
    else if (c == d + 1) v = ln;
    else v = stats[c - d - 2];   // mean e (d values), then mean e^2 (d values)
    X[idx] = (float)v;
  }
}

__global__ void adam_kernel(float* __restrict__ th, float* __restrict__ m, float* __restrict__ v,
                            const float* __restrict__ g, int64_t count, float lr, float b1, float b2, float eps,
                            float c1, float c2) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < count; i += (int64_t)gridDim.x * kT) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

inline int grid_for(int64_t total) {
  int64_t g = (total + kT - 1) / kT;
  if (g > 4096) g = 4096;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

MlpLayout mlp_layout(int d) {
  MlpLayout L{};
  L.d = d;
  L.in_dim = 3 * d + 2;
  const int64_t sizes[6] = {(int64_t)L.in_dim * kHidden, kHidden, (int64_t)kHidden * kHidden, kHidden,
                            (int64_t)kHidden * kOut, kOut};
  int64_t o = 0;
  for (int t = 0; t < 6; ++t) {
    L.off[t] = o;
    o += (sizes[t] + 63) / 64 * 64;
  }
  L.count = o;
  L.block_bytes = ((size_t)o * sizeof(float) + 255) / 256 * 256;
  L.bytes = 3 * L.block_bytes;
  return L;
}

hipError_t mm_bf16(int64_t M, int64_t N, int64_t K, const float* A, int64_t sai, int64_t sak, const float* B,
                   int64_t sbk, int64_t sbj, float* part, int64_t part_cap, int epi, const float* bias,
                   const float* zpre, float* out, float* out2, hipStream_t st) {
  const int64_t tiles = ((M + MT - 1) / MT) * ((N + MT - 1) / MT);
  int64_t ns = (512 + tiles - 1) / tiles;
  const int64_t kchunks = (K + KC - 1) / KC;
  if (ns > kchunks) ns = kchunks;
  if (ns > 128) ns = 128;
  while (ns > 1 && ns * M * N > part_cap) --ns;
  if (ns < 1) ns = 1;
  if (M * N > part_cap) return hipErrorInvalidValue;
  int64_t kps = (K + ns - 1) / ns;
  kps = (kps + KC - 1) / KC * KC;
  ns = (K + kps - 1) / kps;
  if (ns < 1) ns = 1;
  dim3 grid((unsigned)((N + MT - 1) / MT), (unsigned)((M + MT - 1) / MT), (unsigned)ns);
  mm_bf16_kernel<<<grid, kT, 0, st>>>(M, N, K, A, sai, sak, B, sbk, sbj, part, kps);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  mm_epilogue_kernel<<<grid_for(M * N), kT, 0, st>>>(part, (int)ns, M, N, epi, bias, zpre, out, out2);
  return hipGetLastError();
}

hipError_t mlp_features(const double* E, int64_t n, int d, double lambda, float* X, double* colpart, double* stats,
                        unsigned* cnt, hipStream_t st) {
  int64_t g = (n + 255) / 256;
  if (g > kMaxBlocks) g = kMaxBlocks;
  colstat_kernel<<<(unsigned)g, kT, 0, st>>>(E, n, d, colpart, stats, cnt);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  features_kernel<<<grid_for(n * (3 * d + 2)), kT, 0, st>>>(E, n, d, lambda, stats, X);
  return hipGetLastError();
}

hipError_t adam_update(float* theta, float* m, float* v, const float* g, int64_t count, double lr, double beta1,
                       double beta2, double eps, int t, hipStream_t st) {
  const float c1 = (float)(1.0 - pow(beta1, (double)t));
  const float c2 = (float)(1.0 - pow(beta2, (double)t));
  adam_kernel<<<grid_for(count), kT, 0, st>>>(theta, m, v, g, count, (float)lr, (float)beta1, (float)beta2,
                                               (float)eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lk
