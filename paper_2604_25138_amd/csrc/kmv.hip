// Fused attention-kernel product  w = (lambda I + G) p  with G_ij = exp(s <e_i, e_j>)
// formed tile by tile and never stored (Sec. IV-D remark; Alg. 1 step size and
// residual update).  Also the rectangular query-by-site product of the map
// reconstruction (eq. sc-radio-map-reconstruction).
//
// Layout: prepared embeddings are row-major, rows padded with zero columns to
// dp in {16, 32, 64, 128}; zero columns leave every inner product unchanged.
// A launch covers (row block) x (column split); each split writes its partial
// sums, and a second pass adds the splits in a fixed order.
#include "internal.hpp"

namespace lk {

namespace {

constexpr double kLog2e = 1.4426950408889634074;

__global__ void prep_embed_f64_kernel(const double* __restrict__ E, int64_t rows, int d, int dp,
                                      double c, double* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * dp) return;
  int64_t i = idx / dp;
  int col = (int)(idx - i * dp);
  out[idx] = col < d ? c * E[i * d + col] : 0.0;
}

__global__ void prep_embed_f32_kernel(const double* __restrict__ E, int64_t rows, int d, int dp,
                                      double c, float* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * dp) return;
  int64_t i = idx / dp;
  int col = (int)(idx - i * dp);
  out[idx] = col < d ? __double2float_rn(c * E[i * d + col]) : 0.0f;
}

// bfloat16 by round-to-nearest-even from the float32 value (NaN-free inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

__global__ void prep_embed_bf16_kernel(const double* __restrict__ E, int64_t rows, int d, int dp,
                                       double c, uint16_t* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * dp) return;
  int64_t i = idx / dp;
  int col = (int)(idx - i * dp);
  out[idx] = col < d ? f32_to_bf16_rne(__double2float_rn(c * E[i * d + col])) : (uint16_t)0;
}

__device__ __forceinline__ double kexp(double x) { return exp(x); }
__device__ __forceinline__ float kexp(float x) { return __builtin_amdgcn_exp2f(x); }

// One thread per output row; key tiles of 64 rows staged in LDS and read as
// broadcasts.  Used for float64 (and as the float32 product before MFMA).
template <typename T, int DP>
__global__ __launch_bounds__(256) void kmv_valu_kernel(const T* __restrict__ Q, int64_t m,
                                                       const T* __restrict__ K, int64_t n,
                                                       const T* __restrict__ p, T* __restrict__ part,
                                                       int64_t cps, const int* __restrict__ done) {
  if (done != nullptr && *done) return;
  constexpr int BN = 64;
  __shared__ T ks[BN * DP];
  __shared__ T ps[BN];
  const int tid = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 256 + tid;
  T q[DP];
  if (i < m) {
#pragma unroll
    for (int c = 0; c < DP; ++c) q[c] = Q[i * DP + c];
  } else {
#pragma unroll
    for (int c = 0; c < DP; ++c) q[c] = T(0);
  }
  const int64_t j0 = (int64_t)blockIdx.y * cps;
  const int64_t j1 = j0 + cps < n ? j0 + cps : n;
  T acc = T(0);
  for (int64_t jt = j0; jt < j1; jt += BN) {
    __syncthreads();
    const int64_t base = jt * DP;
    const int64_t lim = (j1 - jt) * DP;
    for (int idx = tid; idx < BN * DP; idx += 256) ks[idx] = idx < lim ? K[base + idx] : T(0);
    if (tid < BN) ps[tid] = (jt + tid < j1) ? p[jt + tid] : T(0);
    __syncthreads();
    for (int jj = 0; jj < BN; ++jj) {
      T sc = T(0);
#pragma unroll
      for (int c = 0; c < DP; ++c) sc = fma(q[c], ks[jj * DP + c], sc);
      acc = fma(kexp(sc), ps[jj], acc);
    }
  }
  if (i < m) part[(int64_t)blockIdx.y * m + i] = acc;
}

template <typename T, typename W>
__global__ void kmv_finish_kernel(int64_t m, T lam, const T* __restrict__ p, const T* __restrict__ part,
                                  int nsplit, W* __restrict__ w) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    T s = T(0);
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * m + i];
    w[i] = (W)(p != nullptr ? fma(lam, p[i], s) : s);
  }
}

template <typename S, typename D>
__global__ void convert_kernel(const S* __restrict__ src, D* __restrict__ dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = (D)src[i];
}

inline int grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

template <typename T>
hipError_t launch_valu(int dp, const T* Q, int64_t m, const T* K, int64_t n, const T* p, T* part,
                       const KmvPlan& plan, const int* done, hipStream_t st) {
  dim3 grid((unsigned)((m + 255) / 256), (unsigned)plan.nsplit);
  switch (dp) {
    case 16: kmv_valu_kernel<T, 16><<<grid, 256, 0, st>>>(Q, m, K, n, p, part, plan.cols_per_split, done); break;
    case 32: kmv_valu_kernel<T, 32><<<grid, 256, 0, st>>>(Q, m, K, n, p, part, plan.cols_per_split, done); break;
    case 64: kmv_valu_kernel<T, 64><<<grid, 256, 0, st>>>(Q, m, K, n, p, part, plan.cols_per_split, done); break;
    case 128: kmv_valu_kernel<T, 128><<<grid, 256, 0, st>>>(Q, m, K, n, p, part, plan.cols_per_split, done); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t embed_bytes(int64_t rows, int dp, int prec) {
  size_t el = prec == LAKER_F64 ? 8 : (prec == LAKER_F32 ? 4 : 2);
  return (size_t)rows * (size_t)dp * el;
}

hipError_t prep_embed(const double* E, int64_t rows, int d, int dp, double scale, int prec, void* out,
                      hipStream_t st) {
  const int64_t total = rows * dp;
  const int g = (int)((total + 255) / 256);
  if (total == 0) return hipSuccess;
  if (prec == LAKER_F64) {
    prep_embed_f64_kernel<<<g, 256, 0, st>>>(E, rows, d, dp, sqrt(scale), (double*)out);
  } else if (prec == LAKER_F32) {
    prep_embed_f32_kernel<<<g, 256, 0, st>>>(E, rows, d, dp, sqrt(scale * kLog2e), (float*)out);
  } else {
    prep_embed_bf16_kernel<<<g, 256, 0, st>>>(E, rows, d, dp, sqrt(scale * kLog2e), (uint16_t*)out);
  }
  return hipGetLastError();
}

KmvPlan kmv_plan(int64_t m, int64_t n, int prec) {
  (void)prec;
  const int64_t rowblocks = (m + 255) / 256;
  const int64_t coltiles = (n + 63) / 64;
  int64_t ns = (2048 + rowblocks - 1) / rowblocks;
  if (ns > coltiles) ns = coltiles;
  if (ns > 64) ns = 64;
  if (ns < 1) ns = 1;
  int64_t cps = ((coltiles + ns - 1) / ns) * 64;
  KmvPlan pl;
  pl.cols_per_split = cps;
  pl.nsplit = (int)((n + cps - 1) / cps);
  if (pl.nsplit < 1) pl.nsplit = 1;
  return pl;
}

hipError_t kmv_partials(int prec, int dp, const void* Q, int64_t m, const void* K, int64_t n, const void* p,
                        void* part, const KmvPlan& plan, const int* done, hipStream_t st) {
  if (prec == LAKER_F64)
    return launch_valu<double>(dp, (const double*)Q, m, (const double*)K, n, (const double*)p,
                               (double*)part, plan, done, st);
  if (prec == LAKER_F32)
    return launch_valu<float>(dp, (const float*)Q, m, (const float*)K, n, (const float*)p, (float*)part,
                              plan, done, st);
  return hipErrorInvalidValue;
}

hipError_t kmv_finish(int prec, int64_t m, double lam, const void* p, const void* part, int nsplit, void* w,
                      bool w_double, hipStream_t st) {
  const int g = grid_for(m, 256);
  if (prec == LAKER_F64) {
    kmv_finish_kernel<double, double><<<g, 256, 0, st>>>(m, lam, (const double*)p, (const double*)part,
                                                         nsplit, (double*)w);
  } else if (w_double) {
    kmv_finish_kernel<float, double><<<g, 256, 0, st>>>(m, (float)lam, (const float*)p, (const float*)part,
                                                        nsplit, (double*)w);
  } else {
    kmv_finish_kernel<float, float><<<g, 256, 0, st>>>(m, (float)lam, (const float*)p, (const float*)part,
                                                       nsplit, (float*)w);
  }
  return hipGetLastError();
}

hipError_t convert_vec(const void* src, int src_prec, void* dst, int dst_prec, int64_t n, hipStream_t st) {
  const int g = grid_for(n, 256);
  const bool sd = src_prec == LAKER_F64, dd = dst_prec == LAKER_F64;
  if (sd && dd) convert_kernel<double, double><<<g, 256, 0, st>>>((const double*)src, (double*)dst, n);
  else if (sd) convert_kernel<double, float><<<g, 256, 0, st>>>((const double*)src, (float*)dst, n);
  else if (dd) convert_kernel<float, double><<<g, 256, 0, st>>>((const float*)src, (double*)dst, n);
  else convert_kernel<float, float><<<g, 256, 0, st>>>((const float*)src, (float*)dst, n);
  return hipGetLastError();
}

}  // namespace lk
