// Shared device helpers and the host-side workspace carver of the LAKER library.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stddef.h>
#include <stdint.h>

#include "laker.h"

#define LK_TRY(call)                                  \
  do {                                                \
    hipError_t lk_e_ = (call);                        \
    if (lk_e_ != hipSuccess) return LAKER_EHIP;       \
  } while (0)

#define LK_CHECK_LAUNCH() LK_TRY(hipGetLastError())

namespace lk {

constexpr int kWave = 64;
constexpr int kMaxBlocks = 1024;     // upper bound of blocks taking part in one grid reduction
constexpr int kMaxNr = 1024;         // largest low-rank preconditioner rank
constexpr int kMaxD = 128;           // largest embedding dimension

// Device-resident scalars of one PCG run.  Kernels read `done` first and return
// at once when it is set, so the host can enqueue a chunk of iterations ahead
// of its convergence check.
struct PcgScalars {
  double rzbuf[2];  // r^T theta of iteration k in slot k & 1 (read and written by different launches)
  double pap;       // p^T A p
  double delta;     // step size
  double beta;      // conjugation coefficient
  double rr;        // ||r||^2 (recursive residual)
  double yy;        // ||y||^2 of the right-hand side
  double tol2;      // tol^2 * ||y||^2
  int iters;
  int max_iter;
  int done;         // 0 running, 1 converged, 2 breakdown, 3 iteration cap
  int kcur;         // iterations started: the product launch of iteration k sets it to k + 1
  // conjugation inside the product kernel (symmetric product, low-rank
  // preconditioner): r^T theta of the previous iteration, and 1 until the
  // first step update of a (re)started solve (beta = 0)
  double rzold;
  int first;
  unsigned cnt[8];  // arrival counters of the grid reductions (kept at zero between uses)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Fixed-order block sum (blockDim.x multiple of 64, <= 1024).  Result valid in
// every thread.  `sh` must hold 16 doubles.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const int nw = blockDim.x >> 6;
  double s = 0.0;
  for (int k = 0; k < nw; ++k) s += sh[k];
  return s;
}

// Grid-reduction arrival: returns true in every thread of the last block to
// arrive.  Writers must have stored their partials before calling.
__device__ __forceinline__ bool last_block_arrived(unsigned* cnt) {
  __shared__ int am_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned t = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (t == gridDim.x * gridDim.y * gridDim.z - 1) ? 1 : 0;
  }
  __syncthreads();
  if (am_last) __threadfence();
  return am_last != 0;
}

// As last_block_arrived, for a grid whose first `total` blocks take part.
__device__ __forceinline__ bool last_block_arrived_of(unsigned* cnt, unsigned total) {
  __shared__ int am_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    unsigned t = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (t == total - 1) ? 1 : 0;
  }
  __syncthreads();
  if (am_last) __threadfence();
  return am_last != 0;
}

// Sum of `count` doubles written by other blocks, in index order, by the whole
// block; valid in every thread.
__device__ __forceinline__ double ordered_sum(const double* part, int count, double* sh) {
  double v = 0.0;
  // each thread sums a contiguous stripe, then stripes are combined in order
  const int per = (count + blockDim.x - 1) / blockDim.x;
  const int b = threadIdx.x * per;
  for (int k = 0; k < per; ++k) {
    int idx = b + k;
    if (idx < count) v += __builtin_nontemporal_load(part + idx);
  }
  // ordered combination across threads: wave prefix order is fixed by the xor tree
  return block_sum(v, sh);
}

template <typename T> struct Acc;
template <> struct Acc<double> { using type = double; };
template <> struct Acc<float> { using type = float; };

}  // namespace lk

// ---------------------------------------------------------------------------
// Host: carve a caller-provided workspace into aligned pieces.  The same plan
// code runs to size the workspace (base == nullptr) and to hand out pointers.
// ---------------------------------------------------------------------------
struct WsCarver {
  char* base;
  size_t off = 0;
  explicit WsCarver(void* b) : base(static_cast<char*>(b)) {}
  template <typename T> T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t bytes() const { return (off + 255) & ~size_t(255); }
};

inline int pad_dim(int d) {
  if (d <= 16) return 16;
  if (d <= 32) return 32;
  if (d <= 64) return 64;
  return 128;
}
