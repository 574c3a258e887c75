// Kernel product for several right-hand sides at once:
//     W = (lambda I + G) P,   P = [p_1 ... p_k]   (k <= kMaxRhs columns),
// for the solves of several bands or snapshots that share one set of
// measurement sites (the same E, hence the same G).  Each score tile
// S = Q K^T (MFMA) and its exponentials are formed once and multiplied by the
// k columns' weights, so the MFMA work and the exponentials -- the bulk of a
// product -- are shared by all columns; only the multiply-adds grow with k.
//
// Work split (column-range schedule): a block of four waves owns 64 rows, each
// wave 16 of them, and sweeps the key rows of one column range in 16-key
// tiles (16x16 MFMA tiles: four entries per lane, so that k columns of
// float64 accumulators fit in registers).  float32 / bfloat16 key rows and
// the columns' weights are staged through LDS in stages of KT keys
// (double-buffered, one barrier per stage); float64 key fragments are read
// straight from global memory one tile ahead.  Sums: float32 within a stage
// (float32 / bfloat16), float64 across stages; one float64 partial per
// (column, row, column range), added in a fixed order by the pass that uses
// them, exactly as for one column.
#include <type_traits>

#include "kmv_multi.hpp"

namespace lk {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int kMT = 256;    // threads per block
constexpr int kRows = 64;   // rows per block (16 per wave)

__device__ __forceinline__ float kexp2m(float x) { return __builtin_amdgcn_exp2f(x); }

// Run-state bookkeeping of a PCG step: true when every column has stopped
// (the launch then returns at once); block (0, 0) advances the iteration
// counter of the columns still running.
__device__ __forceinline__ bool multi_all_done(const KmvMultiArgs& A) {
  if (A.S == nullptr) return false;
  for (int q = 0; q < A.k; ++q)
    if (!A.S[q].done) return false;
  return true;
}
__device__ __forceinline__ void multi_step(const KmvMultiArgs& A, int64_t bx, int64_t by) {
  if (A.S != nullptr && A.pcg_step && bx == 0 && by == 0 && threadIdx.x < A.k && !A.S[threadIdx.x].done)
    A.S[threadIdx.x].kcur += 1;
}

// ---- float32 / bfloat16 ------------------------------------------------------
//
// 16x16 tiles: v_mfma_f32_16x16x32_bf16 (a lane (c, h) = (lane % 16, lane / 16)
// supplies row c and 8 consecutive of the 32 depth indices, 8 h ..) and
// v_mfma_f32_16x16x4_f32 (a lane supplies row c, one depth index h of each
// step of four); any assignment of depth indices works as long as the query
// and key fragments use the same one, so each lane reads one contiguous run of
// its rows.  Output: lane (c, h) holds rows 4 h + r (r < 4) of key column c.
template <int PREC, int DP>
struct MStage {
  using ET = typename std::conditional<PREC == LAKER_F32, float, uint16_t>::type;
  static constexpr int ES = (int)sizeof(ET);
  static constexpr int ROWB = DP * ES;
  // key rows per stage: 16 KB of them (at most 128), a multiple of 16
  static constexpr int KT0 = 16384 / ROWB;
  static constexpr int KT = KT0 > 128 ? 128 : (KT0 < 16 ? 16 : KT0 / 16 * 16);
  static constexpr int PITCH = ROWB + 16;            // padded LDS row pitch
  static constexpr int CHUNKS = KT * ROWB / 16;      // 16-byte chunks of a stage's key rows
  static constexpr int PER_T = (CHUNKS + kMT - 1) / kMT;
  // depth steps and the elements a lane supplies per step
  static constexpr int STEPS = PREC == LAKER_F32 ? DP / 4 : (DP + 31) / 32;
  static constexpr int LANE_ELEMS = PREC == LAKER_F32 ? DP / 4 : 8;
};

template <int PREC, int DP>
struct MFrag {
  using St = MStage<PREC, DP>;
  // float32: v[s] is depth index h (DP / 4) + s; bfloat16: w[s] holds depth
  // indices 32 s + 8 h .. + 7 (zero past DP)
  float v[PREC == LAKER_F32 ? DP / 4 : 1];
  v8bf w[PREC == LAKER_F32 ? 1 : St::STEPS];
  __device__ __forceinline__ void load_row(const unsigned char* rowp, int h) {
    if constexpr (PREC == LAKER_F32) {
      const float* src = reinterpret_cast<const float*>(rowp) + h * (DP / 4);
#pragma unroll
      for (int q = 0; q < DP / 16; ++q) {
        const float4 t = *reinterpret_cast<const float4*>(src + 4 * q);
        v[4 * q + 0] = t.x;
        v[4 * q + 1] = t.y;
        v[4 * q + 2] = t.z;
        v[4 * q + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int s = 0; s < St::STEPS; ++s) {
        const int off = 32 * s + 8 * h;
        if (off < DP) {
          w[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4*>(rowp + 2 * off));
        } else {
          u32x4 z = {0u, 0u, 0u, 0u};
          w[s] = __builtin_bit_cast(v8bf, z);
        }
      }
    }
  }
};

template <int PREC, int DP>
__device__ __forceinline__ v4f mtile(const MFrag<PREC, DP>& a, const MFrag<PREC, DP>& b) {
  v4f c = {0.f, 0.f, 0.f, 0.f};
  if constexpr (PREC == LAKER_F32) {
#pragma unroll
    for (int s = 0; s < DP / 4; ++s) c = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[s], b.v[s], c, 0, 0, 0);
  } else {
#pragma unroll
    for (int s = 0; s < MStage<PREC, DP>::STEPS; ++s)
      c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.w[s], b.w[s], c, 0, 0, 0);
  }
  return c;
}

template <int PREC, int DP, int NR>
__global__ __launch_bounds__(kMT) void kmvm32_kernel(KmvMultiArgs A) {
  using St = MStage<PREC, DP>;
  constexpr int KT = St::KT;
  __shared__ __attribute__((aligned(16))) unsigned char keys[2][KT * St::PITCH];
  __shared__ float wts[2][NR][KT];
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  if (multi_all_done(A)) return;
  multi_step(A, bx, by);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 4, c = lane & 15;
  const int64_t row0 = bx * kRows + wv * 16;
  const int64_t j0 = by * A.cps;
  const int64_t j1 = j0 + A.cps < A.n ? j0 + A.cps : A.n;
  const int k = A.k;
  const unsigned char* __restrict__ Qb = reinterpret_cast<const unsigned char*>(A.Q);
  const unsigned char* __restrict__ Kb = reinterpret_cast<const unsigned char*>(A.K);
  const double* __restrict__ P = A.P;

  MFrag<PREC, DP> a;
  {
    int64_t qi = row0 + c;
    if (qi > A.m - 1) qi = A.m - 1;
    a.load_row(Qb + qi * St::ROWB, h);
  }
  double acc[NR][4];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[q][r] = 0.0;

  const int nstages = (int)((j1 - j0 + KT - 1) / KT);
  u32x4 stg[St::PER_T];
  float stw[NR];
  // global -> registers for the stage at key row js (rows clamped to n - 1 in
  // the last stage, their weights zero past the column range)
  auto fetch = [&](int64_t js) {
#pragma unroll
    for (int q = 0; q < St::PER_T; ++q) {
      const int ch = tid + kMT * q;
      if (St::CHUNKS % kMT == 0 || ch < St::CHUNKS) {
        const int rr = ch / (St::ROWB / 16);
        const int cc = ch - rr * (St::ROWB / 16);
        int64_t kr = js + rr;
        if (kr > A.n - 1) kr = A.n - 1;
        stg[q] = *reinterpret_cast<const u32x4*>(Kb + kr * St::ROWB + cc * 16);
      }
    }
    if (tid < KT) {
      const int64_t kj = js + tid;
      const bool ok = kj < j1;
      const int64_t kc = ok ? kj : 0;
#pragma unroll
      for (int q = 0; q < NR; ++q) stw[q] = (ok && q < k) ? (float)P[(int64_t)q * A.n + kc] : 0.f;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < St::PER_T; ++q) {
      const int ch = tid + kMT * q;
      if (St::CHUNKS % kMT == 0 || ch < St::CHUNKS) {
        const int rr = ch / (St::ROWB / 16);
        const int cc = ch - rr * (St::ROWB / 16);
        *reinterpret_cast<u32x4*>(&keys[buf][rr * St::PITCH + cc * 16]) = stg[q];
      }
    }
    if (tid < KT) {
#pragma unroll
      for (int q = 0; q < NR; ++q) wts[buf][q][tid] = stw[q];
    }
  };
  if (nstages > 0) {
    fetch(j0);
    store(0);
    if (nstages > 1) fetch(j0 + KT);
    __syncthreads();
  }
  for (int sidx = 0; sidx < nstages; ++sidx) {
    const int buf = sidx & 1;
    if (sidx + 1 < nstages) store(buf ^ 1);
    if (sidx + 2 < nstages) fetch(j0 + (int64_t)(sidx + 2) * KT);
    float accf[NR][4];
#pragma unroll
    for (int u = 0; u < KT / 16; ++u) {
      MFrag<PREC, DP> b;
      b.load_row(&keys[buf][(u * 16 + c) * St::PITCH], h);
      const v4f sc = mtile<PREC, DP>(a, b);
      float e[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) e[r] = kexp2m(sc[r]);
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const float wq = wts[buf][q][u * 16 + c];
#pragma unroll
        for (int r = 0; r < 4; ++r) accf[q][r] = u == 0 ? e[r] * wq : fmaf(e[r], wq, accf[q][r]);
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[q][r] += (double)accf[q][r];
    __syncthreads();
  }
  // sum over the 16 key columns of each lane group, then lane (c < 4, h)
  // writes row 4 h + c of every column
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = acc[q][r];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      acc[q][r] = v;
    }
  if (c < 4) {
    const int64_t row = row0 + 4 * h + c;
    if (row < A.m) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        if (q < k) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) v = (r == c) ? acc[q][r] : v;
          A.part[((int64_t)q * A.nsplit + by) * A.m + row] = v;
        }
      }
    }
  }
}

// ---- float64 -----------------------------------------------------------------
//
// 16x16x4 f64 MFMA tiles, exp in float64; output: register r of lane
// (c, h) holds row 4 r + h of key column c.
template <int DP>
struct MFrag64 {
  double v[DP / 4];
  __device__ __forceinline__ void load(const double* __restrict__ base, int64_t row, int h) {
    const double2* src = reinterpret_cast<const double2*>(base + row * DP + h * (DP / 4));
#pragma unroll
    for (int q = 0; q < DP / 8; ++q) {
      const double2 t = src[q];
      v[2 * q + 0] = t.x;
      v[2 * q + 1] = t.y;
    }
  }
};

template <int DP>
__device__ __forceinline__ v4d mtile64(const MFrag64<DP>& a, const MFrag64<DP>& b) {
  v4d c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < DP / 4; ++s) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[s], b.v[s], c, 0, 0, 0);
  return c;
}

template <int DP, int NR>
__global__ __launch_bounds__(kMT) void kmvm64_kernel(KmvMultiArgs A) {
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  if (multi_all_done(A)) return;
  multi_step(A, bx, by);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int h = lane >> 4, c = lane & 15;
  const int64_t row0 = bx * kRows + wv * 16;
  const int64_t j0 = by * A.cps;
  const int64_t j1 = j0 + A.cps < A.n ? j0 + A.cps : A.n;
  const int k = A.k;
  const double* __restrict__ Q = reinterpret_cast<const double*>(A.Q);
  const double* __restrict__ K = reinterpret_cast<const double*>(A.K);
  const double* __restrict__ P = A.P;
  MFrag64<DP> a, b, bn;
  {
    int64_t qi = row0 + c;
    if (qi > A.m - 1) qi = A.m - 1;
    a.load(Q, qi, h);
  }
  double acc[NR][4];
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[q][r] = 0.0;
  auto weights = [&](int64_t jt, double* w) {
    const int64_t kj = jt + c;
    const bool ok = kj < j1;
    const int64_t kc = ok ? kj : 0;
#pragma unroll
    for (int q = 0; q < NR; ++q) w[q] = (ok && q < k) ? P[(int64_t)q * A.n + kc] : 0.0;
  };
  if (j0 < j1) {
    double pj[NR], pn[NR];
    weights(j0, pj);
    {
      int64_t kj = j0 + c;
      if (kj > A.n - 1) kj = A.n - 1;
      b.load(K, kj, h);
    }
    for (int64_t jt = j0; jt < j1; jt += 16) {
      const int64_t jn = jt + 16;
      if (jn < j1) {
        weights(jn, pn);
        int64_t kn = jn + c;
        if (kn > A.n - 1) kn = A.n - 1;
        bn.load(K, kn, h);
      }
      const v4d s = mtile64<DP>(a, b);
      double e[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) e[r] = exp(s[r]);
#pragma unroll
      for (int q = 0; q < NR; ++q)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[q][r] = fma(e[r], pj[q], acc[q][r]);
      if (jn < j1) {
        b = bn;
#pragma unroll
        for (int q = 0; q < NR; ++q) pj[q] = pn[q];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NR; ++q)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = acc[q][r];
      v += __shfl_xor(v, 1, 64);
      v += __shfl_xor(v, 2, 64);
      v += __shfl_xor(v, 4, 64);
      v += __shfl_xor(v, 8, 64);
      acc[q][r] = v;
    }
  if (c < 4) {
    const int64_t row = row0 + 4 * c + h;
    if (row < A.m) {
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        if (q < k) {
          double v = 0.0;
#pragma unroll
          for (int r = 0; r < 4; ++r) v = (r == c) ? acc[q][r] : v;
          A.part[((int64_t)q * A.nsplit + by) * A.m + row] = v;
        }
      }
    }
  }
}

// out[q][i] = lam pself[q][i] + sum_s part[q][s][i] (column ranges in order)
__global__ __launch_bounds__(256) void kmvm_finish_kernel(const double* __restrict__ part, int nsplit, int64_t m,
                                                          double lam, const double* __restrict__ pself,
                                                          double* __restrict__ out) {
  const int q = blockIdx.y;
  const double* pp = part + (int64_t)q * nsplit * m;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int t = 0; t < nsplit; ++t) s += pp[(int64_t)t * m + i];
    out[(int64_t)q * m + i] = pself != nullptr ? fma(lam, pself[(int64_t)q * m + i], s) : s;
  }
}

template <int PREC, int DP>
hipError_t launch_m32(int k, dim3 grid, const KmvMultiArgs& A, hipStream_t st) {
  if (k <= 2) kmvm32_kernel<PREC, DP, 2><<<grid, kMT, 0, st>>>(A);
  else if (k <= 4) kmvm32_kernel<PREC, DP, 4><<<grid, kMT, 0, st>>>(A);
  else kmvm32_kernel<PREC, DP, 8><<<grid, kMT, 0, st>>>(A);
  return hipGetLastError();
}

template <int DP>
hipError_t launch_m64(int k, dim3 grid, const KmvMultiArgs& A, hipStream_t st) {
  if (k <= 2) kmvm64_kernel<DP, 2><<<grid, kMT, 0, st>>>(A);
  else if (k <= 4) kmvm64_kernel<DP, 4><<<grid, kMT, 0, st>>>(A);
  else kmvm64_kernel<DP, 8><<<grid, kMT, 0, st>>>(A);
  return hipGetLastError();
}

}  // namespace

KmvMultiPlan kmv_multi_plan(int64_t m, int64_t n) {
  KmvMultiPlan pl{};
  pl.rowblocks = (int)((m + kRows - 1) / kRows);
  // enough blocks to fill the chip several times over: column ranges of at
  // least 512 keys, at most kMaxSplit of them
  int64_t ns = (2048 + pl.rowblocks - 1) / pl.rowblocks;
  const int64_t maxs = (n + 511) / 512;
  if (ns > maxs) ns = maxs;
  if (ns > kMaxSplit) ns = kMaxSplit;
  if (ns < 1) ns = 1;
  int64_t cps = (n + ns - 1) / ns;
  cps = (cps + 127) / 128 * 128;
  pl.cols_per_split = cps;
  pl.nsplit = (int)((n + cps - 1) / cps);
  return pl;
}

size_t kmv_multi_part_elems(int64_t m, int64_t n, int k) {
  const KmvMultiPlan pl = kmv_multi_plan(m, n);
  return (size_t)k * (size_t)pl.nsplit * (size_t)m;
}

hipError_t kmv_multi_run(int prec, int dp, KmvMultiArgs A, hipStream_t st) {
  if (A.k < 1 || A.k > kMaxRhs) return hipErrorInvalidValue;
  const KmvMultiPlan pl = kmv_multi_plan(A.m, A.n);
  A.cps = pl.cols_per_split;
  A.nsplit = pl.nsplit;
  const dim3 grid((unsigned)pl.rowblocks, (unsigned)pl.nsplit);
  hipError_t e;
  if (prec == LAKER_F64) {
    switch (dp) {
      case 16: e = launch_m64<16>(A.k, grid, A, st); break;
      case 32: e = launch_m64<32>(A.k, grid, A, st); break;
      case 64: e = launch_m64<64>(A.k, grid, A, st); break;
      case 128: e = launch_m64<128>(A.k, grid, A, st); break;
      default: return hipErrorInvalidValue;
    }
  } else if (prec == LAKER_F32) {
    switch (dp) {
      case 16: e = launch_m32<LAKER_F32, 16>(A.k, grid, A, st); break;
      case 32: e = launch_m32<LAKER_F32, 32>(A.k, grid, A, st); break;
      case 64: e = launch_m32<LAKER_F32, 64>(A.k, grid, A, st); break;
      case 128: e = launch_m32<LAKER_F32, 128>(A.k, grid, A, st); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (dp) {
      case 16: e = launch_m32<LAKER_BF16, 16>(A.k, grid, A, st); break;
      case 32: e = launch_m32<LAKER_BF16, 32>(A.k, grid, A, st); break;
      case 64: e = launch_m32<LAKER_BF16, 64>(A.k, grid, A, st); break;
      case 128: e = launch_m32<LAKER_BF16, 128>(A.k, grid, A, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  if (e != hipSuccess || !A.finish) return e;
  int64_t g = (A.m + 255) / 256;
  if (g > 1024) g = 1024;
  kmvm_finish_kernel<<<dim3((unsigned)g, (unsigned)A.k), 256, 0, st>>>(A.part, A.nsplit, A.m, A.lam, A.pself,
                                                                       A.out);
  return hipGetLastError();
}

}  // namespace lk
