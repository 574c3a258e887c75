// Fused attention-kernel product  w = (lambda I + G) p  with G_ij = exp(s <e_i, e_j>)
// formed tile by tile on the matrix cores and never stored (Sec. IV-D remark;
// Alg. 1 step size and residual update).  The same kernel computes the
// rectangular query-by-site product of the map reconstruction
// (eq. sc-radio-map-reconstruction).
//
// Layout: prepared embeddings are row-major with rows padded by zero columns to
// dp in {16, 32, 64, 128} (zero columns leave every inner product unchanged).
// float32 / bfloat16 copies are pre-scaled by sqrt(s log2 e) so that the MFMA
// output is directly the exp2 argument; float64 copies by sqrt(s) (exp).
//
// Work split (rectangular kernels): a wave owns 32 rows (16 for float64) and
// sweeps the key tiles of one column range; a block holds four waves.  The
// symmetric kernels below split a 256-row block differently.  The score tile
// S = Q K^T comes from MFMA (32x32x2 f32, 32x32x16 or 16x16x32 bf16, 16x16x4
// f64); each lane then applies exp to its S entries and accumulates
// exp(S) p_j into per-row partial sums (float64 across stages, float32 within
// a stage), which are combined across lanes once at the end.  Column ranges
// write partial sums; a following pass adds them in a fixed order and applies
// lambda p.  Inside PCG the symmetric kernels also form p^T A p from the
// partials they write (one float64 per block), and the step-update pass adds
// the partials of each row itself.
#include <type_traits>

#include "internal.hpp"

namespace lk {

namespace {

constexpr double kLog2e = 1.4426950408889634074;

typedef float v16f __attribute__((ext_vector_type(16)));
typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__global__ void prep_embed_f64_kernel(const double* __restrict__ E, int64_t rows, int d, int dp, double c,
                                      double* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * dp) return;
  int64_t i = idx / dp;
  int col = (int)(idx - i * dp);
  out[idx] = col < d ? c * E[i * d + col] : 0.0;
}

__global__ void prep_embed_f32_kernel(const double* __restrict__ E, int64_t rows, int d, int dp, double c,
                                      float* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * dp) return;
  int64_t i = idx / dp;
  int col = (int)(idx - i * dp);
  out[idx] = col < d ? __double2float_rn(c * E[i * d + col]) : 0.0f;
}

// bfloat16 by round-to-nearest-even from the float32 value (finite inputs).
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

__global__ void prep_embed_bf16_kernel(const double* __restrict__ E, int64_t rows, int d, int dp, double c,
                                       uint16_t* __restrict__ out) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * dp) return;
  int64_t i = idx / dp;
  int col = (int)(idx - i * dp);
  out[idx] = col < d ? f32_to_bf16_rne(__double2float_rn(c * E[i * d + col])) : (uint16_t)0;
}

// ---------------------------------------------------------------------------
// Fragments.  For an MFMA step kk the lane (c, h) -- c = lane % T, h = lane / T
// with T = 32 (16 for f64) -- supplies k-index  h * (dp / H) + (k within step),
// H = 64 / T.  Any assignment of k to steps is valid as long as the Q and K
// fragments use the same one; this one makes each lane's share of a row one
// contiguous run of dp / H elements.
// ---------------------------------------------------------------------------
template <int DP>
struct FragF32 {
  float v[DP / 2];
  __device__ __forceinline__ void load(const float* __restrict__ base, int64_t row, int h) {
    const float4* src = reinterpret_cast<const float4*>(base + row * DP + h * (DP / 2));
#pragma unroll
    for (int q = 0; q < DP / 8; ++q) {
      float4 t = src[q];
      v[4 * q + 0] = t.x;
      v[4 * q + 1] = t.y;
      v[4 * q + 2] = t.z;
      v[4 * q + 3] = t.w;
    }
  }
};

template <int DP>
__device__ __forceinline__ v16f tile_f32(const FragF32<DP>& a, const FragF32<DP>& b) {
  v16f c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < DP / 2; ++kk) c = __builtin_amdgcn_mfma_f32_32x32x2f32(a.v[kk], b.v[kk], c, 0, 0, 0);
  return c;
}

template <int DP>
struct FragBF16 {
  v8bf v[DP / 16];
  __device__ __forceinline__ void load(const uint16_t* __restrict__ base, int64_t row, int h) {
    const u32x4* src = reinterpret_cast<const u32x4*>(base + row * DP + h * (DP / 2));
#pragma unroll
    for (int q = 0; q < DP / 16; ++q) {
      u32x4 t = src[q];
      v[q] = __builtin_bit_cast(v8bf, t);
    }
  }
};

template <int DP>
__device__ __forceinline__ v16f tile_bf16(const FragBF16<DP>& a, const FragBF16<DP>& b) {
  v16f c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < DP / 16; ++kk) c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a.v[kk], b.v[kk], c, 0, 0, 0);
  return c;
}

template <int DP>
struct FragF64 {
  double v[DP / 4];
  __device__ __forceinline__ void load(const double* __restrict__ base, int64_t row, int h) {
    const double2* src = reinterpret_cast<const double2*>(base + row * DP + h * (DP / 4));
#pragma unroll
    for (int q = 0; q < DP / 8; ++q) {
      double2 t = src[q];
      v[2 * q + 0] = t.x;
      v[2 * q + 1] = t.y;
    }
  }
};

template <int DP>
__device__ __forceinline__ v4d tile_f64(const FragF64<DP>& a, const FragF64<DP>& b) {
  v4d c = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < DP / 4; ++kk) c = __builtin_amdgcn_mfma_f64_16x16x4f64(a.v[kk], b.v[kk], c, 0, 0, 0);
  return c;
}

// ---------------------------------------------------------------------------
// Finish: out_i = lam * pself_i + sum_s part[s][i], the column ranges added in a
// fixed order.  A separate launch: completing a reduction inside the product
// with per-block atomic tickets serializes ~40 ns of fence and atomic per
// block, more than this pass costs.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void kmv_finish_kernel(const double* __restrict__ part, PartSum ps, int64_t m,
                                                         double lam, const double* __restrict__ pself,
                                                         double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < m; i += (int64_t)gridDim.x * 256) {
    const double s = ps.row(part, m, i);
    out[i] = pself != nullptr ? fma(lam, pself[i], s) : s;
  }
}

__device__ __forceinline__ float kexp2(float x) { return __builtin_amdgcn_exp2f(x); }

// ---------------------------------------------------------------------------
// float32 / bfloat16 kernel: 32x32 score tiles.
//
// The key rows of a column range are staged through LDS in stages of KT rows,
// double-buffered and shared by the block's four waves: the global loads of
// stage s + 1 are issued before stage s is consumed and written to LDS after
// it, with one barrier per stage.  LDS rows are padded by 16 bytes so that the
// 16-byte fragment reads of 32 consecutive rows fall in distinct banks.
// ---------------------------------------------------------------------------
template <int PREC, int DP>
struct Stage32 {
  using ET = typename std::conditional<PREC == LAKER_F32, float, uint16_t>::type;
  static constexpr int ES = (int)sizeof(ET);
  static constexpr int ROWB = DP * ES;                               // bytes of one key row
#ifndef LAKER_KMV_STAGE_BYTES
#define LAKER_KMV_STAGE_BYTES 16384
#endif
  static constexpr int KT0 = LAKER_KMV_STAGE_BYTES / ROWB;
  static constexpr int KT = KT0 > 128 ? 128 : (KT0 < 32 ? 32 : KT0);  // key rows per stage
  static constexpr int PITCH = ROWB + 16;                            // padded LDS row pitch
  static constexpr int CHUNKS = KT * ROWB / 16;                      // 16-byte chunks per stage
  static constexpr int PER_T = (CHUNKS + 255) / 256;                 // chunks per thread
  static constexpr int BYTES = KT * PITCH + KT * 4;                  // rows + weights (float)
};

template <int PREC, int DP>
__device__ __forceinline__ void kmv32_body(const KmvArgs& A, int64_t bx, int64_t by) {
  using St = Stage32<PREC, DP>;
  using ET = typename St::ET;
  using Frag = typename std::conditional<PREC == LAKER_F32, FragF32<DP>, FragBF16<DP>>::type;
  constexpr int KT = St::KT;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][St::BYTES];
  if (A.S != nullptr && A.S->done) return;
  if (A.pcg_step && bx == 0 && by == 0 && threadIdx.x == 0) A.S->kcur += 1;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 5, c = lane & 31;
  const int64_t rb0 = bx * 128;
  const int64_t row0 = rb0 + wv * 32;
  const int64_t j0 = by * A.cps;
  const int64_t j1 = j0 + A.cps < A.n ? j0 + A.cps : A.n;
  const double* __restrict__ p = A.p;
  const ET* __restrict__ Q = reinterpret_cast<const ET*>(A.Q);
  const unsigned char* __restrict__ Kb = reinterpret_cast<const unsigned char*>(A.K);
  Frag a;
  {
    int64_t qi = row0 + c;
    if (qi > A.m - 1) qi = A.m - 1;
    a.load(Q, qi, h);
  }
  double acc[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0;

  const int nstages = (int)((j1 - j0 + KT - 1) / KT);
  u32x4 stg[St::PER_T];
  double stp = 0.0;
  bool stv = false;
  // global -> registers for the stage starting at key row js.  Rows are
  // contiguous, so chunk ch of a stage sits ch * 16 bytes past its first row;
  // only the last stage of the key rows clamps its rows to n - 1.  The weight
  // is converted and masked (zero past the column range, so that clamped rows
  // add nothing) when it is written to LDS, which keeps the loads in flight.
  auto fetch = [&](int64_t js) {
    const unsigned char* sb = Kb + js * St::ROWB;
    if (js + KT <= A.n) {
#pragma unroll
      for (int q = 0; q < St::PER_T; ++q) {
        const int ch = tid + 256 * q;
        if (St::CHUNKS % 256 == 0 || ch < St::CHUNKS) stg[q] = *reinterpret_cast<const u32x4*>(sb + ch * 16);
      }
    } else {
#pragma unroll
      for (int q = 0; q < St::PER_T; ++q) {
        const int ch = tid + 256 * q;
        if (St::CHUNKS % 256 == 0 || ch < St::CHUNKS) {
          const int rr = ch / (St::ROWB / 16);
          const int cc = ch - rr * (St::ROWB / 16);
          int64_t kr = js + rr;
          if (kr > A.n - 1) kr = A.n - 1;
          stg[q] = *reinterpret_cast<const u32x4*>(Kb + kr * St::ROWB + cc * 16);
        }
      }
    }
    const int64_t kj = js + (tid % KT);
    stv = kj < j1;
    stp = p[kj < A.n ? kj : A.n - 1];
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < St::PER_T; ++q) {
      const int ch = tid + 256 * q;
      if (St::CHUNKS % 256 == 0 || ch < St::CHUNKS) {
        const int rr = ch / (St::ROWB / 16);
        const int cc = ch - rr * (St::ROWB / 16);
        *reinterpret_cast<u32x4*>(&lds[buf][rr * St::PITCH + cc * 16]) = stg[q];
      }
    }
    if (tid < KT) reinterpret_cast<float*>(&lds[buf][KT * St::PITCH])[tid] = stv ? (float)stp : 0.f;
  };
  // Pipeline: at the top of iteration s the registers hold stage s + 1; they
  // are written to the free LDS buffer, the loads of stage s + 2 are issued,
  // stage s is consumed, and one barrier both publishes stage s + 1 and
  // releases the buffer of stage s.
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
    const unsigned char* base = lds[buf];
    const float* pw = reinterpret_cast<const float*>(base + KT * St::PITCH);
    // the stage's products are summed in float32 (KT / 32 terms per lane and
    // row) and the stage sum is added into the float64 accumulator
    float accf[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) accf[r] = 0.f;
#pragma unroll
    for (int u = 0; u < KT / 32; ++u) {
      Frag b;
      const unsigned char* rowp = base + (u * 32 + c) * St::PITCH + h * (St::ROWB / 2);
      if constexpr (PREC == LAKER_F32) {
#pragma unroll
        for (int q = 0; q < DP / 8; ++q) {
          const float4 t = *reinterpret_cast<const float4*>(rowp + 16 * q);
          b.v[4 * q + 0] = t.x;
          b.v[4 * q + 1] = t.y;
          b.v[4 * q + 2] = t.z;
          b.v[4 * q + 3] = t.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < DP / 16; ++q) b.v[q] = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4*>(rowp + 16 * q));
      }
      const float pvf = pw[u * 32 + c];
      v16f sc;
      if constexpr (PREC == LAKER_F32) sc = tile_f32<DP>(a, b);
      else sc = tile_bf16<DP>(a, b);
#pragma unroll
      for (int r = 0; r < 16; ++r) accf[r] = fmaf(kexp2(sc[r]), pvf, accf[r]);
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += (double)accf[r];
    __syncthreads();
  }
  // sum over the 32 lanes of each half (the key columns of the tiles)
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    double v = acc[r];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    v += __shfl_xor(v, 16, 64);
    acc[r] = v;
  }
  double* __restrict__ part = A.part;
  if (c < 16) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) v = (r == c) ? acc[r] : v;
    const int64_t row = row0 + (c >> 2) * 8 + h * 4 + (c & 3);
    if (row < A.m) part[by * A.m + row] = v;
  }
}

template <int PREC, int DP>
__global__ __launch_bounds__(256) void kmv32_kernel(KmvArgs A) {
  kmv32_body<PREC, DP>(A, blockIdx.x, blockIdx.y);
}

// Batched: block b takes tile (problem, row block, column range) = tiles[3 b ..].
template <int PREC, int DP>
__global__ __launch_bounds__(256) void kmv32_batch_kernel(const KmvArgs* __restrict__ As, const int* __restrict__ tiles) {
  const int* t = tiles + 3 * (int64_t)blockIdx.x;
  if (t[0] < 0) return;   // padding tile
  const KmvArgs A = As[t[0]];
  kmv32_body<PREC, DP>(A, t[1], t[2]);
}

// ---------------------------------------------------------------------------
// Symmetric square product (float32 / bfloat16, dp <= 64).  Block b runs the
// stages [T b / G, T (b + 1) / G) of the list of (row block I, column stage
// J >= 2 I), row blocks in the order 0, nrb - 1, 1, nrb - 2, ...  Its eight
// waves own 32 rows each of the 256-row block I; the 128 key rows of a stage are staged through LDS as in the
// rectangular kernel.  For a stage right of the diagonal (J >= 2 I + 2) every
// tile exp2(S) feeds the row sums (weights p_j of the stage's columns) and the
// column sums (weights p_i of the wave's rows); the column sums of the 16
// wave-halves go through LDS and are added in a fixed order by the first 128
// threads while the next stage runs.
// ---------------------------------------------------------------------------
// Block total of the per-thread p^T A p sums of a symmetric launch (NT
// threads), in a fixed order: wave 0 adds the waves' values lane by lane, then
// the lanes by a shuffle tree.
template <int NT = 512>
__device__ __forceinline__ void sym_pap_store(double* papl, double* out) {
  __syncthreads();
  if (threadIdx.x < 64) {
    double s = papl[threadIdx.x];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) s += papl[w * 64 + threadIdx.x];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
    if (threadIdx.x == 0) *out = s;
  }
}

// Inputs of the on-the-fly conjugation (A.theta set), loaded at kernel entry
// so that their latency overlaps the first key-row fetches: this thread's
// r^T theta partials (entries tid + k NT of at most 1024; the index is clamped
// and the value masked when summed) and S->first / S->rzold.
template <int NT = 512>
struct ConjIn {
  double v[1024 / NT];
  double rzold;
  int first;
};
template <int NT = 512>
__device__ __forceinline__ ConjIn<NT> sym_conj_issue(const KmvArgs& A) {
  ConjIn<NT> r{};
  r.first = 1;
  if (A.theta == nullptr) return r;
  const int t = threadIdx.x, g = A.grz;
#pragma unroll
  for (int k = 0; k < 1024 / NT; ++k) r.v[k] = A.rzp[t + k * NT < g ? t + k * NT : g - 1];
  r.rzold = A.S->rzold;
  r.first = A.S->first;
  return r;
}
// beta = r^T theta / S->rzold (0 while S->first), the same in every block
// (fixed-order sum over the block); block 0 records beta and the new r^T theta
// (slot kcur & 1, read by the step update).  Called before kcur advances.
template <int NT = 512>
__device__ __forceinline__ double sym_conj_finish(const KmvArgs& A, const ConjIn<NT>& in, int64_t b) {
  if (A.theta == nullptr) return 0.0;
  __shared__ double sh[16];
  const int t = threadIdx.x, g = A.grz;
  double mine = 0.0;
#pragma unroll
  for (int k = 0; k < 1024 / NT; ++k) mine += t + k * NT < g ? in.v[k] : 0.0;
  const double rz = block_sum(mine, sh);
  const double beta = in.first ? 0.0 : rz / in.rzold;
  if (b == 0 && t == 0) {
    A.S->rzbuf[A.S->kcur & 1] = rz;
    A.S->beta = beta;
  }
  return beta;
}

template <int PREC, int DP>
struct SymStage {
  using ET = typename std::conditional<PREC == LAKER_F32, float, uint16_t>::type;
  static constexpr int ES = (int)sizeof(ET);
  static constexpr int ROWB = DP * ES;
  static constexpr int KT = kSymCols;
  static constexpr int PITCH = ROWB + 16;
  static constexpr int CHUNKS = KT * ROWB / 16;
  static constexpr int STAGERS = 256;  // threads (waves 0-3) that move the key rows
  static constexpr int PER_T = (CHUNKS + STAGERS - 1) / STAGERS;
  static constexpr int BYTES = KT * PITCH + KT * 4;   // key rows, float32 column weights
  static constexpr int CPITCH = 160;   // column-sum rows: wave-halves alternate bank halves
};

template <int PREC, int DP>
__global__ __launch_bounds__(512) void kmvsym_kernel(KmvArgs A, SymPlan P) {
  using St = SymStage<PREC, DP>;
  using ET = typename St::ET;
  using Frag = typename std::conditional<PREC == LAKER_F32, FragF32<DP>, FragBF16<DP>>::type;
  constexpr int KT = St::KT;
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][St::BYTES];
  __shared__ float colbuf[2][16 * St::CPITCH];
  // p^T A p partials (A.pap set): p of the staged columns of three stages in
  // flight, p of the row each lane writes, and one running sum per thread
  __shared__ double pdl[3][KT];
  __shared__ double prl[512];
  __shared__ double papl[512];
  const ConjIn<512> cin = sym_conj_issue<512>(A);
  if (A.S != nullptr && A.S->done) return;
  const int64_t b = blockIdx.x;
  // direction entry j: p_j, or theta_j + beta p_j when conjugating (beta is
  // known once the first key-row fetch has been issued)
  const double* __restrict__ th = A.theta;
  const double* __restrict__ p = A.p;
  double beta = 0.0;
  auto pval = [&](int64_t j) { return th != nullptr ? fma(beta, p[j], th[j]) : p[j]; };
  // (s0 < T for every block: the cursor and first fetches below stay in range
  // also for a block without stages)
  const int64_t s0 = P.T * b / P.grid, s1 = P.T * (b + 1) / P.grid;
  const bool wp = A.pap != nullptr;
  const int64_t L = s1 - s0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 5, c = lane & 31;
  const int64_t n = A.n;
  const int64_t ncs = P.ncs;
  const ET* __restrict__ Q = reinterpret_cast<const ET*>(A.K);
  const unsigned char* __restrict__ Kb = reinterpret_cast<const unsigned char*>(A.K);
  double* __restrict__ part = A.part;

  // cursor of the first stage: position in the row-block order, row block, column stage
  const int64_t nrb = P.nrb;
  int64_t t0 = 0;
  while (sym_pos_start(t0 + 1, nrb, ncs) <= s0) ++t0;
  const int64_t I0 = sym_rowblock_at(t0, nrb);
  const int64_t J0 = 2 * I0 + (s0 - sym_pos_start(t0, nrb, ncs));

  // ---- LDS staging of the key rows of column stage J (as the rectangular kernel)
  u32x4 stg[St::PER_T];
  double stp = 0.0, stt = 0.0;
  bool stv = false;
  // Waves 0-3 move the key rows (global -> registers -> LDS) and waves 2-3 add
  // up the column sums: in a stage the second wave of each SIMD (waves 4-7)
  // finishes its tiles last, and waves 0-3 otherwise wait at the barrier.
  const bool stager = tid < St::STAGERS;
  auto fetch_keys = [&](int64_t J) {
    const int64_t js = J * KT;
    const unsigned char* sb = Kb + js * St::ROWB;
    if (!stager) {
    } else if (js + KT <= n) {
#pragma unroll
      for (int q = 0; q < St::PER_T; ++q) {
        const int ch = tid + St::STAGERS * q;
        if (St::CHUNKS % St::STAGERS == 0 || ch < St::CHUNKS) stg[q] = *reinterpret_cast<const u32x4*>(sb + ch * 16);
      }
    } else {
#pragma unroll
      for (int q = 0; q < St::PER_T; ++q) {
        const int ch = tid + St::STAGERS * q;
        if (St::CHUNKS % St::STAGERS == 0 || ch < St::CHUNKS) {
          const int rr = ch / (St::ROWB / 16);
          const int cc = ch - rr * (St::ROWB / 16);
          int64_t kr = js + rr;
          if (kr > n - 1) kr = n - 1;
          stg[q] = *reinterpret_cast<const u32x4*>(Kb + kr * St::ROWB + cc * 16);
        }
      }
    }
  };
  auto fetch_w = [&](int64_t J) {
    if (tid < KT) {
      const int64_t kj = J * KT + tid;
      stv = kj < n;
      // raw entries: the conjugation waits for the store, a stage later, so
      // that no wait on these loads (and the key rows in flight) comes here
      const int64_t jj = kj < n ? kj : n - 1;
      stp = p[jj];
      if (th != nullptr) stt = th[jj];
    }
  };
  auto fetch = [&](int64_t J) {
    fetch_keys(J);
    fetch_w(J);
  };
  auto store = [&](int buf, int ring) {
    if (stager) {
#pragma unroll
      for (int q = 0; q < St::PER_T; ++q) {
        const int ch = tid + St::STAGERS * q;
        if (St::CHUNKS % St::STAGERS == 0 || ch < St::CHUNKS) {
          const int rr = ch / (St::ROWB / 16);
          const int cc = ch - rr * (St::ROWB / 16);
          *reinterpret_cast<u32x4*>(&lds[buf][rr * St::PITCH + cc * 16]) = stg[q];
        }
      }
    }
    if (tid < KT) {
      const double w = th != nullptr ? fma(beta, stp, stt) : stp;
      reinterpret_cast<float*>(&lds[buf][KT * St::PITCH])[tid] = stv ? (float)w : 0.f;
      if (wp) pdl[ring][tid] = stv ? w : 0.0;
    }
  };
  auto advance = [&](int64_t& t, int64_t& I, int64_t& J) {
    if (++J == ncs) {
      ++t;
      I = sym_rowblock_at(t, nrb);
      J = 2 * I;
    }
  };

  // ---- per row block state: query fragment, row weights, float64 row sums
  Frag a;
  float rw[16];
  double acc[16];
  double prn = 0.0;   // p of the row this lane writes, for the next row block
  int64_t Icur = -1;
  // query fragment and row weights of row block I; issued at the end of the
  // stage before the row block changes (their last readers are that stage's
  // products), so that the loads complete behind its barrier
  // (every load is issued before the first use: rows past n read row n - 1
  // and are masked afterwards)
  auto load_rows = [&](int64_t I) {
    const int64_t row0 = I * kSymRows + wv * 32;
    int64_t qi = row0 + c;
    if (qi > n - 1) qi = n - 1;
    a.load(Q, qi, h);
    const int rn = c >> 1;
    const int64_t rowp = row0 + (rn >> 2) * 8 + h * 4 + (rn & 3);
    double pr[17], tr[17];
#pragma unroll
    for (int r = 0; r < 17; ++r) {
      const int64_t row = r < 16 ? row0 + (r >> 2) * 8 + h * 4 + (r & 3) : rowp;
      const int64_t rr = row < n ? row : n - 1;
      pr[r] = p[rr];
      tr[r] = th != nullptr ? th[rr] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 17; ++r) {
      const int64_t row = r < 16 ? row0 + (r >> 2) * 8 + h * 4 + (r & 3) : rowp;
      const double v = row < n ? (th != nullptr ? fma(beta, pr[r], tr[r]) : pr[r]) : 0.0;
      if (r < 16) rw[r] = (float)v;
      else if (wp) prn = v;
    }
  };
  auto open_rows = [&](int64_t I) {
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0;
    if (wp) prl[tid] = prn;
    Icur = I;
  };
  // row sums over the 32 lanes of each half: a halving exchange (lanes with
  // bit 4 set keep rows 8..15, with bit 3 the upper half of what is left, ...)
  // leaves lane c with row (c >> 1) summed over its 32 lanes after 16 shuffles
  auto flush_rows = [&]() {
    double v8[8], v4[4], v2[2];
    const bool s4 = (c & 16) != 0, s3 = (c & 8) != 0, s2 = (c & 4) != 0, s1 = (c & 2) != 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) v8[j] = (s4 ? acc[j + 8] : acc[j]) + __shfl_xor(s4 ? acc[j] : acc[j + 8], 16, 64);
#pragma unroll
    for (int j = 0; j < 4; ++j) v4[j] = (s3 ? v8[j + 4] : v8[j]) + __shfl_xor(s3 ? v8[j] : v8[j + 4], 8, 64);
#pragma unroll
    for (int j = 0; j < 2; ++j) v2[j] = (s2 ? v4[j + 2] : v4[j]) + __shfl_xor(s2 ? v4[j] : v4[j + 2], 4, 64);
    double v = (s1 ? v2[1] : v2[0]) + __shfl_xor(s1 ? v2[0] : v2[1], 2, 64);
    v += __shfl_xor(v, 1, 64);
    const int64_t slot = b - sym_block_of(sym_pos_start(sym_pos_of(Icur, nrb), nrb, ncs), P.grid, P.T);
    if ((c & 1) == 0) {
      const int r = c >> 1;
      const int64_t row = Icur * kSymRows + wv * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
      if (row < n) {
        part[slot * n + row] = v;
        if (wp) {
          // the block holding the row block's diagonal stage adds lam p_i^2
          const double pr = prl[tid];
          double s = fma(pr, v, papl[tid]);
          if (slot == 0) s = fma(A.lam * pr, pr, s);
          papl[tid] = s;
        }
      }
    }
  };
  // column sums of the stage held in colbuf[buf] (16 wave-halves, fixed order),
  // by waves 2-3
  auto flush_cols = [&](int buf, int ring, int64_t I, int64_t J) {
    const int ct = tid - KT;
    if (ct >= 0 && ct < KT) {
      const int64_t col = J * KT + ct;
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < 16; ++k) v += (double)colbuf[buf][k * St::CPITCH + ct];
      if (col < n) {
        part[(P.rs + I) * n + col] = v;
        if (wp) papl[tid] = fma(pdl[ring][ct], v, papl[tid]);
      }
    }
  };

  // one stage: tiles of the 32 wave rows against the 128 staged key rows.  All
  // key fragments of the stage are read from LDS first, so that the later
  // tiles' reads complete behind the products of the earlier ones.
  auto load_b = [&](Frag& bf, const unsigned char* base, int u) {
    const unsigned char* rowp = base + (u * 32 + c) * St::PITCH + h * (St::ROWB / 2);
    if constexpr (PREC == LAKER_F32) {
#pragma unroll
      for (int q = 0; q < DP / 8; ++q) {
        const float4 t = *reinterpret_cast<const float4*>(rowp + 16 * q);
        bf.v[4 * q + 0] = t.x;
        bf.v[4 * q + 1] = t.y;
        bf.v[4 * q + 2] = t.z;
        bf.v[4 * q + 3] = t.w;
      }
    } else {
#pragma unroll
      for (int q = 0; q < DP / 16; ++q)
        bf.v[q] = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4*>(rowp + 16 * q));
    }
  };
  auto stage = [&](int buf, auto mirror) {
    constexpr bool MIR = decltype(mirror)::value;
    const unsigned char* base = lds[buf];
    const float* pw = reinterpret_cast<const float*>(base + KT * St::PITCH);
    float accf[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) accf[r] = 0.f;
    // (float32 fragments of dp = 64 do not fit in registers four at a time:
    // there each tile reads its own)
    constexpr int NB = (PREC == LAKER_F32 && DP > 32) ? 1 : KT / 32;
    Frag bq[NB];
    float pv[KT / 32];
#pragma unroll
    for (int u = 0; u < KT / 32; ++u) {
      if (NB > 1) load_b(bq[u % NB], base, u);
      pv[u] = pw[u * 32 + c];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < KT / 32; ++u) {
      if (NB == 1) load_b(bq[0], base, u);
      const float pvf = pv[u];
      v16f sc;
      if constexpr (PREC == LAKER_F32) sc = tile_f32<DP>(a, bq[u % NB]);
      else sc = tile_bf16<DP>(a, bq[u % NB]);
      // (first terms are products, not multiply-adds onto zero: the two-operand
      // multiply issues in half the time of a three-operand multiply-add)
      auto madd = [&](float x, float y, float acc0, bool first) { return first ? x * y : fmaf(x, y, acc0); };
      if constexpr (MIR) {
        float g0 = 0.f, g1 = 0.f, g2 = 0.f, g3 = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float t0 = kexp2(sc[r]), t1 = kexp2(sc[4 + r]), t2 = kexp2(sc[8 + r]), t3 = kexp2(sc[12 + r]);
          accf[r] = madd(t0, pvf, accf[r], u == 0);
          accf[4 + r] = madd(t1, pvf, accf[4 + r], u == 0);
          accf[8 + r] = madd(t2, pvf, accf[8 + r], u == 0);
          accf[12 + r] = madd(t3, pvf, accf[12 + r], u == 0);
          g0 = madd(t0, rw[r], g0, r == 0);
          g1 = madd(t1, rw[4 + r], g1, r == 0);
          g2 = madd(t2, rw[8 + r], g2, r == 0);
          g3 = madd(t3, rw[12 + r], g3, r == 0);
        }
        colbuf[buf][(wv * 2 + h) * St::CPITCH + u * 32 + c] = (g0 + g1) + (g2 + g3);
      } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) accf[r] = madd(kexp2(sc[r]), pvf, accf[r], u == 0);
      }
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] += (double)accf[r];
  };

  // ---- pipeline (as the rectangular kernel): registers hold stage k + 1 at
  // the top of iteration k; one barrier per stage
  int64_t tc = t0, Ic = I0, Jc = J0;   // stage k
  int64_t tf = t0, If = I0, Jf = J0;   // next stage to fetch
  // stage s keeps the float64 p of its columns in pdl[s % 3]: written when the
  // stage is stored (iteration s - 1), read when its columns are flushed
  // (iteration s + 1), overwritten by stage s + 3 (iteration s + 2)
  auto ring_next = [](int q) { return q == 2 ? 0 : q + 1; };
  int rcur = 0;
  fetch_keys(Jf);
  beta = sym_conj_finish(A, cin, b);
  if (A.pcg_step && b == 0 && tid == 0) A.S->kcur += 1;
  if (s0 >= s1) {
    if (wp && tid == 0) A.pap[b] = 0.0;
    return;
  }
  if (wp) papl[tid] = 0.0;
  fetch_w(Jf);
  advance(tf, If, Jf);
  store(0, 0);
  if (L > 1) {
    fetch(Jf);
    advance(tf, If, Jf);
  }
  load_rows(I0);
  __syncthreads();
  int64_t Ip = -1, Jp = -1;   // previous off-diagonal stage whose columns are pending
  int rp = 0;
  for (int64_t k = 0; k < L; ++k) {
    const int buf = (int)(k & 1);
    if (k + 1 < L) store(buf ^ 1, ring_next(rcur));
    if (k + 2 < L) {
      fetch(Jf);
      advance(tf, If, Jf);
    }
    if (Ip >= 0) {
      flush_cols(buf ^ 1, rp, Ip, Jp);
      Ip = -1;
    }
    if (Ic != Icur) {
      if (Icur >= 0) flush_rows();
      open_rows(Ic);
    }
    if (Jc >= 2 * Ic + 2) {
      stage(buf, std::true_type{});
      Ip = Ic;
      Jp = Jc;
      rp = rcur;
    } else {
      stage(buf, std::false_type{});
    }
    advance(tc, Ic, Jc);
    rcur = ring_next(rcur);
    if (k + 1 < L && Ic != Icur) load_rows(Ic);
    __syncthreads();
  }
  if (Ip >= 0) flush_cols((int)((L - 1) & 1), rp, Ip, Jp);
  flush_rows();
  if (wp) sym_pap_store(papl, A.pap + b);
}

// ---------------------------------------------------------------------------
// Symmetric square product in bfloat16 on 16x16x32 MFMA tiles (dp = 32, 64).
// The schedule of kmvsym_kernel (row blocks of 256 against column stages of
// 128 on or right of the block diagonal, interleaved row-block order), on a
// grid of 2 kSymGrid blocks of four waves, two blocks per CU.  Each wave owns
// 64 rows as four 16-row tiles, so every key fragment it reads from LDS feeds
// four score tiles (half the fragment reads per kernel entry of the eight-wave
// kernel), and a lane (column q = lane % 16, row group g = lane / 16) holds
// rows 4 g + 0..3 of each row tile: 16 float64 row sums, where 32x32 tiles
// would need 32 for 64 rows.  A block synchronizes four waves per stage
// instead of eight.  The kernel is bound by vector issue: per kernel entry one
// exp2 (two issue slots) and two multiply-adds, plus the MFMA issue.
//
// Fragments: for MFMA step s a lane supplies elements
// g (dp / 4) + 8 s + 0..7 of its row (query rows: A operand, key rows: B);
// the score tile's lane holds S[4 g + i][q], i = 0..3.
// ---------------------------------------------------------------------------
template <int DP>
struct FragB16x {
  static constexpr int S = DP / 32;   // MFMA steps
  v8bf v[S];
  __device__ __forceinline__ void load(const uint16_t* __restrict__ base, int64_t row, int g) {
    const u32x4* src = reinterpret_cast<const u32x4*>(base + row * DP + g * (DP / 4));
#pragma unroll
    for (int q = 0; q < S; ++q) v[q] = __builtin_bit_cast(v8bf, src[q]);
  }
};

template <int DP>
__device__ __forceinline__ v4f tile16_bf16(const FragB16x<DP>& a, const FragB16x<DP>& b) {
  v4f c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < FragB16x<DP>::S; ++s) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.v[s], b.v[s], c, 0, 0, 0);
  return c;
}

// (the body of the single-map and the batched launch; b: the block's index
// in the map's grid)
template <int DP>
__device__ __forceinline__ void kmvsym16_body(const KmvArgs& A, const SymPlan& P, const int64_t b) {
  using St = SymStage<LAKER_BF16, DP>;
  using Frag = FragB16x<DP>;
  constexpr int KT = St::KT;
  constexpr int NT = 256;
  constexpr int RT = 4;                 // 16-row tiles per wave
  constexpr int CROWS = 16;             // column-sum rows: four row groups of four waves
  // (rows 16 banks apart: the four row groups of a wave write disjoint banks,
  // and rows two apart -- the halves of a column's flush -- 32 banks apart)
  constexpr int CPITCH = KT + 16;
  static_assert(St::STAGERS == NT, "every thread stages key rows");
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][St::BYTES];
  __shared__ float colbuf[2][CROWS * CPITCH];
  // p^T A p partials (A.pap set): p of the staged columns of three stages in
  // flight, p of the row each lane writes, and one running sum per thread
  __shared__ double pdl[3][KT];
  __shared__ double prl[NT];
  __shared__ double papl[NT];
  const ConjIn<NT> cin = sym_conj_issue<NT>(A);
  if (A.S != nullptr && A.S->done) return;
  const double* __restrict__ th = A.theta;
  const double* __restrict__ p = A.p;
  double beta = 0.0;
  auto pval = [&](int64_t j) { return th != nullptr ? fma(beta, p[j], th[j]) : p[j]; };
  const int64_t s0 = P.T * b / P.grid, s1 = P.T * (b + 1) / P.grid;
  const bool wp = A.pap != nullptr;
  const int64_t L = s1 - s0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int q = lane & 15, g = lane >> 4;
  const int64_t n = A.n;
  const int64_t ncs = P.ncs;
  const uint16_t* __restrict__ Q = reinterpret_cast<const uint16_t*>(A.K);
  const unsigned char* __restrict__ Kb = reinterpret_cast<const unsigned char*>(A.K);
  // partial slots in float32 (the plan's f32)
  float* __restrict__ partf = reinterpret_cast<float*>(A.part);

  const int64_t nrb = P.nrb;
  int64_t t0 = 0;
  while (sym_pos_start(t0 + 1, nrb, ncs) <= s0) ++t0;
  const int64_t I0 = sym_rowblock_at(t0, nrb);
  const int64_t J0 = 2 * I0 + (s0 - sym_pos_start(t0, nrb, ncs));

  // ---- LDS staging of the key rows of column stage J (every thread)
  u32x4 stg[St::PER_T];
  double stp = 0.0, stt = 0.0;
  bool stv = false;
  auto fetch_keys = [&](int64_t J) {
    const int64_t js = J * KT;
    const unsigned char* sb = Kb + js * St::ROWB;
    if (js + KT <= n) {
#pragma unroll
      for (int u = 0; u < St::PER_T; ++u) {
        const int ch = tid + NT * u;
        if (St::CHUNKS % NT == 0 || ch < St::CHUNKS) stg[u] = *reinterpret_cast<const u32x4*>(sb + ch * 16);
      }
    } else {
#pragma unroll
      for (int u = 0; u < St::PER_T; ++u) {
        const int ch = tid + NT * u;
        if (St::CHUNKS % NT == 0 || ch < St::CHUNKS) {
          const int rr = ch / (St::ROWB / 16);
          const int cc = ch - rr * (St::ROWB / 16);
          int64_t kr = js + rr;
          if (kr > n - 1) kr = n - 1;
          stg[u] = *reinterpret_cast<const u32x4*>(Kb + kr * St::ROWB + cc * 16);
        }
      }
    }
  };
  auto fetch_w = [&](int64_t J) {
    if (tid < KT) {
      const int64_t kj = J * KT + tid;
      stv = kj < n;
      // raw entries: the conjugation waits for the store, a stage later, so
      // that no wait on these loads (and the key rows in flight) comes here
      const int64_t jj = kj < n ? kj : n - 1;
      stp = p[jj];
      if (th != nullptr) stt = th[jj];
    }
  };
  auto fetch = [&](int64_t J) {
    fetch_keys(J);
    fetch_w(J);
  };
  auto store = [&](int buf, int ring) {
#pragma unroll
    for (int u = 0; u < St::PER_T; ++u) {
      const int ch = tid + NT * u;
      if (St::CHUNKS % NT == 0 || ch < St::CHUNKS) {
        const int rr = ch / (St::ROWB / 16);
        const int cc = ch - rr * (St::ROWB / 16);
        *reinterpret_cast<u32x4*>(&lds[buf][rr * St::PITCH + cc * 16]) = stg[u];
      }
    }
    if (tid < KT) {
      const double w = th != nullptr ? fma(beta, stp, stt) : stp;
      reinterpret_cast<float*>(&lds[buf][KT * St::PITCH])[tid] = stv ? (float)w : 0.f;
      if (wp) pdl[ring][tid] = stv ? w : 0.0;
    }
  };
  auto advance = [&](int64_t& t, int64_t& I, int64_t& J) {
    if (++J == ncs) {
      ++t;
      I = sym_rowblock_at(t, nrb);
      J = 2 * I;
    }
  };

  // ---- per row block state.  Row tile k of the wave: rows
  // I kSymRows + 64 wv + 16 k + 0..15; the lane's rows in it: 4 g + 0..3.
  Frag a[RT];
  float rw[RT][4];
  double acc[RT][4];
  double prn = 0.0;   // p of the row this lane writes, for the next row block
  int64_t Icur = -1;
  // the row this lane writes after the row-sum exchange: value j = q of its
  // row group, i.e. row tile q / 4, row 4 g + q % 4 of it
  const int wrow = 16 * (q >> 2) + 4 * g + (q & 3);
  // (every load is issued before the first use: rows past n read row n - 1
  // and are masked afterwards)
  auto load_rows = [&](int64_t I) {
    const int64_t row0 = I * kSymRows + wv * 64;
    double pr[4 * RT + 1], tr[4 * RT + 1];
#pragma unroll
    for (int k = 0; k < RT; ++k) {
      int64_t qi = row0 + 16 * k + q;
      if (qi > n - 1) qi = n - 1;
      a[k].load(Q, qi, g);
    }
#pragma unroll
    for (int j = 0; j <= 4 * RT; ++j) {
      const int64_t row = j < 4 * RT ? row0 + 16 * (j >> 2) + 4 * g + (j & 3) : row0 + wrow;
      const int64_t rr = row < n ? row : n - 1;
      pr[j] = p[rr];
      tr[j] = th != nullptr ? th[rr] : 0.0;
    }
#pragma unroll
    for (int j = 0; j <= 4 * RT; ++j) {
      const int64_t row = j < 4 * RT ? row0 + 16 * (j >> 2) + 4 * g + (j & 3) : row0 + wrow;
      const double v = row < n ? (th != nullptr ? fma(beta, pr[j], tr[j]) : pr[j]) : 0.0;
      if (j < 4 * RT) rw[j >> 2][j & 3] = (float)v;
      else if (wp) prn = v;
    }
  };
  auto open_rows = [&](int64_t I) {
#pragma unroll
    for (int k = 0; k < RT; ++k)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[k][i] = 0.0;
    if (wp) prl[tid] = prn;
    Icur = I;
  };
  // row sums over the 16 lanes of a row group: a halving exchange over the 16
  // values v_j = acc[j / 4][j % 4] (lanes with bit 3 set keep j = 8..15, ...)
  // leaves lane q with value j = q summed over its 16 lanes
  auto flush_rows = [&]() {
    double v8[8], v4[4], v2[2];
    const bool s3 = (q & 8) != 0, s2 = (q & 4) != 0, s1 = (q & 2) != 0, s0b = (q & 1) != 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const double lo = acc[j >> 2][j & 3], hi = acc[(j + 8) >> 2][(j + 8) & 3];
      v8[j] = (s3 ? hi : lo) + __shfl_xor(s3 ? lo : hi, 8, 64);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) v4[j] = (s2 ? v8[j + 4] : v8[j]) + __shfl_xor(s2 ? v8[j] : v8[j + 4], 4, 64);
#pragma unroll
    for (int j = 0; j < 2; ++j) v2[j] = (s1 ? v4[j + 2] : v4[j]) + __shfl_xor(s1 ? v4[j] : v4[j + 2], 2, 64);
    const double v = (s0b ? v2[1] : v2[0]) + __shfl_xor(s0b ? v2[0] : v2[1], 1, 64);
    const int64_t slot = b - sym_block_of(sym_pos_start(sym_pos_of(Icur, nrb), nrb, ncs), P.grid, P.T);
    const int64_t row = Icur * kSymRows + wv * 64 + wrow;
    if (row < n) {
      const float vf = (float)v;
      partf[slot * n + row] = vf;
      if (wp) {
        // the block holding the row block's diagonal stage adds lam p_i^2
        const double pr = prl[tid];
        double s = fma(pr, (double)vf, papl[tid]);
        if (slot == 0) s = fma(A.lam * pr, pr, s);
        papl[tid] = s;
      }
    }
  };
  // column sums of the stage held in colbuf[buf] (16 rows, fixed order): two
  // adjacent lanes per column, one adding rows 0, 1, 4, 5, ..., the other
  // rows 2, 3, 6, 7, ..., then each other's
  auto flush_cols = [&](int buf, int ring, int64_t I, int64_t J) {
    const int ct = tid >> 1, hf = tid & 1;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < CROWS / 2; ++k) v += (double)colbuf[buf][((k >> 1) * 4 + hf * 2 + (k & 1)) * CPITCH + ct];
    v += __shfl_xor(v, 1, 64);
    const int64_t col = J * KT + ct;
    if (hf == 0 && col < n) {
      // float32 slot (the plan's f32); p^T A p takes the stored value
      const float vf = (float)v;
      partf[(P.rs + I) * n + col] = vf;
      if (wp) papl[tid] = fma(pdl[ring][ct], (double)vf, papl[tid]);
    }
  };

  auto load_b = [&](Frag& bf, const unsigned char* base, int v) {
    const unsigned char* rowp = base + (v * 16 + q) * St::PITCH + g * (St::ROWB / 4);
#pragma unroll
    for (int s = 0; s < Frag::S; ++s) bf.v[s] = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4*>(rowp + 16 * s));
  };
  // one stage: the wave's four row tiles against the eight 16-column tiles of
  // the staged key rows
  auto stage = [&](int buf, auto mirror) {
    constexpr bool MIR = decltype(mirror)::value;
    constexpr int NV = KT / 16;
    const unsigned char* base = lds[buf];
    const float* pw = reinterpret_cast<const float*>(base + KT * St::PITCH);
    float accf[RT][4];
    float pv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) pv[v] = pw[v * 16 + q];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      // (one column tile at a time: the other block on the CU covers the
      // fragment reads' latency -- reading the next tile's fragments ahead, in
      // a loop over tile pairs that fits the registers, measured no faster,
      // and unrolled it overflows them)
      __builtin_amdgcn_sched_barrier(0);
      Frag bv;
      load_b(bv, base, v);
      const float pvf = pv[v];
      // (first terms are products, not multiply-adds onto zero)
      auto madd = [&](float x, float y, float acc0, bool first) { return first ? x * y : fmaf(x, y, acc0); };
      // column sums in two chains: row tiles 0, 1 and row tiles 2, 3
      float gk[2];
#pragma unroll
      for (int k = 0; k < RT; ++k) {
        const v4f sc = tile16_bf16<DP>(a[k], bv);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float t = kexp2(sc[i]);
          accf[k][i] = madd(t, pvf, accf[k][i], v == 0);
          if constexpr (MIR) gk[k >> 1] = madd(t, rw[k][i], gk[k >> 1], (k & 1) == 0 && i == 0);
        }
      }
      if constexpr (MIR) colbuf[buf][(wv * 4 + g) * CPITCH + v * 16 + q] = gk[0] + gk[1];
    }
#pragma unroll
    for (int k = 0; k < RT; ++k)
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[k][i] += (double)accf[k][i];
  };

  // ---- pipeline (as the rectangular kernel): registers hold stage k + 1 at
  // the top of iteration k; one barrier per stage
  int64_t tc = t0, Ic = I0, Jc = J0;   // stage k
  int64_t tf = t0, If = I0, Jf = J0;   // next stage to fetch
  // stage s keeps the float64 p of its columns in pdl[s % 3]: written when the
  // stage is stored (iteration s - 1), read when its columns are flushed
  // (iteration s + 1), overwritten by stage s + 3 (iteration s + 2)
  auto ring_next = [](int q) { return q == 2 ? 0 : q + 1; };
  int rcur = 0;
  fetch_keys(Jf);
  beta = sym_conj_finish<NT>(A, cin, b);
  if (A.pcg_step && b == 0 && tid == 0) A.S->kcur += 1;
  if (s0 >= s1) {
    if (wp && tid == 0) A.pap[b] = 0.0;
    return;
  }
  if (wp) papl[tid] = 0.0;
  fetch_w(Jf);
  advance(tf, If, Jf);
  store(0, 0);
  if (L > 1) {
    fetch(Jf);
    advance(tf, If, Jf);
  }
  load_rows(I0);
  __syncthreads();
  int64_t Ip = -1, Jp = -1;   // previous off-diagonal stage whose columns are pending
  int rp = 0;
  for (int64_t k = 0; k < L; ++k) {
    const int buf = (int)(k & 1);
    if (k + 1 < L) store(buf ^ 1, ring_next(rcur));
    if (k + 2 < L) {
      fetch(Jf);
      advance(tf, If, Jf);
    }
    if (Ip >= 0) {
      flush_cols(buf ^ 1, rp, Ip, Jp);
      Ip = -1;
    }
    if (Ic != Icur) {
      if (Icur >= 0) flush_rows();
      open_rows(Ic);
    }
    if (Jc >= 2 * Ic + 2) {
      stage(buf, std::true_type{});
      Ip = Ic;
      Jp = Jc;
      rp = rcur;
    } else {
      stage(buf, std::false_type{});
    }
    advance(tc, Ic, Jc);
    rcur = ring_next(rcur);
    if (k + 1 < L && Ic != Icur) load_rows(Ic);
    __syncthreads();
  }
  if (Ip >= 0) flush_cols((int)((L - 1) & 1), rp, Ip, Jp);
  flush_rows();
  if (wp) sym_pap_store<NT>(papl, A.pap + b);
}

template <int DP>
__global__ __launch_bounds__(256, 2) void kmvsym16_kernel(KmvArgs A, SymPlan P) {
  kmvsym16_body<DP>(A, P, blockIdx.x);
}

// Several maps' products in one launch (the batched solver): grid row y is
// map list[y], with its arguments As[map] and plan Ps[map] (every plan of this
// kernel has the same grid); each block does what it does in the map's own
// launch, so the results are bitwise those of the single launches.
template <int DP>
__global__ __launch_bounds__(256, 2) void kmvsym16_batch_kernel(const KmvArgs* __restrict__ As,
                                                               const SymPlan* __restrict__ Ps,
                                                               const int* __restrict__ list) {
  const int m = list[blockIdx.y];
  kmvsym16_body<DP>(As[m], Ps[m], blockIdx.x);
}

// ---------------------------------------------------------------------------
// Symmetric square product in float64 (dp <= 64): the schedule of the
// float32 / bfloat16 kernel (256-row blocks against 128-column stages on or
// right of the block diagonal, interleaved row-block order, fixed 256-block
// grid).  A wave owns 32 rows as two 16-row tiles of the 16x16x4 f64 MFMA; the
// key fragments come straight from global memory (the f64 MFMA leaves the
// loads ample time), one tile ahead across stage boundaries.  Off-diagonal
// tiles add exp(S)^T p_rows into the stage's columns: each lane sums its
// eight entries, the four lane groups combine by shuffles, the eight waves
// through LDS in a fixed order.
// ---------------------------------------------------------------------------
template <int DP>
__global__ __launch_bounds__(512) void kmvsym64_kernel(KmvArgs A, SymPlan P) {
  constexpr int CT = kSymCols / 16;   // column tiles per stage
  __shared__ double colbuf[2][8 * kSymCols];
  // p^T A p partials (A.pap set): p of the columns of the pending stage and
  // one running sum per thread
  __shared__ double pdl[2][kSymCols];
  __shared__ double papl[512];
  const ConjIn<512> cin = sym_conj_issue<512>(A);
  if (A.S != nullptr && A.S->done) return;
  const int64_t b = blockIdx.x;
  const double beta = sym_conj_finish(A, cin, b);
  if (A.pcg_step && b == 0 && threadIdx.x == 0) A.S->kcur += 1;
  const double* __restrict__ th = A.theta;
  const double* __restrict__ p = A.p;
  auto pval = [&](int64_t j) { return th != nullptr ? fma(beta, p[j], th[j]) : p[j]; };
  const int64_t s0 = P.T * b / P.grid, s1 = P.T * (b + 1) / P.grid;
  const bool wp = A.pap != nullptr;
  if (s0 >= s1) {
    if (wp && threadIdx.x == 0) A.pap[b] = 0.0;
    return;
  }
  const int64_t L = s1 - s0;
  const int tid = threadIdx.x;
  if (wp) papl[tid] = 0.0;
  const int lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 4, c = lane & 15;
  const int64_t n = A.n;
  const int64_t ncs = P.ncs, nrb = P.nrb;
  const double* __restrict__ K = reinterpret_cast<const double*>(A.K);
  double* __restrict__ part = A.part;

  int64_t t0 = 0;
  while (sym_pos_start(t0 + 1, nrb, ncs) <= s0) ++t0;
  const int64_t I0 = sym_rowblock_at(t0, nrb);
  const int64_t J0 = 2 * I0 + (s0 - sym_pos_start(t0, nrb, ncs));
  auto advance = [&](int64_t& t, int64_t& I, int64_t& J) {
    if (++J == ncs) {
      ++t;
      I = sym_rowblock_at(t, nrb);
      J = 2 * I;
    }
  };

  FragF64<DP> a[2];
  double rw[2][4];
  double acc[2][4];
  int64_t Icur = -1;
  auto open_rows = [&](int64_t I) {
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      const int64_t row0 = I * kSymRows + wv * 32 + rt * 16;
      int64_t qi = row0 + c;
      if (qi > n - 1) qi = n - 1;
      a[rt].load(K, qi, h);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + 4 * r + h;
        rw[rt][r] = row < n ? pval(row) : 0.0;
        acc[rt][r] = 0.0;
      }
    }
    Icur = I;
  };
  auto flush_rows = [&]() {
    const int64_t slot = b - sym_block_of(sym_pos_start(sym_pos_of(Icur, nrb), nrb, ncs), P.grid, P.T);
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
      double v4[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double v = acc[rt][r];
        v += __shfl_xor(v, 1, 64);
        v += __shfl_xor(v, 2, 64);
        v += __shfl_xor(v, 4, 64);
        v += __shfl_xor(v, 8, 64);
        v4[r] = v;
      }
      if (c < 4) {
        double v = 0.0, pr = 0.0;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          v = (r == c) ? v4[r] : v;
          pr = (r == c) ? rw[rt][r] : pr;
        }
        const int64_t row = Icur * kSymRows + wv * 32 + rt * 16 + 4 * c + h;
        if (row < n) {
          part[slot * n + row] = v;
          if (wp) {
            // the block holding the row block's diagonal stage adds lam p_i^2
            double s = fma(pr, v, papl[tid]);
            if (slot == 0) s = fma(A.lam * pr, pr, s);
            papl[tid] = s;
          }
        }
      }
    }
  };
  auto flush_cols = [&](int buf, int64_t I, int64_t J) {
    if (tid < kSymCols) {
      const int64_t col = J * kSymCols + tid;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < 8; ++w) v += colbuf[buf][w * kSymCols + tid];
      if (col < n) {
        part[(P.rs + I) * n + col] = v;
        if (wp) papl[tid] = fma(pdl[buf][tid], v, papl[tid]);
      }
    }
  };

  // key tile cursor, one tile ahead of the compute
  int64_t tf = t0, If = I0, Jf = J0;
  int ctf = 0;
  // (the column's p and theta are loaded raw with the tile one tile ahead and
  // combined when the tile becomes current, so no load is waited on early)
  FragF64<DP> bcur, bnext;
  double pcur = 0.0, pnext = 0.0, tnext = 0.0;
  auto load_tile = [&](FragF64<DP>& bf, double& pj, double& tj) {
    int64_t kj = Jf * kSymCols + ctf * 16 + c;
    const bool in = kj < n;
    if (kj > n - 1) kj = n - 1;
    pj = in ? p[kj] : 0.0;
    tj = in && th != nullptr ? th[kj] : 0.0;
    bf.load(K, kj, h);
    if (++ctf == CT) {
      ctf = 0;
      advance(tf, If, Jf);
    }
  };
  auto comb = [&](double pj, double tj) { return th != nullptr ? fma(beta, pj, tj) : pj; };
  load_tile(bcur, pnext, tnext);
  pcur = comb(pnext, tnext);

  int64_t tc = t0, Ic = I0, Jc = J0;
  int64_t Ip = -1, Jp = -1;
  for (int64_t k = 0; k < L; ++k) {
    const int buf = (int)(k & 1);
    if (Ip >= 0) {
      flush_cols(buf ^ 1, Ip, Jp);
      Ip = -1;
    }
    if (Ic != Icur) {
      if (Icur >= 0) flush_rows();
      open_rows(Ic);
    }
    const bool mir = Jc >= 2 * Ic + 2;
#pragma unroll 1
    for (int ct = 0; ct < CT; ++ct) {
      const bool more = k + 1 < L || ct + 1 < CT;
      if (more) load_tile(bnext, pnext, tnext);
      double g = 0.0;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const v4d s = tile_f64<DP>(a[rt], bcur);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const double e = exp(s[r]);
          acc[rt][r] = fma(e, pcur, acc[rt][r]);
          g = fma(e, rw[rt][r], g);
        }
      }
      if (mir) {
        g += __shfl_xor(g, 16, 64);
        g += __shfl_xor(g, 32, 64);
        if (h == 0) colbuf[buf][wv * kSymCols + ct * 16 + c] = g;
        if (wp && wv == 0 && h == 0) pdl[buf][ct * 16 + c] = pcur;
      }
      if (more) {
        bcur = bnext;
        pcur = comb(pnext, tnext);
      }
    }
    if (mir) {
      Ip = Ic;
      Jp = Jc;
    }
    advance(tc, Ic, Jc);
    __syncthreads();
  }
  if (Ip >= 0) flush_cols((int)((L - 1) & 1), Ip, Jp);
  flush_rows();
  if (wp) sym_pap_store(papl, A.pap + b);
}

// ---------------------------------------------------------------------------
// float64 kernel: 16x16 score tiles, exp in float64.
// ---------------------------------------------------------------------------
template <int DP>
__device__ __forceinline__ void kmv64_body(const KmvArgs& A, int64_t bx, int64_t by) {
  if (A.S != nullptr && A.S->done) return;
  if (A.pcg_step && bx == 0 && by == 0 && threadIdx.x == 0) A.S->kcur += 1;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int h = lane >> 4, c = lane & 15;
  const int64_t rb0 = bx * 64;
  const int64_t row0 = rb0 + wv * 16;
  const int64_t j0 = by * A.cps;
  const int64_t j1 = j0 + A.cps < A.n ? j0 + A.cps : A.n;
  const double* __restrict__ p = A.p;
  const double* __restrict__ Q = reinterpret_cast<const double*>(A.Q);
  const double* __restrict__ K = reinterpret_cast<const double*>(A.K);
  FragF64<DP> a, b, bn;
  {
    int64_t qi = row0 + c;
    if (qi > A.m - 1) qi = A.m - 1;
    a.load(Q, qi, h);
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (j0 < j1) {
    int64_t kj = j0 + c;
    double pj = kj < j1 ? p[kj] : 0.0;
    if (kj > A.n - 1) kj = A.n - 1;
    b.load(K, kj, h);
    for (int64_t jt = j0; jt < j1; jt += 16) {
      const int64_t jn = jt + 16;
      double pn = 0.0;
      if (jn < j1) {
        int64_t kn = jn + c;
        pn = kn < j1 ? p[kn] : 0.0;
        if (kn > A.n - 1) kn = A.n - 1;
        bn.load(K, kn, h);
      }
      v4d s = tile_f64<DP>(a, b);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[r] = fma(exp(s[r]), pj, acc[r]);
      b = bn;
      pj = pn;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double v = acc[r];
    v += __shfl_xor(v, 1, 64);
    v += __shfl_xor(v, 2, 64);
    v += __shfl_xor(v, 4, 64);
    v += __shfl_xor(v, 8, 64);
    acc[r] = v;
  }
  double* __restrict__ part = A.part;
  if (c < 4) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) v = (r == c) ? acc[r] : v;
    const int64_t row = row0 + 4 * c + h;   // 16x16x4 f64 output: register r holds row 4 r + lane / 16
    if (row < A.m) part[by * A.m + row] = v;
  }
}

template <int DP>
__global__ __launch_bounds__(256) void kmv64_kernel(KmvArgs A) {
  kmv64_body<DP>(A, blockIdx.x, blockIdx.y);
}

template <int DP>
__global__ __launch_bounds__(256) void kmv64_batch_kernel(const KmvArgs* __restrict__ As, const int* __restrict__ tiles) {
  const int* t = tiles + 3 * (int64_t)blockIdx.x;
  if (t[0] < 0) return;   // padding tile
  const KmvArgs A = As[t[0]];
  kmv64_body<DP>(A, t[1], t[2]);
}

// Batched finish: grid (blocks, problems); problems without a finished output skip.
__global__ __launch_bounds__(256) void kmv_finish_batch_kernel(const KmvArgs* __restrict__ As) {
  const KmvArgs A = As[blockIdx.y];
  if (A.mode != 1) return;
  if (A.S != nullptr && A.S->done) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < A.m; i += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int sp = 0; sp < A.nsplit; ++sp) s += A.part[(int64_t)sp * A.m + i];
    A.out[i] = A.pself != nullptr ? fma(A.lam, A.pself[i], s) : s;
  }
}

template <int PREC>
hipError_t launch32(int dp, dim3 grid, const KmvArgs& A, hipStream_t st) {
  switch (dp) {
    case 16: kmv32_kernel<PREC, 16><<<grid, 256, 0, st>>>(A); break;
    case 32: kmv32_kernel<PREC, 32><<<grid, 256, 0, st>>>(A); break;
    case 64: kmv32_kernel<PREC, 64><<<grid, 256, 0, st>>>(A); break;
    case 128: kmv32_kernel<PREC, 128><<<grid, 256, 0, st>>>(A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch64(int dp, dim3 grid, const KmvArgs& A, hipStream_t st) {
  switch (dp) {
    case 16: kmv64_kernel<16><<<grid, 256, 0, st>>>(A); break;
    case 32: kmv64_kernel<32><<<grid, 256, 0, st>>>(A); break;
    case 64: kmv64_kernel<64><<<grid, 256, 0, st>>>(A); break;
    case 128: kmv64_kernel<128><<<grid, 256, 0, st>>>(A); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch32_batch(int dp, unsigned ntiles, const KmvArgs* As, const int* tiles, hipStream_t st) {
  switch (dp) {
    case 16: kmv32_batch_kernel<PREC, 16><<<ntiles, 256, 0, st>>>(As, tiles); break;
    case 32: kmv32_batch_kernel<PREC, 32><<<ntiles, 256, 0, st>>>(As, tiles); break;
    case 64: kmv32_batch_kernel<PREC, 64><<<ntiles, 256, 0, st>>>(As, tiles); break;
    case 128: kmv32_batch_kernel<PREC, 128><<<ntiles, 256, 0, st>>>(As, tiles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch64_batch(int dp, unsigned ntiles, const KmvArgs* As, const int* tiles, hipStream_t st) {
  switch (dp) {
    case 16: kmv64_batch_kernel<16><<<ntiles, 256, 0, st>>>(As, tiles); break;
    case 32: kmv64_batch_kernel<32><<<ntiles, 256, 0, st>>>(As, tiles); break;
    case 64: kmv64_batch_kernel<64><<<ntiles, 256, 0, st>>>(As, tiles); break;
    case 128: kmv64_batch_kernel<128><<<ntiles, 256, 0, st>>>(As, tiles); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// Stored kernel matrix.  HBM is plentiful (the tiles on or right of the block
// diagonal take 1.09 GB in float64 at n = 16384, of 288 GB), and a product
// that streams them is bound by HBM instead of by the float64 MFMA and exp.
// Layout: the stage list of the symmetric schedule, stage s as one 256 x 128
// row-major tile at s * kSymRows * kSymCols, entries outside n x n zero.
// kmat_build_kernel writes the float64 entries of the fused float64 kernel
// (same fragments, MFMA and exp), rounded to the storage type; the product
// kernel reads them with the symmetric kernel's block runs and partial-sum
// layout, so the finishing pass and the PCG passes are shared.
// ---------------------------------------------------------------------------
constexpr int64_t kTileElems = (int64_t)kSymRows * kSymCols;

template <int DP, typename OT>
__global__ __launch_bounds__(512) void kmat_build_kernel(const double* __restrict__ K, int64_t n, SymPlan P,
                                                         OT* __restrict__ out) {
  constexpr int CT = kSymCols / 16;
  const int64_t b = blockIdx.x;
  const int64_t s0 = P.T * b / P.grid, s1 = P.T * (b + 1) / P.grid;
  if (s0 >= s1) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 4, c = lane & 15;
  const int64_t ncs = P.ncs, nrb = P.nrb;
  int64_t t = 0;
  while (sym_pos_start(t + 1, nrb, ncs) <= s0) ++t;
  int64_t I = sym_rowblock_at(t, nrb);
  int64_t J = 2 * I + (s0 - sym_pos_start(t, nrb, ncs));
  // key tile cursor one tile ahead of the compute (as the fused kernel)
  int64_t tf = t, If = I, Jf = J;
  int ctf = 0;
  FragF64<DP> a[2], bcur, bnext;
  auto load_tile = [&](FragF64<DP>& bf) {
    int64_t kj = Jf * kSymCols + ctf * 16 + c;
    if (kj > n - 1) kj = n - 1;
    bf.load(K, kj, h);
    if (++ctf == CT) {
      ctf = 0;
      if (++Jf == ncs) {
        ++tf;
        If = sym_rowblock_at(tf, nrb);
        Jf = 2 * If;
      }
    }
  };
  load_tile(bcur);
  int64_t Icur = -1;
  for (int64_t s = s0; s < s1; ++s) {
    if (I != Icur) {
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        int64_t qi = I * kSymRows + wv * 32 + rt * 16 + c;
        if (qi > n - 1) qi = n - 1;
        a[rt].load(K, qi, h);
      }
      Icur = I;
    }
    OT* tile = out + s * kTileElems;
#pragma unroll 1
    for (int ct = 0; ct < CT; ++ct) {
      const bool more = s + 1 < s1 || ct + 1 < CT;
      if (more) load_tile(bnext);
      const bool cin = J * kSymCols + ct * 16 + c < n;
#pragma unroll
      for (int rt = 0; rt < 2; ++rt) {
        const v4d sc = tile_f64<DP>(a[rt], bcur);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int lr = wv * 32 + rt * 16 + 4 * r + h;
          const bool in = cin && I * kSymRows + lr < n;
          __builtin_nontemporal_store(in ? (OT)exp(sc[r]) : (OT)0, &tile[(int64_t)lr * kSymCols + ct * 16 + c]);
        }
      }
      if (more) bcur = bnext;
    }
    if (++J == ncs) {
      ++t;
      I = sym_rowblock_at(t, nrb);
      J = 2 * I;
    }
  }
}

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(u & 0xffffffffll), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <typename ET> struct Pair2;
template <> struct Pair2<double> { using type = double2; };
template <> struct Pair2<float> { using type = float2; };

// w = G p from the stored tiles (float64 products of the stored entries,
// float64 sums).  Block runs, row slots and column slots as the symmetric
// kernels.  A wave owns 32 rows of the stage's tile and a lane two adjacent
// columns, so every load instruction reads one whole tile row; the rows are
// read in two halves of 16, the next half always in flight.  Row sums stay
// per lane across the stages of a row block and leave the lanes by a halving
// exchange when it changes; off-diagonal stages also add K^T p_rows into the
// stage's columns (per lane over the wave's rows, then the eight waves in LDS
// in a fixed order, flushed after the stage's barrier).
template <typename ET>
__global__ __launch_bounds__(512) void kmat_matvec_kernel(KmvArgs A, SymPlan P) {
  using E2 = typename Pair2<ET>::type;
  __shared__ double colbuf[2][8 * kSymCols];
  if (A.S != nullptr && A.S->done) return;
  const int64_t b = blockIdx.x;
  if (A.pcg_step && b == 0 && threadIdx.x == 0) A.S->kcur += 1;
  const int64_t s0 = P.T * b / P.grid, s1 = P.T * (b + 1) / P.grid;
  if (s0 >= s1) return;
  const int64_t L = s1 - s0;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int64_t n = A.n;
  const int64_t ncs = P.ncs, nrb = P.nrb;
  const double* __restrict__ p = A.p;
  double* __restrict__ part = A.part;
  const ET* __restrict__ Kt = reinterpret_cast<const ET*>(A.kmat);

  int64_t t0 = 0;
  while (sym_pos_start(t0 + 1, nrb, ncs) <= s0) ++t0;
  const int64_t I0 = sym_rowblock_at(t0, nrb);
  const int64_t J0 = 2 * I0 + (s0 - sym_pos_start(t0, nrb, ncs));
  auto advance = [&](int64_t& t, int64_t& I, int64_t& J) {
    if (++J == ncs) {
      ++t;
      I = sym_rowblock_at(t, nrb);
      J = 2 * I;
    }
  };
  // (streaming loads: the stored G is read once per product and would only
  // evict reusable lines from the caches; measured 10-12% faster)
  auto load_half = [&](int64_t s, int half, E2 (&v)[16]) {
    typedef ET ev2 __attribute__((ext_vector_type(2)));
    const ET* base = Kt + s * kTileElems + (int64_t)(wv * 32 + half * 16) * kSymCols + 2 * lane;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const ev2 t = __builtin_nontemporal_load(reinterpret_cast<const ev2*>(base + r * kSymCols));
      v[r].x = t.x;
      v[r].y = t.y;
    }
  };
  auto load_w = [&](int64_t J, double& w0, double& w1) {
    const int64_t c0 = J * kSymCols + 2 * lane;
    w0 = c0 < n ? p[c0] : 0.0;
    w1 = c0 + 1 < n ? p[c0 + 1] : 0.0;
  };

  double accr[32];
  double prow = 0.0;
  int64_t Icur = -1;
  auto open_rows = [&](int64_t I) {
#pragma unroll
    for (int r = 0; r < 32; ++r) accr[r] = 0.0;
    const int64_t row = I * kSymRows + wv * 32 + (lane & 31);
    prow = row < n ? p[row] : 0.0;
    Icur = I;
  };
  // halving exchange: lane l ends with row (l >> 1) & 31 of the wave's rows
  auto flush_rows = [&]() {
    double v16[16], v8[8], v4[4], v2[2];
    const bool b5 = (lane & 32) != 0, b4 = (lane & 16) != 0, b3 = (lane & 8) != 0, b2 = (lane & 4) != 0,
               b1 = (lane & 2) != 0;
#pragma unroll
    for (int j = 0; j < 16; ++j) v16[j] = (b5 ? accr[j + 16] : accr[j]) + __shfl_xor(b5 ? accr[j] : accr[j + 16], 32, 64);
#pragma unroll
    for (int j = 0; j < 8; ++j) v8[j] = (b4 ? v16[j + 8] : v16[j]) + __shfl_xor(b4 ? v16[j] : v16[j + 8], 16, 64);
#pragma unroll
    for (int j = 0; j < 4; ++j) v4[j] = (b3 ? v8[j + 4] : v8[j]) + __shfl_xor(b3 ? v8[j] : v8[j + 4], 8, 64);
#pragma unroll
    for (int j = 0; j < 2; ++j) v2[j] = (b2 ? v4[j + 2] : v4[j]) + __shfl_xor(b2 ? v4[j] : v4[j + 2], 4, 64);
    double v = (b1 ? v2[1] : v2[0]) + __shfl_xor(b1 ? v2[0] : v2[1], 2, 64);
    v += __shfl_xor(v, 1, 64);
    const int64_t slot = b - sym_block_of(sym_pos_start(sym_pos_of(Icur, nrb), nrb, ncs), P.grid, P.T);
    const int64_t row = Icur * kSymRows + wv * 32 + ((lane >> 1) & 31);
    if ((lane & 1) == 0 && row < n) part[slot * n + row] = v;
  };
  auto flush_cols = [&](int buf, int64_t I, int64_t J) {
    if (tid < kSymCols) {
      const int64_t col = J * kSymCols + tid;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < 8; ++w) v += colbuf[buf][w * kSymCols + tid];
      if (col < n) part[(P.rs + I) * n + col] = v;
    }
  };
  // rows 16 half .. 16 half + 15 of the wave: row sums, and (mirror) the
  // column sums weighted by the rows' p
  auto half_rows = [&](const E2 (&v)[16], int half, double w0, double w1, bool mir, double& g0, double& g1) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const double x = (double)v[r].x, y = (double)v[r].y;
      accr[half * 16 + r] = fma(y, w1, fma(x, w0, accr[half * 16 + r]));
      if (mir) {
        const double pr = readlane_f64(prow, half * 16 + r);
        g0 = fma(x, pr, g0);
        g1 = fma(y, pr, g1);
      }
    }
  };

  E2 v0[16], v1[16];
  double w0 = 0.0, w1 = 0.0, wn0 = 0.0, wn1 = 0.0;
  int64_t tc = t0, Ic = I0, Jc = J0;
  int64_t tn = t0, In = I0, Jn = J0;   // next stage (for its column weights)
  load_half(s0, 0, v0);
  load_w(Jn, wn0, wn1);
  advance(tn, In, Jn);
  int64_t Ip = -1, Jp = -1;
  for (int64_t k = 0; k < L; ++k) {
    const int buf = (int)(k & 1);
    const int64_t s = s0 + k;
    load_half(s, 1, v1);
    w0 = wn0;
    w1 = wn1;
    if (Ip >= 0) {
      flush_cols(buf ^ 1, Ip, Jp);
      Ip = -1;
    }
    if (Ic != Icur) {
      if (Icur >= 0) flush_rows();
      open_rows(Ic);
    }
    const bool mir = Jc >= 2 * Ic + 2;
    double g0 = 0.0, g1 = 0.0;
    if (mir) half_rows(v0, 0, w0, w1, true, g0, g1);
    else half_rows(v0, 0, w0, w1, false, g0, g1);
    if (k + 1 < L) {
      load_half(s + 1, 0, v0);
      load_w(Jn, wn0, wn1);
      advance(tn, In, Jn);
    }
    if (mir) {
      half_rows(v1, 1, w0, w1, true, g0, g1);
      colbuf[buf][wv * kSymCols + 2 * lane] = g0;
      colbuf[buf][wv * kSymCols + 2 * lane + 1] = g1;
      Ip = Ic;
      Jp = Jc;
    } else {
      half_rows(v1, 1, w0, w1, false, g0, g1);
    }
    advance(tc, Ic, Jc);
    __syncthreads();
  }
  if (Ip >= 0) flush_cols((int)((L - 1) & 1), Ip, Jp);
  flush_rows();
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

int kmv_rows_per_block(int prec) { return prec == LAKER_F64 ? 64 : 128; }

KmvPlan kmv_plan(int64_t m, int64_t n, int prec) {
  const int rpb = kmv_rows_per_block(prec);
  const int tile = prec == LAKER_F64 ? 16 : 32;
  const int64_t rowblocks = (m + rpb - 1) / rpb;
  const int64_t coltiles = (n + tile - 1) / tile;
  // about LAKER_KMV_BLOCKS blocks of four waves (512: two per CU, two waves
  // per SIMD), with few column ranges to add up afterwards
#ifndef LAKER_KMV_BLOCKS
#define LAKER_KMV_BLOCKS 512
#endif
  int64_t ns = (LAKER_KMV_BLOCKS + rowblocks - 1) / rowblocks;
  if (ns > coltiles) ns = coltiles;
  if (ns > kMaxSplit) ns = kMaxSplit;
  if (ns < 1) ns = 1;
  int64_t cps = ((coltiles + ns - 1) / ns) * tile;
  KmvPlan pl{};
  pl.cols_per_split = cps;
  pl.nsplit = (int)((n + cps - 1) / cps);
  if (pl.nsplit < 1) pl.nsplit = 1;
  pl.rowblocks = (int)rowblocks;
  return pl;
}

// Symmetric schedule for the square product of n rows, or sym = 0 when the
// rectangular one applies: dp > 64, fewer stages than blocks, or more row
// blocks than the column slots are sized for.
static SymPlan sym_plan(int64_t n, int grid = kSymGrid) {
  SymPlan sp{};
  sp.nrb = (int)((n + kSymRows - 1) / kSymRows);
  sp.ncs = (int)((n + kSymCols - 1) / kSymCols);
  sp.T = (int64_t)sp.nrb * sp.ncs - (int64_t)sp.nrb * (sp.nrb - 1);
  sp.grid = grid;
  sp.rs = 0;
  for (int64_t t = 0; t < sp.nrb; ++t) {
    const int64_t b0 = sym_block_of(sym_pos_start(t, sp.nrb, sp.ncs), sp.grid, sp.T);
    const int64_t b1 = sym_block_of(sym_pos_start(t + 1, sp.nrb, sp.ncs) - 1, sp.grid, sp.T);
    if (b1 - b0 + 1 > sp.rs) sp.rs = (int)(b1 - b0 + 1);
  }
  return sp;
}

// The symmetric schedule pays off once the MFMA work dominates or the stage
// runs are long: float32 / float64 products from two stages per block on
// (n >= ~5800), bfloat16 ones from six (n >= ~9800).  Measured on stand-alone
// products, symmetric against column-range, in us (d = 64):
//   n = 4096:   f32 40 / 34,   f64 76 / 81
//   n = 8192:   bf16 30 / 28,  f32 74 / 93,   f64 166 / 273
//   n = 10000:  bf16 38 / 43
//   n = 12000:  bf16 43 / 53,  f32 122 / 231, f64 284 / 715
//   n = 16384:  bf16 60 / 71,  f32 200 / 329, f64 499 / 978
static int64_t sym_min_stages(int prec) { return prec == LAKER_BF16 ? 6 : 2; }

static bool sym_applies(int64_t n, int dp, int prec) {
  if (dp > 64) return false;
  const int64_t nrb = (n + kSymRows - 1) / kSymRows;
  if (nrb > kSymMaxRowBlocks) return false;
  const int64_t ncs = (n + kSymCols - 1) / kSymCols;
  return nrb * ncs - nrb * (nrb - 1) >= sym_min_stages(prec) * kSymGrid;
}

// bfloat16 products of dp = 32 and 64 run the four-wave 16x16 kernel on twice
// as many blocks (two per CU); the others kSymGrid blocks of eight waves
static bool sym16_applies(int dp, int prec) { return prec == LAKER_BF16 && (dp == 32 || dp == 64); }
static int sym_grid(int dp, int prec) { return sym16_applies(dp, prec) ? 2 * kSymGrid : kSymGrid; }

bool kmv_sym16(int dp, int prec) { return sym16_applies(dp, prec); }

hipError_t kmv_run_sym16_batch(int dp, int count, const KmvArgs* As_dev, const SymPlan* Ps_dev,
                               const int* list_dev, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  if (!sym16_applies(dp, LAKER_BF16) || count > 65535) return hipErrorInvalidValue;
  const dim3 grid((unsigned)(2 * kSymGrid), (unsigned)count);
  if (dp == 32) kmvsym16_batch_kernel<32><<<grid, 256, 0, st>>>(As_dev, Ps_dev, list_dev);
  else kmvsym16_batch_kernel<64><<<grid, 256, 0, st>>>(As_dev, Ps_dev, list_dev);
  return hipGetLastError();
}

KmvPlan kmv_plan_square(int64_t n, int dp, int prec) {
  KmvPlan pl = kmv_plan(n, n, prec);
  if (sym_applies(n, dp, prec)) {
    pl.sym = 1;
    pl.sp = sym_plan(n, sym_grid(dp, prec));
    pl.sp.f32 = sym16_applies(dp, prec) ? 1 : 0;
  }
  return pl;
}

size_t kmv_part_elems(int64_t m, int64_t n) {
  const int64_t rows = n > m ? n : m;
  size_t e = (size_t)kMaxSplit * rows;
  if (sym_applies(n, 64, LAKER_F64)) {   // the loosest threshold
    for (int grid : {kSymGrid, 2 * kSymGrid}) {
      const SymPlan sp = sym_plan(n, grid);
      const size_t es = (size_t)(sp.rs + sp.nrb) * n;
      if (es > e) e = es;
    }
  }
  return e;
}

hipError_t launch_sym64(int dp, const KmvArgs& A, const SymPlan& sp, hipStream_t st) {
  switch (dp) {
    case 16: kmvsym64_kernel<16><<<sp.grid, 512, 0, st>>>(A, sp); break;
    case 32: kmvsym64_kernel<32><<<sp.grid, 512, 0, st>>>(A, sp); break;
    case 64: kmvsym64_kernel<64><<<sp.grid, 512, 0, st>>>(A, sp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC>
hipError_t launch_sym(int dp, const KmvArgs& A, const SymPlan& sp, hipStream_t st) {
  // the plan's grid belongs to the kernel's block shape
  if (sp.grid != sym_grid(dp, PREC)) return hipErrorInvalidValue;
  if (sym16_applies(dp, PREC)) {
    if (dp == 32) kmvsym16_kernel<32><<<sp.grid, 256, 0, st>>>(A, sp);
    else kmvsym16_kernel<64><<<sp.grid, 256, 0, st>>>(A, sp);
    return hipGetLastError();
  }
  switch (dp) {
    case 16: kmvsym_kernel<PREC, 16><<<sp.grid, 512, 0, st>>>(A, sp); break;
    case 32: kmvsym_kernel<PREC, 32><<<sp.grid, 512, 0, st>>>(A, sp); break;
    case 64: kmvsym_kernel<PREC, 64><<<sp.grid, 512, 0, st>>>(A, sp); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

bool kmat_applies(int64_t n, int dp) { return sym_applies(n, dp, LAKER_F64); }

size_t kmat_bytes(int64_t n, int prec) {
  const SymPlan sp = sym_plan(n);
  return (size_t)sp.T * (size_t)kTileElems * (prec == LAKER_F64 ? sizeof(double) : sizeof(float));
}

template <typename OT>
static hipError_t launch_kmat_build(int dp, const double* e64, int64_t n, const SymPlan& sp, OT* out, hipStream_t st) {
  switch (dp) {
    case 16: kmat_build_kernel<16, OT><<<sp.grid, 512, 0, st>>>(e64, n, sp, out); break;
    case 32: kmat_build_kernel<32, OT><<<sp.grid, 512, 0, st>>>(e64, n, sp, out); break;
    case 64: kmat_build_kernel<64, OT><<<sp.grid, 512, 0, st>>>(e64, n, sp, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t kmat_build(int dp, const double* e64, int64_t n, int prec, void* out, hipStream_t st) {
  if (!kmat_applies(n, dp) || out == nullptr) return hipErrorInvalidValue;
  const SymPlan sp = sym_plan(n);
  if (prec == LAKER_F64) return launch_kmat_build<double>(dp, e64, n, sp, (double*)out, st);
  if (prec == LAKER_F32) return launch_kmat_build<float>(dp, e64, n, sp, (float*)out, st);
  return hipErrorInvalidValue;
}

hipError_t kmv_run(int prec, int dp, const KmvPlan& pl, KmvArgs A, hipStream_t st) {
  A.cps = pl.cols_per_split;
  A.nsplit = pl.nsplit;
  A.ps = part_sum(pl);
  // the p^T A p partials and the on-the-fly conjugation belong to the
  // symmetric kernels inside PCG only
  if ((A.pap != nullptr || A.theta != nullptr) && !pl.sym) return hipErrorInvalidValue;
  if (A.theta != nullptr && (A.S == nullptr || !A.pcg_step)) return hipErrorInvalidValue;
  hipError_t e;
  if (A.kmat != nullptr) {
    // stored tiles: float64 or float32 entries, no in-kernel p^T A p or conjugation
    if (!pl.sym || A.Q != A.K || A.m != A.n || A.pap != nullptr || A.theta != nullptr) return hipErrorInvalidValue;
    if (prec == LAKER_F64) kmat_matvec_kernel<double><<<pl.sp.grid, 512, 0, st>>>(A, pl.sp);
    else if (prec == LAKER_F32) kmat_matvec_kernel<float><<<pl.sp.grid, 512, 0, st>>>(A, pl.sp);
    else return hipErrorInvalidValue;
    e = hipGetLastError();
  } else if (pl.sym) {
    // the symmetric schedule covers the square self-product only
    if (A.Q != A.K || A.m != A.n) return hipErrorInvalidValue;
    if (prec == LAKER_F64) e = launch_sym64(dp, A, pl.sp, st);
    else if (prec == LAKER_F32) e = launch_sym<LAKER_F32>(dp, A, pl.sp, st);
    else e = launch_sym<LAKER_BF16>(dp, A, pl.sp, st);
  } else {
    dim3 grid((unsigned)pl.rowblocks, (unsigned)pl.nsplit);
    if (prec == LAKER_F64) e = launch64(dp, grid, A, st);
    else if (prec == LAKER_F32) e = launch32<LAKER_F32>(dp, grid, A, st);
    else e = launch32<LAKER_BF16>(dp, grid, A, st);
  }
  if (e != hipSuccess || A.mode == 0) return e;
  int64_t g = (A.m + 255) / 256;
  if (g > 4096) g = 4096;
  kmv_finish_kernel<<<(unsigned)g, 256, 0, st>>>(A.part, A.ps, A.m, A.lam, A.pself, A.out);
  return hipGetLastError();
}

hipError_t kmv_run_batch(int prec, int dp, int count, const KmvArgs* As_dev, const int* tiles_dev, int ntiles,
                         bool finish, int64_t max_m, hipStream_t st) {
  hipError_t e;
  if (ntiles > 0) {
    if (prec == LAKER_F64) e = launch64_batch(dp, (unsigned)ntiles, As_dev, tiles_dev, st);
    else if (prec == LAKER_F32) e = launch32_batch<LAKER_F32>(dp, (unsigned)ntiles, As_dev, tiles_dev, st);
    else e = launch32_batch<LAKER_BF16>(dp, (unsigned)ntiles, As_dev, tiles_dev, st);
    if (e != hipSuccess) return e;
  }
  if (!finish) return hipSuccess;
  int64_t g = (max_m + 255) / 256;
  if (g > 1024) g = 1024;
  kmv_finish_batch_kernel<<<dim3((unsigned)g, (unsigned)count), 256, 0, st>>>(As_dev);
  return hipGetLastError();
}

}  // namespace lk
