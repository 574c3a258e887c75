// Random-direction products U = (lambda I + G) Z for N_r right-hand sides
// (eq. random_directions; Alg. 1, first step of preconditioner learning) on the
// matrix cores, flash-attention style: per key tile J the score tile is
// S'^T = K_J Q_I^T (MFMA), E = exp2(S') stays in registers, and O_I += E Z_J is a
// second MFMA, so neither G nor E is ever stored.
//
// The first MFMA is issued with the key rows as the A operand, so that each
// lane's exp values belong to one query row i and the key set
//   j(h, r) = 8 (r / 4) + 4 h + (r % 4),  r = 0..15,  h = lane / 32
// of the 32 x 32 accumulator layout.  The second MFMA contracts over j; its A
// operand takes those values as they are, and the B operand (the Z tile) is
// read from LDS in the same j order, so no data moves between lanes.
//
// Arithmetic: float32 (32x32x2 f32 for both products) or bfloat16 (32x32x16
// bf16, exp values and Z rounded to bfloat16), float32 accumulation.  These
// directions only shape the preconditioner; any SPD P leaves the PCG solution
// unchanged.
#include <type_traits>

#include "mrhs.hpp"

namespace lk {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

constexpr int NC = 64;    // output columns (directions) per block
constexpr int KJ = 32;    // keys per tile

__device__ __forceinline__ uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void z_convert_f32_kernel(const double* __restrict__ Z, float* __restrict__ out, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = __double2float_rn(Z[i]);
}

__global__ void z_convert_bf16_kernel(const double* __restrict__ Z, uint16_t* __restrict__ out, int64_t total) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = bf16_rne(__double2float_rn(Z[i]));
}

template <int PREC, int DP>
struct MrhsT {
  using ET = typename std::conditional<PREC == LAKER_F32, float, uint16_t>::type;
  static constexpr int ES = (int)sizeof(ET);
  static constexpr int ROWB = DP * ES;
  static constexpr int KPITCH = ROWB + 16;                 // padded key-row pitch (bytes)
  // Z tile: f32 as Zs[j][c] (pitch NC + 1 floats); bf16 transposed as ZsT[c][j] (pitch 40 bf16)
  static constexpr int ZBYTES = PREC == LAKER_F32 ? KJ * (NC + 1) * 4 : NC * 40 * 2;
};

template <int PREC, int DP>
__global__ __launch_bounds__(256) void mrhs_kernel(const void* __restrict__ Ehv, int64_t n,
                                                   const void* __restrict__ Zrv, const double* __restrict__ Z64,
                                                   int nr, double lam, double* __restrict__ U) {
  using T = MrhsT<PREC, DP>;
  using ET = typename T::ET;
  __shared__ __attribute__((aligned(16))) unsigned char ks[KJ * T::KPITCH];
  __shared__ __attribute__((aligned(16))) unsigned char zs[T::ZBYTES];
  const int tid = threadIdx.x;
  const int lane = tid & 63, wv = tid >> 6;
  const int h = lane >> 5, c = lane & 31;
  const int64_t row0 = (int64_t)blockIdx.x * 128 + wv * 32;
  const int c0 = blockIdx.y * NC;
  const ET* __restrict__ Eh = reinterpret_cast<const ET*>(Ehv);
  const ET* __restrict__ Zr = reinterpret_cast<const ET*>(Zrv);

  // query fragment (B operand of the score MFMA): row row0 + c, k-half h
  float qf[PREC == LAKER_F32 ? DP / 2 : 1];
  v8bf qb[PREC == LAKER_F32 ? 1 : DP / 16];
  {
    int64_t qi = row0 + c;
    if (qi > n - 1) qi = n - 1;
    if constexpr (PREC == LAKER_F32) {
      const float4* src = reinterpret_cast<const float4*>(reinterpret_cast<const float*>(Ehv) + qi * DP + h * (DP / 2));
#pragma unroll
      for (int q = 0; q < DP / 8; ++q) {
        const float4 t = src[q];
        qf[4 * q] = t.x;
        qf[4 * q + 1] = t.y;
        qf[4 * q + 2] = t.z;
        qf[4 * q + 3] = t.w;
      }
    } else {
      const u32x4* src = reinterpret_cast<const u32x4*>(reinterpret_cast<const uint16_t*>(Ehv) + qi * DP + h * (DP / 2));
#pragma unroll
      for (int q = 0; q < DP / 16; ++q) qb[q] = __builtin_bit_cast(v8bf, src[q]);
    }
  }
  v16f acc0 = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  v16f acc1 = acc0;

  for (int64_t jt = 0; jt < n; jt += KJ) {
    __syncthreads();
    // key rows jt .. jt + 31 (clamped) -> ks
    for (int ch = tid; ch < KJ * (T::ROWB / 16); ch += 256) {
      const int rr = ch / (T::ROWB / 16), cc = ch % (T::ROWB / 16);
      int64_t kr = jt + rr;
      if (kr > n - 1) kr = n - 1;
      *reinterpret_cast<u32x4*>(&ks[rr * T::KPITCH + cc * 16]) =
          *reinterpret_cast<const u32x4*>(reinterpret_cast<const unsigned char*>(Eh) + kr * T::ROWB + cc * 16);
    }
    // Z tile rows jt .. jt + 31, columns c0 .. c0 + 63 (zero outside) -> zs
    for (int e = tid; e < KJ * NC; e += 256) {
      const int jj = e / NC, cc = e % NC;
      const int64_t j = jt + jj;
      ET v = ET(0);
      if (j < n && c0 + cc < nr) v = Zr[j * nr + c0 + cc];
      if constexpr (PREC == LAKER_F32) reinterpret_cast<float*>(zs)[jj * (NC + 1) + cc] = v;
      else reinterpret_cast<uint16_t*>(zs)[cc * 40 + jj] = v;
    }
    __syncthreads();
    // S'^T = K_J Q^T: A operand = key row c of the tile, B operand = query row c
    v16f s = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const unsigned char* krow = ks + c * T::KPITCH + h * (T::ROWB / 2);
    if constexpr (PREC == LAKER_F32) {
#pragma unroll
      for (int q = 0; q < DP / 8; ++q) {
        const float4 t = *reinterpret_cast<const float4*>(krow + 16 * q);
        s = __builtin_amdgcn_mfma_f32_32x32x2f32(t.x, qf[4 * q], s, 0, 0, 0);
        s = __builtin_amdgcn_mfma_f32_32x32x2f32(t.y, qf[4 * q + 1], s, 0, 0, 0);
        s = __builtin_amdgcn_mfma_f32_32x32x2f32(t.z, qf[4 * q + 2], s, 0, 0, 0);
        s = __builtin_amdgcn_mfma_f32_32x32x2f32(t.w, qf[4 * q + 3], s, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int q = 0; q < DP / 16; ++q) {
        const v8bf kf = __builtin_bit_cast(v8bf, *reinterpret_cast<const u32x4*>(krow + 16 * q));
        s = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf, qb[q], s, 0, 0, 0);
      }
    }
    // lane (c, h): s[r] = score of query row c with key j(h, r)
    float e[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) e[r] = __builtin_amdgcn_exp2f(s[r]);
    // O += E Z_J for the two 32-column output tiles
    if constexpr (PREC == LAKER_F32) {
      const float* zf = reinterpret_cast<const float*>(zs);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int j = 8 * (r >> 2) + 4 * h + (r & 3);
        acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(e[r], zf[j * (NC + 1) + c], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(e[r], zf[j * (NC + 1) + 32 + c], acc1, 0, 0, 0);
      }
    } else {
      const uint16_t* zt = reinterpret_cast<const uint16_t*>(zs);
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        u32x4 ab;
        ab[0] = (uint32_t)bf16_rne(e[8 * st + 0]) | ((uint32_t)bf16_rne(e[8 * st + 1]) << 16);
        ab[1] = (uint32_t)bf16_rne(e[8 * st + 2]) | ((uint32_t)bf16_rne(e[8 * st + 3]) << 16);
        ab[2] = (uint32_t)bf16_rne(e[8 * st + 4]) | ((uint32_t)bf16_rne(e[8 * st + 5]) << 16);
        ab[3] = (uint32_t)bf16_rne(e[8 * st + 6]) | ((uint32_t)bf16_rne(e[8 * st + 7]) << 16);
        const v8bf a8 = __builtin_bit_cast(v8bf, ab);
        // keys 16 st + 4 h + 0..3 and 16 st + 8 + 4 h + 0..3 of column c (and c + 32)
        const uint16_t* z0 = zt + c * 40 + 16 * st + 4 * h;
        const uint16_t* z1 = zt + (32 + c) * 40 + 16 * st + 4 * h;
        u32x4 b0, b1;
        const u32x2 p00 = *reinterpret_cast<const u32x2*>(z0);
        const u32x2 p01 = *reinterpret_cast<const u32x2*>(z0 + 8);
        const u32x2 p10 = *reinterpret_cast<const u32x2*>(z1);
        const u32x2 p11 = *reinterpret_cast<const u32x2*>(z1 + 8);
        b0[0] = p00[0];
        b0[1] = p00[1];
        b0[2] = p01[0];
        b0[3] = p01[1];
        b1[0] = p10[0];
        b1[1] = p10[1];
        b1[2] = p11[0];
        b1[3] = p11[1];
        acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, __builtin_bit_cast(v8bf, b0), acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a8, __builtin_bit_cast(v8bf, b1), acc1, 0, 0, 0);
      }
    }
  }
  // lane (c, h): acc[r] = O[row (r/4)*8 + 4h + r%4][column c (+32)]
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int64_t i = row0 + 8 * (r >> 2) + 4 * h + (r & 3);
    if (i >= n) continue;
    const int k0 = c0 + c, k1 = c0 + 32 + c;
    if (k0 < nr) U[i * nr + k0] = fma(lam, Z64[i * nr + k0], (double)acc0[r]);
    if (k1 < nr) U[i * nr + k1] = fma(lam, Z64[i * nr + k1], (double)acc1[r]);
  }
}

template <int PREC>
hipError_t launch(int dp, dim3 grid, const void* Eh, int64_t n, const void* Zr, const double* Z64, int nr,
                  double lam, double* U, hipStream_t st) {
  switch (dp) {
    case 16: mrhs_kernel<PREC, 16><<<grid, 256, 0, st>>>(Eh, n, Zr, Z64, nr, lam, U); break;
    case 32: mrhs_kernel<PREC, 32><<<grid, 256, 0, st>>>(Eh, n, Zr, Z64, nr, lam, U); break;
    case 64: mrhs_kernel<PREC, 64><<<grid, 256, 0, st>>>(Eh, n, Zr, Z64, nr, lam, U); break;
    case 128: mrhs_kernel<PREC, 128><<<grid, 256, 0, st>>>(Eh, n, Zr, Z64, nr, lam, U); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

size_t mrhs_z_bytes(int64_t n, int nr) { return (size_t)n * nr * 4; }

hipError_t mrhs_mfma(int prec, int dp, const void* Eh, int64_t n, const double* Z, void* Zr, int nr, double lam,
                     double* U, hipStream_t st) {
  const int64_t total = n * (int64_t)nr;
  int64_t g = (total + 255) / 256;
  if (g > 8192) g = 8192;
  if (prec == LAKER_F32) z_convert_f32_kernel<<<(unsigned)g, 256, 0, st>>>(Z, (float*)Zr, total);
  else z_convert_bf16_kernel<<<(unsigned)g, 256, 0, st>>>(Z, (uint16_t*)Zr, total);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((n + 127) / 128), (unsigned)((nr + NC - 1) / NC));
  if (prec == LAKER_F32) return launch<LAKER_F32>(dp, grid, Eh, n, Zr, Z, nr, lam, U, st);
  return launch<LAKER_BF16>(dp, grid, Eh, n, Zr, Z, nr, lam, U, st);
}

}  // namespace lk
