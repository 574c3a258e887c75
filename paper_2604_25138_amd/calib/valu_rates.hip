// Issue-rate calibration of the vector ALU and the matrix cores on the GPU it
// runs on: the denominators of the ALU roofline of the fused kernel products.
//
// The fused products spend their vector time on exp2 (one per distinct kernel
// entry) and float32 multiply-adds (one per ordered pair); their score tiles
// run on bfloat16 MFMA.  This program measures, per compute unit and clock:
//   * unpacked float32 multiply-adds (the library is built without packed
//     float32 instructions),
//   * v_exp_f32 (the hardware exp2),
//   * exp2 followed by 1, 2 or 4 dependent multiply-adds (do they overlap?),
//   * 32x32x16 bfloat16 MFMA alone and with 16 / 32 exp2 per 4 MFMA in the
//     same wave (does the matrix core run beside the vector ALU?), and the
//     same for eight 16x16x32 MFMA (the same flops in twice the instructions)
//     and for the older 16x16x16 / 32x32x8 forms,
//   * the symmetric product's work per 1024 kernel entries (16 per lane): the
//     score MFMA of either tile shape with 16 exp2 and 32 multiply-adds,
// at 1, 2, 4 and 8 waves per SIMD.  Each thread keeps 8 independent chains so
// that latency does not hide the issue rate, and writes one float at the end.
//
// Build: hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang
//        -packed-fp32-ops valu_rates.hip -o valu_rates
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>

#define CHECK(x)                                                                  \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));         \
      std::exit(1);                                                               \
    }                                                                             \
  } while (0)

typedef float v16f __attribute__((ext_vector_type(16)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;
constexpr int kThreads = 256;   // four waves: one per SIMD

__global__ __launch_bounds__(kThreads) void fma_rate(float* out, int iters, float a, float b) {
  float x[kChains];
  for (int j = 0; j < kChains; ++j) x[j] = threadIdx.x * 1e-3f + j;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = fmaf(x[j], a, b);
  }
  float s = 0.f;
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// x <- 2^-x converges (to ~0.64) and stays finite; the negation is a source
// modifier of the exp instruction
__global__ __launch_bounds__(kThreads) void exp_rate(float* out, int iters) {
  float x[kChains];
  for (int j = 0; j < kChains; ++j) x[j] = threadIdx.x * 1e-3f + j * 0.01f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = __builtin_amdgcn_exp2f(-x[j]);
  }
  float s = 0.f;
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

template <int NF>
__global__ __launch_bounds__(kThreads) void exp_fma_rate(float* out, int iters, float a) {
  float x[kChains], y[kChains];
  for (int j = 0; j < kChains; ++j) {
    x[j] = threadIdx.x * 1e-3f + j * 0.01f;
    y[j] = j;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) {
      const float t = __builtin_amdgcn_exp2f(-x[j]);
      x[j] = t;
#pragma unroll
      for (int f = 0; f < NF; ++f) y[j] = fmaf(y[j], a, t);
    }
  }
  float s = 0.f;
  for (int j = 0; j < kChains; ++j) s += x[j] + y[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// four independent 32x32x16 bfloat16 MFMA per iteration, and NE exp2 on
// sixteen independent chains
template <int NE>
__global__ __launch_bounds__(kThreads) void mfma_exp_rate(float* out, int iters) {
  v8bf av, bv;
  for (int j = 0; j < 8; ++j) {
    av[j] = (__bf16)(threadIdx.x * 1e-3f);
    bv[j] = (__bf16)(j * 1e-3f);
  }
  v16f c0 = {}, c1 = {}, c2 = {}, c3 = {};
  float x[16];
  for (int j = 0; j < 16; ++j) x[j] = threadIdx.x * 1e-3f + j * 0.01f;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c3, 0, 0, 0);
#pragma unroll
    for (int e = 0; e < NE; ++e) x[e % 16] = __builtin_amdgcn_exp2f(-x[e % 16]);
  }
  float s = 0.f;
  for (int j = 0; j < 16; ++j) s += c0[j] + c1[j] + c2[j] + c3[j] + x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// the same flops as eight independent 16x16x32 bfloat16 MFMA (the symmetric
// product's tile), with NE exp2 per iteration
typedef float v4f __attribute__((ext_vector_type(4)));
template <int NE>
__global__ __launch_bounds__(kThreads) void mfma16_exp_rate(float* out, int iters) {
  v8bf av, bv;
  for (int j = 0; j < 8; ++j) {
    av[j] = (__bf16)(threadIdx.x * 1e-3f);
    bv[j] = (__bf16)(j * 1e-3f);
  }
  v4f c[8];
  for (int k = 0; k < 8; ++k) c[k] = v4f{0.f, 0.f, 0.f, 0.f};
  float x[16];
  for (int j = 0; j < 16; ++j) x[j] = threadIdx.x * 1e-3f + j * 0.01f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c[k], 0, 0, 0);
#pragma unroll
    for (int e = 0; e < NE; ++e) x[e % 16] = __builtin_amdgcn_exp2f(-x[e % 16]);
  }
  float s = 0.f;
  for (int k = 0; k < 8; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  for (int j = 0; j < 16; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// the same flops as sixteen 16x16x16 or eight 32x32x8 bfloat16 MFMA (the
// older instructions, half the K)
typedef short v4s __attribute__((ext_vector_type(4)));
template <int NE>
__global__ __launch_bounds__(kThreads) void mfma16k16_exp_rate(float* out, int iters) {
  v4s av, bv;
  for (int j = 0; j < 4; ++j) {
    av[j] = (short)(threadIdx.x + j);
    bv[j] = (short)(j * 3 + 1);
  }
  v4f c[16];
  for (int k = 0; k < 16; ++k) c[k] = v4f{0.f, 0.f, 0.f, 0.f};
  float x[16];
  for (int j = 0; j < 16; ++j) x[j] = threadIdx.x * 1e-3f + j * 0.01f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 16; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, c[k], 0, 0, 0);
#pragma unroll
    for (int e = 0; e < NE; ++e) x[e % 16] = __builtin_amdgcn_exp2f(-x[e % 16]);
  }
  float s = 0.f;
  for (int k = 0; k < 16; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
  for (int j = 0; j < 16; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}
template <int NE>
__global__ __launch_bounds__(kThreads) void mfma32k8_exp_rate(float* out, int iters) {
  v4s av, bv;
  for (int j = 0; j < 4; ++j) {
    av[j] = (short)(threadIdx.x + j);
    bv[j] = (short)(j * 3 + 1);
  }
  v16f c[8];
  for (int k = 0; k < 8; ++k) c[k] = v16f{};
  float x[16];
  for (int j = 0; j < 16; ++j) x[j] = threadIdx.x * 1e-3f + j * 0.01f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) c[k] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, c[k], 0, 0, 0);
#pragma unroll
    for (int e = 0; e < NE; ++e) x[e % 16] = __builtin_amdgcn_exp2f(-x[e % 16]);
  }
  float s = 0.f;
  for (int k = 0; k < 8; ++k)
    for (int j = 0; j < 16; ++j) s += c[k][j];
  for (int j = 0; j < 16; ++j) s += x[j];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// The symmetric product's work per 1024 kernel entries at d = 64, on
// independent chains: NM32 32x32x16 MFMA (4: one score tile) or NM16 16x16x32
// MFMA (8: four score tiles), 16 exp2 and 32 multiply-adds (row and column
// sums) per lane.
template <int NM32, int NM16>
__global__ __launch_bounds__(kThreads) void tile_mix_rate(float* out, int iters, float a) {
  v8bf av, bv;
  for (int j = 0; j < 8; ++j) {
    av[j] = (__bf16)(threadIdx.x * 1e-3f);
    bv[j] = (__bf16)(j * 1e-3f);
  }
  v16f c[4];
  v4f d[8];
  for (int k = 0; k < 4; ++k) c[k] = v16f{};
  for (int k = 0; k < 8; ++k) d[k] = v4f{0.f, 0.f, 0.f, 0.f};
  float x[16], y[16];
  for (int j = 0; j < 16; ++j) {
    x[j] = threadIdx.x * 1e-3f + j * 0.01f;
    y[j] = j;
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < NM32; ++k) c[k & 3] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, c[k & 3], 0, 0, 0);
#pragma unroll
    for (int k = 0; k < NM16; ++k) d[k & 7] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, d[k & 7], 0, 0, 0);
#pragma unroll
    for (int e = 0; e < 16; ++e) x[e] = __builtin_amdgcn_exp2f(-x[e]);
#pragma unroll
    for (int f = 0; f < 32; ++f) y[f & 15] = fmaf(y[f & 15], a, x[(f * 7) & 15]);
  }
  float s = 0.f;
  for (int j = 0; j < 16; ++j) s += x[j] + y[j] + c[0][j] + c[1][j] + c[2][j] + c[3][j];
  for (int k = 0; k < 8; ++k) s += d[k][0] + d[k][1] + d[k][2] + d[k][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

int main() {
  int cus = 0, khz = 0;
  CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, 0));
  CHECK(hipDeviceGetAttribute(&khz, hipDeviceAttributeClockRate, 0));
  std::printf("compute units %d, clock %d MHz\n", cus, khz / 1000);
  std::printf("| waves / SIMD | test | ms | per CU per clock |\n|---:|---|---:|---:|\n");
  hipEvent_t e0, e1;
  CHECK(hipEventCreate(&e0));
  CHECK(hipEventCreate(&e1));
  const int iters = 4096;
  for (int wps = 1; wps <= 8; wps *= 2) {
    const int blocks = cus * wps;
    float* out = nullptr;
    CHECK(hipMalloc(&out, (size_t)blocks * kThreads * sizeof(float)));
    // per_thread_iter: counted operations per thread and loop iteration
    auto run = [&](const char* name, auto launch, double per_thread_iter, const char* unit) {
      launch();
      CHECK(hipGetLastError());
      CHECK(hipDeviceSynchronize());
      CHECK(hipEventRecord(e0));
      for (int r = 0; r < 5; ++r) launch();
      CHECK(hipEventRecord(e1));
      CHECK(hipEventSynchronize(e1));
      float ms = 0.f;
      CHECK(hipEventElapsedTime(&ms, e0, e1));
      ms /= 5;
      const double ops = (double)blocks * kThreads * iters * per_thread_iter;
      const double rate = ops / (ms * 1e-3) / cus / (khz * 1e3);
      std::printf("| %d | %s | %.3f | %.1f %s |\n", wps, name, ms, rate, unit);
    };
    run("fp32 multiply-add", [&] { fma_rate<<<blocks, kThreads>>>(out, iters, 0.999f, 1e-3f); }, kChains,
        "lane-FMA");
    run("exp2", [&] { exp_rate<<<blocks, kThreads>>>(out, iters); }, kChains, "lane-exp2");
    run("exp2 + 1 FMA", [&] { exp_fma_rate<1><<<blocks, kThreads>>>(out, iters, 0.999f); }, kChains, "lane-exp2");
    run("exp2 + 2 FMA", [&] { exp_fma_rate<2><<<blocks, kThreads>>>(out, iters, 0.999f); }, kChains, "lane-exp2");
    run("exp2 + 4 FMA", [&] { exp_fma_rate<4><<<blocks, kThreads>>>(out, iters, 0.999f); }, kChains, "lane-exp2");
    // a wave's four 32x32x16 MFMA are 4 * 32768 flops: per thread, a 64th
    run("bf16 MFMA", [&] { mfma_exp_rate<0><<<blocks, kThreads>>>(out, iters); }, 4.0 * 32768 / 64, "flop");
    run("bf16 MFMA + 16 exp2", [&] { mfma_exp_rate<16><<<blocks, kThreads>>>(out, iters); }, 4.0 * 32768 / 64,
        "flop");
    run("bf16 MFMA + 32 exp2", [&] { mfma_exp_rate<32><<<blocks, kThreads>>>(out, iters); }, 4.0 * 32768 / 64,
        "flop");
    // eight 16x16x32 MFMA: 8 * 16384 flops per wave, the same as four 32x32x16
    run("bf16 MFMA 16x16x32", [&] { mfma16_exp_rate<0><<<blocks, kThreads>>>(out, iters); }, 8.0 * 16384 / 64,
        "flop");
    run("bf16 MFMA 16x16x32 + 16 exp2", [&] { mfma16_exp_rate<16><<<blocks, kThreads>>>(out, iters); },
        8.0 * 16384 / 64, "flop");
    run("bf16 MFMA 16x16x32 + 32 exp2", [&] { mfma16_exp_rate<32><<<blocks, kThreads>>>(out, iters); },
        8.0 * 16384 / 64, "flop");
    run("bf16 MFMA 16x16x16", [&] { mfma16k16_exp_rate<0><<<blocks, kThreads>>>(out, iters); }, 16.0 * 8192 / 64,
        "flop");
    run("bf16 MFMA 16x16x16 + 16 exp2", [&] { mfma16k16_exp_rate<16><<<blocks, kThreads>>>(out, iters); },
        16.0 * 8192 / 64, "flop");
    run("bf16 MFMA 32x32x8", [&] { mfma32k8_exp_rate<0><<<blocks, kThreads>>>(out, iters); }, 8.0 * 16384 / 64,
        "flop");
    run("bf16 MFMA 32x32x8 + 16 exp2", [&] { mfma32k8_exp_rate<16><<<blocks, kThreads>>>(out, iters); },
        8.0 * 16384 / 64, "flop");
    // per 1024 kernel entries: 16 per lane
    run("16 exp2 + 32 FMA per lane", [&] { tile_mix_rate<0, 0><<<blocks, kThreads>>>(out, iters, 0.999f); }, 16.0,
        "entries");
    run("+ 4 MFMA 32x32x16", [&] { tile_mix_rate<4, 0><<<blocks, kThreads>>>(out, iters, 0.999f); }, 16.0,
        "entries");
    run("+ 8 MFMA 16x16x32", [&] { tile_mix_rate<0, 8><<<blocks, kThreads>>>(out, iters, 0.999f); }, 16.0,
        "entries");
    CHECK(hipFree(out));
  }
  return 0;
}
