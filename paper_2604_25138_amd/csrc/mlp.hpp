// The per-point network of the learned preconditioner (mlp.hip): layout of the
// model buffer, a bfloat16 MFMA matrix product with fused epilogues, feature
// construction and the Adam update.
#pragma once

#include "common.hpp"

namespace lk {

constexpr int kHidden = 256;       // width of both hidden layers
constexpr int kRank = 64;          // rank of the learned low-rank part
constexpr int kOut = kRank + 1;    // network outputs per point: v_i (kRank) and log delta_i

// Parameters W1 (in x H), b1 (H), W2 (H x H), b2 (H), W3 (H x kOut), b3 (kOut),
// weights stored fan_in x fan_out, float32, each tensor 64-element aligned.
// Model buffer: [theta | Adam m | Adam v], three blocks of `count` floats, each
// block 256-byte aligned.
struct MlpLayout {
  int d;
  int in_dim;          // 3 d + 2
  int64_t off[6];      // element offsets of W1 b1 W2 b2 W3 b3 in a block
  int64_t count;       // floats in one block
  size_t block_bytes;  // bytes of one block (256-aligned)
  size_t bytes;        // bytes of the model buffer
};
MlpLayout mlp_layout(int d);

// Epilogues of mm_bf16 (C = the f32 sum of the products):
//   kEpiLinear: out = C + bias                     (bias may be null)
//   kEpiSilu:   out2 = C + bias (pre-activation),  out = silu(C + bias)
//   kEpiSiluBack: out = C * silu'(zpre)
enum { kEpiLinear = 0, kEpiSilu = 1, kEpiSiluBack = 2 };

// out (M x N, row-major f32, leading dimension N) = epilogue(op(A) op(B)) with
//   op(A)(i, k) = A[i * sai + k * sak],  op(B)(k, j) = B[k * sbk + j * sbj];
// both operands are rounded to bfloat16 when staged and multiplied on MFMA
// with float32 accumulation.  `part` holds part_cap floats of split-K partials.
hipError_t mm_bf16(int64_t M, int64_t N, int64_t K, const float* A, int64_t sai, int64_t sak, const float* B,
                   int64_t sbk, int64_t sbj, float* part, int64_t part_cap, int epi, const float* bias,
                   const float* zpre, float* out, float* out2, hipStream_t st);

// Network inputs x_i = [e_i, log lambda, log(n)/10, mean_j e_j, mean_j e_j^2]
// (n x in_dim float32) from the float64 embeddings.  colpart holds
// 2 d kMaxBlocks doubles, stats 2 d doubles.
hipError_t mlp_features(const double* E, int64_t n, int d, double lambda, float* X, double* colpart, double* stats,
                        unsigned* cnt, hipStream_t st);

// One Adam step on `count` parameters (theta, m, v updated in place from g),
// step t >= 1 (bias correction).
hipError_t adam_update(float* theta, float* m, float* v, const float* g, int64_t count, double lr, double beta1,
                       double beta2, double eps, int t, hipStream_t st);

}  // namespace lk
