// The learned rank-64-plus-diagonal preconditioner (learned.hip): network
// forward and backward, the probe loss and its gradient through the Woodbury
// solve, the preconditioner buffer, and Sigma^{1/2} Z of a fitted CCCP
// preconditioner (the training target).
#pragma once

#include "mlp.hpp"
#include "pcg.hpp"

namespace lk {

struct LearnedWs {
  // network (float32)
  float* X;      // n x in_dim inputs
  float* Z1;     // n x H pre-activations of layer 1
  float* H1;     // n x H
  float* Z2;
  float* H2;
  float* O;      // n x kOut outputs
  float* dO;     // n x kOut
  float* dZ2;    // n x H
  float* dZ1;    // n x H
  float* grad;   // gradient block (MlpLayout::count floats)
  float* part;   // split-K partials of the network products
  int64_t part_cap;
  float* one;    // a single 1.0f (row of ones for bias gradients)
  double* colpart;
  double* stats;
  // loss side (float64)
  double* V;     // n x R
  double* DV;    // D^{-1} V
  double* Di;    // 1 / delta
  double* delta;
  double* Kc;    // R x R capacitance, then its inverse
  double* Kside;
  double* Y;     // n x m
  double* G;     // n x m: -2 (Z - Y) / (n m), then H = S^{-1} G
  double* S1;    // R x m
  double* S2;
  double* YtV;   // m x R
  double* HtV;
  double* dV;    // n x R
  double* gpart; // partials of the float64 products
  int64_t gpart_cap;
  double* lpart; // per-block loss partials
  double* scal;  // [0] loss, [1] log det of the capacitance
  int* flag;
  unsigned* gbar;
  unsigned* cnt;
  size_t total;
};
LearnedWs plan_learned_ws(void* base, int64_t n, int d, int m);

// Network output O (n x kOut) for the problem's embeddings.
laker_status learned_forward(const Problem& pb, const MlpLayout& L, const float* theta, const LearnedWs& w,
                             hipStream_t st);

// Loss ||Z - S^{-1} U||^2 / (n m) into w.scal[0] and its gradient into w.grad
// (after learned_forward).
laker_status learned_loss_grad(const Problem& pb, const MlpLayout& L, const float* theta, const double* Z,
                               const double* U, int m, const LearnedWs& w, hipStream_t st);

// P = S^{-1} = D^{-1} + Bt B^T with B = D^{-1} V, Bt = -B K^{-1} into the
// preconditioner buffer (after learned_forward).
laker_status learned_build(const Problem& pb, const LearnedWs& w, const PrecondLayout& P, hipStream_t st);

// Sigma^{1/2} Z = Sigma (P Z) for a fitted CCCP preconditioner
// (Sigma = b I + B B^T, P = b^{-1/2} I + Bt B^T).
struct SigmaHalfWs {
  double* t;     // nrp x m
  double* PZ;    // n x m
  double* part;
  int64_t part_cap;
  size_t total;
};
SigmaHalfWs plan_sigma_half_ws(void* base, int64_t n, int nr, int m);
laker_status sigma_half(const PrecondLayout& P, int64_t n, int nr, int m, const double* Z, double* U,
                        const SigmaHalfWs& w, hipStream_t st);

}  // namespace lk
