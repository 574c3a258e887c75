// The learned rank-64-plus-diagonal preconditioner.
//
// A per-point network maps x_i = [e_i, log lambda, log(n)/10, mean e, mean e^2]
// to o_i = (v_i, log delta_i); S = diag(delta) + V V^T is a surrogate of the
// CCCP matrix Sigma_star^{1/2} (Sec. IV), SPD for every weight vector, and the
// preconditioner is P = S^{-1}, applied through the Woodbury identity with the
// R x R capacitance K = I + V^T D^{-1} V:
//     P = D^{-1} + Bt B^T,   B = D^{-1} V,   Bt = -B K^{-1}.
// Training minimises L = ||Z - S^{-1} U||_F^2 / (n m) over Gaussian probes Z
// with U = Sigma_star^{1/2} Z taken from fitted CCCP preconditioners; with
// Y = S^{-1} U, G = -2 (Z - Y) / (n m) and H = S^{-1} G,
//     dL/d delta_i = -sum_k H_ik Y_ik,   dL/dV = -(H (Y^T V) + Y (H^T V)).
// The network runs on bfloat16 MFMA with float32 accumulation and float32
// master weights; the loss side (Woodbury solves and the gradient of S) runs in
// float64.
#include "learned.hpp"

#include <math.h>

#include <algorithm>

#include "dense.hpp"

namespace lk {

namespace {

constexpr int kT = 256;

inline int grid_for(int64_t total) {
  int64_t g = (total + kT - 1) / kT;
  if (g > 4096) g = 4096;
  return (int)(g < 1 ? 1 : g);
}

// V (float64) and the diagonal from the network output
__global__ void split_kernel(const float* __restrict__ O, int64_t n, double* __restrict__ V,
                             double* __restrict__ DV, double* __restrict__ Di, double* __restrict__ delta) {
  const int64_t total = n * kOut;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t i = idx / kOut;
    const int c = (int)(idx - i * kOut);
    const double ld = (double)O[i * kOut + kRank];
    const double di = exp(-ld);
    if (c < kRank) {
      const double v = (double)O[idx];
      V[i * kRank + c] = v;
      DV[i * kRank + c] = di * v;
    } else {
      Di[i] = di;
      delta[i] = exp(ld);
    }
  }
}

__global__ void fill_one_kernel(float* p) {
  if (threadIdx.x == 0) p[0] = 1.0f;
}

__global__ void identity_kernel(double* __restrict__ K, int r) {
  for (int idx = blockIdx.x * kT + threadIdx.x; idx < r * r; idx += gridDim.x * kT)
    K[idx] = (idx / r == idx % r) ? 1.0 : 0.0;
}

// out = Di (row scale) * X, n x m
__global__ void rowscale_kernel(const double* __restrict__ X, const double* __restrict__ Di, double* __restrict__ out,
                                int64_t n, int m) {
  const int64_t total = n * m;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT)
    out[idx] = Di[idx / m] * X[idx];
}

// G = -2 (Z - Y) / (n m); loss = sum (Z - Y)^2 / (n m) into scal[0]
__global__ __launch_bounds__(kT) void loss_kernel(const double* __restrict__ Z, const double* __restrict__ Y,
                                                  double* __restrict__ G, int64_t total, double inv,
                                                  double* __restrict__ lpart, double* __restrict__ scal,
                                                  unsigned* cnt) {
  __shared__ double sh[16];
  double s = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const double r = Z[idx] - Y[idx];
    s = fma(r, r, s);
    G[idx] = -2.0 * r * inv;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) lpart[blockIdx.x] = s;
  if (last_block_arrived(cnt)) {
    const double t = ordered_sum(lpart, gridDim.x, sh);
    if (threadIdx.x == 0) {
      scal[0] = t * inv;
      *cnt = 0;
    }
  }
}

// dO = [dV, (-sum_k H_ik Y_ik) delta_i] in float32
__global__ void dout_kernel(const double* __restrict__ dV, const double* __restrict__ H, const double* __restrict__ Y,
                            const double* __restrict__ delta, int64_t n, int m, float* __restrict__ dO) {
  const int64_t total = n * kOut;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t i = idx / kOut;
    const int c = (int)(idx - i * kOut);
    if (c < kRank) {
      dO[idx] = (float)dV[i * kRank + c];
    } else {
      double s = 0.0;
      for (int k = 0; k < m; ++k) s = fma(H[i * m + k], Y[i * m + k], s);
      dO[idx] = (float)(-s * delta[i]);
    }
  }
}

__global__ void scale_by_kernel(const double* __restrict__ X, const double* __restrict__ sp, double* __restrict__ out,
                                int64_t total) {
  const double s = sp[0];
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT)
    out[idx] = s * X[idx];
}

__global__ void learned_finish_kernel(const double* __restrict__ DV, const double* __restrict__ Bt,
                                      const double* __restrict__ Di, int64_t n, float* __restrict__ B32,
                                      float* __restrict__ Bt32, double* __restrict__ dinv, double* __restrict__ hdr) {
  const int64_t total = n * kRank;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    B32[idx] = (float)DV[idx];
    Bt32[idx] = (float)Bt[idx];
    if (idx < n) dinv[idx] = Di[idx];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int k = 0; k < 32; ++k) hdr[k] = 0.0;
  }
}

// float64 product with a split picked for the partial buffer
hipError_t g64(int64_t M, int64_t N, int64_t K, const double* A, int64_t sai, int64_t sak, const double* B,
               int64_t sbk, int64_t sbj, double* C, int64_t ldc, double alpha, const double* alpha_dev, double beta,
               double* part, int64_t cap, hipStream_t st) {
  int ns = gemm_pick_split(M, N, K, cap);
  return gemm_f64(M, N, K, A, sai, sak, B, sbk, sbj, C, ldc, alpha, alpha_dev, beta, part, ns, st);
}

// out = S^{-1} X (n x m) by Woodbury; out may alias X.  Kc holds K^{-1}.
laker_status woodbury(const LearnedWs& w, int64_t n, int m, const double* X, double* out, hipStream_t st) {
  rowscale_kernel<<<grid_for(n * m), kT, 0, st>>>(X, w.Di, out, n, m);
  LK_CHECK_LAUNCH();
  LK_TRY(g64(kRank, m, n, w.V, 1, kRank, out, m, 1, w.S1, m, 1.0, nullptr, 0.0, w.gpart, w.gpart_cap, st));
  LK_TRY(g64(kRank, m, kRank, w.Kc, kRank, 1, w.S1, m, 1, w.S2, m, 1.0, nullptr, 0.0, w.gpart, w.gpart_cap, st));
  LK_TRY(g64(n, m, kRank, w.DV, kRank, 1, w.S2, m, 1, out, m, -1.0, nullptr, 1.0, w.gpart, w.gpart_cap, st));
  return LAKER_OK;
}

// V, D^{-1}, and K^{-1} = (I + V^T D^{-1} V)^{-1} into w.Kc
laker_status capacitance(const LearnedWs& w, int64_t n, hipStream_t st) {
  split_kernel<<<grid_for(n * kOut), kT, 0, st>>>(w.O, n, w.V, w.DV, w.Di, w.delta);
  LK_CHECK_LAUNCH();
  identity_kernel<<<grid_for(kRank * kRank), kT, 0, st>>>(w.Kc, kRank);
  LK_CHECK_LAUNCH();
  LK_TRY(g64(kRank, kRank, n, w.V, 1, kRank, w.DV, kRank, 1, w.Kc, kRank, 1.0, nullptr, 1.0, w.gpart, w.gpart_cap,
             st));
  LK_TRY(hipMemsetAsync(w.gbar, 0, sizeof(unsigned), st));
  LK_TRY(hipMemsetAsync(w.flag, 0, sizeof(int), st));
  double* As[1] = {w.Kc};
  double* Ss[1] = {w.Kside};
  double* Ls[1] = {w.scal + 1};
  LK_TRY(spd_inverse_sweep(1, As, Ss, Ls, kRank, w.flag, w.gbar, 0u, st));
  return LAKER_OK;
}

}  // namespace

LearnedWs plan_learned_ws(void* base, int64_t n, int d, int m) {
  WsCarver c(base);
  LearnedWs w{};
  const MlpLayout L = mlp_layout(d);
  const int64_t mm = m > 0 ? m : 1;
  w.X = c.take<float>((size_t)n * L.in_dim);
  w.Z1 = c.take<float>((size_t)n * kHidden);
  w.H1 = c.take<float>((size_t)n * kHidden);
  w.Z2 = c.take<float>((size_t)n * kHidden);
  w.H2 = c.take<float>((size_t)n * kHidden);
  w.O = c.take<float>((size_t)n * kOut);
  w.dO = c.take<float>((size_t)n * kOut);
  w.dZ2 = c.take<float>((size_t)n * kHidden);
  w.dZ1 = c.take<float>((size_t)n * kHidden);
  w.grad = c.take<float>((size_t)L.count);
  w.part_cap = std::max<int64_t>((int64_t)n * kHidden * 2, (int64_t)128 * kHidden * kHidden);
  w.part = c.take<float>((size_t)w.part_cap);
  w.one = c.take<float>(64);
  w.colpart = c.take<double>((size_t)kMaxBlocks * 2 * d);
  w.stats = c.take<double>((size_t)2 * d);
  w.V = c.take<double>((size_t)n * kRank);
  w.DV = c.take<double>((size_t)n * kRank);
  w.Di = c.take<double>((size_t)n);
  w.delta = c.take<double>((size_t)n);
  w.Kc = c.take<double>((size_t)kRank * kRank);
  w.Kside = c.take<double>(gj_side_elems(kRank));
  w.Y = c.take<double>((size_t)n * mm);
  w.G = c.take<double>((size_t)n * mm);
  w.S1 = c.take<double>((size_t)kRank * mm);
  w.S2 = c.take<double>((size_t)kRank * mm);
  w.YtV = c.take<double>((size_t)mm * kRank);
  w.HtV = c.take<double>((size_t)mm * kRank);
  w.dV = c.take<double>((size_t)n * kRank);
  w.gpart_cap = std::max<int64_t>((int64_t)4 << 20, 2 * (int64_t)n * std::max<int64_t>(mm, kRank));
  w.gpart = c.take<double>((size_t)w.gpart_cap);
  w.lpart = c.take<double>(kMaxBlocks);
  w.scal = c.take<double>(8);
  w.flag = c.take<int>(16);
  w.gbar = c.take<unsigned>(16);
  w.cnt = c.take<unsigned>(16);
  w.total = c.bytes();
  return w;
}

laker_status learned_forward(const Problem& pb, const MlpLayout& L, const float* theta, const LearnedWs& w,
                             hipStream_t st) {
  const int64_t n = pb.n;
  LK_TRY(hipMemsetAsync(w.cnt, 0, 16 * sizeof(unsigned), st));
  LK_TRY(mlp_features(pb.E, n, pb.d, pb.lambda, w.X, w.colpart, w.stats, w.cnt, st));
  const float* W1 = theta + L.off[0];
  const float* b1 = theta + L.off[1];
  const float* W2 = theta + L.off[2];
  const float* b2 = theta + L.off[3];
  const float* W3 = theta + L.off[4];
  const float* b3 = theta + L.off[5];
  LK_TRY(mm_bf16(n, kHidden, L.in_dim, w.X, L.in_dim, 1, W1, kHidden, 1, w.part, w.part_cap, kEpiSilu, b1, nullptr,
                 w.H1, w.Z1, st));
  LK_TRY(mm_bf16(n, kHidden, kHidden, w.H1, kHidden, 1, W2, kHidden, 1, w.part, w.part_cap, kEpiSilu, b2, nullptr,
                 w.H2, w.Z2, st));
  LK_TRY(mm_bf16(n, kOut, kHidden, w.H2, kHidden, 1, W3, kOut, 1, w.part, w.part_cap, kEpiLinear, b3, nullptr, w.O,
                 nullptr, st));
  return LAKER_OK;
}

laker_status learned_loss_grad(const Problem& pb, const MlpLayout& L, const float* theta, const double* Z,
                               const double* U, int m, const LearnedWs& w, hipStream_t st) {
  const int64_t n = pb.n;
  laker_status e = capacitance(w, n, st);
  if (e != LAKER_OK) return e;
  // Y = S^{-1} U; loss and G
  e = woodbury(w, n, m, U, w.Y, st);
  if (e != LAKER_OK) return e;
  {
    int64_t g = (n * m + kT * 4 - 1) / (kT * 4);
    if (g > kMaxBlocks) g = kMaxBlocks;
    loss_kernel<<<(unsigned)g, kT, 0, st>>>(Z, w.Y, w.G, n * m, 1.0 / ((double)n * m), w.lpart, w.scal, w.cnt);
    LK_CHECK_LAUNCH();
  }
  // H = S^{-1} G (in place)
  e = woodbury(w, n, m, w.G, w.G, st);
  if (e != LAKER_OK) return e;
  // dV = -(H (Y^T V) + Y (H^T V))
  LK_TRY(g64(m, kRank, n, w.Y, 1, m, w.V, kRank, 1, w.YtV, kRank, 1.0, nullptr, 0.0, w.gpart, w.gpart_cap, st));
  LK_TRY(g64(m, kRank, n, w.G, 1, m, w.V, kRank, 1, w.HtV, kRank, 1.0, nullptr, 0.0, w.gpart, w.gpart_cap, st));
  LK_TRY(g64(n, kRank, m, w.G, m, 1, w.YtV, kRank, 1, w.dV, kRank, -1.0, nullptr, 0.0, w.gpart, w.gpart_cap, st));
  LK_TRY(g64(n, kRank, m, w.Y, m, 1, w.HtV, kRank, 1, w.dV, kRank, -1.0, nullptr, 1.0, w.gpart, w.gpart_cap, st));
  dout_kernel<<<grid_for(n * kOut), kT, 0, st>>>(w.dV, w.G, w.Y, w.delta, n, m, w.dO);
  LK_CHECK_LAUNCH();
  // backward through the network
  LK_TRY(hipMemsetAsync(w.grad, 0, sizeof(float) * L.count, st));
  fill_one_kernel<<<1, 64, 0, st>>>(w.one);
  LK_CHECK_LAUNCH();
  float* gW1 = w.grad + L.off[0];
  float* gb1 = w.grad + L.off[1];
  float* gW2 = w.grad + L.off[2];
  float* gb2 = w.grad + L.off[3];
  float* gW3 = w.grad + L.off[4];
  float* gb3 = w.grad + L.off[5];
  const float* W2 = theta + L.off[2];
  const float* W3 = theta + L.off[4];
  // layer 3: dW3 = H2^T dO, db3 = 1^T dO, dZ2 = (dO W3^T) * silu'(Z2)
  LK_TRY(mm_bf16(kHidden, kOut, n, w.H2, 1, kHidden, w.dO, kOut, 1, w.part, w.part_cap, kEpiLinear, nullptr, nullptr,
                 gW3, nullptr, st));
  LK_TRY(mm_bf16(1, kOut, n, w.one, 0, 0, w.dO, kOut, 1, w.part, w.part_cap, kEpiLinear, nullptr, nullptr, gb3,
                 nullptr, st));
  LK_TRY(mm_bf16(n, kHidden, kOut, w.dO, kOut, 1, W3, 1, kOut, w.part, w.part_cap, kEpiSiluBack, nullptr, w.Z2, w.dZ2,
                 nullptr, st));
  // layer 2
  LK_TRY(mm_bf16(kHidden, kHidden, n, w.H1, 1, kHidden, w.dZ2, kHidden, 1, w.part, w.part_cap, kEpiLinear, nullptr,
                 nullptr, gW2, nullptr, st));
  LK_TRY(mm_bf16(1, kHidden, n, w.one, 0, 0, w.dZ2, kHidden, 1, w.part, w.part_cap, kEpiLinear, nullptr, nullptr, gb2,
                 nullptr, st));
  LK_TRY(mm_bf16(n, kHidden, kHidden, w.dZ2, kHidden, 1, W2, 1, kHidden, w.part, w.part_cap, kEpiSiluBack, nullptr,
                 w.Z1, w.dZ1, nullptr, st));
  // layer 1
  LK_TRY(mm_bf16(L.in_dim, kHidden, n, w.X, 1, L.in_dim, w.dZ1, kHidden, 1, w.part, w.part_cap, kEpiLinear, nullptr,
                 nullptr, gW1, nullptr, st));
  LK_TRY(mm_bf16(1, kHidden, n, w.one, 0, 0, w.dZ1, kHidden, 1, w.part, w.part_cap, kEpiLinear, nullptr, nullptr, gb1,
                 nullptr, st));
  return LAKER_OK;
}

laker_status learned_build(const Problem& pb, const LearnedWs& w, const PrecondLayout& P, hipStream_t st) {
  const int64_t n = pb.n;
  laker_status e = capacitance(w, n, st);
  if (e != LAKER_OK) return e;
  // B = D^{-1} V (row stride kRank = nrp), Bt = -B K^{-1}
  LK_TRY(hipMemcpyAsync(P.B64, w.DV, sizeof(double) * n * kRank, hipMemcpyDeviceToDevice, st));
  LK_TRY(g64(n, kRank, kRank, w.DV, kRank, 1, w.Kc, kRank, 1, P.Bt64, kRank, -1.0, nullptr, 0.0, w.gpart,
             w.gpart_cap, st));
  learned_finish_kernel<<<grid_for(n * kRank), kT, 0, st>>>(w.DV, P.Bt64, w.Di, n, P.B32, P.Bt32, P.dinv64, P.hdr);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

SigmaHalfWs plan_sigma_half_ws(void* base, int64_t n, int nr, int m) {
  WsCarver c(base);
  SigmaHalfWs w{};
  const int nrp = pad_nr(nr);
  w.t = c.take<double>((size_t)nrp * m);
  w.PZ = c.take<double>((size_t)n * m);
  w.part_cap = std::max<int64_t>((int64_t)4 << 20, (int64_t)n * m);
  w.part = c.take<double>((size_t)w.part_cap);
  w.total = c.bytes();
  return w;
}

laker_status sigma_half(const PrecondLayout& P, int64_t n, int nr, int m, const double* Z, double* U,
                        const SigmaHalfWs& w, hipStream_t st) {
  const int nrp = pad_nr(nr);
  // PZ = c0 Z + Bt (B^T Z)
  LK_TRY(g64(nrp, m, n, P.B64, 1, nrp, Z, m, 1, w.t, m, 1.0, nullptr, 0.0, w.part, w.part_cap, st));
  scale_by_kernel<<<grid_for(n * m), kT, 0, st>>>(Z, P.hdr, w.PZ, n * m);
  LK_CHECK_LAUNCH();
  LK_TRY(g64(n, m, nrp, P.Bt64, nrp, 1, w.t, m, 1, w.PZ, m, 1.0, nullptr, 1.0, w.part, w.part_cap, st));
  // U = b PZ + B (B^T PZ)
  LK_TRY(g64(nrp, m, n, P.B64, 1, nrp, w.PZ, m, 1, w.t, m, 1.0, nullptr, 0.0, w.part, w.part_cap, st));
  scale_by_kernel<<<grid_for(n * m), kT, 0, st>>>(w.PZ, P.hdr + 2, U, n * m);
  LK_CHECK_LAUNCH();
  LK_TRY(g64(n, m, nrp, P.B64, nrp, 1, w.t, m, 1, U, m, 1.0, nullptr, 1.0, w.part, w.part_cap, st));
  return LAKER_OK;
}

}  // namespace lk
