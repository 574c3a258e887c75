// Preconditioned conjugate gradient on (lambda I + G) alpha = y (Sec. IV-E, Alg. 1).
//
// Every step runs on the device: the products A p, the inner products, the
// updates of alpha, r and p, the stopping test on the recursive residual and the
// preconditioner.  Scalars (delta, beta, ||r||^2, ...) live in device memory and
// each grid reduction is finished by the last block to arrive, in a fixed
// order.  The host enqueues `check_every` iterations at a time and then reads
// the `done` flag; kernels launched after convergence return at once.
//
// The Krylov vectors are float64 in every precision mode: only the kernel
// product changes arithmetic (float64, or float32 / bfloat16 scores with
// float64 accumulation).  At kappa(A) ~ 1e8, float32 accumulation of the
// products or float32 recurrences roughly double the iteration count, because
// their rounding noise is of the order of lambda |p| in the directions CG
// resolves last.
#include <mutex>
#include <vector>

#include "pcg.hpp"

namespace lk {

namespace {

constexpr int kThreads = 256;

// A non-blocking stream per device on which PCG chunks are captured into graphs
// (capture needs a stream other than the null stream; the graphs are launched on
// the caller's stream).
hipStream_t capture_stream() {
  static hipStream_t streams[64] = {};
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (streams[dev] == nullptr && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

// blocks of the low-rank apply: 16 rows per block pass, at most kMaxBlocks blocks
inline int apply_blocks(int64_t n) {
  int64_t g = (n + 15) / 16;
  if (g > kMaxBlocks) g = kMaxBlocks;
  return (int)(g < 1 ? 1 : g);
}

inline int red_blocks(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > kMaxBlocks) g = kMaxBlocks;
  if (g < 1) g = 1;
  return (int)g;
}

// Grid reductions: every kernel writes one float64 partial per block with a
// plain store; the kernel that needs the total (launched after it, so the
// partials are visible) adds them in a fixed order in each of its blocks, and
// block 0 records the scalar.  No atomics or fences inside the loop.

// r = y - w (or y when w is null); p = 0; partials of ||y||^2 and ||r||^2.
__global__ __launch_bounds__(kThreads) void pcg_init_kernel(const double* __restrict__ y, const double* __restrict__ w,
                                                            double* __restrict__ r, double* __restrict__ p, int64_t n,
                                                            double* __restrict__ yyp, double* __restrict__ rrp) {
  __shared__ double sh[16];
  double yy = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double yi = y[i];
    const double ri = w != nullptr ? yi - w[i] : yi;
    r[i] = ri;
    p[i] = 0.0;
    yy += yi * yi;
    rr += ri * ri;
  }
  yy = block_sum(yy, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    yyp[blockIdx.x] = yy;
    rrp[blockIdx.x] = rr;
  }
}

// One block: ||y||^2, ||r^0||^2, the tolerance and the initial state.
__global__ __launch_bounds__(kThreads) void pcg_start_kernel(PcgScalars* S, const double* __restrict__ yyp,
                                                             const double* __restrict__ rrp, int g, double tol,
                                                             int max_iter) {
  __shared__ double sh[16];
  const double yy = ordered_sum(yyp, g, sh);
  const double rr = ordered_sum(rrp, g, sh);
  if (threadIdx.x == 0) {
    S->yy = yy;
    S->rr = rr;
    S->tol2 = tol * tol * yy;
    S->iters = 0;
    S->max_iter = max_iter;
    S->beta = 0.0;
    S->kcur = 0;
    S->done = (yy == 0.0 || rr <= tol * tol * yy) ? 1 : 0;
  }
}

// Ap = lambda p + sum of the column-range partials; partials of p^T A p.
__global__ __launch_bounds__(kThreads) void pcg_ap_kernel(const double* __restrict__ p, const double* __restrict__ part,
                                                          int nsplit, double* __restrict__ Ap, int64_t n, double lam,
                                                          double* __restrict__ pap_p, const PcgScalars* S) {
  if (S->done) return;
  __shared__ double sh[16];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * n + i];
    const double pi = p[i];
    const double a = fma(lam, pi, s);
    Ap[i] = a;
    acc += pi * a;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) pap_p[blockIdx.x] = acc;
}

// delta = r^T theta / p^T A p; alpha += delta p; r -= delta Ap (Alg. 1);
// partials of ||r||^2 and, for Jacobi, theta = r / diag and r^T theta.
template <int KIND>
__global__ __launch_bounds__(kThreads) void pcg_update_kernel(double* __restrict__ alpha, double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ Ap,
                                                              const double* __restrict__ dinv,
                                                              double* __restrict__ theta, int64_t n, PcgScalars* S,
                                                              const double* __restrict__ pap_p, int gp,
                                                              double* __restrict__ rrp, double* __restrict__ rzp) {
  if (S->done) return;
  __shared__ double sh[16];
  const int k = S->kcur - 1;
  const double pap = ordered_sum(pap_p, gp, sh);
  const double dl = S->rzbuf[k & 1] / pap;
  if (!(pap > 0.0) || !isfinite(dl)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) S->done = 2;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->pap = pap;
    S->delta = dl;
  }
  double rr = 0.0, rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    alpha[i] = fma(dl, p[i], alpha[i]);
    const double ri = fma(-dl, Ap[i], r[i]);
    r[i] = ri;
    rr += ri * ri;
    if (KIND == LAKER_PRECOND_JACOBI) {
      const double ti = ri * dinv[i];
      theta[i] = ti;
      rz += ri * ti;
    }
  }
  rr = block_sum(rr, sh);
  if (KIND == LAKER_PRECOND_JACOBI) rz = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    rrp[blockIdx.x] = rr;
    rzp[blockIdx.x] = rz;
  }
}

// Stopping test of iteration k on the recursive residual (Alg. 1), evaluated
// identically by every block; block 0 records it.  Returns true to continue.
__device__ bool pcg_decide(int k, PcgScalars* S, const double* __restrict__ rrp, int g, double* sh) {
  const double rr = ordered_sum(rrp, g, sh);
  int d = 0;
  if (!isfinite(rr)) d = 2;
  else if (rr <= S->tol2) d = 1;
  else if (k + 1 >= S->max_iter) d = 3;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->rr = rr;
    S->iters = k + 1;
    if (d) S->done = d;
  }
  return d == 0;
}

// p = theta + beta p with beta = r_new^T theta_new / r^T theta.  With
// init set: p = theta and r^T theta is stored for iteration 0.  For P = I and
// Jacobi this kernel also takes the stopping decision of iteration k.
template <int KIND>
__global__ __launch_bounds__(kThreads) void pcg_pupdate_kernel(int init, const double* __restrict__ theta,
                                                               double* __restrict__ p, int64_t n, PcgScalars* S,
                                                               const double* __restrict__ rrp, int grr,
                                                               const double* __restrict__ rzp, int grz) {
  if (S->done) return;
  __shared__ double sh[16];
  const int k = S->kcur - 1;
  if (!init && KIND != LAKER_PRECOND_CCCP && !pcg_decide(k, S, rrp, grr, sh)) return;
  const double rz = ordered_sum(KIND == LAKER_PRECOND_NONE ? rrp : rzp, KIND == LAKER_PRECOND_NONE ? grr : grz, sh);
  const int slot = init ? 0 : ((k + 1) & 1);
  const double b = init ? 0.0 : rz / S->rzbuf[k & 1];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->rzbuf[slot] = rz;
    S->beta = b;
  }
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    p[i] = fma(b, p[i], theta[i]);
}

// theta = r / diag (Jacobi) with r^T theta partials, for the start of the iteration.
__global__ __launch_bounds__(kThreads) void jacobi_apply_kernel(const double* __restrict__ r,
                                                                const double* __restrict__ dinv,
                                                                double* __restrict__ theta, int64_t n,
                                                                const PcgScalars* S, double* __restrict__ rzp) {
  if (S->done) return;
  __shared__ double sh[16];
  double rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double ri = r[i];
    const double ti = ri * dinv[i];
    theta[i] = ti;
    rz += ri * ti;
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) rzp[blockIdx.x] = rz;
}

// Low-rank preconditioner  theta = c0 r + Bt (B^T r)  with B, Bt stored n x nrp
// row-major (nrp = N_r rounded up to a multiple of 4, zero padding), as float64
// or float32 (MT); products are accumulated in float64.
//
// t = B^T r, first half: block b owns rows [64 b, 64 b + 64).  A thread owns
// four consecutive columns (one 16-byte load per row, 8 bytes for float64
// pairs twice) and the block's threads are split into row groups when fewer
// than 256 threads cover the columns; groups are combined in LDS in a fixed
// order into one float64 partial row per block.
constexpr int kTRows = 64;

template <typename MT>
__global__ __launch_bounds__(kThreads) void lr_t_partial_kernel(const MT* __restrict__ B, const double* __restrict__ r,
                                                                int64_t n, int nrp, double* __restrict__ tpart,
                                                                const PcgScalars* S) {
  if (S != nullptr && S->done) return;
  __shared__ double red[kMaxNr];
  const int tid = threadIdx.x;
  const int cq = nrp / 4;                       // column quads
  int tpr = 1;                                  // threads per row group (power of two >= cq)
  while (tpr < cq) tpr <<= 1;
  const int groups = kThreads / tpr;
  const int g = tid / tpr, q = tid % tpr;
  const int64_t i0 = (int64_t)blockIdx.x * kTRows;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (q < cq) {
#pragma unroll 8
    for (int rr = g; rr < kTRows; rr += groups) {
      const int64_t i = i0 + rr;
      if (i < n) {
        const double ri = r[i];
        const MT* row = B + i * nrp + 4 * q;
        a0 = fma((double)row[0], ri, a0);
        a1 = fma((double)row[1], ri, a1);
        a2 = fma((double)row[2], ri, a2);
        a3 = fma((double)row[3], ri, a3);
      }
    }
  }
  // fixed-order combination of the row groups
  for (int gg = 0; gg < groups; ++gg) {
    if (g == gg && q < cq) {
      if (gg == 0) {
        red[4 * q + 0] = a0;
        red[4 * q + 1] = a1;
        red[4 * q + 2] = a2;
        red[4 * q + 3] = a3;
      } else {
        red[4 * q + 0] += a0;
        red[4 * q + 1] += a1;
        red[4 * q + 2] += a2;
        red[4 * q + 3] += a3;
      }
    }
    __syncthreads();
  }
  for (int k = tid; k < nrp; k += kThreads) tpart[(int64_t)blockIdx.x * nrp + k] = red[k];
}

// PCG update fused with the first half of the low-rank preconditioner: block
// b owns rows [64 b, 64 b + 64): delta from the p^T A p partials, alpha += delta p,
// r -= delta Ap, the ||r||^2 partial, and t_b = B[rows]^T r[rows] from the
// fresh r kept in LDS.  The stopping decision is taken by the next pass.
template <typename MT>
__global__ __launch_bounds__(kThreads) void pcg_update_t_kernel(double* __restrict__ alpha,
                                                                double* __restrict__ r, const double* __restrict__ p,
                                                                const double* __restrict__ Ap,
                                                                const MT* __restrict__ B, int nrp, int64_t n,
                                                                PcgScalars* S, const double* __restrict__ pap_p,
                                                                int gp, double* __restrict__ rrp,
                                                                double* __restrict__ tpart) {
  if (S->done) return;
  __shared__ double sh[16];
  __shared__ double rs[kTRows];
  __shared__ double red[kMaxNr];
  const int tid = threadIdx.x;
  const int k = S->kcur - 1;
  const double pap = ordered_sum(pap_p, gp, sh);
  const double dl = S->rzbuf[k & 1] / pap;
  if (!(pap > 0.0) || !isfinite(dl)) {
    if (blockIdx.x == 0 && tid == 0) S->done = 2;
    return;
  }
  if (blockIdx.x == 0 && tid == 0) {
    S->pap = pap;
    S->delta = dl;
  }
  const int64_t i0 = (int64_t)blockIdx.x * kTRows;
  double rr = 0.0;
  if (tid < kTRows) {
    const int64_t i = i0 + tid;
    double ri = 0.0;
    if (i < n) {
      alpha[i] = fma(dl, p[i], alpha[i]);
      ri = fma(-dl, Ap[i], r[i]);
      r[i] = ri;
    }
    rs[tid] = ri;
    rr = ri * ri;
  }
  rr = block_sum(rr, sh);     // contains the barrier that publishes rs
  if (tid == 0) rrp[blockIdx.x] = rr;
  const int cq = nrp / 4;
  int tpr = 1;
  while (tpr < cq) tpr <<= 1;
  const int groups = kThreads / tpr;
  const int g = tid / tpr, q = tid % tpr;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (q < cq) {
#pragma unroll 8
    for (int rr2 = g; rr2 < kTRows; rr2 += groups) {
      const int64_t i = i0 + rr2;
      if (i < n) {
        const double ri = rs[rr2];
        const MT* row = B + i * nrp + 4 * q;
        a0 = fma((double)row[0], ri, a0);
        a1 = fma((double)row[1], ri, a1);
        a2 = fma((double)row[2], ri, a2);
        a3 = fma((double)row[3], ri, a3);
      }
    }
  }
  for (int gg = 0; gg < groups; ++gg) {
    if (g == gg && q < cq) {
      if (gg == 0) {
        red[4 * q + 0] = a0;
        red[4 * q + 1] = a1;
        red[4 * q + 2] = a2;
        red[4 * q + 3] = a3;
      } else {
        red[4 * q + 0] += a0;
        red[4 * q + 1] += a1;
        red[4 * q + 2] += a2;
        red[4 * q + 3] += a3;
      }
    }
    __syncthreads();
  }
  for (int c = tid; c < nrp; c += kThreads) tpart[(int64_t)blockIdx.x * nrp + c] = red[c];
}

// t[k] = sum_b tpart[b][k] in a fixed order: a block owns 16 columns; its 16
// row groups of 16 threads each sum every 16th partial row, then combine in LDS.
__global__ __launch_bounds__(kThreads) void lr_t_finish_kernel(const double* __restrict__ tpart, int nb, int nrp,
                                                               double* __restrict__ t, PcgScalars* S,
                                                               const double* __restrict__ rrp, int grr) {
  if (S != nullptr && S->done) return;
  __shared__ double red[16][17];
  __shared__ double shd[16];
  // inside the loop this pass takes the stopping decision of the current iteration first
  if (rrp != nullptr && !pcg_decide(S->kcur - 1, S, rrp, grr, shd)) return;
  const int g = threadIdx.x >> 4, cl = threadIdx.x & 15;
  const int col = blockIdx.x * 16 + cl;
  double s = 0.0;
  if (col < nrp)
    for (int b = g; b < nb; b += 16) s += tpart[(int64_t)b * nrp + col];
  red[g][cl] = s;
  __syncthreads();
  if (g == 0 && col < nrp) {
    double v = 0.0;
    for (int gg = 0; gg < 16; ++gg) v += red[gg][cl];
    t[col] = v;
  }
}

// theta = c r + Bt t (c = c0, or dinv_i for a diagonal-plus-low-rank
// preconditioner): 16 lanes per row (four rows per wave), 16-byte loads,
// t in LDS; partials of r^T theta.
template <typename MT>
__global__ __launch_bounds__(kThreads) void lr_apply_kernel(const MT* __restrict__ Bt, const double* __restrict__ t,
                                                            const double* __restrict__ r, double* __restrict__ theta,
                                                            int64_t n, int nrp, const double* __restrict__ c0p,
                                                            const double* __restrict__ dinv, const PcgScalars* S,
                                                            double* __restrict__ rzp) {
  if (S != nullptr && S->done) return;
  constexpr int VEC = 16 / (int)sizeof(MT);
  __shared__ double sh[16];
  __shared__ double ts[kMaxNr];
  const double c0 = c0p[0];
  for (int k = threadIdx.x; k < nrp; k += kThreads) ts[k] = t[k];
  __syncthreads();
  const int sub = threadIdx.x & 15;
  const int rl = threadIdx.x >> 4;                  // row slot within the block (16 per pass)
  const int nvec = nrp / VEC;
  double rz = 0.0;
  for (int64_t i0 = (int64_t)blockIdx.x * 16; i0 < n; i0 += (int64_t)gridDim.x * 16) {
    const int64_t i = i0 + rl;
    double acc = 0.0;
    if (i < n) {
      // all of the lane's loads are issued before the first use
      constexpr int MAXV = kMaxNr / VEC / 16;
      const MT* row = Bt + i * nrp;
      if constexpr (VEC == 4) {
        float4 x[MAXV];
#pragma unroll
        for (int j = 0; j < MAXV; ++j)
          if (sub + 16 * j < nvec) x[j] = *reinterpret_cast<const float4*>(row + 4 * (sub + 16 * j));
#pragma unroll
        for (int j = 0; j < MAXV; ++j) {
          if (sub + 16 * j < nvec) {
            const int v = sub + 16 * j;
            acc = fma((double)x[j].x, ts[4 * v + 0], acc);
            acc = fma((double)x[j].y, ts[4 * v + 1], acc);
            acc = fma((double)x[j].z, ts[4 * v + 2], acc);
            acc = fma((double)x[j].w, ts[4 * v + 3], acc);
          }
        }
      } else {
        double2 x[MAXV];
#pragma unroll
        for (int j = 0; j < MAXV; ++j)
          if (sub + 16 * j < nvec) x[j] = *reinterpret_cast<const double2*>(row + 2 * (sub + 16 * j));
#pragma unroll
        for (int j = 0; j < MAXV; ++j) {
          if (sub + 16 * j < nvec) {
            const int v = sub + 16 * j;
            acc = fma(x[j].x, ts[2 * v + 0], acc);
            acc = fma(x[j].y, ts[2 * v + 1], acc);
          }
        }
      }
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 8, 64);
    if (sub == 0 && i < n) {
      const double ri = r[i];
      const double th = fma(dinv != nullptr ? dinv[i] : c0, ri, acc);
      theta[i] = th;
      rz += ri * th;
    }
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0 && rzp != nullptr) rzp[blockIdx.x] = rz;
}

// ||y - w||^2 and ||y||^2 (float64), for the true residual; r = y - w if r is set.
__global__ __launch_bounds__(kThreads) void resid_kernel(const double* __restrict__ y, const double* __restrict__ w,
                                                         double* __restrict__ r, int64_t n,
                                                         double* __restrict__ bpart, unsigned* cnt, double* out2) {
  __shared__ double sh[16];
  double rr = 0.0, yy = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double yi = y[i];
    const double ri = w != nullptr ? yi - w[i] : yi;
    if (r != nullptr) r[i] = ri;
    rr += ri * ri;
    yy += yi * yi;
  }
  rr = block_sum(rr, sh);
  yy = block_sum(yy, sh);
  if (threadIdx.x == 0) {
    bpart[blockIdx.x] = rr;
    bpart[kMaxBlocks + blockIdx.x] = yy;
  }
  if (last_block_arrived(cnt)) {
    const double srr = ordered_sum(bpart, gridDim.x, sh);
    const double syy = ordered_sum(bpart + kMaxBlocks, gridDim.x, sh);
    if (threadIdx.x == 0) {
      out2[0] = srr;
      out2[1] = syy;
      *cnt = 0;
    }
  }
}

__global__ void axpy_kernel(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    x[i] += d[i];
}

// theta = P r for the low-rank preconditioner (three passes); with rrp set the
// middle pass first takes the stopping decision of iteration k, and the first
// pass is skipped when `skip_partial` says the fused update already wrote the
// t partials.
template <typename MT>
laker_status enqueue_lowrank(const PrecondView& P, const double* r, double* theta, int64_t n, PcgScalars* S,
                             const double* rrp, int grr, double* rzp, double* tpart, double* t, bool skip_partial,
                             hipStream_t st) {
  const int nb = (int)((n + kTRows - 1) / kTRows);
  if (!skip_partial) {
    lr_t_partial_kernel<MT><<<nb, kThreads, 0, st>>>((const MT*)P.B, r, n, P.nrp, tpart, S);
    LK_CHECK_LAUNCH();
  }
  lr_t_finish_kernel<<<(P.nrp + 15) / 16, kThreads, 0, st>>>(tpart, nb, P.nrp, t, S, rrp, grr);
  LK_CHECK_LAUNCH();
  lr_apply_kernel<MT><<<(unsigned)apply_blocks(n), kThreads, 0, st>>>((const MT*)P.Bt, t, r, theta, n, P.nrp, P.c0p,
                                                                      (const double*)P.dinv, S, rzp);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

laker_status enqueue_lowrank_any(const PrecondView& P, const double* r, double* theta, int64_t n, PcgScalars* S,
                                 const double* rrp, int grr, double* rzp, double* tpart, double* t,
                                 bool skip_partial, hipStream_t st) {
  if (P.f32) return enqueue_lowrank<float>(P, r, theta, n, S, rrp, grr, rzp, tpart, t, skip_partial, st);
  return enqueue_lowrank<double>(P, r, theta, n, S, rrp, grr, rzp, tpart, t, skip_partial, st);
}

}  // namespace

SolveWs plan_solve_ws(void* base, int64_t n, int d, int64_t m) {
  WsCarver c(base);
  SolveWs w;
  const int dp = pad_dim(d);
  const int64_t rows = n > m ? n : m;
  const int64_t mq = m > 0 ? m : 1;
  w.e64 = c.take<double>((size_t)n * dp);
  w.e32 = c.take<float>((size_t)n * dp);
  w.e16 = c.take<uint16_t>((size_t)n * dp);
  w.q64 = c.take<double>((size_t)mq * dp);
  w.q32 = c.take<float>((size_t)mq * dp);
  w.q16 = c.take<uint16_t>((size_t)mq * dp);
  w.part = c.take<double>((size_t)kMaxSplit * rows);
  w.r = c.take<double>(n);
  w.p = c.take<double>(n);
  w.ap = c.take<double>(n);
  w.theta = c.take<double>(n);
  w.w64 = c.take<double>(rows);
  w.rout = c.take<double>(n);
  w.dalpha = c.take<double>(n);
  w.S = c.take<PcgScalars>(1);
  w.bpart = c.take<double>(2 * kMaxBlocks);
  w.yyp = c.take<double>(kMaxBlocks);
  // partials of ||r||^2 come from up to max(kMaxBlocks, n / kTRows) blocks
  const int64_t nrrp = (n + kTRows - 1) / kTRows > kMaxBlocks ? (n + kTRows - 1) / kTRows : kMaxBlocks;
  w.rrp = c.take<double>((size_t)nrrp);
  w.rzp = c.take<double>(kMaxBlocks);
  w.papp = c.take<double>(kMaxBlocks);
  w.tpart = c.take<double>((size_t)((n + kTRows - 1) / kTRows) * kMaxNr);
  w.t = c.take<double>(kMaxNr);
  w.misc = c.take<double>(16);
  w.cnt = c.take<unsigned>(16);
  w.total = c.bytes();
  return w;
}

KmvArgs kmv_args(const void* Q, int64_t m, const void* K, int64_t n, const double* p, const SolveWs& ws) {
  KmvArgs A{};
  A.Q = Q;
  A.m = m;
  A.K = K;
  A.n = n;
  A.p = p;
  A.part = ws.part;
  A.mode = 1;
  return A;
}

const void* prepared(const SolveWs& ws, int prec) {
  return prec == LAKER_F64 ? (const void*)ws.e64 : (prec == LAKER_F32 ? (const void*)ws.e32 : (const void*)ws.e16);
}

laker_status true_residual(const Problem& pb, const SolveWs& ws, const double* y, const double* alpha,
                           double* r_out, double* relres, bool have_alpha, hipStream_t st) {
  const int g = red_blocks(pb.n);
  const double* wv = nullptr;
  if (have_alpha) {
    KmvPlan pl = kmv_plan(pb.n, pb.n, LAKER_F64);
    KmvArgs A = kmv_args(ws.e64, pb.n, ws.e64, pb.n, alpha, ws);
    A.lam = pb.lambda;
    A.pself = alpha;
    A.out = ws.w64;
    LK_TRY(kmv_run(LAKER_F64, pb.dp, pl, A, st));
    wv = ws.w64;
  }
  resid_kernel<<<g, kThreads, 0, st>>>(y, wv, r_out, pb.n, ws.bpart, ws.cnt, ws.misc);
  LK_CHECK_LAUNCH();
  double h[2];
  LK_TRY(hipMemcpyAsync(h, ws.misc, sizeof(h), hipMemcpyDeviceToHost, st));
  LK_TRY(hipStreamSynchronize(st));
  *relres = h[1] > 0 ? sqrt(h[0] / h[1]) : 0.0;
  return LAKER_OK;
}

laker_status pcg_run(const Problem& pb, const SolveWs& ws, const PrecondView& P, const double* rhs, double* alpha,
                     bool warm, double tol, int max_iter, int check_every, int prec, bool use_graph, bool profile,
                     laker_stats* stats, hipStream_t st) {
  const int64_t n = pb.n;
  const int g = red_blocks(n);
  const int ga = apply_blocks(n);
  double* r = ws.r;
  double* p = ws.p;
  double* Ap = ws.ap;
  double* th = ws.theta;
  PcgScalars* S = ws.S;
  const void* eh = prepared(ws, prec);
  const KmvPlan pl = kmv_plan(n, n, prec);
  const bool lowrank = P.kind == LAKER_PRECOND_CCCP || P.kind == LAKER_PRECOND_LEARNED;
  const double* dinv = (const double*)P.dinv;

  // r^0 = y - A alpha^0
  const double* wv = nullptr;
  if (warm) {
    KmvArgs A = kmv_args(eh, n, eh, n, alpha, ws);
    A.lam = pb.lambda;
    A.pself = alpha;
    A.out = Ap;
    LK_TRY(kmv_run(prec, pb.dp, pl, A, st));
    wv = Ap;
  } else {
    LK_TRY(hipMemsetAsync(alpha, 0, sizeof(double) * n, st));
  }
  pcg_init_kernel<<<g, kThreads, 0, st>>>(rhs, wv, r, p, n, ws.yyp, ws.rrp);
  LK_CHECK_LAUNCH();
  pcg_start_kernel<<<1, kThreads, 0, st>>>(S, ws.yyp, ws.rrp, g, tol, max_iter);
  LK_CHECK_LAUNCH();
  // theta^0 = P r^0, p^0 = theta^0, r^T theta stored for iteration 0
  if (P.kind == LAKER_PRECOND_JACOBI) {
    jacobi_apply_kernel<<<g, kThreads, 0, st>>>(r, dinv, th, n, S, ws.rzp);
    LK_CHECK_LAUNCH();
    pcg_pupdate_kernel<LAKER_PRECOND_JACOBI><<<g, kThreads, 0, st>>>(1, th, p, n, S, ws.rrp, g, ws.rzp, g);
  } else if (P.kind == LAKER_PRECOND_NONE) {
    pcg_pupdate_kernel<LAKER_PRECOND_NONE><<<g, kThreads, 0, st>>>(1, r, p, n, S, ws.rrp, g, ws.rzp, g);
  } else {
    laker_status e = enqueue_lowrank_any(P, r, th, n, S, nullptr, 0, ws.rzp, ws.tpart, ws.t, false, st);
    if (e != LAKER_OK) return e;
    pcg_pupdate_kernel<LAKER_PRECOND_CCCP><<<g, kThreads, 0, st>>>(1, th, p, n, S, ws.rrp, g, ws.rzp, ga);
  }
  LK_CHECK_LAUNCH();

  KmvArgs Ak = kmv_args(eh, n, eh, n, p, ws);
  Ak.mode = 0;
  Ak.S = S;
  Ak.pcg_step = 1;
  const int nbt = (int)((n + kTRows - 1) / kTRows);
  // one PCG iteration; every argument is fixed, the iteration index lives on the device
  // profiling: a pair of events around each kernel product (eager launches only)
  std::vector<hipEvent_t> pev;
  const bool prof = profile && !use_graph;
  auto enqueue_iteration = [&](hipStream_t s2) -> laker_status {
    if (prof) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      LK_TRY(hipEventCreate(&e0));
      LK_TRY(hipEventCreate(&e1));
      pev.push_back(e0);
      pev.push_back(e1);
      LK_TRY(hipEventRecord(e0, s2));
      LK_TRY(kmv_run(prec, pb.dp, pl, Ak, s2));
      LK_TRY(hipEventRecord(e1, s2));
    } else {
      LK_TRY(kmv_run(prec, pb.dp, pl, Ak, s2));
    }
    pcg_ap_kernel<<<g, kThreads, 0, s2>>>(p, ws.part, pl.nsplit, Ap, n, pb.lambda, ws.papp, S);
    LK_CHECK_LAUNCH();
    if (P.kind == LAKER_PRECOND_JACOBI) {
      pcg_update_kernel<LAKER_PRECOND_JACOBI><<<g, kThreads, 0, s2>>>(alpha, r, p, Ap, dinv, th, n, S, ws.papp, g,
                                                                      ws.rrp, ws.rzp);
      LK_CHECK_LAUNCH();
      pcg_pupdate_kernel<LAKER_PRECOND_JACOBI><<<g, kThreads, 0, s2>>>(0, th, p, n, S, ws.rrp, g, ws.rzp, g);
    } else if (P.kind == LAKER_PRECOND_NONE) {
      pcg_update_kernel<LAKER_PRECOND_NONE><<<g, kThreads, 0, s2>>>(alpha, r, p, Ap, nullptr, th, n, S, ws.papp, g,
                                                                    ws.rrp, ws.rzp);
      LK_CHECK_LAUNCH();
      pcg_pupdate_kernel<LAKER_PRECOND_NONE><<<g, kThreads, 0, s2>>>(0, r, p, n, S, ws.rrp, g, ws.rzp, g);
    } else {
      if (P.f32)
        pcg_update_t_kernel<float><<<nbt, kThreads, 0, s2>>>(alpha, r, p, Ap, (const float*)P.B, P.nrp, n, S,
                                                             ws.papp, g, ws.rrp, ws.tpart);
      else
        pcg_update_t_kernel<double><<<nbt, kThreads, 0, s2>>>(alpha, r, p, Ap, (const double*)P.B, P.nrp, n, S,
                                                              ws.papp, g, ws.rrp, ws.tpart);
      LK_CHECK_LAUNCH();
      laker_status e = enqueue_lowrank_any(P, r, th, n, S, ws.rrp, nbt, ws.rzp, ws.tpart, ws.t, true, s2);
      if (e != LAKER_OK) return e;
      pcg_pupdate_kernel<LAKER_PRECOND_CCCP><<<g, kThreads, 0, s2>>>(0, th, p, n, S, ws.rrp, g, ws.rzp, ga);
    }
    LK_CHECK_LAUNCH();
    return LAKER_OK;
  };

  // The chunk of `check_every` iterations is captured once into a HIP graph
  // (on a capture stream of the library) and replayed on `st`: the launches
  // of a chunk then leave the host together.  Without graphs the kernels are
  // enqueued one by one.
  hipGraphExec_t gexec = nullptr;
  if (use_graph) {
    hipStream_t cs = capture_stream();
    hipGraph_t graph = nullptr;
    bool ok = cs != nullptr && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      laker_status e = LAKER_OK;
      for (int c = 0; c < check_every && e == LAKER_OK; ++c) e = enqueue_iteration(cs);
      ok = hipStreamEndCapture(cs, &graph) == hipSuccess && e == LAKER_OK;
      if (ok) ok = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) == hipSuccess;
      if (graph != nullptr) (void)hipGraphDestroy(graph);
    }
    if (!ok) {
      (void)hipGetLastError();
      if (gexec != nullptr) (void)hipGraphExecDestroy(gexec);
      return LAKER_EHIP;
    }
  }
  PcgScalars hs;
  int k = 0;
  laker_status loop_status = LAKER_OK;
  // Eager chunks shrink near convergence: the next chunk is the number of
  // iterations the residual decay of the last chunk predicts are still needed
  // (plus one), so few launches are enqueued past the converged iteration.
  int chunk = check_every;
  double last_rr = -1.0;
  int last_it = 0;
  for (;;) {
    if (gexec != nullptr) {
      if (hipGraphLaunch(gexec, st) != hipSuccess) {
        loop_status = LAKER_EHIP;
        break;
      }
      k += check_every;
    } else {
      for (int c = 0; c < chunk; ++c) {
        loop_status = enqueue_iteration(st);
        if (loop_status != LAKER_OK) break;
      }
      if (loop_status != LAKER_OK) break;
      k += chunk;
    }
    if (hipMemcpyAsync(&hs, S, sizeof(hs), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      loop_status = LAKER_EHIP;
      break;
    }
    if (hs.done || k >= max_iter + check_every) break;
    chunk = check_every;
    if (last_rr > 0.0 && hs.rr > 0.0 && hs.rr < last_rr && hs.iters > last_it && hs.tol2 > 0.0) {
      const double per_it = log(hs.rr / last_rr) / (double)(hs.iters - last_it);
      const double need = log(hs.tol2 / hs.rr) / per_it;
      if (need >= 0.0 && need < (double)check_every) chunk = (int)ceil(need) + 1;
      if (chunk < 1) chunk = 1;
      if (chunk > check_every) chunk = check_every;
    }
    last_rr = hs.rr;
    last_it = hs.iters;
  }
  if (gexec != nullptr) (void)hipGraphExecDestroy(gexec);
  if (prof) {
    // products of iterations that ran, and all launches (the ones enqueued after
    // convergence return at entry)
    double tot = 0.0, tot_all = 0.0;
    int cnt = 0, cnt_all = 0;
    for (size_t q = 0; q + 1 < pev.size(); q += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, pev[q], pev[q + 1]) != hipSuccess) continue;
      tot_all += ms;
      ++cnt_all;
      if ((int)(q / 2) < hs.iters) {
        tot += ms;
        ++cnt;
      }
    }
    for (hipEvent_t e : pev) (void)hipEventDestroy(e);
    if (stats != nullptr) {
      if (cnt > 0) {
        const double prev = stats->kmv_ms * stats->kmv_count;
        stats->kmv_count += cnt;
        stats->kmv_ms = (prev + tot) / stats->kmv_count;
      }
      if (cnt_all > 0) {
        const double prev = stats->kmv_launch_ms * stats->kmv_launches;
        stats->kmv_launches += cnt_all;
        stats->kmv_launch_ms = (prev + tot_all) / stats->kmv_launches;
      }
    }
  }
  if (loop_status != LAKER_OK) return loop_status;
  if (stats) {
    stats->iters += hs.iters;
    stats->relres = hs.yy > 0 ? sqrt(hs.rr / hs.yy) : 0.0;
  }
  if (hs.done == 2) return LAKER_EBREAKDOWN;
  if (hs.done == 1) return LAKER_OK;
  return LAKER_ENOCONV;
}

laker_status axpy_inplace(double* x, const double* d, int64_t n, hipStream_t st) {
  axpy_kernel<<<red_blocks(n), kThreads, 0, st>>>(x, d, n);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

laker_status apply_lowrank_once(const PrecondView& P, const double* r, double* theta, int64_t n, const SolveWs& ws,
                                hipStream_t st) {
  return enqueue_lowrank_any(P, r, theta, n, nullptr, nullptr, 0, nullptr, ws.tpart, ws.t, false, st);
}

}  // namespace lk
