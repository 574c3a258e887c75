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
#include "pcg.hpp"

namespace lk {

namespace {

constexpr int kThreads = 256;

inline int red_blocks(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  if (g > kMaxBlocks) g = kMaxBlocks;
  if (g < 1) g = 1;
  return (int)g;
}

// one wave per row, up to 1024 blocks of four waves
inline int apply_blocks(int64_t n) {
  int64_t g = (n + 3) / 4;
  if (g > kMaxBlocks) g = kMaxBlocks;
  return (int)(g < 1 ? 1 : g);
}

// r = y - w (or r = y when w is null); S->yy = ||y||^2, S->rr = ||r||^2;
// resets the iteration state; p = 0.
__global__ __launch_bounds__(kThreads) void pcg_init_kernel(const double* __restrict__ y, const double* __restrict__ w,
                                                            double* __restrict__ r, double* __restrict__ p, int64_t n,
                                                            double tol, int max_iter, PcgScalars* S,
                                                            double* __restrict__ bpart) {
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
    bpart[blockIdx.x] = yy;
    bpart[kMaxBlocks + blockIdx.x] = rr;
  }
  if (last_block_arrived(&S->cnt[0])) {
    const double syy = ordered_sum(bpart, gridDim.x, sh);
    const double srr = ordered_sum(bpart + kMaxBlocks, gridDim.x, sh);
    if (threadIdx.x == 0) {
      S->yy = syy;
      S->rr = srr;
      S->tol2 = tol * tol * syy;
      S->iters = 0;
      S->max_iter = max_iter;
      S->rz = 1.0;     // so that the first preconditioner pass sets p = theta
      S->beta = 0.0;
      S->done = (srr <= tol * tol * syy) ? 1 : (syy == 0.0 ? 1 : 0);
      S->cnt[0] = 0;
    }
  }
}

// alpha += delta p; r -= delta Ap; ||r||^2; stopping test (Alg. 1: before the
// preconditioner is applied).  For P = I and Jacobi the preconditioned
// residual and r^T theta are formed here too and beta is set.
template <int KIND>
__global__ __launch_bounds__(kThreads) void pcg_update_kernel(double* __restrict__ alpha, double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ Ap,
                                                              const double* __restrict__ dinv,
                                                              double* __restrict__ theta, int64_t n, PcgScalars* S,
                                                              double* __restrict__ bpart) {
  if (S->done) return;
  __shared__ double sh[16];
  const double dl = S->delta;
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
    bpart[blockIdx.x] = rr;
    bpart[kMaxBlocks + blockIdx.x] = rz;
  }
  if (last_block_arrived(&S->cnt[2])) {
    const double srr = ordered_sum(bpart, gridDim.x, sh);
    const double srz = KIND == LAKER_PRECOND_JACOBI ? ordered_sum(bpart + kMaxBlocks, gridDim.x, sh) : srr;
    if (threadIdx.x == 0) {
      S->rr = srr;
      const int it = S->iters + 1;
      S->iters = it;
      if (!isfinite(srr)) S->done = 2;
      else if (srr <= S->tol2) S->done = 1;
      else if (it >= S->max_iter) S->done = 3;
      if (KIND == LAKER_PRECOND_NONE || KIND == LAKER_PRECOND_JACOBI) {
        S->beta = srz / S->rz;
        S->rz = srz;
      }
      S->cnt[2] = 0;
    }
  }
}

// First half of the low-rank preconditioner: t = B^T r.  Block b sums rows
// [32 b, 32 b + 32): each wave takes every fourth row, each lane the columns
// k = lane + 64 c; the four waves are combined in LDS and written as one
// float64 partial row.  A second kernel adds the block partials in order.
// MT is the storage type of B (float64, or float32 for the reduced-precision
// solves); products are accumulated in float64.
constexpr int kTRows = 32;

template <typename MT>
__global__ __launch_bounds__(kThreads) void lr_t_partial_kernel(const MT* __restrict__ B, const double* __restrict__ r,
                                                                int64_t n, int nr, double* __restrict__ tpart,
                                                                const PcgScalars* S) {
  if (S != nullptr && S->done) return;
  constexpr int MAXC = kMaxNr / 64;
  __shared__ double red[4][kMaxNr];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t i0 = (int64_t)blockIdx.x * kTRows;
  double acc[MAXC];
#pragma unroll
  for (int c = 0; c < MAXC; ++c) acc[c] = 0.0;
  for (int rr = wv; rr < kTRows; rr += 4) {
    const int64_t i = i0 + rr;
    if (i >= n) break;
    const double ri = r[i];
    const MT* row = B + i * nr;
#pragma unroll
    for (int c = 0; c < MAXC; ++c) {
      const int k = lane + 64 * c;
      if (k < nr) acc[c] = fma((double)row[k], ri, acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < MAXC; ++c) {
    const int k = lane + 64 * c;
    if (k < nr) red[wv][k] = acc[c];
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nr; k += kThreads)
    tpart[(int64_t)blockIdx.x * nr + k] = (red[0][k] + red[1][k]) + (red[2][k] + red[3][k]);
}

// t[k] = sum_b tpart[b][k] in a fixed order: block handles 64 columns, the four
// waves take every fourth partial row, then combine in LDS.
__global__ __launch_bounds__(kThreads) void lr_t_finish_kernel(const double* __restrict__ tpart, int nb, int nr,
                                                               double* __restrict__ t, const PcgScalars* S) {
  if (S != nullptr && S->done) return;
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  double s = 0.0;
  if (k < nr)
    for (int b = wv; b < nb; b += 4) s += tpart[(int64_t)b * nr + k];
  red[wv][lane] = s;
  __syncthreads();
  if (wv == 0 && k < nr) t[k] = (red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane]);
}

// Second half: theta = c0 r + Bt t, one wave per row; r^T theta and beta.
template <typename MT>
__global__ __launch_bounds__(kThreads) void lr_apply_kernel(const MT* __restrict__ Bt, const double* __restrict__ t,
                                                            const double* __restrict__ r, double* __restrict__ theta,
                                                            int64_t n, int nr, const double* __restrict__ c0p,
                                                            PcgScalars* S, double* __restrict__ bpart, int set_beta) {
  if (S != nullptr && S->done) return;
  __shared__ double sh[16];
  __shared__ double ts[kMaxNr];
  const double c0 = c0p[0];
  for (int k = threadIdx.x; k < nr; k += kThreads) ts[k] = t[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t wstride = (int64_t)gridDim.x * (kThreads / 64);
  double rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + wv; i < n; i += wstride) {
    double acc = 0.0;
    const MT* row = Bt + i * nr;
    for (int k = lane; k < nr; k += 64) acc = fma((double)row[k], ts[k], acc);
    acc = wave_sum(acc);
    if (lane == 0) {
      const double ri = r[i];
      const double th = fma(c0, ri, acc);
      theta[i] = th;
      rz += ri * th;
    }
  }
  rz = block_sum(rz, sh);
  if (S == nullptr) return;
  if (threadIdx.x == 0) bpart[blockIdx.x] = rz;
  if (last_block_arrived(&S->cnt[3])) {
    const double srz = ordered_sum(bpart, gridDim.x, sh);
    if (threadIdx.x == 0) {
      if (set_beta) {
        S->beta = srz / S->rz;
        S->rz = srz;
      }
      S->cnt[3] = 0;
    }
  }
}

// p = theta + beta p
__global__ __launch_bounds__(kThreads) void pcg_pupdate_kernel(const double* __restrict__ theta, double* __restrict__ p,
                                                               int64_t n, const PcgScalars* S) {
  if (S->done) return;
  const double b = S->beta;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    p[i] = fma(b, p[i], theta[i]);
}

// Initial preconditioned residual when P = I or Jacobi: theta = P r, rz, beta.
template <int KIND>
__global__ __launch_bounds__(kThreads) void simple_precond_kernel(const double* __restrict__ r,
                                                                  const double* __restrict__ dinv,
                                                                  double* __restrict__ theta, int64_t n,
                                                                  PcgScalars* S, double* __restrict__ bpart) {
  if (S->done) return;
  __shared__ double sh[16];
  double rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double ri = r[i];
    const double ti = KIND == LAKER_PRECOND_JACOBI ? ri * dinv[i] : ri;
    theta[i] = ti;
    rz += ri * ti;
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = rz;
  if (last_block_arrived(&S->cnt[4])) {
    const double srz = ordered_sum(bpart, gridDim.x, sh);
    if (threadIdx.x == 0) {
      S->beta = srz / S->rz;
      S->rz = srz;
      S->cnt[4] = 0;
    }
  }
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

template <typename MT>
laker_status enqueue_lowrank(const PrecondView& P, const double* r, double* theta, int64_t n, PcgScalars* S,
                             double* bpart, double* tpart, double* t, int set_beta, hipStream_t st) {
  const int nb = (int)((n + kTRows - 1) / kTRows);
  lr_t_partial_kernel<MT><<<nb, kThreads, 0, st>>>((const MT*)P.B, r, n, P.nr, tpart, S);
  LK_CHECK_LAUNCH();
  lr_t_finish_kernel<<<(P.nr + 63) / 64, kThreads, 0, st>>>(tpart, nb, P.nr, t, S);
  LK_CHECK_LAUNCH();
  lr_apply_kernel<MT><<<apply_blocks(n), kThreads, 0, st>>>((const MT*)P.Bt, t, r, theta, n, P.nr, P.c0p, S, bpart,
                                                            set_beta);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

laker_status enqueue_precond(const PrecondView& P, const double* r, double* theta, int64_t n, PcgScalars* S,
                             const SolveWs& ws, hipStream_t st) {
  if (P.f32) return enqueue_lowrank<float>(P, r, theta, n, S, ws.bpart, ws.tpart, ws.t, 1, st);
  return enqueue_lowrank<double>(P, r, theta, n, S, ws.bpart, ws.tpart, ws.t, 1, st);
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
  w.rb_cnt = c.take<unsigned>((size_t)(rows + 63) / 64 + 1);
  w.rbpart = c.take<double>((size_t)(rows + 63) / 64 + 1);
  w.r = c.take<double>(n);
  w.p = c.take<double>(n);
  w.ap = c.take<double>(n);
  w.theta = c.take<double>(n);
  w.w64 = c.take<double>(rows);
  w.rout = c.take<double>(n);
  w.dalpha = c.take<double>(n);
  w.S = c.take<PcgScalars>(1);
  w.bpart = c.take<double>(2 * kMaxBlocks);
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
  A.rb_cnt = ws.rb_cnt;
  A.rbpart = ws.rbpart;
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
                     bool warm, double tol, int max_iter, int check_every, int prec, laker_stats* stats,
                     hipStream_t st) {
  const int64_t n = pb.n;
  const int g = red_blocks(n);
  double* r = ws.r;
  double* p = ws.p;
  double* Ap = ws.ap;
  double* th = ws.theta;
  PcgScalars* S = ws.S;
  const void* eh = prepared(ws, prec);
  const KmvPlan pl = kmv_plan(n, n, prec);

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
  pcg_init_kernel<<<g, kThreads, 0, st>>>(rhs, wv, r, p, n, tol, max_iter, S, ws.bpart);
  LK_CHECK_LAUNCH();
  // theta^0 = P r^0, p^0 = theta^0
  const double* dinv = (const double*)P.dinv;
  if (P.kind == LAKER_PRECOND_JACOBI) {
    simple_precond_kernel<LAKER_PRECOND_JACOBI><<<g, kThreads, 0, st>>>(r, dinv, th, n, S, ws.bpart);
    LK_CHECK_LAUNCH();
  } else if (P.kind == LAKER_PRECOND_NONE) {
    simple_precond_kernel<LAKER_PRECOND_NONE><<<g, kThreads, 0, st>>>(r, nullptr, th, n, S, ws.bpart);
    LK_CHECK_LAUNCH();
  } else {
    laker_status e = enqueue_precond(P, r, th, n, S, ws, st);
    if (e != LAKER_OK) return e;
  }
  pcg_pupdate_kernel<<<g, kThreads, 0, st>>>(th, p, n, S);
  LK_CHECK_LAUNCH();

  // A p, p^T A p and the step size in one launch
  KmvArgs Ak = kmv_args(eh, n, eh, n, p, ws);
  Ak.mode = 2;
  Ak.lam = pb.lambda;
  Ak.pself = p;
  Ak.out = Ap;
  Ak.S = S;
  PcgScalars hs;
  int enq = 0;
  for (;;) {
    for (int k = 0; k < check_every; ++k) {
      LK_TRY(kmv_run(prec, pb.dp, pl, Ak, st));
      if (P.kind == LAKER_PRECOND_JACOBI) {
        pcg_update_kernel<LAKER_PRECOND_JACOBI><<<g, kThreads, 0, st>>>(alpha, r, p, Ap, dinv, th, n, S, ws.bpart);
        LK_CHECK_LAUNCH();
        pcg_pupdate_kernel<<<g, kThreads, 0, st>>>(th, p, n, S);
      } else if (P.kind == LAKER_PRECOND_NONE) {
        pcg_update_kernel<LAKER_PRECOND_NONE><<<g, kThreads, 0, st>>>(alpha, r, p, Ap, nullptr, th, n, S, ws.bpart);
        LK_CHECK_LAUNCH();
        pcg_pupdate_kernel<<<g, kThreads, 0, st>>>(r, p, n, S);
      } else {
        pcg_update_kernel<LAKER_PRECOND_CCCP><<<g, kThreads, 0, st>>>(alpha, r, p, Ap, nullptr, th, n, S, ws.bpart);
        LK_CHECK_LAUNCH();
        laker_status e = enqueue_precond(P, r, th, n, S, ws, st);
        if (e != LAKER_OK) return e;
        pcg_pupdate_kernel<<<g, kThreads, 0, st>>>(th, p, n, S);
      }
      LK_CHECK_LAUNCH();
    }
    enq += check_every;
    LK_TRY(hipMemcpyAsync(&hs, S, sizeof(hs), hipMemcpyDeviceToHost, st));
    LK_TRY(hipStreamSynchronize(st));
    if (hs.done || enq >= max_iter + check_every) break;
  }
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
  if (P.f32) return enqueue_lowrank<float>(P, r, theta, n, nullptr, ws.bpart, ws.tpart, ws.t, 0, st);
  return enqueue_lowrank<double>(P, r, theta, n, nullptr, ws.bpart, ws.tpart, ws.t, 0, st);
}

}  // namespace lk
