// Preconditioned conjugate gradient on (lambda I + G) alpha = y (Sec. IV-E, Alg. 1).
//
// Every step runs on the device: the products A p, the inner products, the
// updates of alpha, r and p, the stopping test on the recursive residual and the
// preconditioner.  Scalars (delta, beta, ||r||^2, ...) live in device memory and
// each grid reduction is finished by the last block to arrive, in a fixed
// order.  The host enqueues `check_every` iterations at a time and then reads
// the `done` flag; kernels launched after convergence return at once.
#include "pcg.hpp"

namespace lk {

namespace {

constexpr int kThreads = 256;

inline int red_blocks(int64_t n) {
  int64_t g = (n + kThreads * 4 - 1) / (kThreads * 4);
  if (g > kMaxBlocks) g = kMaxBlocks;
  if (g < 1) g = 1;
  return (int)g;
}

// r = y - w (or r = y when w is null); S->yy = ||y||^2, S->rr = ||r||^2;
// resets the iteration state.
template <typename V>
__global__ __launch_bounds__(kThreads) void pcg_init_kernel(const double* __restrict__ y,
                                                            const V* __restrict__ w, V* __restrict__ r,
                                                            V* __restrict__ p, int64_t n, double tol,
                                                            int max_iter, PcgScalars* S,
                                                            double* __restrict__ bpart) {
  __shared__ double sh[16];
  double yy = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double yi = y[i];
    V ri = w != nullptr ? (V)(yi - (double)w[i]) : (V)yi;
    r[i] = ri;
    p[i] = V(0);
    yy += yi * yi;
    rr += (double)ri * (double)ri;
  }
  yy = block_sum(yy, sh);
  rr = block_sum(rr, sh);
  if (threadIdx.x == 0) {
    bpart[blockIdx.x] = yy;
    bpart[kMaxBlocks + blockIdx.x] = rr;
  }
  if (last_block_arrived(&S->cnt[0])) {
    double syy = ordered_sum(bpart, gridDim.x, sh);
    double srr = ordered_sum(bpart + kMaxBlocks, gridDim.x, sh);
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

// Ap = lambda p + sum of the column-split partials; p^T A p; delta = rz / pAp.
template <typename V>
__global__ __launch_bounds__(kThreads) void pcg_ap_kernel(const V* __restrict__ p, const V* __restrict__ part,
                                                          int nsplit, V* __restrict__ Ap, int64_t n, V lam,
                                                          PcgScalars* S, double* __restrict__ bpart) {
  if (S->done) return;
  __shared__ double sh[16];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    V s = V(0);
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * n + i];
    V pi = p[i];
    V a = fma(lam, pi, s);
    Ap[i] = a;
    acc += (double)pi * (double)a;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = acc;
  if (last_block_arrived(&S->cnt[1])) {
    double pap = ordered_sum(bpart, gridDim.x, sh);
    if (threadIdx.x == 0) {
      S->pap = pap;
      double dl = S->rz / pap;
      S->delta = dl;
      if (!(pap > 0.0) || !isfinite(dl)) S->done = 2;
      S->cnt[1] = 0;
    }
  }
}

// alpha += delta p; r -= delta Ap; ||r||^2; stopping test (Alg. 1: before the
// preconditioner is applied).  For P = I and Jacobi the preconditioned
// residual and r^T theta are formed here too and beta is set.
template <typename V, int KIND>
__global__ __launch_bounds__(kThreads) void pcg_update_kernel(double* __restrict__ alpha, V* __restrict__ r,
                                                              const V* __restrict__ p, const V* __restrict__ Ap,
                                                              const V* __restrict__ dinv, V* __restrict__ theta,
                                                              int64_t n, PcgScalars* S,
                                                              double* __restrict__ bpart) {
  if (S->done) return;
  __shared__ double sh[16];
  const double dl = S->delta;
  const V dv = (V)dl;
  double rr = 0.0, rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    V pi = p[i];
    alpha[i] += dl * (double)pi;
    V ri = fma(-dv, Ap[i], r[i]);
    r[i] = ri;
    rr += (double)ri * (double)ri;
    if (KIND == LAKER_PRECOND_JACOBI) {
      V ti = ri * dinv[i];
      theta[i] = ti;
      rz += (double)ri * (double)ti;
    }
  }
  rr = block_sum(rr, sh);
  if (KIND == LAKER_PRECOND_JACOBI) rz = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    bpart[blockIdx.x] = rr;
    bpart[kMaxBlocks + blockIdx.x] = rz;
  }
  if (last_block_arrived(&S->cnt[2])) {
    double srr = ordered_sum(bpart, gridDim.x, sh);
    double srz = KIND == LAKER_PRECOND_JACOBI ? ordered_sum(bpart + kMaxBlocks, gridDim.x, sh) : srr;
    if (threadIdx.x == 0) {
      S->rr = srr;
      int it = S->iters + 1;
      S->iters = it;
      if (!isfinite(srr)) S->done = 2;
      else if (srr <= S->tol2) S->done = 1;
      else if (it >= S->max_iter) S->done = 3;
      if (KIND != LAKER_PRECOND_CCCP && KIND != LAKER_PRECOND_LEARNED) {
        S->beta = srz / S->rz;
        S->rz = srz;
      }
      S->cnt[2] = 0;
    }
  }
}

// First half of the low-rank preconditioner: t = B^T r.  Blocks own
// contiguous row chunks; the last block adds the chunk partials in order.
template <typename V>
__global__ __launch_bounds__(kThreads) void lr_t_kernel(const V* __restrict__ B, const V* __restrict__ r,
                                                        int64_t n, int nr, int64_t rows_per_block,
                                                        double* __restrict__ tpart, double* __restrict__ t,
                                                        PcgScalars* S, unsigned* cnt) {
  if (S != nullptr && S->done) return;
  const int64_t i0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t i1 = i0 + rows_per_block < n ? i0 + rows_per_block : n;
  for (int k = threadIdx.x; k < nr; k += kThreads) {
    V acc = V(0);
    for (int64_t i = i0; i < i1; ++i) acc = fma(B[i * nr + k], r[i], acc);
    tpart[(int64_t)blockIdx.x * nr + k] = (double)acc;
  }
  if (last_block_arrived(cnt)) {
    for (int k = threadIdx.x; k < nr; k += kThreads) {
      double s = 0.0;
      for (unsigned b = 0; b < gridDim.x; ++b) s += __builtin_nontemporal_load(tpart + (int64_t)b * nr + k);
      t[k] = s;
    }
    if (threadIdx.x == 0) *cnt = 0;
  }
}

// Second half: theta = c0 r + Bt t, one wave per row; r^T theta and beta.
template <typename V>
__global__ __launch_bounds__(kThreads) void lr_apply_kernel(const V* __restrict__ Bt, const double* __restrict__ t,
                                                            const V* __restrict__ r, V* __restrict__ theta,
                                                            int64_t n, int nr, const double* __restrict__ c0p,
                                                            PcgScalars* S,
                                                            double* __restrict__ bpart, int set_beta) {
  if (S != nullptr && S->done) return;
  __shared__ double sh[16];
  __shared__ V ts[kMaxNr];
  const V c0 = (V)c0p[0];
  for (int k = threadIdx.x; k < nr; k += kThreads) ts[k] = (V)t[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int64_t wstride = (int64_t)gridDim.x * (kThreads / 64);
  double rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * (kThreads / 64) + wv; i < n; i += wstride) {
    V acc = V(0);
    const V* row = Bt + i * nr;
    for (int k = lane; k < nr; k += 64) acc = fma(row[k], ts[k], acc);
    acc = wave_sum(acc);
    if (lane == 0) {
      V ri = r[i];
      V th = fma(c0, ri, acc);
      theta[i] = th;
      rz += (double)ri * (double)th;
    }
  }
  rz = block_sum(rz, sh);
  if (S == nullptr) return;
  if (threadIdx.x == 0) bpart[blockIdx.x] = rz;
  if (last_block_arrived(&S->cnt[3])) {
    double srz = ordered_sum(bpart, gridDim.x, sh);
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
template <typename V>
__global__ __launch_bounds__(kThreads) void pcg_pupdate_kernel(const V* __restrict__ theta, V* __restrict__ p,
                                                               int64_t n, const PcgScalars* S) {
  if (S->done) return;
  const V b = (V)S->beta;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    p[i] = fma(b, p[i], theta[i]);
}

// Initial preconditioned residual when P = I or Jacobi: theta = P r, rz, beta.
template <typename V, int KIND>
__global__ __launch_bounds__(kThreads) void simple_precond_kernel(const V* __restrict__ r, const V* __restrict__ dinv,
                                                                  V* __restrict__ theta, int64_t n, PcgScalars* S,
                                                                  double* __restrict__ bpart) {
  if (S->done) return;
  __shared__ double sh[16];
  double rz = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    V ri = r[i];
    V ti = KIND == LAKER_PRECOND_JACOBI ? ri * dinv[i] : ri;
    theta[i] = ti;
    rz += (double)ri * (double)ti;
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = rz;
  if (last_block_arrived(&S->cnt[4])) {
    double srz = ordered_sum(bpart, gridDim.x, sh);
    if (threadIdx.x == 0) {
      S->beta = srz / S->rz;
      S->rz = srz;
      S->cnt[4] = 0;
    }
  }
}

// out = ||y - w||^2 / ||y||^2 components (float64), for the true residual.
__global__ __launch_bounds__(kThreads) void resid_kernel(const double* __restrict__ y, const double* __restrict__ w,
                                                         double* __restrict__ r, int64_t n,
                                                         double* __restrict__ bpart, unsigned* cnt,
                                                         double* out2) {
  __shared__ double sh[16];
  double rr = 0.0, yy = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    double yi = y[i];
    double ri = w != nullptr ? yi - w[i] : yi;
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
    double srr = ordered_sum(bpart, gridDim.x, sh);
    double syy = ordered_sum(bpart + kMaxBlocks, gridDim.x, sh);
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

template <typename V>
laker_status enqueue_precond(const PrecondView& P, const V* r, V* theta, int64_t n, PcgScalars* S,
                             double* bpart, double* tpart, double* t, hipStream_t st) {
  const int g = red_blocks(n);
  if (P.kind == LAKER_PRECOND_CCCP || P.kind == LAKER_PRECOND_LEARNED) {
    const V* B = (const V*)P.B;
    const V* Bt = (const V*)P.Bt;
    int64_t rpb = (n + 255) / 256;
    if (rpb < 32) rpb = 32;
    int gt = (int)((n + rpb - 1) / rpb);
    lr_t_kernel<V><<<gt, kThreads, 0, st>>>(B, r, n, P.nr, rpb, tpart, t, S, &S->cnt[5]);
    LK_CHECK_LAUNCH();
    lr_apply_kernel<V><<<g, kThreads, 0, st>>>(Bt, t, r, theta, n, P.nr, P.c0p, S, bpart, 1);
    LK_CHECK_LAUNCH();
  }
  return LAKER_OK;
}

}  // namespace

SolveWs plan_solve_ws(void* base, int64_t n, int d, int64_t m) {
  WsCarver c(base);
  SolveWs w;
  const int dp = pad_dim(d);
  const int64_t rows = n > m ? n : m;
  w.e64 = c.take<double>((size_t)n * dp);
  w.e32 = c.take<float>((size_t)n * dp);
  w.e16 = c.take<uint16_t>((size_t)n * dp);
  w.q64 = c.take<double>((size_t)(m > 0 ? m : 1) * dp);
  w.q32 = c.take<float>((size_t)(m > 0 ? m : 1) * dp);
  w.q16 = c.take<uint16_t>((size_t)(m > 0 ? m : 1) * dp);
  w.part = c.take<double>((size_t)64 * rows);
  w.r = c.take<double>(n);
  w.p = c.take<double>(n);
  w.ap = c.take<double>(n);
  w.theta = c.take<double>(n);
  w.vtmp = c.take<double>(rows);
  w.w64 = c.take<double>(rows);
  w.rout = c.take<double>(n);
  w.dalpha = c.take<double>(n);
  w.S = c.take<PcgScalars>(1);
  w.bpart = c.take<double>(2 * kMaxBlocks);
  w.tpart = c.take<double>((size_t)256 * kMaxNr);
  w.t = c.take<double>(kMaxNr);
  w.misc = c.take<double>(16);
  w.cnt = c.take<unsigned>(16);
  w.total = c.bytes();
  return w;
}

laker_status true_residual(const Problem& pb, const SolveWs& ws, const double* y, const double* alpha,
                           double* r_out, double* relres, bool have_alpha, hipStream_t st) {
  const int g = red_blocks(pb.n);
  const double* wv = nullptr;
  if (have_alpha) {
    KmvPlan pl = kmv_plan(pb.n, pb.n, LAKER_F64);
    LK_TRY(kmv_partials(LAKER_F64, pb.dp, ws.e64, pb.n, ws.e64, pb.n, alpha, ws.part, pl, nullptr, st));
    LK_TRY(kmv_finish(LAKER_F64, pb.n, pb.lambda, alpha, ws.part, pl.nsplit, ws.w64, true, st));
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

template <typename V>
static laker_status pcg_core(const Problem& pb, const SolveWs& ws, const PrecondView& P, const double* rhs,
                             double* alpha, bool warm, double tol, int max_iter, int check_every, int vprec,
                             laker_stats* stats, hipStream_t st) {
  const int64_t n = pb.n;
  const int g = red_blocks(n);
  V* r = (V*)ws.r;
  V* p = (V*)ws.p;
  V* Ap = (V*)ws.ap;
  V* th = (V*)ws.theta;
  V* part = (V*)ws.part;
  PcgScalars* S = ws.S;
  const void* eh = vprec == LAKER_F64 ? (const void*)ws.e64 : (vprec == LAKER_F32 ? (const void*)ws.e32 : (const void*)ws.e16);
  const int kprec = vprec;
  KmvPlan pl = kmv_plan(n, n, kprec);

  // r^0 = y - A alpha^0
  const V* wv = nullptr;
  if (warm) {
    V* av = (V*)ws.vtmp;
    LK_TRY(convert_vec(alpha, LAKER_F64, av, sizeof(V) == 8 ? LAKER_F64 : LAKER_F32, n, st));
    LK_TRY(kmv_partials(kprec, pb.dp, eh, n, eh, n, av, part, pl, nullptr, st));
    LK_TRY(kmv_finish(kprec, n, pb.lambda, av, part, pl.nsplit, Ap, false, st));
    wv = Ap;
  } else {
    LK_TRY(hipMemsetAsync(alpha, 0, sizeof(double) * n, st));
  }
  pcg_init_kernel<V><<<g, kThreads, 0, st>>>(rhs, wv, r, p, n, tol, max_iter, S, ws.bpart);
  LK_CHECK_LAUNCH();
  // theta^0 = P r^0, p^0 = theta^0
  const V* dinv = (const V*)P.dinv;
  if (P.kind == LAKER_PRECOND_JACOBI) {
    simple_precond_kernel<V, LAKER_PRECOND_JACOBI><<<g, kThreads, 0, st>>>(r, dinv, th, n, S, ws.bpart);
    LK_CHECK_LAUNCH();
  } else if (P.kind == LAKER_PRECOND_NONE) {
    simple_precond_kernel<V, LAKER_PRECOND_NONE><<<g, kThreads, 0, st>>>(r, nullptr, th, n, S, ws.bpart);
    LK_CHECK_LAUNCH();
  } else {
    laker_status e = enqueue_precond<V>(P, r, th, n, S, ws.bpart, ws.tpart, ws.t, st);
    if (e != LAKER_OK) return e;
  }
  pcg_pupdate_kernel<V><<<g, kThreads, 0, st>>>(th, p, n, S);
  LK_CHECK_LAUNCH();

  PcgScalars hs;
  int enq = 0;
  for (;;) {
    for (int k = 0; k < check_every; ++k) {
      LK_TRY(kmv_partials(kprec, pb.dp, eh, n, eh, n, p, part, pl, &S->done, st));
      pcg_ap_kernel<V><<<g, kThreads, 0, st>>>(p, part, pl.nsplit, Ap, n, (V)pb.lambda, S, ws.bpart);
      LK_CHECK_LAUNCH();
      if (P.kind == LAKER_PRECOND_JACOBI) {
        pcg_update_kernel<V, LAKER_PRECOND_JACOBI><<<g, kThreads, 0, st>>>(alpha, r, p, Ap, dinv, th, n, S, ws.bpart);
        LK_CHECK_LAUNCH();
        pcg_pupdate_kernel<V><<<g, kThreads, 0, st>>>(th, p, n, S);
      } else if (P.kind == LAKER_PRECOND_NONE) {
        pcg_update_kernel<V, LAKER_PRECOND_NONE><<<g, kThreads, 0, st>>>(alpha, r, p, Ap, nullptr, th, n, S, ws.bpart);
        LK_CHECK_LAUNCH();
        pcg_pupdate_kernel<V><<<g, kThreads, 0, st>>>(r, p, n, S);
      } else {
        pcg_update_kernel<V, LAKER_PRECOND_CCCP><<<g, kThreads, 0, st>>>(alpha, r, p, Ap, nullptr, th, n, S, ws.bpart);
        LK_CHECK_LAUNCH();
        laker_status e = enqueue_precond<V>(P, r, th, n, S, ws.bpart, ws.tpart, ws.t, st);
        if (e != LAKER_OK) return e;
        pcg_pupdate_kernel<V><<<g, kThreads, 0, st>>>(th, p, n, S);
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

laker_status pcg_run(const Problem& pb, const SolveWs& ws, const PrecondView& P, const double* rhs, double* alpha,
                     bool warm, double tol, int max_iter, int check_every, int prec, laker_stats* stats,
                     hipStream_t st) {
  if (prec == LAKER_F64)
    return pcg_core<double>(pb, ws, P, rhs, alpha, warm, tol, max_iter, check_every, prec, stats, st);
  return pcg_core<float>(pb, ws, P, rhs, alpha, warm, tol, max_iter, check_every, prec, stats, st);
}

laker_status axpy_inplace(double* x, const double* d, int64_t n, hipStream_t st) {
  axpy_kernel<<<red_blocks(n), kThreads, 0, st>>>(x, d, n);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

laker_status apply_lowrank_once(const PrecondView& P, const double* r, double* theta, int64_t n,
                                const SolveWs& ws, hipStream_t st) {
  int64_t rpb = (n + 255) / 256;
  if (rpb < 32) rpb = 32;
  int gt = (int)((n + rpb - 1) / rpb);
  lr_t_kernel<double><<<gt, kThreads, 0, st>>>((const double*)P.B, r, n, P.nr, rpb, ws.tpart, ws.t, nullptr, ws.cnt + 1);
  LK_CHECK_LAUNCH();
  lr_apply_kernel<double><<<red_blocks(n), kThreads, 0, st>>>((const double*)P.Bt, ws.t, r, theta, n, P.nr, P.c0p,
                                                              nullptr, ws.bpart, 0);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

}  // namespace lk
