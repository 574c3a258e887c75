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
#include "pcg_body.hpp"

namespace lk {

namespace {

using pcgk::kThreads;
using pcgk::kTRows;

// A non-blocking stream per device on which PCG chunks are captured into graphs
// (capture needs a stream other than the null stream; the graphs are launched on
// the caller's stream).
hipStream_t capture_stream_impl() {
  static hipStream_t streams[64] = {};
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (streams[dev] == nullptr && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

using namespace pcgk;

__global__ __launch_bounds__(kThreads) void pcg_init_kernel(const double* __restrict__ y, const double* __restrict__ w,
                                                            double* __restrict__ r, double* __restrict__ p, int64_t n,
                                                            double* __restrict__ yyp, double* __restrict__ rrp) {
  pcg_init_body(blockIdx.x, gridDim.x, y, w, r, p, n, yyp, rrp);
}

__global__ __launch_bounds__(kThreads) void pcg_start_kernel(PcgScalars* S, const double* __restrict__ yyp,
                                                             const double* __restrict__ rrp, int g, double tol,
                                                             int max_iter) {
  pcg_start_body(blockIdx.x, gridDim.x, S, yyp, rrp, g, tol, max_iter);
}

__global__ __launch_bounds__(kThreads) void pcg_ap_kernel(const double* __restrict__ p, const double* __restrict__ part,
                                                          PartSum ps, double* __restrict__ Ap, int64_t n, double lam,
                                                          double* __restrict__ pap_p, const PcgScalars* S) {
  pcg_ap_body(blockIdx.x, gridDim.x, p, part, ps, Ap, n, lam, pap_p, S);
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void pcg_update_kernel(double* __restrict__ alpha, double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ Ap,
                                                              const double* __restrict__ part, PartSum ps, double lam,
                                                              const double* __restrict__ dinv,
                                                              double* __restrict__ theta, int64_t n, PcgScalars* S,
                                                              const double* __restrict__ pap_p, int gp,
                                                              double* __restrict__ rrp, double* __restrict__ rzp) {
  pcg_update_body<KIND>(blockIdx.x, gridDim.x, alpha, r, p, Ap, part, ps, lam, dinv, theta, n, S, pap_p, gp, rrp,
                        rzp);
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void pcg_pupdate_kernel(int init, const double* __restrict__ theta,
                                                               double* __restrict__ p, int64_t n, PcgScalars* S,
                                                               const double* __restrict__ rrp, int grr,
                                                               const double* __restrict__ rzp, int grz) {
  pcg_pupdate_body<KIND>(blockIdx.x, gridDim.x, init, theta, p, n, S, rrp, grr, rzp, grz);
}

__global__ __launch_bounds__(kThreads) void jacobi_apply_kernel(const double* __restrict__ r,
                                                                const double* __restrict__ dinv,
                                                                double* __restrict__ theta, int64_t n,
                                                                const PcgScalars* S, double* __restrict__ rzp) {
  jacobi_apply_body(blockIdx.x, gridDim.x, r, dinv, theta, n, S, rzp);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void lr_t_partial_kernel(const MT* __restrict__ B, const double* __restrict__ r,
                                                                int64_t n, int nrp, double* __restrict__ tpart,
                                                                const PcgScalars* S) {
  lr_t_partial_body<MT>(blockIdx.x, gridDim.x, B, r, n, nrp, tpart, S);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void pcg_update_t_kernel(double* __restrict__ alpha,
                                                                double* __restrict__ r, double* __restrict__ p,
                                                                const double* __restrict__ theta,
                                                                const double* __restrict__ Ap,
                                                                const double* __restrict__ part, PartSum ps,
                                                                double lam,
                                                                const MT* __restrict__ B, int nrp, int64_t n,
                                                                PcgScalars* S, const double* __restrict__ pap_p,
                                                                int gp, double* __restrict__ rrp,
                                                                double* __restrict__ tpart) {
  pcg_update_t_body<MT>(blockIdx.x, gridDim.x, alpha, r, p, theta, Ap, part, ps, lam, B, nrp, n, S, pap_p, gp, rrp,
                        tpart);
}

__global__ __launch_bounds__(kThreads) void lr_t_finish_kernel(const double* __restrict__ tpart, int nb, int nrp,
                                                               double* __restrict__ t, PcgScalars* S,
                                                               const double* __restrict__ rrp, int grr) {
  lr_t_finish_body(blockIdx.x, gridDim.x, tpart, nb, nrp, t, S, rrp, grr);
}

template <typename MT, int MAXR>
__global__ __launch_bounds__(kThreads) void lr_apply_kernel(const MT* __restrict__ Bt, const double* __restrict__ t,
                                                            const double* __restrict__ r, double* __restrict__ theta,
                                                            int64_t n, int nrp, const double* __restrict__ c0p,
                                                            const double* __restrict__ dinv, const PcgScalars* S,
                                                            double* __restrict__ rzp) {
  lr_apply_body<MT, MAXR>(blockIdx.x, gridDim.x, Bt, t, r, theta, n, nrp, c0p, dinv, S, rzp);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void lr_apply_t_kernel(const double* __restrict__ tpart, int nb,
                                                              const MT* __restrict__ Bt, const double* __restrict__ r,
                                                              double* __restrict__ theta, int64_t n, int nrp,
                                                              const double* __restrict__ c0p,
                                                              const double* __restrict__ dinv, PcgScalars* S,
                                                              const double* __restrict__ rrp, int grr,
                                                              double* __restrict__ rzp) {
  lr_apply_t_body<MT>(blockIdx.x, tpart, nb, Bt, r, theta, n, nrp, c0p, dinv, S, rrp, grr, rzp);
}

__global__ __launch_bounds__(kThreads) void resid_kernel(const double* __restrict__ y, const double* __restrict__ w,
                                                         double* __restrict__ r, int64_t n,
                                                         double* __restrict__ bpart, unsigned* cnt, double* out2) {
  resid_body(blockIdx.x, gridDim.x, y, w, r, n, bpart, cnt, out2);
}

__global__ void axpy_kernel(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
  axpy_body(blockIdx.x, gridDim.x, x, d, n);
}

// After iteration k (k = kcur - 1): its step size and the conjugation
// coefficient the run state holds.  Launches after the run has stopped see the
// same k and rewrite the same values.
__global__ void lanczos_record_kernel(const PcgScalars* S, double* __restrict__ coef, int cap) {
  if (threadIdx.x != 0) return;
  const int k = S->kcur - 1;
  if (k < 0 || k >= cap || S->done == 2) return;
  coef[2 * k] = S->delta;
  coef[2 * k + 1] = S->beta;
}

// Lanczos tridiagonal of m CG steps with step sizes a_k and conjugation
// coefficients b_k (p_{k+1} = z_{k+1} + b_k p_k):
//   T_00 = 1 / a_0,  T_kk = 1 / a_k + b_{k-1} / a_{k-1},  T_{k-1,k} = sqrt(b_{k-1}) / a_{k-1}.
// Its eigenvalues are the Ritz values of P A on the Krylov space.  With the
// conjugation done inside the next product (shifted = 1) the coefficient
// recorded after iteration k is b_{k-1}; otherwise it is b_k.
__device__ __forceinline__ void tri_entry(const double* coef, int k, int shifted, double& diag, double& off2) {
  const double ak = coef[2 * k];
  diag = 1.0 / ak;
  off2 = 0.0;
  if (k > 0) {
    const double am = coef[2 * (k - 1)];
    const double bm = shifted ? coef[2 * k + 1] : coef[2 * (k - 1) + 1];
    diag += bm / am;
    off2 = bm / (am * am);
  }
}

// Number of eigenvalues of T below x (Sturm sequence of the LDL^T pivots).
__device__ int tri_count_below(const double* coef, int m, int shifted, double x) {
  int c = 0;
  double dprev = 1.0;
  for (int k = 0; k < m; ++k) {
    double dk, e2;
    tri_entry(coef, k, shifted, dk, e2);
    double d = dk - x - (k > 0 ? e2 / dprev : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0.0) ++c;
    dprev = d;
  }
  return c;
}

// out[0] = smallest, out[1] = largest eigenvalue of T, by bisection inside the
// Gershgorin interval (thread 0: the smallest, thread 1: the largest).
__global__ void tridiag_extremes_kernel(const double* __restrict__ coef, int m, int shifted,
                                        double* __restrict__ out) {
  const int t = threadIdx.x;
  if (t > 1) return;
  double lo = 0.0, hi = 0.0;
  for (int k = 0; k < m; ++k) {
    double dk, e2;
    tri_entry(coef, k, shifted, dk, e2);
    const double el = k > 0 ? sqrt(e2) : 0.0;
    double er = 0.0;
    if (k + 1 < m) {
      double dn, en2;
      tri_entry(coef, k + 1, shifted, dn, en2);
      er = sqrt(en2);
    }
    const double a = dk - el - er, b = dk + el + er;
    if (k == 0 || a < lo) lo = a;
    if (k == 0 || b > hi) hi = b;
  }
  if (lo < 0.0) lo = 0.0;
  // smallest: the least x with count(x) >= 1; largest: the least x with count(x) >= m
  const int target = t == 0 ? 1 : m;
  double a = lo, b = hi * (1.0 + 1e-12) + 1e-300;
  for (int it = 0; it < 200 && b - a > 1e-15 * fabs(b); ++it) {
    const double mid = 0.5 * (a + b);
    if (tri_count_below(coef, m, shifted, mid) >= target) b = mid;
    else a = mid;
  }
  out[t] = 0.5 * (a + b);
}

// theta = P r for the low-rank preconditioner (t partials, t, theta: three
// passes, or two when the apply finishes t itself, lr_fused_t); with rrp set
// the pass that finishes t first takes the stopping decision of iteration k,
// and the first pass is skipped when `skip_partial` says the fused update
// already wrote the t partials.
template <typename MT>
laker_status enqueue_lowrank(const PrecondView& P, const double* r, double* theta, int64_t n, PcgScalars* S,
                             const double* rrp, int grr, double* rzp, double* tpart, double* t, bool skip_partial,
                             hipStream_t st) {
  const int nb = (int)((n + kTRows - 1) / kTRows);
  if (!skip_partial) {
    lr_t_partial_kernel<MT><<<nb, kThreads, 0, st>>>((const MT*)P.B, r, n, P.nrp, tpart, S);
    LK_CHECK_LAUNCH();
  }
  if (lr_fused_t(n, P.nrp)) {
    // t finished inside the apply (nb blocks of 64 rows; r^T theta partials: nb)
    lr_apply_t_kernel<MT><<<nb, kThreads, 0, st>>>(tpart, nb, (const MT*)P.Bt, r, theta, n, P.nrp, P.c0p,
                                                   (const double*)P.dinv, S, rrp, grr, rzp);
    LK_CHECK_LAUNCH();
    return LAKER_OK;
  }
  lr_t_finish_kernel<<<(P.nrp + 15) / 16, kThreads, 0, st>>>(tpart, nb, P.nrp, t, S, rrp, grr);
  LK_CHECK_LAUNCH();
  // (ranks up to 64, the learned preconditioner's, keep more rows in flight)
  if (P.nrp <= 64)
    lr_apply_kernel<MT, 64><<<(unsigned)apply_blocks(n), kThreads, 0, st>>>((const MT*)P.Bt, t, r, theta, n, P.nrp,
                                                                            P.c0p, (const double*)P.dinv, S, rzp);
  else
    lr_apply_kernel<MT, kMaxNr><<<(unsigned)apply_blocks(n), kThreads, 0, st>>>((const MT*)P.Bt, t, r, theta, n,
                                                                                P.nrp, P.c0p, (const double*)P.dinv,
                                                                                S, rzp);
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
  SolveWs w{};
  const int dp = pad_dim(d);
  const int64_t rows = n > m ? n : m;
  const int64_t mq = m > 0 ? m : 1;
  w.e64 = c.take<double>((size_t)n * dp);
  w.e32 = c.take<float>((size_t)n * dp);
  w.e16 = c.take<uint16_t>((size_t)n * dp);
  w.q64 = c.take<double>((size_t)mq * dp);
  w.q32 = c.take<float>((size_t)mq * dp);
  w.q16 = c.take<uint16_t>((size_t)mq * dp);
  w.part = c.take<double>(kmv_part_elems(m, n));
  w.r = c.take<double>(n);
  w.p = c.take<double>(n);
  w.ap = c.take<double>(n);
  w.theta = c.take<double>(n);
  w.w64 = c.take<double>(rows);
  w.rout = c.take<double>(n);
  w.dalpha = c.take<double>(n);
  w.fp = c.take<double>(n);
  w.fq = c.take<double>(n);
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
  w.fring = c.take<double>(2 * (size_t)kFcgHist * (size_t)n);
  w.fpq = c.take<double>(kFcgHist);
  w.fdz = c.take<double>(kFcgHist);
  w.fpart = c.take<double>((size_t)kFcgHist * kMaxBlocks);
  w.lcoef = c.take<double>(2 * (size_t)kLanczosCap);
  w.lout = c.take<double>(4);
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
  // square products of the solve stream the stored G when there is one
  if (Q == K && m == n) {
    if (Q == ws.e64) A.kmat = ws.kmat64;
    else if (Q == ws.e32) A.kmat = ws.kmat32;
  }
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
    KmvPlan pl = kmv_plan_square(pb.n, pb.dp, LAKER_F64);
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
                     laker_stats* stats, hipStream_t st, bool defer, int stall_window, bool lanczos) {
  const int64_t n = pb.n;
  const int g = red_blocks(n);
  const bool lowrank0 = P.kind == LAKER_PRECOND_CCCP || P.kind == LAKER_PRECOND_LEARNED;
  // partials of r^T theta: one per block of the preconditioner apply
  const int ga = lowrank0 && lr_fused_t(n, P.nrp) ? (int)((n + kTRows - 1) / kTRows) : apply_blocks(n);
  double* r = ws.r;
  double* p = ws.p;
  double* Ap = ws.ap;
  double* th = ws.theta;
  PcgScalars* S = ws.S;
  const void* eh = prepared(ws, prec);
  const KmvPlan pl = kmv_plan_square(n, pb.dp, prec);
  const bool lowrank = P.kind == LAKER_PRECOND_CCCP || P.kind == LAKER_PRECOND_LEARNED;
  // symmetric product with a low-rank preconditioner: the product kernel
  // conjugates the direction itself (p = theta + beta p) and the step update
  // stores it, so the iteration has no separate direction pass
  const bool stored = kmv_args(eh, n, eh, n, p, ws).kmat != nullptr;
  const bool fold = pl.sym && !stored;
  const bool fused = lowrank && fold;
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
    // (conjugated: p^0 = theta^0 + 0 p with p = 0 from the start pass)
    if (!fused) pcg_pupdate_kernel<LAKER_PRECOND_CCCP><<<g, kThreads, 0, st>>>(1, th, p, n, S, ws.rrp, g, ws.rzp, ga);
  }
  LK_CHECK_LAUNCH();

  KmvArgs Ak = kmv_args(eh, n, eh, n, p, ws);
  Ak.mode = 0;
  Ak.S = S;
  Ak.pcg_step = 1;
  // a symmetric product forms p^T A p itself and the step update adds each
  // row's partials (no separate pass for A p); else (also for a product
  // that streams the stored G) a pass finishes A p and its p^T A p partials
  const PartSum ps = part_sum(pl);
  const double* Apu = fold ? nullptr : Ap;
  const int gp = fold ? pl.sp.grid : g;
  if (fold) {
    Ak.pap = ws.papp;
    Ak.lam = pb.lambda;
  }
  if (fused) {
    Ak.theta = th;
    Ak.rzp = ws.rzp;
    Ak.grz = ga;
  }
  const double* thu = fused ? th : nullptr;
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
    if (!fold) {
      pcg_ap_kernel<<<g, kThreads, 0, s2>>>(p, ws.part, ps, Ap, n, pb.lambda, ws.papp, S);
      LK_CHECK_LAUNCH();
    }
    if (P.kind == LAKER_PRECOND_JACOBI) {
      pcg_update_kernel<LAKER_PRECOND_JACOBI><<<g, kThreads, 0, s2>>>(alpha, r, p, Apu, ws.part, ps, pb.lambda, dinv,
                                                                      th, n, S, ws.papp, gp, ws.rrp, ws.rzp);
      LK_CHECK_LAUNCH();
      pcg_pupdate_kernel<LAKER_PRECOND_JACOBI><<<g, kThreads, 0, s2>>>(0, th, p, n, S, ws.rrp, g, ws.rzp, g);
    } else if (P.kind == LAKER_PRECOND_NONE) {
      pcg_update_kernel<LAKER_PRECOND_NONE><<<g, kThreads, 0, s2>>>(alpha, r, p, Apu, ws.part, ps, pb.lambda, nullptr,
                                                                    th, n, S, ws.papp, gp, ws.rrp, ws.rzp);
      LK_CHECK_LAUNCH();
      pcg_pupdate_kernel<LAKER_PRECOND_NONE><<<g, kThreads, 0, s2>>>(0, r, p, n, S, ws.rrp, g, ws.rzp, g);
    } else {
      if (P.f32)
        pcg_update_t_kernel<float><<<nbt, kThreads, 0, s2>>>(alpha, r, p, thu, Apu, ws.part, ps, pb.lambda,
                                                             (const float*)P.B, P.nrp, n, S, ws.papp, gp, ws.rrp,
                                                             ws.tpart);
      else
        pcg_update_t_kernel<double><<<nbt, kThreads, 0, s2>>>(alpha, r, p, thu, Apu, ws.part, ps, pb.lambda,
                                                              (const double*)P.B, P.nrp, n, S, ws.papp, gp, ws.rrp,
                                                              ws.tpart);
      LK_CHECK_LAUNCH();
      laker_status e = enqueue_lowrank_any(P, r, th, n, S, ws.rrp, nbt, ws.rzp, ws.tpart, ws.t, true, s2);
      if (e != LAKER_OK) return e;
      if (!fused) pcg_pupdate_kernel<LAKER_PRECOND_CCCP><<<g, kThreads, 0, s2>>>(0, th, p, n, S, ws.rrp, g, ws.rzp, ga);
    }
    LK_CHECK_LAUNCH();
    if (lanczos) {
      lanczos_record_kernel<<<1, 64, 0, s2>>>(S, ws.lcoef, kLanczosCap);
      LK_CHECK_LAUNCH();
    }
    return LAKER_OK;
  };

  // The chunk of `check_every` iterations is captured once into a HIP graph
  // (on a capture stream of the library) and replayed on `st`: the launches
  // of a chunk then leave the host together.  Without graphs the kernels are
  // enqueued one by one.
  hipGraphExec_t gexec = nullptr;
  if (use_graph) {
    hipStream_t cs = capture_stream_impl();
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
  if (defer && gexec == nullptr && !prof && check_every >= max_iter) {
    // one chunk holds every iteration the cap allows (the cap ends the loop
    // on the device; later launches return at entry)
    for (int c = 0; c < check_every; ++c) {
      const laker_status e = enqueue_iteration(st);
      if (e != LAKER_OK) return e;
    }
    return LAKER_OK;
  }
  PcgScalars hs{};   // (zero until the first read-back: error paths see no iterations)
  int k = 0;
  laker_status loop_status = LAKER_OK;
  // Eager chunks shrink near convergence: the next chunk is the number of
  // iterations the residual decay of the last chunk predicts are still needed
  // (plus one), so few launches are enqueued past the converged iteration.
  int chunk = check_every;
  double last_rr = -1.0;
  int last_it = 0;
  StallTest stall;
  stall.window = stall_window;
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
    if (stall.stalled(hs.iters, sqrt(hs.rr))) {
      loop_status = LAKER_ESTALL;
      break;
    }
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
  if (loop_status != LAKER_OK && loop_status != LAKER_ESTALL) return loop_status;
  if (stats) {
    stats->iters += hs.iters;
    stats->relres = hs.yy > 0 ? sqrt(hs.rr / hs.yy) : 0.0;
  }
  if (lanczos && stats != nullptr && hs.iters > 0) {
    const int m = hs.iters < kLanczosCap ? hs.iters : kLanczosCap;
    tridiag_extremes_kernel<<<1, 64, 0, st>>>(ws.lcoef, m, fused ? 1 : 0, ws.lout);
    LK_CHECK_LAUNCH();
    double h2[2] = {0.0, 0.0};
    LK_TRY(hipMemcpyAsync(h2, ws.lout, sizeof(h2), hipMemcpyDeviceToHost, st));
    LK_TRY(hipStreamSynchronize(st));
    stats->lanczos_steps = m;
    stats->eig_min = h2[0];
    stats->eig_max = h2[1];
    stats->cond_est = h2[0] > 0.0 ? h2[1] / h2[0] : 0.0;
  }
  if (loop_status == LAKER_ESTALL) return LAKER_ESTALL;
  if (hs.done == 2) return LAKER_EBREAKDOWN;
  if (hs.done == 1) return LAKER_OK;
  return LAKER_ENOCONV;
}

hipStream_t pcg_capture_stream() { return capture_stream_impl(); }

laker_status axpy_inplace(double* x, const double* d, int64_t n, hipStream_t st) {
  axpy_kernel<<<red_blocks(n), kThreads, 0, st>>>(x, d, n);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

laker_status apply_lowrank_once(const PrecondView& P, const double* r, double* theta, int64_t n, const SolveWs& ws,
                                hipStream_t st) {
  return enqueue_lowrank_any(P, r, theta, n, nullptr, nullptr, 0, nullptr, ws.tpart, ws.t, false, st);
}

namespace {
__global__ void clear_scalars_kernel(PcgScalars* S) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *S = PcgScalars{};
}
}  // namespace

laker_status precond_apply_once(const PrecondView& P, const double* r, double* theta, int64_t n, double* tpart,
                                double* t, PcgScalars* S, double* rzp, hipStream_t st) {
  if (P.kind == LAKER_PRECOND_JACOBI) {
    // the Jacobi pass reads the run state first: a cleared one (not done)
    clear_scalars_kernel<<<1, 64, 0, st>>>(S);
    LK_CHECK_LAUNCH();
    jacobi_apply_kernel<<<red_blocks(n), kThreads, 0, st>>>(r, (const double*)P.dinv, theta, n, S, rzp);
    LK_CHECK_LAUNCH();
    return LAKER_OK;
  }
  if (P.kind != LAKER_PRECOND_CCCP && P.kind != LAKER_PRECOND_LEARNED) return LAKER_EINVAL;
  return enqueue_lowrank_any(P, r, theta, n, nullptr, nullptr, 0, nullptr, tpart, t, false, st);
}

}  // namespace lk
