// PCG (Alg. 1) for several right-hand sides on one map: k measurement vectors
// y_1 .. y_k (bands or snapshots) taken at the same sites share E, G and the
// preconditioner.  Each column runs its own PCG recurrence -- its own step
// sizes, conjugation coefficients, stopping test and retirement, exactly the
// iteration of the single-column solver -- while the kernel product of an
// iteration is one launch for all columns (kmv_multi.hip: score tiles and
// exponentials formed once, multiplied by the k directions).  The vector
// passes are the single solver's per-block bodies with the column as the
// second grid dimension.
#include <math.h>

#include <vector>

#include "kmv_multi.hpp"
#include "pcg_body.hpp"

using namespace lk;
using namespace lk::pcgk;

namespace {

bool mfinite_pos(double x) { return isfinite(x) && x > 0.0; }

// Carved workspace of the multi-column solve (k columns of n rows).
struct MultiWs {
  void* emb;          // prepared embeddings of the products' precision
  double* e64;        // float64 prepared embeddings (true residuals)
  double* part;       // product partials
  double* R;          // residuals, directions, products, preconditioned residuals (n x k each)
  double* P;
  double* AP;
  double* TH;
  double* W;          // (lambda I + G) alpha for the true residuals
  PcgScalars* S;      // k run states
  double* yyp;        // per-column block partials (kMaxBlocks each)
  double* rrp;
  double* rzp;
  double* papp;
  double* tpart;      // per column: (n / 64) x nrp partial rows of t = B^T r
  double* t;          // per column: kMaxNr
  double* rpart;      // per column: 2 kMaxBlocks (||y - A alpha||^2, ||y||^2 partials)
  double* rout;       // per column: the two sums
  size_t total;
};

MultiWs plan_multi_ws(void* base, int64_t n, int d, int k, int prec) {
  WsCarver c(base);
  MultiWs w{};
  const int dp = pad_dim(d);
  const size_t el = prec == LAKER_F64 ? 8 : (prec == LAKER_F32 ? 4 : 2);
  w.emb = c.take<unsigned char>((size_t)n * dp * el);
  w.e64 = c.take<double>((size_t)n * dp);
  w.part = c.take<double>(kmv_multi_part_elems(n, n, k));
  w.R = c.take<double>((size_t)n * k);
  w.P = c.take<double>((size_t)n * k);
  w.AP = c.take<double>((size_t)n * k);
  w.TH = c.take<double>((size_t)n * k);
  w.W = c.take<double>((size_t)n * k);
  w.S = c.take<PcgScalars>((size_t)k);
  w.yyp = c.take<double>((size_t)k * kMaxBlocks);
  w.rrp = c.take<double>((size_t)k * kMaxBlocks);
  w.rzp = c.take<double>((size_t)k * kMaxBlocks);
  w.papp = c.take<double>((size_t)k * kMaxBlocks);
  w.tpart = c.take<double>((size_t)k * (size_t)((n + kTRows - 1) / kTRows) * kMaxNr);
  w.t = c.take<double>((size_t)k * kMaxNr);
  w.rpart = c.take<double>((size_t)k * 2 * kMaxBlocks);
  w.rout = c.take<double>((size_t)k * 2);
  w.total = c.bytes();
  return w;
}

// ---- per-column wrappers of the single solver's bodies (column = blockIdx.y)

__global__ __launch_bounds__(kThreads) void m_init_kernel(const double* __restrict__ Y, double* __restrict__ R,
                                                          double* __restrict__ P, double* __restrict__ alpha,
                                                          int64_t n, double* __restrict__ yyp,
                                                          double* __restrict__ rrp) {
  const int64_t q = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads)
    alpha[q * n + i] = 0.0;
  pcg_init_body(blockIdx.x, gridDim.x, Y + q * n, nullptr, R + q * n, P + q * n, n, yyp + q * kMaxBlocks,
                rrp + q * kMaxBlocks);
}

__global__ __launch_bounds__(kThreads) void m_start_kernel(PcgScalars* S, const double* __restrict__ yyp,
                                                           const double* __restrict__ rrp, int g, double tol,
                                                           int max_iter) {
  const int q = blockIdx.x;
  pcg_start_body(0, 1, S + q, yyp + (int64_t)q * kMaxBlocks, rrp + (int64_t)q * kMaxBlocks, g, tol, max_iter);
}

__global__ __launch_bounds__(kThreads) void m_ap_kernel(const double* __restrict__ P, const double* __restrict__ part,
                                                        PartSum ps, double* __restrict__ AP, int64_t n, double lam,
                                                        double* __restrict__ papp, const PcgScalars* S) {
  const int64_t q = blockIdx.y;
  pcg_ap_body(blockIdx.x, gridDim.x, P + q * n, part + q * ps.nsplit * n, ps, AP + q * n, n, lam,
              papp + q * kMaxBlocks, S + q);
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void m_update_kernel(double* __restrict__ alpha, double* __restrict__ R,
                                                            const double* __restrict__ P,
                                                            const double* __restrict__ AP, PartSum ps, double lam,
                                                            const double* __restrict__ dinv,
                                                            double* __restrict__ TH, int64_t n, PcgScalars* S,
                                                            const double* __restrict__ papp, int gp,
                                                            double* __restrict__ rrp, double* __restrict__ rzp) {
  const int64_t q = blockIdx.y;
  pcg_update_body<KIND>(blockIdx.x, gridDim.x, alpha + q * n, R + q * n, P + q * n, AP + q * n, nullptr, ps, lam,
                        dinv, TH + q * n, n, S + q, papp + q * kMaxBlocks, gp, rrp + q * kMaxBlocks,
                        rzp + q * kMaxBlocks);
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void m_pupdate_kernel(int init, const double* __restrict__ TH,
                                                             double* __restrict__ P, int64_t n, PcgScalars* S,
                                                             const double* __restrict__ rrp, int grr,
                                                             const double* __restrict__ rzp, int grz) {
  const int64_t q = blockIdx.y;
  pcg_pupdate_body<KIND>(blockIdx.x, gridDim.x, init, TH + q * n, P + q * n, n, S + q, rrp + q * kMaxBlocks, grr,
                         rzp + q * kMaxBlocks, grz);
}

__global__ __launch_bounds__(kThreads) void m_jacobi_kernel(const double* __restrict__ R,
                                                            const double* __restrict__ dinv,
                                                            double* __restrict__ TH, int64_t n, const PcgScalars* S,
                                                            double* __restrict__ rzp) {
  const int64_t q = blockIdx.y;
  jacobi_apply_body(blockIdx.x, gridDim.x, R + q * n, dinv, TH + q * n, n, S + q, rzp + q * kMaxBlocks);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void m_t_partial_kernel(const MT* __restrict__ B, const double* __restrict__ R,
                                                               int64_t n, int nrp, double* __restrict__ tpart,
                                                               const PcgScalars* S) {
  const int64_t q = blockIdx.y;
  const int64_t nbt = (n + kTRows - 1) / kTRows;
  lr_t_partial_body<MT>(blockIdx.x, gridDim.x, B, R + q * n, n, nrp, tpart + q * nbt * nrp, S + q);
}

__global__ __launch_bounds__(kThreads) void m_t_finish_kernel(const double* __restrict__ tpart, int nb, int nrp,
                                                              double* __restrict__ t, PcgScalars* S,
                                                              const double* __restrict__ rrp, int grr) {
  const int64_t q = blockIdx.y;
  lr_t_finish_body(blockIdx.x, gridDim.x, tpart + q * (int64_t)nb * nrp, nb, nrp, t + q * kMaxNr, S + q,
                   rrp != nullptr ? rrp + q * kMaxBlocks : nullptr, grr);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void m_apply_kernel(const MT* __restrict__ Bt, const double* __restrict__ t,
                                                           const double* __restrict__ R, double* __restrict__ TH,
                                                           int64_t n, int nrp, const double* __restrict__ c0p,
                                                           const double* __restrict__ dinv, const PcgScalars* S,
                                                           double* __restrict__ rzp) {
  const int64_t q = blockIdx.y;
  lr_apply_body<MT>(blockIdx.x, gridDim.x, Bt, t + q * kMaxNr, R + q * n, TH + q * n, n, nrp, c0p, dinv, S + q,
                    rzp + q * kMaxBlocks);
}

// true residuals: per-column block partials of ||y - w||^2 and ||y||^2, then
// one block per column adds them in order
__global__ __launch_bounds__(kThreads) void m_resid_partial_kernel(const double* __restrict__ Y,
                                                                   const double* __restrict__ W, int64_t n,
                                                                   double* __restrict__ rpart) {
  __shared__ double sh[16];
  const int64_t q = blockIdx.y;
  double rr = 0.0, yy = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double yi = Y[q * n + i];
    const double ri = yi - W[q * n + i];
    rr += ri * ri;
    yy += yi * yi;
  }
  rr = block_sum(rr, sh);
  yy = block_sum(yy, sh);
  if (threadIdx.x == 0) {
    rpart[q * 2 * kMaxBlocks + blockIdx.x] = rr;
    rpart[q * 2 * kMaxBlocks + kMaxBlocks + blockIdx.x] = yy;
  }
}

__global__ __launch_bounds__(kThreads) void m_resid_finish_kernel(const double* __restrict__ rpart, int g,
                                                                  double* __restrict__ out) {
  __shared__ double sh[16];
  const int64_t q = blockIdx.x;
  const double rr = ordered_sum(rpart + q * 2 * kMaxBlocks, g, sh);
  const double yy = ordered_sum(rpart + q * 2 * kMaxBlocks + kMaxBlocks, g, sh);
  if (threadIdx.x == 0) {
    out[2 * q] = rr;
    out[2 * q + 1] = yy;
  }
}

struct MultiView {
  int kind;
  int nr, nrp;
  const double* c0p;
  const void* B;
  const void* Bt;
  const double* dinv;
  int f32;
};

laker_status make_multi_view(const laker_precond* pc, int64_t n, int prec, MultiView* out) {
  MultiView v{};
  v.kind = LAKER_PRECOND_NONE;
  if (pc != nullptr && pc->kind != LAKER_PRECOND_NONE) {
    if (pc->data == nullptr || pc->n != n) return LAKER_EINVAL;
    PrecondLayout L = precond_layout(pc->data, n, pc->n_r);
    if (pc->bytes < L.total) return LAKER_ENOMEM;
    v.kind = pc->kind;
    v.c0p = L.hdr;
    if (pc->kind == LAKER_PRECOND_JACOBI) {
      v.dinv = L.dinv64;
    } else if (pc->kind == LAKER_PRECOND_CCCP || pc->kind == LAKER_PRECOND_LEARNED) {
      if (pc->n_r < 1 || pc->n_r > kMaxNr) return LAKER_EINVAL;
      v.nr = pc->n_r;
      v.nrp = pad_nr(pc->n_r);
      // CCCP factors as the single solver reads them (float32 copies below
      // float64 products); the learned factors in float64 always
      const bool f64 = prec == LAKER_F64 || pc->kind == LAKER_PRECOND_LEARNED;
      v.f32 = f64 ? 0 : 1;
      v.B = f64 ? (const void*)L.B64 : (const void*)L.B32;
      v.Bt = f64 ? (const void*)L.Bt64 : (const void*)L.Bt32;
      if (pc->kind == LAKER_PRECOND_LEARNED) v.dinv = L.dinv64;
    } else {
      return LAKER_EINVAL;
    }
  }
  *out = v;
  return LAKER_OK;
}

template <typename MT>
laker_status m_lowrank(const MultiView& V, const MultiWs& W, int64_t n, int k, bool decide, int g, hipStream_t st) {
  const int nbt = (int)((n + kTRows - 1) / kTRows);
  m_t_partial_kernel<MT><<<dim3(nbt, k), kThreads, 0, st>>>((const MT*)V.B, W.R, n, V.nrp, W.tpart, W.S);
  LK_CHECK_LAUNCH();
  m_t_finish_kernel<<<dim3((V.nrp + 15) / 16, k), kThreads, 0, st>>>(W.tpart, nbt, V.nrp, W.t, W.S,
                                                                     decide ? W.rrp : nullptr, g);
  LK_CHECK_LAUNCH();
  m_apply_kernel<MT><<<dim3(apply_blocks(n), k), kThreads, 0, st>>>((const MT*)V.Bt, W.t, W.R, W.TH, n, V.nrp, V.c0p,
                                                                    V.dinv, W.S, W.rzp);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

laker_status check_multi_problem(const laker_problem* p) {
  if (p == nullptr || p->E == nullptr) return LAKER_EINVAL;
  if (p->n < 1 || p->d < 1 || p->d > kMaxD) return LAKER_EINVAL;
  if (!mfinite_pos(p->lambda) || !mfinite_pos(p->scale)) return LAKER_EINVAL;
  return LAKER_OK;
}

}  // namespace

extern "C" {

size_t laker_multi_workspace_bytes(int64_t n, int32_t d, int32_t k) {
  if (n < 1 || d < 1 || d > kMaxD || k < 1 || k > kMaxRhs) return 0;
  // the float64 copy is the largest embedding copy a product reads
  return plan_multi_ws(nullptr, n, d, k, LAKER_F64).total;
}

laker_status laker_kernel_matvec_multi(const laker_problem* prob, int32_t k, const double* P, double* W,
                                       int32_t precision, void* workspace, size_t workspace_bytes, void* stream) {
  laker_status e = check_multi_problem(prob);
  if (e != LAKER_OK) return e;
  if (k < 1 || k > kMaxRhs || P == nullptr || W == nullptr || workspace == nullptr) return LAKER_EINVAL;
  if (precision != LAKER_F64 && precision != LAKER_F32 && precision != LAKER_BF16) return LAKER_EINVAL;
  const MultiWs M = plan_multi_ws(workspace, prob->n, prob->d, k, precision);
  if (workspace_bytes < plan_multi_ws(nullptr, prob->n, prob->d, k, LAKER_F64).total) return LAKER_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  const int dp = pad_dim(prob->d);
  LK_TRY(prep_embed(prob->E, prob->n, prob->d, dp, prob->scale, precision, M.emb, st));
  KmvMultiArgs A{};
  A.Q = M.emb;
  A.m = prob->n;
  A.K = M.emb;
  A.n = prob->n;
  A.P = P;
  A.part = M.part;
  A.k = k;
  A.finish = 1;
  A.lam = prob->lambda;
  A.pself = P;
  A.out = W;
  LK_TRY(kmv_multi_run(precision, dp, A, st));
  return LAKER_OK;
}

laker_status laker_pcg_solve_multi(const laker_problem* prob, const laker_precond* precond, int32_t k,
                                   const double* Y, double* Alpha, const laker_pcg_opts* opts, void* workspace,
                                   size_t workspace_bytes, laker_stats* stats, void* stream) {
  laker_status e = check_multi_problem(prob);
  if (e != LAKER_OK) return e;
  if (k < 1 || k > kMaxRhs || Y == nullptr || Alpha == nullptr || opts == nullptr || workspace == nullptr ||
      stats == nullptr)
    return LAKER_EINVAL;
  if (opts->precision != LAKER_F64 && opts->precision != LAKER_F32 && opts->precision != LAKER_BF16)
    return LAKER_EINVAL;
  if (!(opts->tol >= 0.0) || opts->max_iter < 1 || opts->refine != 0 || opts->warm_start || opts->graph ||
      opts->lanczos || opts->stall_window)
    return LAKER_EINVAL;
  const int64_t n = prob->n;
  MultiView V{};
  e = make_multi_view(precond, n, opts->precision, &V);
  if (e != LAKER_OK) return e;
  if (workspace_bytes < plan_multi_ws(nullptr, n, prob->d, k, LAKER_F64).total) return LAKER_ENOMEM;
  const MultiWs W = plan_multi_ws(workspace, n, prob->d, k, opts->precision);
  hipStream_t st = (hipStream_t)stream;
  const int dp = pad_dim(prob->d);
  const int prec = opts->precision;
  const int g = red_blocks(n);
  const bool lowrank = V.kind == LAKER_PRECOND_CCCP || V.kind == LAKER_PRECOND_LEARNED;
  const int ga = lowrank ? apply_blocks(n) : g;
  for (int q = 0; q < k; ++q) stats[q] = laker_stats{};
  LK_TRY(prep_embed(prob->E, n, prob->d, dp, prob->scale, prec, W.emb, st));
  LK_TRY(prep_embed(prob->E, n, prob->d, dp, prob->scale, LAKER_F64, W.e64, st));
  LK_TRY(hipMemsetAsync(W.S, 0, sizeof(PcgScalars) * k, st));

  // r^0 = y, alpha^0 = 0; theta^0 = P r^0, p^0 = theta^0
  m_init_kernel<<<dim3(g, k), kThreads, 0, st>>>(Y, W.R, W.P, Alpha, n, W.yyp, W.rrp);
  LK_CHECK_LAUNCH();
  m_start_kernel<<<k, kThreads, 0, st>>>(W.S, W.yyp, W.rrp, g, opts->tol, opts->max_iter);
  LK_CHECK_LAUNCH();
  if (V.kind == LAKER_PRECOND_JACOBI) {
    m_jacobi_kernel<<<dim3(g, k), kThreads, 0, st>>>(W.R, V.dinv, W.TH, n, W.S, W.rzp);
    LK_CHECK_LAUNCH();
    m_pupdate_kernel<LAKER_PRECOND_JACOBI><<<dim3(g, k), kThreads, 0, st>>>(1, W.TH, W.P, n, W.S, W.rrp, g, W.rzp, g);
  } else if (V.kind == LAKER_PRECOND_NONE) {
    m_pupdate_kernel<LAKER_PRECOND_NONE><<<dim3(g, k), kThreads, 0, st>>>(1, W.R, W.P, n, W.S, W.rrp, g, W.rzp, g);
  } else {
    e = V.f32 ? m_lowrank<float>(V, W, n, k, false, g, st) : m_lowrank<double>(V, W, n, k, false, g, st);
    if (e != LAKER_OK) return e;
    m_pupdate_kernel<LAKER_PRECOND_CCCP><<<dim3(g, k), kThreads, 0, st>>>(1, W.TH, W.P, n, W.S, W.rrp, g, W.rzp, ga);
  }
  LK_CHECK_LAUNCH();

  const KmvMultiPlan pl = kmv_multi_plan(n, n);
  PartSum ps{};
  ps.nsplit = pl.nsplit;
  ps.sym = 0;
  KmvMultiArgs A{};
  A.Q = W.emb;
  A.m = n;
  A.K = W.emb;
  A.n = n;
  A.P = W.P;
  A.part = W.part;
  A.k = k;
  A.S = W.S;
  A.pcg_step = 1;
  A.finish = 0;
  auto iteration = [&]() -> laker_status {
    LK_TRY(kmv_multi_run(prec, dp, A, st));
    m_ap_kernel<<<dim3(g, k), kThreads, 0, st>>>(W.P, W.part, ps, W.AP, n, prob->lambda, W.papp, W.S);
    LK_CHECK_LAUNCH();
    if (V.kind == LAKER_PRECOND_JACOBI) {
      m_update_kernel<LAKER_PRECOND_JACOBI><<<dim3(g, k), kThreads, 0, st>>>(
          Alpha, W.R, W.P, W.AP, ps, prob->lambda, V.dinv, W.TH, n, W.S, W.papp, g, W.rrp, W.rzp);
      LK_CHECK_LAUNCH();
      m_pupdate_kernel<LAKER_PRECOND_JACOBI><<<dim3(g, k), kThreads, 0, st>>>(0, W.TH, W.P, n, W.S, W.rrp, g, W.rzp,
                                                                              g);
    } else if (V.kind == LAKER_PRECOND_NONE) {
      m_update_kernel<LAKER_PRECOND_NONE><<<dim3(g, k), kThreads, 0, st>>>(
          Alpha, W.R, W.P, W.AP, ps, prob->lambda, nullptr, W.TH, n, W.S, W.papp, g, W.rrp, W.rzp);
      LK_CHECK_LAUNCH();
      m_pupdate_kernel<LAKER_PRECOND_NONE><<<dim3(g, k), kThreads, 0, st>>>(0, W.R, W.P, n, W.S, W.rrp, g, W.rzp, g);
    } else {
      m_update_kernel<LAKER_PRECOND_CCCP><<<dim3(g, k), kThreads, 0, st>>>(
          Alpha, W.R, W.P, W.AP, ps, prob->lambda, nullptr, W.TH, n, W.S, W.papp, g, W.rrp, W.rzp);
      LK_CHECK_LAUNCH();
      laker_status e2 = V.f32 ? m_lowrank<float>(V, W, n, k, true, g, st) : m_lowrank<double>(V, W, n, k, true, g, st);
      if (e2 != LAKER_OK) return e2;
      m_pupdate_kernel<LAKER_PRECOND_CCCP><<<dim3(g, k), kThreads, 0, st>>>(0, W.TH, W.P, n, W.S, W.rrp, g, W.rzp,
                                                                            ga);
    }
    LK_CHECK_LAUNCH();
    return LAKER_OK;
  };

  const int check = opts->check_every > 0 ? opts->check_every : 16;
  std::vector<PcgScalars> hs(k);
  int done_iters = 0;
  for (;;) {
    for (int c = 0; c < check; ++c) {
      e = iteration();
      if (e != LAKER_OK) return e;
    }
    done_iters += check;
    LK_TRY(hipMemcpyAsync(hs.data(), W.S, sizeof(PcgScalars) * k, hipMemcpyDeviceToHost, st));
    LK_TRY(hipStreamSynchronize(st));
    bool all = true;
    for (int q = 0; q < k; ++q) all = all && hs[q].done != 0;
    if (all || done_iters >= opts->max_iter + check) break;
  }

  // true residuals ||y_q - (lambda I + G) alpha_q|| / ||y_q|| in float64
  KmvMultiArgs T{};
  T.Q = W.e64;
  T.m = n;
  T.K = W.e64;
  T.n = n;
  T.P = Alpha;
  T.part = W.part;
  T.k = k;
  T.finish = 1;
  T.lam = prob->lambda;
  T.pself = Alpha;
  T.out = W.W;
  LK_TRY(kmv_multi_run(LAKER_F64, dp, T, st));
  m_resid_partial_kernel<<<dim3(g, k), kThreads, 0, st>>>(Y, W.W, n, W.rpart);
  LK_CHECK_LAUNCH();
  m_resid_finish_kernel<<<k, kThreads, 0, st>>>(W.rpart, g, W.rout);
  LK_CHECK_LAUNCH();
  std::vector<double> ro(2 * (size_t)k);
  LK_TRY(hipMemcpyAsync(ro.data(), W.rout, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, st));
  LK_TRY(hipStreamSynchronize(st));
  laker_status worst = LAKER_OK;
  for (int q = 0; q < k; ++q) {
    laker_stats& s = stats[q];
    s.iters = hs[q].iters;
    s.relres = hs[q].yy > 0.0 ? sqrt(hs[q].rr / hs[q].yy) : 0.0;
    s.relres_true = ro[2 * q + 1] > 0.0 ? sqrt(ro[2 * q] / ro[2 * q + 1]) : 0.0;
    laker_status sq = hs[q].done == 1 ? LAKER_OK : (hs[q].done == 2 ? LAKER_EBREAKDOWN : LAKER_ENOCONV);
    s.status = sq;
    if (sq == LAKER_EBREAKDOWN || (sq == LAKER_ENOCONV && worst == LAKER_OK)) worst = sq;
  }
  return worst;
}

}  // extern "C"
