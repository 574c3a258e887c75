// Entry points of the C ABI declared in laker.h: argument validation,
// workspace carving and orchestration of the device kernels.
#include <math.h>

#include "fit.hpp"

#include <vector>

#include "bpcg.hpp"

using namespace lk;

namespace {

bool finite_pos(double x) { return isfinite(x) && x > 0.0; }

laker_status check_problem(const laker_problem* p) {
  if (p == nullptr || p->E == nullptr) return LAKER_EINVAL;
  if (p->n < 1 || p->d < 1 || p->d > kMaxD) return LAKER_EINVAL;
  if (!finite_pos(p->lambda) || !finite_pos(p->scale)) return LAKER_EINVAL;
  return LAKER_OK;
}

Problem to_problem(const laker_problem* p) {
  Problem q;
  q.n = p->n;
  q.d = p->d;
  q.dp = pad_dim(p->d);
  q.lambda = p->lambda;
  q.scale = p->scale;
  q.E = p->E;
  return q;
}

bool valid_precision(int32_t prec) { return prec == LAKER_F64 || prec == LAKER_F32 || prec == LAKER_BF16; }

laker_status make_view(const laker_precond* precond, int64_t n, int32_t precision, PrecondView* out) {
  PrecondView view{};
  view.kind = LAKER_PRECOND_NONE;
  if (precond != nullptr && precond->kind != LAKER_PRECOND_NONE) {
    if (precond->data == nullptr || precond->n != n) return LAKER_EINVAL;
    PrecondLayout L = precond_layout(precond->data, n, precond->n_r);
    if (precond->bytes < L.total) return LAKER_ENOMEM;
    const bool f64 = precision == LAKER_F64;
    view.f32 = f64 ? 0 : 1;
    view.kind = precond->kind;
    view.nr = precond->n_r;
    view.nrp = pad_nr(precond->n_r);
    view.c0p = L.hdr;
    if (precond->kind == LAKER_PRECOND_JACOBI) {
      view.dinv = L.dinv64;
    } else if (precond->kind == LAKER_PRECOND_CCCP || precond->kind == LAKER_PRECOND_LEARNED) {
      if (precond->n_r < 1 || precond->n_r > kMaxNr) return LAKER_EINVAL;
      view.B = f64 ? (const void*)L.B64 : (const void*)L.B32;
      view.Bt = f64 ? (const void*)L.Bt64 : (const void*)L.Bt32;
      if (precond->kind == LAKER_PRECOND_LEARNED) {
        // D^{-1} + Bt B^T cancels to the ratio of the largest to the smallest
        // eigenvalue of S on range(V); per-point diagonals can make that ratio
        // exceed what float32 factors resolve, so the rank-64 factors are read
        // in float64 in every precision (2 n 64 doubles per apply)
        view.dinv = L.dinv64;
        view.f32 = 0;
        view.B = (const void*)L.B64;
        view.Bt = (const void*)L.Bt64;
      }
    } else {
      return LAKER_EINVAL;
    }
  }
  *out = view;
  return LAKER_OK;
}

}  // namespace

namespace lk {

PrecondLayout precond_layout(void* base, int64_t n, int nr) {
  WsCarver c(base);
  PrecondLayout L;
  L.hdr = c.take<double>(32);
  const int nrp = pad_nr(nr);
  L.B64 = c.take<double>((size_t)n * nrp);
  L.Bt64 = c.take<double>((size_t)n * nrp);
  L.B32 = c.take<float>((size_t)n * nrp);
  L.Bt32 = c.take<float>((size_t)n * nrp);
  L.dinv64 = c.take<double>(n);
  L.total = c.bytes();
  return L;
}

}  // namespace lk

extern "C" {

const char* laker_status_str(int32_t s) {
  switch (s) {
    case LAKER_OK: return "ok";
    case LAKER_EINVAL: return "invalid argument";
    case LAKER_ENOMEM: return "workspace or buffer too small";
    case LAKER_EHIP: return "HIP runtime error";
    case LAKER_EBREAKDOWN: return "numerical breakdown";
    case LAKER_ENOCONV: return "iteration cap reached before the tolerance";
    case LAKER_ESTALL: return "the residual stalled";
    default: return "unknown status";
  }
}

size_t laker_precond_bytes(int64_t n, int32_t n_r) {
  if (n < 1 || n_r < 0) return 0;
  return precond_layout(nullptr, n, n_r).total;
}

size_t laker_fit_workspace_bytes(int64_t n, int32_t d, int32_t n_r) {
  if (n < 1 || d < 1 || d > kMaxD || n_r < 1) return 0;
  return plan_fit_ws(nullptr, n, d, n_r).total;
}

size_t laker_kmat_bytes(int64_t n, int32_t d, int32_t precision) {
  if (n < 1 || d < 1 || d > 128) return 0;
  if (precision != LAKER_F64 && precision != LAKER_F32) return 0;
  if (!kmat_applies(n, pad_dim(d))) return 0;
  return kmat_bytes(n, precision);
}

size_t laker_solve_workspace_bytes(int64_t n, int32_t d, int64_t m) {
  if (n < 1 || d < 1 || d > kMaxD || m < 0) return 0;
  return plan_solve_ws(nullptr, n, d, m).total;
}

laker_status laker_kernel_matvec(const laker_problem* prob, const double* p, double* w, int32_t precision,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (p == nullptr || w == nullptr || workspace == nullptr || !valid_precision(precision)) return LAKER_EINVAL;
  SolveWs W = plan_solve_ws(workspace, prob->n, prob->d, 0);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  Problem pb = to_problem(prob);
  hipStream_t st = (hipStream_t)stream;
  KmvPlan pl = kmv_plan_square(pb.n, pb.dp, precision);
  void* eh = precision == LAKER_F64 ? (void*)W.e64 : (precision == LAKER_F32 ? (void*)W.e32 : (void*)W.e16);
  LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, precision, eh, st));
  KmvArgs A = kmv_args(eh, pb.n, eh, pb.n, p, W);
  A.lam = pb.lambda;
  A.pself = p;
  A.out = w;
  LK_TRY(kmv_run(precision, pb.dp, pl, A, st));
  return LAKER_OK;
}

// ---- preconditioner apply ------------------------------------------------------
}  // extern "C"

namespace {

struct ApplyWs {
  double* tpart;
  double* t;
  PcgScalars* S;
  double* rzp;
  size_t total;
};
ApplyWs plan_apply_ws(void* base, int64_t n, int nr) {
  WsCarver c(base);
  ApplyWs a;
  a.tpart = c.take<double>((size_t)((n + 63) / 64) * (size_t)pad_nr(nr > 0 ? nr : 1));
  a.t = c.take<double>(kMaxNr);
  a.S = c.take<PcgScalars>(1);
  a.rzp = c.take<double>(kMaxBlocks);
  a.total = c.bytes();
  return a;
}

}  // namespace

extern "C" {

size_t laker_precond_apply_workspace_bytes(int64_t n, int32_t n_r) {
  if (n < 1 || n_r < 0 || n_r > kMaxNr) return 0;
  return plan_apply_ws(nullptr, n, n_r).total;
}

laker_status laker_precond_apply(const laker_precond* precond, const double* r, double* theta, int32_t precision,
                                 void* workspace, size_t workspace_bytes, void* stream) {
  if (precond == nullptr || r == nullptr || theta == nullptr || precond->n < 1) return LAKER_EINVAL;
  if (!valid_precision(precision)) return LAKER_EINVAL;
  const int64_t n = precond->n;
  hipStream_t st = (hipStream_t)stream;
  if (precond->kind == LAKER_PRECOND_NONE) {
    LK_TRY(hipMemcpyAsync(theta, r, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    return LAKER_OK;
  }
  if (workspace == nullptr) return LAKER_EINVAL;
  PrecondView view{};
  laker_status e = make_view(precond, n, precision, &view);
  if (e != LAKER_OK) return e;
  ApplyWs W = plan_apply_ws(workspace, n, view.nr);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  return precond_apply_once(view, r, theta, n, W.tpart, W.t, W.S, W.rzp, st);
}

laker_status laker_fit_precond(const laker_problem* prob, const double* Z, const laker_cccp_opts* opts,
                               laker_precond* out, void* workspace, size_t workspace_bytes, laker_stats* stats,
                               void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (Z == nullptr || opts == nullptr || out == nullptr || out->data == nullptr || workspace == nullptr)
    return LAKER_EINVAL;
  const int nr = opts->n_r;
  if (nr < 1 || nr > kMaxNr || nr > prob->n) return LAKER_EINVAL;
  if (!(opts->gamma >= 0.0) || !isfinite(opts->gamma)) return LAKER_EINVAL;
  if (!(opts->rho >= 0.0 && opts->rho <= 1.0)) return LAKER_EINVAL;
  if (!finite_pos(opts->eps) || !(opts->tol >= 0.0) || opts->max_iter < 1) return LAKER_EINVAL;
  if (!valid_precision(opts->precision)) return LAKER_EINVAL;
  FitWs W = plan_fit_ws(workspace, prob->n, prob->d, nr);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  PrecondLayout L = precond_layout(out->data, prob->n, nr);
  if (out->bytes < L.total) return LAKER_ENOMEM;
  Problem pb = to_problem(prob);
  out->kind = LAKER_PRECOND_CCCP;
  out->n = prob->n;
  out->n_r = nr;
  laker_stats local{};
  laker_stats* sp = stats != nullptr ? stats : &local;
  sp->cccp_iters = 0;
  laker_status r = fit_cccp(pb, Z, *opts, W, L, sp, (hipStream_t)stream);
  sp->status = r;
  return r;
}

// State buffer of the online fit: (a, b), w, then the directions U (rows up to
// the buffer's end), so that the first two sit at fixed offsets.
namespace {
struct OnlineLayout {
  double* ab;
  double* w;
  double* U;
  size_t u_off;
};
OnlineLayout online_layout(void* base, int nr) {
  WsCarver c(base);
  OnlineLayout L;
  L.ab = c.take<double>(2);
  L.w = c.take<double>(nr);
  L.u_off = (c.bytes());
  L.U = base != nullptr ? reinterpret_cast<double*>(static_cast<char*>(base) + L.u_off) : nullptr;
  return L;
}
}  // namespace

size_t laker_online_state_bytes(int64_t n_cap, int32_t n_r) {
  if (n_cap < 1 || n_r < 1 || n_r > kMaxNr) return 0;
  return online_layout(nullptr, n_r).u_off + sizeof(double) * (size_t)n_cap * (size_t)n_r;
}

laker_status laker_fit_precond_online(const laker_problem* prob, int64_t n_prev, const double* Z,
                                      const laker_cccp_opts* opts, void* state, size_t state_bytes,
                                      laker_precond* out, void* workspace, size_t workspace_bytes,
                                      laker_stats* stats, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (Z == nullptr || opts == nullptr || state == nullptr || out == nullptr || out->data == nullptr ||
      workspace == nullptr)
    return LAKER_EINVAL;
  const int nr = opts->n_r;
  if (nr < 1 || nr > kMaxNr || nr > prob->n || n_prev < 0 || n_prev > prob->n) return LAKER_EINVAL;
  if (n_prev > 0 && nr > n_prev) return LAKER_EINVAL;
  if (!(opts->gamma >= 0.0) || !isfinite(opts->gamma)) return LAKER_EINVAL;
  if (!(opts->rho >= 0.0 && opts->rho <= 1.0)) return LAKER_EINVAL;
  if (!finite_pos(opts->eps) || !(opts->tol >= 0.0) || opts->max_iter < 1) return LAKER_EINVAL;
  // the state keeps float64 directions: the products are float64
  if (opts->precision != LAKER_F64) return LAKER_EINVAL;
  if (state_bytes < laker_online_state_bytes(prob->n, nr)) return LAKER_ENOMEM;
  FitWs W = plan_fit_ws(workspace, prob->n, prob->d, nr);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  PrecondLayout L = precond_layout(out->data, prob->n, nr);
  if (out->bytes < L.total) return LAKER_ENOMEM;
  const OnlineLayout SL = online_layout(state, nr);
  OnlineFit on;
  on.U = SL.U;
  on.w = SL.w;
  on.ab = SL.ab;
  on.n_prev = n_prev;
  out->kind = LAKER_PRECOND_CCCP;
  out->n = prob->n;
  out->n_r = nr;
  laker_stats local{};
  laker_stats* sp = stats != nullptr ? stats : &local;
  sp->cccp_iters = 0;
  laker_status r = fit_cccp(to_problem(prob), Z, *opts, W, L, sp, (hipStream_t)stream, &on);
  sp->status = r;
  return r;
}

laker_status laker_jacobi_precond(const laker_problem* prob, laker_precond* out, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (out == nullptr || out->data == nullptr) return LAKER_EINVAL;
  PrecondLayout L = precond_layout(out->data, prob->n, 0);
  if (out->bytes < L.total) return LAKER_ENOMEM;
  out->kind = LAKER_PRECOND_JACOBI;
  out->n = prob->n;
  out->n_r = 0;
  return fit_jacobi(to_problem(prob), L, (hipStream_t)stream);
}

laker_status laker_pcg_solve(const laker_problem* prob, const laker_precond* precond, const double* y, double* alpha,
                             const laker_pcg_opts* opts, void* workspace, size_t workspace_bytes, laker_stats* stats,
                             void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (y == nullptr || alpha == nullptr || opts == nullptr || workspace == nullptr) return LAKER_EINVAL;
  if (!valid_precision(opts->precision)) return LAKER_EINVAL;
  if (!(opts->tol >= 0.0) || opts->max_iter < 1) return LAKER_EINVAL;
  if (opts->refine < 0 || opts->refine > 2 || opts->inner_max_iter < 0) return LAKER_EINVAL;
  if (opts->refine && (opts->ir_max < 1 || !(opts->inner_tol > 0.0))) return LAKER_EINVAL;
  if (opts->refine == 1 && opts->ir_max > 64) return LAKER_EINVAL;
  if (opts->stall_window < 0 || opts->lanczos < 0 || opts->lanczos > 1) return LAKER_EINVAL;
  if (opts->outer_history < 0 || opts->outer_history > 8 || opts->escalate < 0 || opts->escalate > 1)
    return LAKER_EINVAL;
  if (opts->lanczos && opts->refine) return LAKER_EINVAL;
  PrecondView view{};
  e = make_view(precond, prob->n, opts->precision, &view);
  if (e != LAKER_OK) return e;
  if (opts->materialized < 0 || opts->materialized > 1) return LAKER_EINVAL;
  SolveWs W = plan_solve_ws(workspace, prob->n, prob->d, 0);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  // stored G after the carved workspace (float64; float32 too for float32 products)
  if (opts->materialized) {
    const size_t b64 = laker_kmat_bytes(prob->n, prob->d, LAKER_F64);
    if (b64 > 0) {
      size_t need = ((W.total + 255) & ~size_t(255)) + b64;
      const size_t off64 = need - b64;
      size_t off32 = 0;
      if (opts->precision == LAKER_F32) {
        const size_t b32 = laker_kmat_bytes(prob->n, prob->d, LAKER_F32);
        off32 = (need + 255) & ~size_t(255);
        need = off32 + b32;
      }
      if (workspace_bytes < need) return LAKER_ENOMEM;
      W.kmat64 = (char*)workspace + off64;
      if (off32 > 0) W.kmat32 = (char*)workspace + off32;
    }
  }
  Problem pb = to_problem(prob);
  hipStream_t st = (hipStream_t)stream;
  laker_stats local{};
  laker_stats* sp = stats != nullptr ? stats : &local;
  sp->iters = 0;
  sp->ir_steps = 0;
  sp->relres = 0.0;
  sp->relres_true = 0.0;
  sp->kmv_ms = 0.0;
  sp->kmv_count = 0;
  sp->kmv_launches = 0;
  sp->kmv_launch_ms = 0.0;
  sp->escalations = 0;
  sp->lanczos_steps = 0;
  sp->eig_min = sp->eig_max = sp->cond_est = 0.0;
  const int check = opts->check_every > 0 ? opts->check_every : 16;
  LK_TRY(hipMemsetAsync(W.S, 0, sizeof(PcgScalars), st));
  LK_TRY(hipMemsetAsync(W.cnt, 0, 16 * sizeof(unsigned), st));
  LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, LAKER_F64, W.e64, st));
  if (opts->precision == LAKER_F32)
    LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, LAKER_F32, W.e32, st));
  else if (opts->precision == LAKER_BF16)
    LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, LAKER_BF16, W.e16, st));
  if (W.kmat64 != nullptr) LK_TRY(kmat_build(pb.dp, W.e64, pb.n, LAKER_F64, W.kmat64, st));
  if (W.kmat32 != nullptr) LK_TRY(kmat_build(pb.dp, W.e64, pb.n, LAKER_F32, W.kmat32, st));
  laker_status r;
  if (!opts->refine) {
    r = pcg_run(pb, W, view, y, alpha, opts->warm_start != 0, opts->tol, opts->max_iter, check, opts->precision,
                opts->graph != 0, opts->profile != 0, sp, st, false, opts->stall_window, opts->lanczos != 0);
    if (r == LAKER_OK || r == LAKER_ENOCONV || r == LAKER_ESTALL) {
      double rt = 0.0;
      laker_status r2 = true_residual(pb, W, y, alpha, nullptr, &rt, true, st);
      if (r2 != LAKER_OK) return r2;
      sp->relres_true = rt;
    }
  } else if (opts->refine == 2) {
    r = fcg_run(pb, W, view, y, alpha, *opts, check, sp, st);
    if (r == LAKER_EHIP) return r;
  } else {
    if (!opts->warm_start) LK_TRY(hipMemsetAsync(alpha, 0, sizeof(double) * pb.n, st));
    r = LAKER_ENOCONV;
    int used = 0;
    int prec_now = opts->precision;
    StallTest stall;
    stall.window = opts->stall_window;
    for (int s = 0; s <= opts->ir_max; ++s) {
      double rel = 0.0;
      laker_status r2 = true_residual(pb, W, y, alpha, W.rout, &rel, s > 0 || opts->warm_start, st);
      if (r2 != LAKER_OK) return r2;
      if (s < 64) sp->ir_relres[s] = rel;
      sp->relres_true = rel;
      sp->relres = rel;
      sp->ir_steps = s;
      if (rel <= opts->tol) {
        r = LAKER_OK;
        break;
      }
      if (s == opts->ir_max || used >= opts->max_iter) break;
      if (stall.stalled(used, rel)) {
        r = LAKER_ESTALL;
        break;
      }
      // no progress over two refinement steps: the inner products are too
      // coarse for this system (the correction they give does not contract the
      // float64 residual); continue with the next finer arithmetic
      if (s >= 2 && rel >= sp->ir_relres[s - 2] && prec_now != LAKER_F64) {
        prec_now = prec_now == LAKER_BF16 ? LAKER_F32 : LAKER_F64;
        sp->escalations += 1;
        if (prec_now == LAKER_F32) LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, LAKER_F32, W.e32, st));
      }
      // the correction need not be solved more accurately than the outer
      // tolerance still requires
      double itol = opts->inner_tol;
      const double need = 0.5 * opts->tol / rel;
      if (need > itol) itol = need;
      laker_stats inner{};
      int cap = opts->max_iter - used;
      if (opts->inner_max_iter > 0 && cap > opts->inner_max_iter) cap = opts->inner_max_iter;
      laker_status ri = pcg_run(pb, W, view, W.rout, W.dalpha, false, itol, cap, check,
                                prec_now, opts->graph != 0, opts->profile != 0, &inner, st);
      used += inner.iters;
      sp->iters = used;
      if (inner.kmv_count > 0) {
        const double prev = sp->kmv_ms * sp->kmv_count;
        sp->kmv_count += inner.kmv_count;
        sp->kmv_ms = (prev + inner.kmv_ms * inner.kmv_count) / sp->kmv_count;
      }
      if (inner.kmv_launches > 0) {
        const double prev = sp->kmv_launch_ms * sp->kmv_launches;
        sp->kmv_launches += inner.kmv_launches;
        sp->kmv_launch_ms = (prev + inner.kmv_launch_ms * inner.kmv_launches) / sp->kmv_launches;
      }
      // A breakdown of the inner PCG (p^T A p <= 0 in the reduced-precision
      // product: its rounding exceeds lambda in the near-null directions) ends
      // that inner solve with the correction accumulated so far, which the
      // float64 residual then evaluates like any other.
      if (ri == LAKER_EHIP || ri == LAKER_EINVAL) return ri;
      if (ri == LAKER_EBREAKDOWN && prec_now == LAKER_F64) return ri;
      r2 = axpy_inplace(alpha, W.dalpha, pb.n, st);
      if (r2 != LAKER_OK) return r2;
    }
  }
  LK_TRY(hipStreamSynchronize(st));
  sp->status = r;
  return r;
}

laker_status laker_predict(const laker_problem* prob, const double* alpha, int64_t m, const double* Eq, double* rhat,
                           int32_t precision, void* workspace, size_t workspace_bytes, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (alpha == nullptr || Eq == nullptr || rhat == nullptr || workspace == nullptr || m < 1) return LAKER_EINVAL;
  if (!valid_precision(precision)) return LAKER_EINVAL;
  SolveWs W = plan_solve_ws(workspace, prob->n, prob->d, m);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  Problem pb = to_problem(prob);
  hipStream_t st = (hipStream_t)stream;
  KmvPlan pl = kmv_plan(m, pb.n, precision);
  void* eh = precision == LAKER_F64 ? (void*)W.e64 : (precision == LAKER_F32 ? (void*)W.e32 : (void*)W.e16);
  void* qh = precision == LAKER_F64 ? (void*)W.q64 : (precision == LAKER_F32 ? (void*)W.q32 : (void*)W.q16);
  LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, precision, eh, st));
  LK_TRY(prep_embed(Eq, m, pb.d, pb.dp, pb.scale, precision, qh, st));
  KmvArgs A = kmv_args(qh, m, eh, pb.n, alpha, W);
  A.lam = 0.0;
  A.out = rhat;
  LK_TRY(kmv_run(precision, pb.dp, pl, A, st));
  return LAKER_OK;
}

}  // extern "C"

// ---- learned preconditioner -------------------------------------------------

#include "learned.hpp"

namespace {

laker_status learned_flag(const LearnedWs& w, hipStream_t st) {
  int f = 0;
  LK_TRY(hipMemcpyAsync(&f, w.flag, sizeof(int), hipMemcpyDeviceToHost, st));
  LK_TRY(hipStreamSynchronize(st));
  return f ? LAKER_EBREAKDOWN : LAKER_OK;
}

}  // namespace

extern "C" {

laker_status laker_mlp_layout_query(int32_t d, laker_mlp_layout* out) {
  if (out == nullptr || d < 1 || d > kMaxD) return LAKER_EINVAL;
  MlpLayout L = mlp_layout(d);
  out->d = L.d;
  out->in_dim = L.in_dim;
  out->count = L.count;
  for (int t = 0; t < 6; ++t) out->off[t] = L.off[t];
  out->block_bytes = L.block_bytes;
  out->bytes = L.bytes;
  return LAKER_OK;
}

size_t laker_learned_workspace_bytes(int64_t n, int32_t d, int32_t m) {
  if (n < 1 || d < 1 || d > kMaxD || m < 0) return 0;
  return plan_learned_ws(nullptr, n, d, m).total;
}

laker_status laker_learned_forward(const laker_problem* prob, const void* model, float* out, void* workspace,
                                   size_t workspace_bytes, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (model == nullptr || out == nullptr || workspace == nullptr) return LAKER_EINVAL;
  LearnedWs W = plan_learned_ws(workspace, prob->n, prob->d, 0);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  MlpLayout L = mlp_layout(prob->d);
  e = learned_forward(to_problem(prob), L, (const float*)model, W, st);
  if (e != LAKER_OK) return e;
  LK_TRY(hipMemcpyAsync(out, W.O, sizeof(float) * prob->n * kOut, hipMemcpyDeviceToDevice, st));
  return LAKER_OK;
}

laker_status laker_learned_train_step(const laker_problem* prob, void* model, int32_t m, const double* Z,
                                      const double* U, const laker_train_opts* opts, float* grad_out,
                                      double* loss_out, void* workspace, size_t workspace_bytes, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (model == nullptr || Z == nullptr || U == nullptr || opts == nullptr || workspace == nullptr || m < 1)
    return LAKER_EINVAL;
  if (opts->update && (opts->step < 1 || !finite_pos(opts->lr) || !(opts->beta1 >= 0.0 && opts->beta1 < 1.0) ||
                       !(opts->beta2 >= 0.0 && opts->beta2 < 1.0) || !finite_pos(opts->eps)))
    return LAKER_EINVAL;
  LearnedWs W = plan_learned_ws(workspace, prob->n, prob->d, m);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  MlpLayout L = mlp_layout(prob->d);
  Problem pb = to_problem(prob);
  float* theta = (float*)model;
  e = learned_forward(pb, L, theta, W, st);
  if (e != LAKER_OK) return e;
  e = learned_loss_grad(pb, L, theta, Z, U, m, W, st);
  if (e != LAKER_OK) return e;
  if (grad_out != nullptr)
    LK_TRY(hipMemcpyAsync(grad_out, W.grad, sizeof(float) * L.count, hipMemcpyDeviceToDevice, st));
  if (opts->update) {
    char* base = (char*)model;
    LK_TRY(adam_update(theta, (float*)(base + L.block_bytes), (float*)(base + 2 * L.block_bytes), W.grad, L.count,
                       opts->lr, opts->beta1, opts->beta2, opts->eps, opts->step, st));
  }
  if (loss_out != nullptr) {
    LK_TRY(hipMemcpyAsync(loss_out, W.scal, sizeof(double), hipMemcpyDeviceToHost, st));
    return learned_flag(W, st);
  }
  return LAKER_OK;
}

laker_status laker_learned_precond(const laker_problem* prob, const void* model, laker_precond* out,
                                   void* workspace, size_t workspace_bytes, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (model == nullptr || out == nullptr || out->data == nullptr || workspace == nullptr) return LAKER_EINVAL;
  if (prob->n < kRank) return LAKER_EINVAL;
  LearnedWs W = plan_learned_ws(workspace, prob->n, prob->d, 0);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  PrecondLayout P = precond_layout(out->data, prob->n, kRank);
  if (out->bytes < P.total) return LAKER_ENOMEM;
  hipStream_t st = (hipStream_t)stream;
  MlpLayout L = mlp_layout(prob->d);
  Problem pb = to_problem(prob);
  e = learned_forward(pb, L, (const float*)model, W, st);
  if (e != LAKER_OK) return e;
  e = learned_build(pb, W, P, st);
  if (e != LAKER_OK) return e;
  out->kind = LAKER_PRECOND_LEARNED;
  out->n = prob->n;
  out->n_r = kRank;
  return learned_flag(W, st);
}

size_t laker_learned_solve_workspace_bytes(int64_t n, int32_t d, int32_t n_r, int32_t precision,
                                           int32_t materialized) {
  if (n < 1 || d < 1 || d > kMaxD || n_r < 1 || n_r > kMaxNr || !valid_precision(precision)) return 0;
  size_t need = laker_solve_workspace_bytes(n, d, 0);
  if (materialized) {
    const size_t b64 = laker_kmat_bytes(n, d, LAKER_F64);
    if (b64 > 0) {
      need = ((need + 255) & ~size_t(255)) + b64;
      if (precision == LAKER_F32) need = ((need + 255) & ~size_t(255)) + laker_kmat_bytes(n, d, LAKER_F32);
    }
  }
  const size_t a = laker_learned_workspace_bytes(n, d, 0);
  const size_t b = laker_fit_workspace_bytes(n, d, n_r);
  if (a > need) need = a;
  if (b > need) need = b;
  return need;
}

laker_status laker_learned_solve(const laker_problem* prob, const void* model, const double* Z,
                                 const laker_cccp_opts* cccp, const double* y, double* alpha,
                                 const laker_pcg_opts* opts, laker_precond* precond, void* workspace,
                                 size_t workspace_bytes, laker_stats* stats, void* stream) {
  laker_status e = check_problem(prob);
  if (e != LAKER_OK) return e;
  if (model == nullptr || Z == nullptr || cccp == nullptr || y == nullptr || alpha == nullptr || opts == nullptr ||
      precond == nullptr || precond->data == nullptr || workspace == nullptr)
    return LAKER_EINVAL;
  if (prob->n < kRank || cccp->n_r < 1 || cccp->n_r > kMaxNr || cccp->n_r > prob->n) return LAKER_EINVAL;
  if (opts->warm_start || opts->lanczos) return LAKER_EINVAL;
  const int nr_buf = cccp->n_r > kRank ? cccp->n_r : kRank;
  if (precond->bytes < laker_precond_bytes(prob->n, nr_buf)) return LAKER_ENOMEM;
  const size_t need = laker_learned_solve_workspace_bytes(prob->n, prob->d, cccp->n_r, opts->precision,
                                                          opts->materialized);
  if (need == 0) return LAKER_EINVAL;
  if (workspace_bytes < need) return LAKER_ENOMEM;
  laker_stats local{};
  laker_stats* sp = stats != nullptr ? stats : &local;
  *sp = laker_stats{};
  // 1. the learned preconditioner, and the solve with it under the stall test
  e = laker_learned_precond(prob, model, precond, workspace, workspace_bytes, stream);
  int reason = 0;
  int learned_iters = 0;
  if (e == LAKER_EBREAKDOWN) {
    reason = 2;
  } else if (e != LAKER_OK) {
    return e;
  } else {
    e = laker_pcg_solve(prob, precond, y, alpha, opts, workspace, workspace_bytes, sp, stream);
    learned_iters = sp->iters;
    if (e == LAKER_OK) {
      sp->learned_iters = learned_iters;
      return LAKER_OK;
    }
    if (e == LAKER_ESTALL || e == LAKER_ENOCONV) reason = 1;
    else if (e == LAKER_EBREAKDOWN) reason = 2;
    else return e;
  }
  // 2. fallback: the CCCP fit of Alg. 1 into the same buffer, and the solve
  // from the learned solve's iterate (from zero after a breakdown of the build)
  laker_stats fit{};
  e = laker_fit_precond(prob, Z, cccp, precond, workspace, workspace_bytes, &fit, stream);
  if (e != LAKER_OK) return e;
  laker_pcg_opts o2 = *opts;
  o2.stall_window = 0;
  o2.warm_start = (reason == 1 || (reason == 2 && learned_iters > 0)) ? 1 : 0;
  laker_stats s2{};
  e = laker_pcg_solve(prob, precond, y, alpha, &o2, workspace, workspace_bytes, &s2, stream);
  s2.iters += learned_iters;
  s2.fell_back = reason;
  s2.learned_iters = learned_iters;
  s2.cccp_iters = fit.cccp_iters;
  *sp = s2;
  return e;
}

size_t laker_sigma_half_workspace_bytes(int64_t n, int32_t n_r, int32_t m) {
  if (n < 1 || n_r < 1 || n_r > kMaxNr || m < 1) return 0;
  return plan_sigma_half_ws(nullptr, n, n_r, m).total;
}

laker_status laker_precond_sigma_half(const laker_precond* precond, int32_t m, const double* Z, double* U,
                                      void* workspace, size_t workspace_bytes, void* stream) {
  if (precond == nullptr || precond->data == nullptr || precond->kind != LAKER_PRECOND_CCCP) return LAKER_EINVAL;
  if (Z == nullptr || U == nullptr || workspace == nullptr || m < 1 || precond->n < 1) return LAKER_EINVAL;
  if (precond->n_r < 1 || precond->n_r > kMaxNr) return LAKER_EINVAL;
  PrecondLayout P = precond_layout(precond->data, precond->n, precond->n_r);
  if (precond->bytes < P.total) return LAKER_ENOMEM;
  SigmaHalfWs W = plan_sigma_half_ws(workspace, precond->n, precond->n_r, m);
  if (workspace_bytes < W.total) return LAKER_ENOMEM;
  return sigma_half(P, precond->n, precond->n_r, m, Z, U, W, (hipStream_t)stream);
}

}  // extern "C"

// ---- batched solve ------------------------------------------------------------

extern "C" {

size_t laker_batch_workspace_bytes(int32_t count, const int64_t* n, int32_t d) {
  if (count < 1 || n == nullptr || d < 1 || d > kMaxD) return 0;
  for (int b = 0; b < count; ++b)
    if (n[b] < 1) return 0;
  return plan_batch_ws(count, n, d, nullptr, nullptr, nullptr);
}

laker_status laker_pcg_solve_batched(int32_t count, const laker_problem* probs, const laker_precond* preconds,
                                     const double* const* y, double* const* alpha, const laker_pcg_opts* opts,
                                     laker_batch_opts* bopts, void* workspace, size_t workspace_bytes,
                                     laker_stats* stats, void* stream) {
  if (count < 1 || probs == nullptr || y == nullptr || alpha == nullptr || opts == nullptr || workspace == nullptr ||
      stats == nullptr)
    return LAKER_EINVAL;
  if (!valid_precision(opts->precision) || !(opts->tol >= 0.0) || opts->max_iter < 1) return LAKER_EINVAL;
  if (opts->refine < 0 || opts->refine > 1) return LAKER_EINVAL;
  if (opts->refine && (opts->ir_max < 1 || opts->ir_max > 64 || !(opts->inner_tol > 0.0))) return LAKER_EINVAL;
  if (opts->warm_start || opts->lanczos || opts->stall_window) return LAKER_EINVAL;
  if (opts->materialized < 0 || opts->materialized > 1) return LAKER_EINVAL;
  std::vector<int64_t> ns(count);
  std::vector<Problem> pbs(count);
  std::vector<PrecondView> views(count);
  for (int b = 0; b < count; ++b) {
    laker_status e = check_problem(&probs[b]);
    if (e != LAKER_OK) return e;
    if (probs[b].d != probs[0].d || y[b] == nullptr || alpha[b] == nullptr) return LAKER_EINVAL;
    ns[b] = probs[b].n;
    pbs[b] = to_problem(&probs[b]);
    e = make_view(preconds != nullptr ? &preconds[b] : nullptr, probs[b].n, opts->precision, &views[b]);
    if (e != LAKER_OK) return e;
    if (views[b].kind != views[0].kind || views[b].f32 != views[0].f32) return LAKER_EINVAL;
  }
  std::vector<size_t> off(count);
  BatchWs bw{};
  size_t need = plan_batch_ws(count, ns.data(), probs[0].d, off.data(), workspace, &bw);
  // stored G of the maps it applies to, after the batch workspace, in map order
  std::vector<size_t> koff(count, 0);
  if (opts->materialized) {
    for (int b = 0; b < count; ++b) {
      const size_t kb = laker_kmat_bytes(ns[b], probs[0].d, LAKER_F64);
      if (kb == 0) continue;
      koff[b] = (need + 255) & ~size_t(255);
      need = koff[b] + kb;
    }
  }
  if (workspace_bytes < need) return LAKER_ENOMEM;
  std::vector<SolveWs> wss(count);
  for (int b = 0; b < count; ++b) {
    wss[b] = plan_solve_ws((char*)workspace + off[b], ns[b], probs[0].d, 0);
    if (koff[b] > 0) wss[b].kmat64 = (char*)workspace + koff[b];
  }
  BatchOpts bo{};
  bo.cps = bopts != nullptr ? bopts->cols_per_split : 0;
  bo.xcd_order = bopts != nullptr ? bopts->xcd_order : 0;
  if (bo.cps > 0 && bo.cps < 32) return LAKER_EINVAL;
  for (int b = 0; b < count && bo.cps > 0; ++b)
    if ((ns[b] + bo.cps - 1) / bo.cps > kMaxSplit) return LAKER_EINVAL;
  int used = 0;
  laker_status r = pcg_batch(count, pbs.data(), wss.data(), views.data(), y, alpha, *opts, bo, bw, stats, &used,
                             (hipStream_t)stream);
  if (bopts != nullptr) bopts->cols_used = used;
  return r;
}

}  // extern "C"
