// Internal interfaces of the solver, the fit and the entry points.
#pragma once

#include "internal.hpp"

namespace lk {

struct Problem {
  int64_t n;
  int d;
  int dp;
  double lambda;
  double scale;
  const double* E;
};

constexpr int kFcgHist = 8;   // directions the truncated flexible CG can keep

// Carved solve workspace.
struct SolveWs {
  double* e64;
  float* e32;
  uint16_t* e16;
  double* q64;
  float* q32;
  uint16_t* q16;
  double* part;     // column-range partials, up to kMaxSplit x max(n, m)
  double* r;
  double* p;
  double* ap;
  double* theta;
  double* w64;
  double* rout;
  double* dalpha;
  double* fp;       // flexible outer CG: direction and its product (float64)
  double* fq;
  PcgScalars* S;
  double* bpart;
  double* yyp;      // per-block partials of ||y||^2, ||r||^2, r^T theta, p^T A p
  double* rrp;
  double* rzp;
  double* papp;
  double* tpart;
  double* t;
  double* misc;
  unsigned* cnt;
  double* fring;    // truncated flexible CG: kFcgHist directions, then their products (n each)
  double* fpq;      //   p_i^T q_i per slot
  double* fdz;      //   z^T q_i of the current step
  double* fpart;    //   block partials of those (kFcgHist x kMaxBlocks)
  double* lcoef;    // Lanczos estimate: (step size, conjugation coefficient) per iteration
  double* lout;     // its extreme Ritz values
  size_t total;
  // stored G (float64 / float32 tiles, kmat_build) placed after the carved
  // workspace when the solve asks for it; null otherwise
  void* kmat64;
  void* kmat32;
};
SolveWs plan_solve_ws(void* base, int64_t n, int d, int64_t m);
KmvArgs kmv_args(const void* Q, int64_t m, const void* K, int64_t n, const double* p, const SolveWs& ws);
const void* prepared(const SolveWs& ws, int prec);

// Preconditioner as the solver sees it, in one vector precision.
//   CCCP / learned:  theta = c0 r + Bt (B^T r)   (B, Bt: n x nr row-major)
//   Jacobi:          theta = dinv .* r
struct PrecondView {
  int kind;
  int nr;
  int nrp;             // row stride of B, Bt: nr rounded up to a multiple of 4
  const double* c0p;   // device pointer to c0
  const void* B;
  const void* Bt;
  const void* dinv;
  int f32;             // B, Bt stored as float32 (products still accumulated in float64)
};

// Layout of the preconditioner buffer (all offsets 256-byte aligned):
//   header (32 doubles: [0] = b^{-1/2}, [1] = a, [2] = b, [3] = CCCP iterations, ...),
//   B64, Bt64 (n x nrp float64), B32, Bt32 (n x nrp float32), dinv64 (n), with
//   nrp = nr rounded up to a multiple of 4 and zero padding columns.
struct PrecondLayout {
  double* hdr;
  double* B64;
  double* Bt64;
  float* B32;
  float* Bt32;
  double* dinv64;
  size_t total;
};
PrecondLayout precond_layout(void* base, int64_t n, int nr);
inline int pad_nr(int nr) { return (nr + 3) & ~3; }

// defer: when one chunk covers max_iter (eager launches, no profiling), the
// iterations are only enqueued: the call returns LAKER_OK at once and the
// caller reads ws.S (iters, done) after its own next synchronisation.
// stall_window > 0: LAKER_ESTALL when ||r|| fell by less than 2x over the last
// stall_window iterations (checked at each read-back).  lanczos: record the
// step sizes and conjugation coefficients and fill stats->eig_min, eig_max,
// cond_est, lanczos_steps from the Lanczos tridiagonal they define.
constexpr int kLanczosCap = 8192;
laker_status pcg_run(const Problem& pb, const SolveWs& ws, const PrecondView& P, const double* rhs, double* alpha,
                     bool warm, double tol, int max_iter, int check_every, int prec, bool use_graph,
                     bool profile, laker_stats* stats, hipStream_t st, bool defer = false, int stall_window = 0,
                     bool lanczos = false);

// Residual history of a solve for the stall test: stalled() is true when the
// newest residual is above half the residual of the latest record at least
// `window` iterations older.
struct StallTest {
  int window = 0;
  int n = 0;
  int it[4096];
  double res[4096];
  bool stalled(int iters, double resid) {
    if (window <= 0) return false;
    bool s = false;
    for (int k = n - 1; k >= 0; --k) {
      if (it[k] <= iters - window) {
        s = resid > 0.5 * res[k];
        break;
      }
    }
    if (n == 4096) {
      // keep every second record (the test reads the latest old-enough one)
      for (int k = 0; k < 2048; ++k) {
        it[k] = it[2 * k + 1];
        res[k] = res[2 * k + 1];
      }
      n = 2048;
    }
    it[n] = iters;
    res[n] = resid;
    ++n;
    return s;
  }
};
laker_status true_residual(const Problem& pb, const SolveWs& ws, const double* y, const double* alpha,
                           double* r_out, double* relres, bool have_alpha, hipStream_t st);
laker_status axpy_inplace(double* x, const double* d, int64_t n, hipStream_t st);

// Flexible outer CG in float64 whose preconditioner is the inner PCG in
// `precision` (fcg.hip); stats as for the refinement loop.
laker_status fcg_run(const Problem& pb, const SolveWs& ws, const PrecondView& P, const double* y, double* alpha,
                     const laker_pcg_opts& o, int check, laker_stats* sp, hipStream_t st);
// The library's non-blocking stream (per device) on which iteration chunks are
// captured into HIP graphs.
hipStream_t pcg_capture_stream();
laker_status apply_lowrank_once(const PrecondView& P, const double* r, double* theta, int64_t n,
                                const SolveWs& ws, hipStream_t st);
// theta = P r once, with the kernels of the PCG loop (low-rank: the t partials,
// t and the apply, or the apply that finishes t itself; Jacobi: the diagonal
// pass, which takes its run state from S and writes r^T theta partials to rzp)
laker_status precond_apply_once(const PrecondView& P, const double* r, double* theta, int64_t n, double* tpart,
                                double* t, PcgScalars* S, double* rzp, hipStream_t st);

}  // namespace lk
