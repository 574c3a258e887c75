// Internal interface of the preconditioner fit (fit.hip).
#pragma once

#include "pcg.hpp"

namespace lk {

struct CccpState {
  double a, b, tau, change;   // Sigma = b I + a U_bar diag(w) U_bar^T; last relative change
  double ld_y, ld_z;          // log det of the matrices inverted by the Denman-Beavers step
  double db_change;           // ||I - Z Y||_F / sqrt(N_r) of the square-root iteration
  double sq_c;                // ||R||_F, the scale of the square-root iteration
  int iters, done, gjflag, db_iters;
  unsigned cnt[4];
};

struct FitWs {
  double* e64;
  float* elow;            // float32 / bfloat16 prepared embeddings
  unsigned char* zlow;    // float32 / bfloat16 copy of Z
  double* part;
  int64_t part_cap;
  double* U;
  double* cpart;
  double* norms;
  double* C;
  double* M;
  double* Y;
  double* Zm;
  double* Yi;
  double* Zi;
  double* Gs;
  double* side;           // 2 N_r x N_r partner buffers of the inverse sweeps
  unsigned* gbar;         // grid-barrier counter of the inverse sweeps
  double* q;
  double* w;
  double* wnew;
  CccpState* S;
  double* bpart;
  unsigned* cnt;
  size_t total;
};
FitWs plan_fit_ws(void* base, int64_t n, int d, int nr);

// State of a fit that later fits extend with appended sites: the unscaled
// directions U = (lambda I + G) Z of the sites so far (float64, rows in site
// order) and the CCCP weights (w, a, b) it ended with.
struct OnlineFit {
  double* U;        // n_cap x n_r
  double* w;        // n_r
  double* ab;       // a, b
  int64_t n_prev;   // sites of the previous fit (0: this fit starts the state)
};

laker_status fit_cccp(const Problem& pb, const double* Z, const laker_cccp_opts& o, const FitWs& ws,
                      const PrecondLayout& L, laker_stats* stats, hipStream_t st, const OnlineFit* on = nullptr);
laker_status fit_jacobi(const Problem& pb, const PrecondLayout& L, hipStream_t st);

}  // namespace lk
