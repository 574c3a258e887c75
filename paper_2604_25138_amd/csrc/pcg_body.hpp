// Per-block bodies of the PCG kernels (pcg.hip launches them one problem per
// grid, bpcg.hip with a problem index per grid row).  Each body receives its
// block index `blk` and the block count `nblk` of its problem's grid, so the
// same body gives the same partial sums in either launch form.
#pragma once

#include <type_traits>

#include "pcg.hpp"

namespace lk {
namespace pcgk {

constexpr int kThreads = 256;

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
__device__ __forceinline__ void pcg_init_body(int blk, int nblk, const double* __restrict__ y, const double* __restrict__ w,
                                                            double* __restrict__ r, double* __restrict__ p, int64_t n,
                                                            double* __restrict__ yyp, double* __restrict__ rrp) {
  __shared__ double sh[16];
  double yy = 0.0, rr = 0.0;
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
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
    yyp[blk] = yy;
    rrp[blk] = rr;
  }
}

// One block: ||y||^2, ||r^0||^2, the tolerance and the initial state.
__device__ __forceinline__ void pcg_start_body(int blk, int nblk, PcgScalars* S, const double* __restrict__ yyp,
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
    S->rzold = 0.0;
    S->first = 1;
    S->done = (yy == 0.0 || rr <= tol * tol * yy) ? 1 : 0;
  }
}

// Ap = lambda p + sum of the column-range partials; partials of p^T A p.
__device__ __forceinline__ void pcg_ap_body(int blk, int nblk, const double* __restrict__ p, const double* __restrict__ part,
                                                          const PartSum& ps, double* __restrict__ Ap, int64_t n, double lam,
                                                          double* __restrict__ pap_p, const PcgScalars* S) {
  if (S->done) return;
  __shared__ double sh[16];
  double acc = 0.0;
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
    const double s = ps.row(part, n, i);
    const double pi = p[i];
    const double a = fma(lam, pi, s);
    Ap[i] = a;
    acc += pi * a;
  }
  acc = block_sum(acc, sh);
  if (threadIdx.x == 0) pap_p[blk] = acc;
}

// delta = r^T theta / p^T A p; alpha += delta p; r -= delta Ap (Alg. 1);
// partials of ||r||^2 and, for Jacobi, theta = r / diag and r^T theta.
// Ap null: the product was symmetric, its kernel wrote the p^T A p partials,
// and Ap_i = lam p_i + the product's partials of row i is formed here.
template <int KIND>
__device__ __forceinline__ void pcg_update_body(int blk, int nblk, double* __restrict__ alpha, double* __restrict__ r,
                                                              const double* __restrict__ p,
                                                              const double* __restrict__ Ap,
                                                              const double* __restrict__ part, const PartSum& ps,
                                                              double lam,
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
    if (blk == 0 && threadIdx.x == 0) S->done = 2;
    return;
  }
  if (blk == 0 && threadIdx.x == 0) {
    S->pap = pap;
    S->delta = dl;
  }
  double rr = 0.0, rz = 0.0;
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
    const double pi = p[i];
    const double a = Ap != nullptr ? Ap[i] : fma(lam, pi, ps.row(part, n, i));
    alpha[i] = fma(dl, pi, alpha[i]);
    const double ri = fma(-dl, a, r[i]);
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
    rrp[blk] = rr;
    rzp[blk] = rz;
  }
}

// Sum of thread tid's stripe of `count` grid-reduction partials, in the order
// ordered_sum takes them (a contiguous stripe of per = ceil(count / kThreads)
// entries), of which the first four were loaded ahead into v4; the rest of a
// longer stripe (count > 4 kThreads, e.g. the ||r||^2 partials of more than
// 65536 rows) are read here, after them.
__device__ __forceinline__ double stripe_sum(const double (&v4)[4], const double* __restrict__ part, int count,
                                             int tid, int per) {
  double v = 0.0;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (u < per && tid * per + u < count) v += v4[u];
  for (int u = 4; u < per; ++u)
    if (tid * per + u < count) v += part[tid * per + u];
  return v;
}

// Stopping test of iteration k on the recursive residual (Alg. 1), evaluated
// identically by every block; block 0 records it.  Returns true to continue.
__device__ __forceinline__ bool pcg_decide_rr(int blk, int k, PcgScalars* S, double rr) {
  int d = 0;
  if (!isfinite(rr)) d = 2;
  else if (rr <= S->tol2) d = 1;
  else if (k + 1 >= S->max_iter) d = 3;
  if (blk == 0 && threadIdx.x == 0) {
    S->rr = rr;
    S->iters = k + 1;
    if (d) S->done = d;
  }
  return d == 0;
}
__device__ __forceinline__ bool pcg_decide(int blk, int k, PcgScalars* S, const double* __restrict__ rrp, int g,
                                           double* sh) {
  return pcg_decide_rr(blk, k, S, ordered_sum(rrp, g, sh));
}

// p = theta + beta p with beta = r_new^T theta_new / r^T theta.  With
// init set: p = theta and r^T theta is stored for iteration 0.  For P = I and
// Jacobi this kernel also takes the stopping decision of iteration k.
template <int KIND>
__device__ __forceinline__ void pcg_pupdate_body(int blk, int nblk, int init, const double* __restrict__ theta,
                                                               double* __restrict__ p, int64_t n, PcgScalars* S,
                                                               const double* __restrict__ rrp, int grr,
                                                               const double* __restrict__ rzp, int grz) {
  if (S->done) return;
  __shared__ double sh[16];
  const int k = S->kcur - 1;
  if (!init && KIND != LAKER_PRECOND_CCCP && !pcg_decide(blk, k, S, rrp, grr, sh)) return;
  const double rz = ordered_sum(KIND == LAKER_PRECOND_NONE ? rrp : rzp, KIND == LAKER_PRECOND_NONE ? grr : grz, sh);
  const int slot = init ? 0 : ((k + 1) & 1);
  const double b = init ? 0.0 : rz / S->rzbuf[k & 1];
  if (blk == 0 && threadIdx.x == 0) {
    S->rzbuf[slot] = rz;
    S->beta = b;
  }
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads)
    p[i] = fma(b, p[i], theta[i]);
}

// theta = r / diag (Jacobi) with r^T theta partials, for the start of the iteration.
__device__ __forceinline__ void jacobi_apply_body(int blk, int nblk, const double* __restrict__ r,
                                                                const double* __restrict__ dinv,
                                                                double* __restrict__ theta, int64_t n,
                                                                const PcgScalars* S, double* __restrict__ rzp) {
  if (S->done) return;
  __shared__ double sh[16];
  double rz = 0.0;
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
    const double ri = r[i];
    const double ti = ri * dinv[i];
    theta[i] = ti;
    rz += ri * ti;
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) rzp[blk] = rz;
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

// red[k] = sum over row groups gg = 0, 1, ... of group gg's column sums, added
// in group order: every group stores its four sums into its own LDS row, one
// barrier, then each column is added up by one thread (the loads are
// independent and issue back to back).  Ends with the result in red[0 .. nrp).
__device__ __forceinline__ void combine_groups(double* red, int g, int q, int cq, int groups, int nrp, double a0,
                                               double a1, double a2, double a3) {
  __shared__ double rows[kThreads * 4];   // groups x (4 tpr) <= 4 kThreads
  const int w = 4 * (kThreads / groups);  // row width 4 tpr
  if (q < cq) {
    rows[g * w + 4 * q + 0] = a0;
    rows[g * w + 4 * q + 1] = a1;
    rows[g * w + 4 * q + 2] = a2;
    rows[g * w + 4 * q + 3] = a3;
  }
  __syncthreads();
  for (int k = threadIdx.x; k < nrp; k += kThreads) {
    double v = rows[k];
    for (int gg = 1; gg < groups; ++gg) v += rows[gg * w + k];
    red[k] = v;
  }
  __syncthreads();
}

template <typename MT>
__device__ __forceinline__ void lr_t_partial_body(int blk, int nblk, const MT* __restrict__ B, const double* __restrict__ r,
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
  const int64_t i0 = (int64_t)blk * kTRows;
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
  // fixed-order combination of the row groups (group 0 first)
  combine_groups(red, g, q, cq, groups, nrp, a0, a1, a2, a3);
  for (int k = tid; k < nrp; k += kThreads) tpart[(int64_t)blk * nrp + k] = red[k];
}

// PCG update fused with the first half of the low-rank preconditioner: block
// b owns rows [64 b, 64 b + 64): delta from the p^T A p partials, alpha += delta p,
// r -= delta Ap, the ||r||^2 partial, and t_b = B[rows]^T r[rows] from the
// fresh r kept in LDS.  The stopping decision is taken by the next pass.
// Ap null: as in pcg_update_body, with the block's four waves adding every
// fourth partial of the 64 rows (coalesced rows of the partial buffer).
// theta set: the product kernel of this iteration conjugated the direction on
// the fly (p = theta + beta p, beta in S); this pass stores that direction in
// place, with the same arithmetic, and moves r^T theta to S->rzold.
template <typename MT>
__device__ __forceinline__ void pcg_update_t_body(int blk, int nblk, double* __restrict__ alpha,
                                                                double* __restrict__ r, double* __restrict__ p,
                                                                const double* __restrict__ theta,
                                                                const double* __restrict__ Ap,
                                                                const double* __restrict__ part, const PartSum& ps,
                                                                double lam,
                                                                const MT* __restrict__ B, int nrp, int64_t n,
                                                                PcgScalars* S, const double* __restrict__ pap_p,
                                                                int gp, double* __restrict__ rrp,
                                                                double* __restrict__ tpart) {
  if (S->done) return;
  __shared__ double sh[16];
  __shared__ double rs[kTRows];
  __shared__ double red[kMaxNr];
  __shared__ double apq[kThreads / kTRows][kTRows];
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blk * kTRows;
  // Loads that do not depend on this iteration's scalars go first, so that
  // their latencies overlap: this thread's stripe of the p^T A p partials (as
  // ordered_sum takes them, the first four), the block's rows of p, theta,
  // alpha, r (or Ap), then the row sums of the product's partials.
    const int per = (gp + kThreads - 1) / kThreads;
  double pv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = tid * per + u;
    pv[u] = u < per && idx < gp ? pap_p[idx] : 0.0;
  }
  const int64_t iw = i0 + tid;
  const bool row_in = tid < kTRows && iw < n;
  double pi = 0.0, ti = 0.0, ali = 0.0, ri0 = 0.0, api = 0.0;
  if (row_in) {
    pi = p[iw];
    if (theta != nullptr) ti = theta[iw];
    ali = alpha[iw];
    ri0 = r[iw];
    if (Ap != nullptr) api = Ap[iw];
  }
  // the thread's rows of B for t = B^T r (when they fit in registers: at
  // most four rows, N_r <= 64), loaded now, used once r is updated
  const int cq = nrp / 4;
  int tpr = 1;
  while (tpr < cq) tpr <<= 1;
  const int groups = kThreads / tpr;
  const int g = tid / tpr, q = tid % tpr;
  constexpr int PRE = 4;
  const bool pre = kTRows <= PRE * groups;
  MT bv[PRE][4];
#pragma unroll
  for (int j = 0; j < PRE; ++j) {
    const int rr2 = g + j * groups;
    const bool in = pre && q < cq && rr2 < kTRows && i0 + rr2 < n;
    const MT* row = B + (in ? (i0 + rr2) * nrp + 4 * q : 0);
#pragma unroll
    for (int c = 0; c < 4; ++c) bv[j][c] = in ? row[c] : (MT)0;
  }
  if (Ap == nullptr) {
    const int64_t i = i0 + (tid % kTRows);
    apq[tid / kTRows][tid % kTRows] =
        i < n ? ps.row_strided_all<24>(part, n, i, tid / kTRows, kThreads / kTRows) : 0.0;
  }
  const double pap = block_sum(stripe_sum(pv, pap_p, gp, tid, per), sh);   // (its barriers also publish apq)
  const int k = S->kcur - 1;
  const double dl = S->rzbuf[k & 1] / pap;
  if (!(pap > 0.0) || !isfinite(dl)) {
    if (blk == 0 && tid == 0) S->done = 2;
    return;
  }
  if (blk == 0 && tid == 0) {
    S->pap = pap;
    S->delta = dl;
    if (theta != nullptr) {
      S->rzold = S->rzbuf[k & 1];
      S->first = 0;
    }
  }
  double rr = 0.0;
  if (tid < kTRows) {
    double ri = 0.0;
    if (row_in) {
      if (theta != nullptr) {
        pi = fma(S->beta, pi, ti);
        p[iw] = pi;
      }
      static_assert(kThreads / kTRows == 4, "four partial sums per row");
      const double a = Ap != nullptr ? api
                                     : fma(lam, pi, (apq[0][tid] + apq[1][tid]) + (apq[2][tid] + apq[3][tid]));
      alpha[iw] = fma(dl, pi, ali);
      ri = fma(-dl, a, ri0);
      r[iw] = ri;
    }
    rs[tid] = ri;
    rr = ri * ri;
  }
  rr = block_sum(rr, sh);     // contains the barrier that publishes rs
  if (tid == 0) rrp[blk] = rr;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (pre && q < cq) {
#pragma unroll
    for (int j = 0; j < PRE; ++j) {
      const int rr2 = g + j * groups;
      if (rr2 < kTRows && i0 + rr2 < n) {
        const double ri = rs[rr2];
        a0 = fma((double)bv[j][0], ri, a0);
        a1 = fma((double)bv[j][1], ri, a1);
        a2 = fma((double)bv[j][2], ri, a2);
        a3 = fma((double)bv[j][3], ri, a3);
      }
    }
  } else if (q < cq) {
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
  combine_groups(red, g, q, cq, groups, nrp, a0, a1, a2, a3);
  for (int c = tid; c < nrp; c += kThreads) tpart[(int64_t)blk * nrp + c] = red[c];
}

// t[k] = sum_b tpart[b][k] in a fixed order: a block owns 16 columns; its 16
// row groups of 16 threads each sum every 16th partial row, then combine in LDS.
__device__ __forceinline__ void lr_t_finish_body(int blk, int nblk, const double* __restrict__ tpart, int nb, int nrp,
                                                               double* __restrict__ t, PcgScalars* S,
                                                               const double* __restrict__ rrp, int grr) {
  if (S != nullptr && S->done) return;
  __shared__ double red[16][17];
  __shared__ double shd[16];
  const int tid = threadIdx.x;
  const int g = tid >> 4, cl = tid & 15;
  const int col = blk * 16 + cl;
  // Inside the loop this pass first takes the stopping decision of the
  // current iteration.  Its ||r||^2 partials (this thread's stripe, as
  // ordered_sum takes them, the first four) and, for up to 256 partial
  // rows, the t partials are loaded before it, so that the latencies overlap.
    const int per = rrp != nullptr ? (grr + kThreads - 1) / kThreads : 0;
  double rv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = tid * per + u;
    rv[u] = u < per && idx < grr ? rrp[idx] : 0.0;
  }
  constexpr int PRE = 16;
  const bool pre = nb <= 16 * PRE;
  double tv[PRE];
#pragma unroll
  for (int u = 0; u < PRE; ++u) {
    const int b = g + 16 * u;
    tv[u] = pre && col < nrp && b < nb ? tpart[(int64_t)b * nrp + col] : 0.0;
  }
  if (rrp != nullptr) {
    if (!pcg_decide_rr(blk, S->kcur - 1, S, block_sum(stripe_sum(rv, rrp, grr, tid, per), shd))) return;
  }
  double s = 0.0;
  if (pre) {
#pragma unroll
    for (int u = 0; u < PRE; ++u)
      if (col < nrp && g + 16 * u < nb) s += tv[u];
  } else if (col < nrp) {
    // partial rows g, g + 16, ... added in order; loads issued eight at a time
    int b = g;
    for (; b + 16 * 7 < nb; b += 16 * 8) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = tpart[(int64_t)(b + 16 * u) * nrp + col];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
    for (; b < nb; b += 16) s += tpart[(int64_t)b * nrp + col];
  }
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
template <typename MT, int MAXR = kMaxNr>
__device__ __forceinline__ void lr_apply_body(int blk, int nblk, const MT* __restrict__ Bt, const double* __restrict__ t,
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
  // (ranks up to MAXR; a pass issues MAXV loads per thread)
  constexpr int MAXV = (MAXR + VEC * 16 - 1) / (VEC * 16);
  using VT = typename std::conditional<VEC == 4, float4, double2>::type;
  // UNR passes at a time, so that about four row loads per thread are in
  // flight (at rank 64 one pass issues a single load, too few to stream Bt);
  // all of them are issued before the first use, and the passes are then
  // finished in order, as one at a time would
  constexpr int UNR = MAXV >= 4 ? 1 : 4 / MAXV;
  const int64_t stride = (int64_t)nblk * 16;
  double rz = 0.0;
  for (int64_t i0 = (int64_t)blk * 16; i0 < n; i0 += stride * UNR) {
    VT x[UNR][MAXV];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int64_t i = i0 + u * stride + rl;
      const MT* row = Bt + i * nrp;
#pragma unroll
      for (int j = 0; j < MAXV; ++j)
        if (i < n && sub + 16 * j < nvec) x[u][j] = *reinterpret_cast<const VT*>(row + VEC * (sub + 16 * j));
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int64_t i = i0 + u * stride + rl;
      double acc = 0.0;
      if (i < n) {
#pragma unroll
        for (int j = 0; j < MAXV; ++j) {
          if (sub + 16 * j < nvec) {
            const int v = sub + 16 * j;
            if constexpr (VEC == 4) {
              acc = fma((double)x[u][j].x, ts[4 * v + 0], acc);
              acc = fma((double)x[u][j].y, ts[4 * v + 1], acc);
              acc = fma((double)x[u][j].z, ts[4 * v + 2], acc);
              acc = fma((double)x[u][j].w, ts[4 * v + 3], acc);
            } else {
              acc = fma(x[u][j].x, ts[2 * v + 0], acc);
              acc = fma(x[u][j].y, ts[2 * v + 1], acc);
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
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0 && rzp != nullptr) rzp[blk] = rz;
}

// theta = c r + Bt t with t = B^T r finished here, for N_r <= 64 and at most
// kFuseRows partial rows of t: every block adds all the partial rows itself,
// in one fixed order (thread (q, c) takes column c of rows q, q + 4, ...; the
// four sums are then added in q order), so t needs no pass and launch of its
// own.  Block b owns rows [64 b, 64 b + 64), four passes of 16 rows (16 lanes
// per row, as lr_apply_body).  With rrp set it first takes the stopping
// decision of iteration k, as the separate finishing pass does; the loads of
// the decision's and of t's partials are issued before it.
constexpr int kFuseRows = 256;
__host__ __device__ inline bool lr_fused_t(int64_t n, int nrp) { return nrp <= 64 && (n + kTRows - 1) / kTRows <= kFuseRows; }

// t = B^T r from the t partials in the fused apply's order (thread (q, c):
// column c of rows q, q + 4, ...; then the four sums in q order), into
// ts[0 .. nrp);
// with rrp set, the stopping decision of iteration k first.  Returns false
// when the iteration has stopped.  One whole block of kThreads.
__device__ __forceinline__ bool t_fused_order(int blk, const double* __restrict__ tpart, int nb, int nrp,
                                              PcgScalars* S, const double* __restrict__ rrp, int grr, double* ts,
                                              double* sh) {
  constexpr int MAXR = kFuseRows / 4;
  __shared__ double red[4][64];
  const int tid = threadIdx.x;
  const int q = tid >> 6, c = tid & 63;
    const int per = rrp != nullptr ? (grr + kThreads - 1) / kThreads : 0;
  double rv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int idx = tid * per + u;
    rv[u] = u < per && idx < grr ? rrp[idx] : 0.0;
  }
  double tv[MAXR];
#pragma unroll
  for (int u = 0; u < MAXR; ++u) {
    const int row = q + 4 * u;
    tv[u] = c < nrp && row < nb ? tpart[(int64_t)row * nrp + c] : 0.0;
  }
  if (rrp != nullptr) {
    if (!pcg_decide_rr(blk, S->kcur - 1, S, block_sum(stripe_sum(rv, rrp, grr, tid, per), sh))) return false;
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < MAXR; ++u)
    if (c < nrp && q + 4 * u < nb) s += tv[u];
  red[q][c] = s;
  __syncthreads();
  if (tid < nrp) ts[tid] = (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]);
  __syncthreads();
  return true;
}

// The same t as a separate pass (one block), for the batched solver, whose
// maps share one launch: there every block of every map adding all partial
// rows would multiply the L2 reads.  t_in of lr_apply_t_body then takes it.
__device__ __forceinline__ void lr_t_finish_fused_order_body(const double* __restrict__ tpart, int nb, int nrp,
                                                             double* __restrict__ t, PcgScalars* S,
                                                             const double* __restrict__ rrp, int grr) {
  if (S != nullptr && S->done) return;
  __shared__ double sh[16];
  __shared__ double ts[64];
  if (!t_fused_order(0, tpart, nb, nrp, S, rrp, grr, ts, sh)) return;
  if (threadIdx.x < nrp) t[threadIdx.x] = ts[threadIdx.x];
}

template <typename MT>
__device__ __forceinline__ void lr_apply_t_body(int blk, const double* __restrict__ tpart, int nb,
                                                const MT* __restrict__ Bt, const double* __restrict__ r,
                                                double* __restrict__ theta, int64_t n, int nrp,
                                                const double* __restrict__ c0p, const double* __restrict__ dinv,
                                                PcgScalars* S, const double* __restrict__ rrp, int grr,
                                                double* __restrict__ rzp, const double* __restrict__ t_in = nullptr) {
  if (S != nullptr && S->done) return;
  constexpr int VEC = 16 / (int)sizeof(MT);
  constexpr int MAXV = 64 / VEC / 16;
  using VT = typename std::conditional<VEC == 4, float4, double2>::type;
  __shared__ double sh[16];
  __shared__ double ts[64];
  const int tid = threadIdx.x;
  const int sub = tid & 15, rl = tid >> 4;
  const int nvec = nrp / VEC;
  // the block's rows of Bt, r and the diagonal for all four passes are loaded
  // first: none depends on t, so their latency overlaps the t reduction
  VT x[4][MAXV];
  double rv4[4], cv4[4];
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    const int64_t i = (int64_t)blk * 64 + pass * 16 + rl;
    rv4[pass] = 0.0;
    cv4[pass] = 0.0;
    if (i < n) {
      const MT* row = Bt + i * nrp;
#pragma unroll
      for (int j = 0; j < MAXV; ++j)
        if (sub + 16 * j < nvec) x[pass][j] = *reinterpret_cast<const VT*>(row + VEC * (sub + 16 * j));
      if (sub == 0) {
        rv4[pass] = r[i];
        cv4[pass] = dinv != nullptr ? dinv[i] : c0p[0];
      }
    }
  }
  if (t_in != nullptr) {
    // t already finished (in the fused order) by a separate pass
    if (tid < nrp) ts[tid] = t_in[tid];
    __syncthreads();
  } else if (!t_fused_order(blk, tpart, nb, nrp, S, rrp, grr, ts, sh)) {
    return;
  }
  double rz = 0.0;
#pragma unroll
  for (int pass = 0; pass < 4; ++pass) {
    const int64_t i = (int64_t)blk * 64 + pass * 16 + rl;
    double acc = 0.0;
    if (i < n) {
#pragma unroll
      for (int j = 0; j < MAXV; ++j) {
        if (sub + 16 * j < nvec) {
          const int v = sub + 16 * j;
          if constexpr (VEC == 4) {
            acc = fma((double)x[pass][j].x, ts[4 * v + 0], acc);
            acc = fma((double)x[pass][j].y, ts[4 * v + 1], acc);
            acc = fma((double)x[pass][j].z, ts[4 * v + 2], acc);
            acc = fma((double)x[pass][j].w, ts[4 * v + 3], acc);
          } else {
            acc = fma(x[pass][j].x, ts[2 * v + 0], acc);
            acc = fma(x[pass][j].y, ts[2 * v + 1], acc);
          }
        }
      }
    }
    acc += __shfl_xor(acc, 1, 64);
    acc += __shfl_xor(acc, 2, 64);
    acc += __shfl_xor(acc, 4, 64);
    acc += __shfl_xor(acc, 8, 64);
    if (sub == 0 && i < n) {
      const double ri = rv4[pass];
      const double th = fma(cv4[pass], ri, acc);
      theta[i] = th;
      rz += ri * th;
    }
  }
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0 && rzp != nullptr) rzp[blk] = rz;
}

// ||y - w||^2 and ||y||^2 (float64), for the true residual; r = y - w if r is set.
__device__ __forceinline__ void resid_body(int blk, int nblk, const double* __restrict__ y, const double* __restrict__ w,
                                                         double* __restrict__ r, int64_t n,
                                                         double* __restrict__ bpart, unsigned* cnt, double* out2) {
  __shared__ double sh[16];
  double rr = 0.0, yy = 0.0;
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads) {
    const double yi = y[i];
    const double ri = w != nullptr ? yi - w[i] : yi;
    if (r != nullptr) r[i] = ri;
    rr += ri * ri;
    yy += yi * yi;
  }
  rr = block_sum(rr, sh);
  yy = block_sum(yy, sh);
  if (threadIdx.x == 0) {
    bpart[blk] = rr;
    bpart[kMaxBlocks + blk] = yy;
  }
  if (last_block_arrived_of(cnt, (unsigned)nblk)) {
    const double srr = ordered_sum(bpart, nblk, sh);
    const double syy = ordered_sum(bpart + kMaxBlocks, nblk, sh);
    if (threadIdx.x == 0) {
      out2[0] = srr;
      out2[1] = syy;
      *cnt = 0;
    }
  }
}

__device__ __forceinline__ void axpy_body(int blk, int nblk, double* __restrict__ x, const double* __restrict__ d, int64_t n) {
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += (int64_t)nblk * kThreads)
    x[i] += d[i];
}


}  // namespace pcgk
}  // namespace lk
