// Preconditioner fit of Alg. 1 ("Attention Kernel Regression Learning"):
//   u_k = (lambda I + G) z_k,  u_bar_k = u_k / ||u_k||          (eq. random_directions)
//   shrinkage-CCCP from Sigma_0 = I                             (eqs. kernel_shrinkage_cccp_F/Sigma/normalization)
//   P = Sigma_star^{-1/2}                                        (eq. preconditioner-Sigmma)
//
// Sigma_t is carried exactly in low-rank form b I + a U_bar diag(w) U_bar^T:
// one step computes q_k = u_k^T Sigma^{-1} u_k = (M^{-1} C)_kk / (a w_k) with
// C = U_bar^T U_bar and M = (b/a) diag(1/w) + C (Woodbury), then
// w_k = 1/(q_k + eps), tau = tr(Sigma_tilde)/n, a = (1-rho) c n / (N_r tau),
// b = ((1-rho) c gamma + rho) / tau, c = 1/(1 + gamma/n).
// With B = sqrt(a) U_bar diag(sqrt(w)) and R = b I + B^T B, the inverse square
// root is P = b^{-1/2} I + B Gs B^T, Gs = -b^{-1/2} R^{-1/2} (sqrt(b) I + R^{1/2})^{-1};
// R^{+-1/2} come from the scaled Denman-Beavers iteration, which needs only SPD
// inverses.  The solver applies P as c0 r + Bt (B^T r) with Bt = B Gs.
#include "fit.hpp"

#include <algorithm>
#include <utility>

#include "dense.hpp"
#include "mrhs.hpp"

namespace lk {

namespace {

constexpr int kT = 256;

// part[s][i][k] = sum_{j in split s} exp(<q_i, e_j>) Z[j][k]   (float64, on the
// f64 MFMA; queries q (mq rows), keys e (nk rows, Z row-aligned with them):
// the same rows for a fit, the old and the appended sites for the online update).  A wave owns 16 rows (i) and NCT 16-column tiles of Z and walks
// the split's keys (j) 16 at a time: the score tile is formed transposed,
// S^T = (key rows) (query rows)^T by DP / 4 steps of the 16x16x4 f64 MFMA, so
// that its output -- register r of lane l holds key 4 r + l / 16 against row
// l % 16 -- is, after exp, the lane's A operand of step r of the product with
// Z (row l % 16, k-slot l / 16 = key 4 r + l / 16); the B operand of that step
// is Z[key 4 r + l / 16][column l % 16 of the tile].  Each score tile and its
// exp feed all NCT column tiles, so they are formed once per 16 NCT columns of
// Z.  Key and Z rows come straight from L2: the four waves of a block read the
// same ones.
typedef double v4d_ __attribute__((ext_vector_type(4)));
template <int DP, int NCT>
__global__ __launch_bounds__(256) void mrhs_f64m_kernel(const double* __restrict__ Eq, int64_t mq,
                                                        const double* __restrict__ Ek, int64_t nk,
                                                        const double* __restrict__ Z, int nr,
                                                        double* __restrict__ part, int64_t cps) {
  constexpr int S = DP / 4;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int c = lane & 15, h = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * 64 + wv * 16;
  const int c0 = blockIdx.y * (16 * NCT);
  const int64_t j0 = (int64_t)blockIdx.z * cps;
  const int64_t j1 = j0 + cps < nk ? j0 + cps : nk;
  // query fragment (B operand of the score): element h (DP / 4) + s of row row0 + c
  double qf[S];
  {
    int64_t r = row0 + c;
    if (r > mq - 1) r = mq - 1;
    const double* src = Eq + r * DP + h * S;
#pragma unroll
    for (int s = 0; s < S; ++s) qf[s] = src[s];
  }
  // the lane's Z column in tile t, clamped to the last column (masked on store)
  int zc[NCT];
#pragma unroll
  for (int t = 0; t < NCT; ++t) zc[t] = c0 + 16 * t + c < nr ? c0 + 16 * t + c : nr - 1;
  v4d_ acc[NCT];
#pragma unroll
  for (int t = 0; t < NCT; ++t) acc[t] = v4d_{0.0, 0.0, 0.0, 0.0};
  for (int64_t k0 = j0; k0 < j1; k0 += 16) {
    double kf[S];
    {
      int64_t kr = k0 + c;
      if (kr > nk - 1) kr = nk - 1;
      const double* src = Ek + kr * DP + h * S;
#pragma unroll
      for (int s = 0; s < S; ++s) kf[s] = src[s];
    }
    v4d_ sc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s = 0; s < S; ++s) sc = __builtin_amdgcn_mfma_f64_16x16x4f64(kf[s], qf[s], sc, 0, 0, 0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t key = k0 + 4 * r + h;
      const double x = key < j1 ? exp(sc[r]) : 0.0;
      const double* zrow = Z + (key < nk ? key : nk - 1) * (int64_t)nr;
#pragma unroll
      for (int t = 0; t < NCT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, zrow[zc[t]], acc[t], 0, 0, 0);
    }
  }
  // register r of lane l: row row0 + 4 r + l / 16, column c0 + 16 t + l % 16
  double* out = part + (int64_t)blockIdx.z * mq * nr;
#pragma unroll
  for (int t = 0; t < NCT; ++t) {
    const int col = c0 + 16 * t + c;
    if (col >= nr) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + 4 * r + h;
      if (row < mq) out[row * nr + col] = acc[t][r];
    }
  }
}


// U = lambda Z + sum_s part[s]
__global__ void mrhs_finish_kernel(const double* __restrict__ part, int nsplit, const double* __restrict__ Z,
                                   double lam, int64_t total, double* __restrict__ U) {
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * total + idx];
    U[idx] = fma(lam, Z[idx], s);
  }
}

// Column sums of squares of the n x nr matrix U (row chunks, ordered finish),
// then norms.
__global__ __launch_bounds__(256) void colsq_kernel(const double* __restrict__ U, int64_t n, int nr, int64_t rpb,
                                                    double* __restrict__ cpart, double* __restrict__ norms,
                                                    unsigned* cnt) {
  const int64_t i0 = (int64_t)blockIdx.x * rpb;
  const int64_t i1 = i0 + rpb < n ? i0 + rpb : n;
  for (int k = threadIdx.x; k < nr; k += kT) {
    double s = 0.0;
    for (int64_t i = i0; i < i1; ++i) {
      double u = U[i * nr + k];
      s = fma(u, u, s);
    }
    cpart[(int64_t)blockIdx.x * nr + k] = s;
  }
  if (last_block_arrived(cnt)) {
    for (int k = threadIdx.x; k < nr; k += kT) {
      double s = 0.0;
      for (unsigned b = 0; b < gridDim.x; ++b) s += __builtin_nontemporal_load(cpart + (int64_t)b * nr + k);
      norms[k] = sqrt(s);
    }
    if (threadIdx.x == 0) *cnt = 0;
  }
}

__global__ void colscale_kernel(double* __restrict__ U, int64_t n, int nr, const double* __restrict__ norms) {
  const int64_t total = n * nr;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    int k = (int)(idx % nr);
    U[idx] = U[idx] / norms[k];
  }
}

// M = (b/a) diag(1/w) + C
__global__ void cccp_build_m_kernel(const double* __restrict__ C, const double* __restrict__ w,
                                    const CccpState* __restrict__ S, double* __restrict__ M, int nr) {
  if (S->done) return;
  const double ba = S->b / S->a;
  const int64_t total = (int64_t)nr * nr;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    int64_t i = idx / nr, j = idx - i * nr;
    M[idx] = C[idx] + (i == j ? ba / w[i] : 0.0);
  }
}

// q_k = (M^{-1} C)_kk / (a w_k), or q_k = C_kk while Sigma = I; one wave per k.
__global__ __launch_bounds__(256) void cccp_q_kernel(const double* __restrict__ Minv, const double* __restrict__ C,
                                                     const double* __restrict__ w, const CccpState* __restrict__ S,
                                                     double* __restrict__ q, int nr, int first) {
  if (S->done) return;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= nr) return;
  if (first) {
    if (lane == 0) q[k] = C[(int64_t)k * nr + k];
    return;
  }
  double s = 0.0;
  const double* mr = Minv + (int64_t)k * nr;
  const double* cr = C + (int64_t)k * nr;   // C symmetric: column k = row k
  for (int j = lane; j < nr; j += 64) s = fma(mr[j], cr[j], s);
  s = wave_sum(s);
  if (lane == 0) q[k] = s / (S->a * w[k]);
}

// q_k from the refined solve X = M^{-1} C:  q_k = (X_kk + (Minv R)_kk) / (a w_k)
// with R = C - M X the residual of the last refinement step; one wave per k.
__global__ __launch_bounds__(256) void cccp_q_refined_kernel(const double* __restrict__ Minv,
                                                             const double* __restrict__ X,
                                                             const double* __restrict__ R,
                                                             const double* __restrict__ w,
                                                             const CccpState* __restrict__ S,
                                                             double* __restrict__ q, int nr) {
  if (S->done) return;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= nr) return;
  double s = 0.0;
  const double* mr = Minv + (int64_t)k * nr;
  for (int j = lane; j < nr; j += 64) s = fma(mr[j], R[(int64_t)j * nr + k], s);
  s = wave_sum(s);
  if (lane == 0) q[k] = (X[(int64_t)k * nr + k] + s) / (S->a * w[k]);
}

// w <- 1/(q + eps); tau, a, b; exact Frobenius change of Sigma; stopping test.
// One block of 1024 threads, fixed-order sums.
__global__ __launch_bounds__(1024) void cccp_update_kernel(const double* __restrict__ C, const double* __restrict__ q,
                                                           double* __restrict__ w, double* __restrict__ wnew,
                                                           CccpState* S, int nr, double n, double gamma, double rho,
                                                           double eps, double tol, int max_iter) {
  if (S->done) return;
  __shared__ double sh[16];
  const int tid = threadIdx.x;
  const double a0 = S->a, b0 = S->b;
  double swc = 0.0;
  for (int k = tid; k < nr; k += 1024) {
    double wn = 1.0 / (q[k] + eps);
    wnew[k] = wn;
    swc += wn * C[(int64_t)k * nr + k];
  }
  swc = block_sum(swc, sh);
  const double c = 1.0 / (1.0 + gamma / n);
  const double tau = (1.0 - rho) * c * (swc / nr + gamma) + rho;
  const double a1 = (1.0 - rho) * c * n / (nr * tau);
  const double b1 = ((1.0 - rho) * c * gamma + rho) / tau;
  __syncthreads();
  // D = a1 wnew - a0 w ; F = a0 w.  Wave v takes rows v, v + 16, ...; its lanes
  // the columns.
  double t_dc = 0.0, t_fc = 0.0, t_dd = 0.0, t_ff = 0.0;
  const int lane = tid & 63, wv = tid >> 6;
  for (int k = wv; k < nr; k += 16) {
    const double dk = a1 * wnew[k] - a0 * w[k], fk = a0 * w[k];
    const double* __restrict__ Ck = C + (int64_t)k * nr;
    for (int l = lane; l < nr; l += 64) {
      const double ckl = Ck[l];
      const double dl = a1 * wnew[l] - a0 * w[l], fl = a0 * w[l];
      const double c2 = ckl * ckl;
      t_dd = fma(dk * dl, c2, t_dd);
      t_ff = fma(fk * fl, c2, t_ff);
      if (k == l) {
        t_dc += dk * ckl;
        t_fc += fk * ckl;
      }
    }
  }
  t_dd = block_sum(t_dd, sh);
  t_ff = block_sum(t_ff, sh);
  t_dc = block_sum(t_dc, sh);
  t_fc = block_sum(t_fc, sh);
  __syncthreads();
  const double db = b1 - b0;
  const double num = n * db * db + 2.0 * db * t_dc + t_dd;
  const double den = n * b0 * b0 + 2.0 * b0 * t_fc + t_ff;
  const double change = sqrt(fmax(num, 0.0) / den);
  for (int k = tid; k < nr; k += 1024) w[k] = wnew[k];
  if (tid == 0) {
    S->a = a1;
    S->b = b1;
    S->tau = tau;
    S->change = change;
    int it = S->iters + 1;
    S->iters = it;
    if (!isfinite(change) || !(tau > 0.0)) S->done = 2;
    else if (change <= tol) S->done = 1;
    else if (it >= max_iter) S->done = 3;
  }
}

__global__ void cccp_init_kernel(CccpState* S, double* w, int nr) {
  for (int k = threadIdx.x; k < nr; k += blockDim.x) w[k] = 0.0;
  if (threadIdx.x == 0) {
    S->a = 0.0;
    S->b = 1.0;
    S->tau = 1.0;
    S->change = 0.0;
    S->iters = 0;
    S->done = 0;
    S->gjflag = 0;
    S->db_iters = 0;
    S->db_change = 0.0;
  }
}

// B = sqrt(a) U_bar diag(sqrt(w))  (n x nr, stored with row stride nrp, zero padding)
__global__ void make_b_kernel(const double* __restrict__ Ub, const double* __restrict__ w,
                              const CccpState* __restrict__ S, double* __restrict__ B, int64_t n, int nr, int nrp) {
  const double sa = sqrt(S->a);
  const int64_t total = n * nrp;
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t i = idx / nrp;
    const int k = (int)(idx - i * nrp);
    B[idx] = k < nr ? sa * Ub[i * nr + k] * sqrt(w[k]) : 0.0;
  }
}

// Y = b I + a diag(sqrt w) C diag(sqrt w) (= b I + B^T B),  Zm = I
// R = b I + B^T B = b I + a diag(sqrt w) C diag(sqrt w) into Y, Zm = I, and
// c = ||R||_F (>= the largest eigenvalue of R) into S->sq_c.
__global__ __launch_bounds__(256) void sq_init_kernel(const double* __restrict__ C, const double* __restrict__ w,
                                                      CccpState* S, double* __restrict__ Y, double* __restrict__ Zm,
                                                      int nr, double* __restrict__ bpart) {
  __shared__ double sh[16];
  const double a = S->a, b = S->b;
  double ss = 0.0;
  const int total = nr * nr;
  for (int idx = blockIdx.x * kT + threadIdx.x; idx < total; idx += gridDim.x * kT) {
    const int i = idx / nr, j = idx - i * nr;
    const double r = a * sqrt(w[i] * w[j]) * C[idx] + (i == j ? b : 0.0);
    Y[idx] = r;
    Zm[idx] = (i == j) ? 1.0 : 0.0;
    ss = fma(r, r, ss);
  }
  ss = block_sum(ss, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = ss;
  if (last_block_arrived(&S->cnt[0])) {
    const double t = ordered_sum(bpart, gridDim.x, sh);
    if (threadIdx.x == 0) {
      S->sq_c = sqrt(t);
      S->db_iters = 0;
      S->cnt[0] = 0;
    }
  }
}

// X <- X / c (mode 0), X * sqrt(c) (mode 1), X / sqrt(c) (mode 2), c = S->sq_c
__global__ void sq_scale_kernel(double* __restrict__ X, const CccpState* __restrict__ S, int mode, int total) {
  const double c = S->sq_c;
  const double f = mode == 0 ? 1.0 / c : (mode == 1 ? sqrt(c) : 1.0 / sqrt(c));
  for (int idx = blockIdx.x * kT + threadIdx.x; idx < total; idx += gridDim.x * kT) X[idx] *= f;
}

// Coupled Newton-Schulz step, middle part: P = Z Y given, T = (3 I - P) / 2 in
// place, and ||I - P||_F / sqrt(N) into S->db_change.
__global__ __launch_bounds__(256) void sq_t_kernel(double* __restrict__ P, CccpState* S, int nr,
                                                   double* __restrict__ bpart) {
  __shared__ double sh[16];
  double ss = 0.0;
  const int total = nr * nr;
  for (int idx = blockIdx.x * kT + threadIdx.x; idx < total; idx += gridDim.x * kT) {
    const int i = idx / nr, j = idx - i * nr;
    const double e = (i == j ? 1.0 : 0.0) - P[idx];
    ss = fma(e, e, ss);
    P[idx] = (i == j ? 1.5 : 0.0) - 0.5 * P[idx];
  }
  ss = block_sum(ss, sh);
  if (threadIdx.x == 0) bpart[blockIdx.x] = ss;
  if (last_block_arrived(&S->cnt[0])) {
    const double t = ordered_sum(bpart, gridDim.x, sh);
    if (threadIdx.x == 0) {
      S->db_change = sqrt(t / nr);
      S->db_iters += 1;
      S->cnt[0] = 0;
    }
  }
}

__global__ void add_sqrtb_diag_kernel(const double* __restrict__ Y, const CccpState* __restrict__ S,
                                      double* __restrict__ W, int nr) {
  const int64_t total = (int64_t)nr * nr;
  const double sb = sqrt(S->b);
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    const int64_t i = idx / nr, j = idx - i * nr;
    W[idx] = Y[idx] + (i == j ? sb : 0.0);
  }
}

__global__ void write_header_kernel(const CccpState* __restrict__ S, double* __restrict__ hdr) {
  if (threadIdx.x == 0) {
    hdr[0] = 1.0 / sqrt(S->b);
    hdr[1] = S->a;
    hdr[2] = S->b;
    hdr[3] = (double)S->iters;
    hdr[4] = S->change;
    hdr[5] = (double)S->db_iters;
    hdr[6] = S->db_change;
  }
}

// Jacobi: dinv_i = 1 / (lambda + exp(s <e_i, e_i>)).
__global__ void jacobi_kernel(const double* __restrict__ E, int64_t n, int d, double s, double lam,
                              double* __restrict__ d64) {
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    double acc = 0.0;
    for (int c = 0; c < d; ++c) acc = fma(E[i * d + c], E[i * d + c], acc);
    double v = 1.0 / (lam + exp(s * acc));
    d64[i] = v;
  }
}

__global__ void to_f32_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t total) {
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT)
    dst[idx] = (float)src[idx];
}

inline int ew_grid(int64_t total) {
  int64_t g = (total + kT - 1) / kT;
  if (g > 8192) g = 8192;
  return (int)(g < 1 ? 1 : g);
}


// U[i] = base[i] + sum_s part[s][i] over mq x nr entries, where base is
// lambda Zs (Zs set: the rows' own directions) or the previous U (in place)
__global__ void mrhs_rect_finish_kernel(const double* __restrict__ part, int nsplit, const double* __restrict__ Zs,
                                        double lam, int64_t total, double* __restrict__ U) {
  for (int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x; idx < total; idx += (int64_t)gridDim.x * kT) {
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * total + idx];
    U[idx] = Zs != nullptr ? fma(lam, Zs[idx], s) : U[idx] + s;
  }
}

// Warm start of the CCCP iteration from a previous fit's (a, b, w).
__global__ void cccp_init_warm_kernel(CccpState* S, double* w, const double* w0, const double* ab, int nr) {
  for (int k = threadIdx.x; k < nr; k += blockDim.x) w[k] = w0[k];
  if (threadIdx.x == 0) {
    S->a = ab[0];
    S->b = ab[1];
    S->tau = 1.0;
    S->change = 0.0;
    S->iters = 0;
    S->done = 0;
    S->gjflag = 0;
    S->db_iters = 0;
    S->db_change = 0.0;
  }
}

__global__ void cccp_save_kernel(const CccpState* S, const double* w, double* w0, double* ab, int nr) {
  for (int k = threadIdx.x; k < nr; k += blockDim.x) w0[k] = w[k];
  if (threadIdx.x == 0) {
    ab[0] = S->a;
    ab[1] = S->b;
  }
}

inline int64_t mrhs_partial_cap(int64_t n, int nr) {
  int64_t a = 4 * n * (int64_t)nr;
  int64_t b = 16 * (int64_t)nr * nr;
  int64_t c = (int64_t)1 << 22;
  int64_t m = a > b ? a : b;
  return m > c ? m : c;
}

// columns of Z per block of the f64 MFMA directions product: 16 NCT, NCT = 8
// (4 for dp = 128, whose fragments take twice the registers)
inline int mrhs_nct(int dp) { return dp == 128 ? 4 : 8; }

hipError_t launch_mrhs(int dp, const double* Eq, int64_t mq, const double* Ek, int64_t nk, const double* Z, int nr,
                       double* part, int nsplit, int64_t cps, hipStream_t st) {
  const int cols = 16 * mrhs_nct(dp);
  dim3 grid((unsigned)((mq + 63) / 64), (unsigned)((nr + cols - 1) / cols), (unsigned)nsplit);
  switch (dp) {
    case 16: mrhs_f64m_kernel<16, 8><<<grid, 256, 0, st>>>(Eq, mq, Ek, nk, Z, nr, part, cps); break;
    case 32: mrhs_f64m_kernel<32, 8><<<grid, 256, 0, st>>>(Eq, mq, Ek, nk, Z, nr, part, cps); break;
    case 64: mrhs_f64m_kernel<64, 8><<<grid, 256, 0, st>>>(Eq, mq, Ek, nk, Z, nr, part, cps); break;
    case 128: mrhs_f64m_kernel<128, 4><<<grid, 256, 0, st>>>(Eq, mq, Ek, nk, Z, nr, part, cps); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// part[s] = G(Eq, Ek) Z over nsplit key ranges of cps keys, then
// U = base + sum_s part[s] (mq x nr); the split keeps mq nr nsplit within cap
hipError_t rect_directions(int dp, const double* Eq, int64_t mq, const double* Ek, int64_t nk, const double* Z,
                           int nr, const double* Zs, double lam, double* U, double* part, int64_t cap,
                           hipStream_t st) {
  if (mq < 1 || nk < 1) return hipSuccess;
  const int64_t rowtiles = (mq + 63) / 64, coltiles = (nr + 16 * mrhs_nct(dp) - 1) / (16 * mrhs_nct(dp));
  int64_t ns = (1024 + rowtiles * coltiles - 1) / (rowtiles * coltiles);
  const int64_t jt = (nk + 31) / 32;
  if (ns > jt) ns = jt;
  if (ns > 64) ns = 64;
  while (ns > 1 && ns * mq * nr > cap) --ns;
  if (ns < 1) ns = 1;
  if (mq * nr > cap) return hipErrorInvalidValue;
  const int64_t cps = (((nk + ns - 1) / ns) + 31) / 32 * 32;
  ns = (nk + cps - 1) / cps;
  hipError_t e = launch_mrhs(dp, Eq, mq, Ek, nk, Z, nr, part, (int)ns, cps, st);
  if (e != hipSuccess) return e;
  mrhs_rect_finish_kernel<<<ew_grid(mq * nr), kT, 0, st>>>(part, (int)ns, Zs, lam, mq * nr, U);
  return hipGetLastError();
}

}  // namespace

FitWs plan_fit_ws(void* base, int64_t n, int d, int nr) {
  WsCarver c(base);
  FitWs w;
  const int dp = pad_dim(d);
  w.e64 = c.take<double>((size_t)n * dp);
  w.elow = c.take<float>((size_t)n * dp);
  w.zlow = c.take<unsigned char>(mrhs_z_bytes(n, nr));
  w.part_cap = mrhs_partial_cap(n, nr);
  w.part = c.take<double>((size_t)w.part_cap);
  w.U = c.take<double>((size_t)n * nr);
  w.cpart = c.take<double>((size_t)256 * nr);
  w.norms = c.take<double>(nr);
  w.C = c.take<double>((size_t)nr * nr);
  w.M = c.take<double>((size_t)nr * nr);
  w.Y = c.take<double>((size_t)nr * nr);
  w.Zm = c.take<double>((size_t)nr * nr);
  w.Yi = c.take<double>((size_t)nr * nr);
  w.Zi = c.take<double>((size_t)nr * nr);
  w.Gs = c.take<double>((size_t)nr * nr);
  w.side = c.take<double>(2 * gj_side_elems(nr));
  w.gbar = c.take<unsigned>(64);
  w.q = c.take<double>(nr);
  w.w = c.take<double>(nr);
  w.wnew = c.take<double>(nr);
  w.S = c.take<CccpState>(1);
  w.bpart = c.take<double>(2 * kMaxBlocks);
  w.cnt = c.take<unsigned>(16);
  w.total = c.bytes();
  return w;
}

laker_status fit_cccp(const Problem& pb, const double* Z, const laker_cccp_opts& o, const FitWs& ws,
                      const PrecondLayout& L, laker_stats* stats, hipStream_t st, const OnlineFit* on) {
  const int64_t n = pb.n;
  const int nr = o.n_r;
  const bool warm = on != nullptr && on->n_prev > 0;
  // 1-2. U = (lambda I + G) Z: float64 tiles, or float32 / bfloat16 MFMA tiles.
  // Sites appended to a previous fit (rows n_prev ..): only the products with
  // the new rows are formed, in float64:
  //   U[old] += G[old, new] Z[new],   U[new] = G[new, all] Z + lambda Z[new]
  if (warm) {
    const int64_t n0 = on->n_prev, m = n - n0;
    LK_TRY(prep_embed(pb.E, n, pb.d, pb.dp, pb.scale, LAKER_F64, ws.e64, st));
    const double* e_new = ws.e64 + n0 * pb.dp;
    LK_TRY(rect_directions(pb.dp, ws.e64, n0, e_new, m, Z + n0 * nr, nr, nullptr, 0.0, on->U, ws.part, ws.part_cap,
                           st));
    LK_TRY(rect_directions(pb.dp, e_new, m, ws.e64, n, Z, nr, Z + n0 * nr, pb.lambda, on->U + n0 * nr, ws.part,
                           ws.part_cap, st));
    LK_TRY(hipMemcpyAsync(ws.U, on->U, sizeof(double) * n * nr, hipMemcpyDeviceToDevice, st));
  } else if (o.precision == LAKER_F64) {
    LK_TRY(prep_embed(pb.E, n, pb.d, pb.dp, pb.scale, LAKER_F64, ws.e64, st));
    const int64_t rowtiles = (n + 63) / 64, coltiles = (nr + 16 * mrhs_nct(pb.dp) - 1) / (16 * mrhs_nct(pb.dp));
    int64_t ns = (1024 + rowtiles * coltiles - 1) / (rowtiles * coltiles);
    int64_t jt = (n + 31) / 32;
    if (ns > jt) ns = jt;
    if (ns > 64) ns = 64;
    while (ns > 1 && ns * n * nr > ws.part_cap) --ns;
    if (ns < 1) ns = 1;
    int64_t cps = (((n + ns - 1) / ns) + 31) / 32 * 32;
    ns = (n + cps - 1) / cps;
    LK_TRY(launch_mrhs(pb.dp, ws.e64, n, ws.e64, n, Z, nr, ws.part, (int)ns, cps, st));
    mrhs_finish_kernel<<<ew_grid(n * nr), kT, 0, st>>>(ws.part, (int)ns, Z, pb.lambda, n * nr, ws.U);
    LK_CHECK_LAUNCH();
  } else {
    LK_TRY(prep_embed(pb.E, n, pb.d, pb.dp, pb.scale, o.precision, ws.elow, st));
    LK_TRY(mrhs_mfma(o.precision, pb.dp, ws.elow, n, Z, ws.zlow, nr, pb.lambda, ws.U, st));
  }
  if (on != nullptr && !warm) LK_TRY(hipMemcpyAsync(on->U, ws.U, sizeof(double) * n * nr, hipMemcpyDeviceToDevice, st));
  // 3. U_bar = U / ||U||  (column-wise)
  {
    int64_t rpb = (n + 255) / 256;
    if (rpb < 16) rpb = 16;
    int gb = (int)((n + rpb - 1) / rpb);
    LK_TRY(hipMemsetAsync(ws.cnt, 0, 16 * sizeof(unsigned), st));
    colsq_kernel<<<gb, kT, 0, st>>>(ws.U, n, nr, rpb, ws.cpart, ws.norms, ws.cnt);
    LK_CHECK_LAUNCH();
    colscale_kernel<<<ew_grid(n * nr), kT, 0, st>>>(ws.U, n, nr, ws.norms);
    LK_CHECK_LAUNCH();
  }
  // 4. C = U_bar^T U_bar
  {
    int ns = gemm_pick_split(nr, nr, n, ws.part_cap);
    LK_TRY(gemm_f64(nr, nr, n, ws.U, 1, nr, ws.U, nr, 1, ws.C, nr, 1.0, nullptr, 0.0, ws.part, ns, st));
  }
  // 5. CCCP iterations
  if (warm) cccp_init_warm_kernel<<<1, 256, 0, st>>>(ws.S, ws.w, on->w, on->ab, nr);
  else cccp_init_kernel<<<1, 256, 0, st>>>(ws.S, ws.w, nr);
  LK_CHECK_LAUNCH();
  // grid-barrier counter of the inverse sweeps: zero here, then advanced by a
  // known amount per sweep
  LK_TRY(hipMemsetAsync(ws.gbar, 0, sizeof(unsigned), st));
  unsigned gbase = 0;
  auto inverse = [&](int count, double* A0, double* A1, double* ld0, double* ld1) -> hipError_t {
    double* As[2] = {A0, A1};
    double* Ss[2] = {ws.side, ws.side + gj_side_elems(nr)};
    double* Ls[2] = {ld0, ld1};
    hipError_t e = spd_inverse_sweep(count, As, Ss, Ls, nr, &ws.S->gjflag, ws.gbar, gbase, st);
    gbase += gj_barriers(nr, count);
    return e;
  };
  LK_TRY(hipMemsetAsync(ws.S->cnt, 0, sizeof(ws.S->cnt), st));
  CccpState hs;
  const int qgrid = (nr + 3) / 4;
  const size_t mbq = (size_t)nr * nr * sizeof(double);
  int nsq = gemm_pick_split(nr, nr, nr, ws.part_cap);
  if (nsq > 4) nsq = 4;
  for (int t = 0; t < o.max_iter; ++t) {
    if (t > 0 || warm) {
      // q_k = (M^{-1} C)_kk / (a w_k) from the solve M X = C: the blocked
      // Gauss-Jordan inverse Minv of M is accurate in norm, but the diagonal of
      // Minv C cancels (it is 1 - (b/a) Minv_kk / w_k), so the solve is refined
      // twice with Minv as the approximate inverse (X <- X + Minv (C - M X)),
      // which brings q to the accuracy of a direct solve of M X = C
      cccp_build_m_kernel<<<ew_grid((int64_t)nr * nr), kT, 0, st>>>(ws.C, ws.w, ws.S, ws.M, nr);
      LK_CHECK_LAUNCH();
      LK_TRY(hipMemcpyAsync(ws.Yi, ws.M, mbq, hipMemcpyDeviceToDevice, st));
      LK_TRY(inverse(1, ws.M, nullptr, &ws.S->ld_y, nullptr));
      LK_TRY(gemm_f64(nr, nr, nr, ws.M, nr, 1, ws.C, nr, 1, ws.Zi, nr, 1.0, nullptr, 0.0, ws.part, nsq, st));
      for (int rs = 0; rs < 2; ++rs) {
        LK_TRY(hipMemcpyAsync(ws.Gs, ws.C, mbq, hipMemcpyDeviceToDevice, st));
        LK_TRY(gemm_f64(nr, nr, nr, ws.Yi, nr, 1, ws.Zi, nr, 1, ws.Gs, nr, -1.0, nullptr, 1.0, ws.part, nsq, st));
        if (rs == 1) break;
        LK_TRY(gemm_f64(nr, nr, nr, ws.M, nr, 1, ws.Gs, nr, 1, ws.Zi, nr, 1.0, nullptr, 1.0, ws.part, nsq, st));
      }
      cccp_q_refined_kernel<<<qgrid, 256, 0, st>>>(ws.M, ws.Zi, ws.Gs, ws.w, ws.S, ws.q, nr);
    } else {
      cccp_q_kernel<<<qgrid, 256, 0, st>>>(ws.M, ws.C, ws.w, ws.S, ws.q, nr, 1);
    }
    LK_CHECK_LAUNCH();
    cccp_update_kernel<<<1, 1024, 0, st>>>(ws.C, ws.q, ws.w, ws.wnew, ws.S, nr, (double)n, o.gamma, o.rho, o.eps,
                                           o.tol, o.max_iter);
    LK_CHECK_LAUNCH();
    LK_TRY(hipMemcpyAsync(&hs, ws.S, sizeof(hs), hipMemcpyDeviceToHost, st));
    LK_TRY(hipStreamSynchronize(st));
    if (hs.gjflag) return LAKER_EBREAKDOWN;
    if (hs.done) break;
  }
  if (hs.done == 2) return LAKER_EBREAKDOWN;
  if (stats) stats->cccp_iters = hs.iters;
  if (on != nullptr) {
    cccp_save_kernel<<<1, 256, 0, st>>>(ws.S, ws.w, on->w, on->ab, nr);
    LK_CHECK_LAUNCH();
  }
  // 6. B and R = b I + B^T B; coupled Newton-Schulz iteration on R / c
  //    (c = ||R||_F, so the spectrum lies in (0, 1]):
  //      P = Z Y,  T = (3 I - P) / 2,  Y <- Y T,  Z <- T Z,
  //    with Y -> (R/c)^{1/2} and Z -> (R/c)^{-1/2}; GEMMs only.
  const int nrp = pad_nr(nr);
  make_b_kernel<<<ew_grid(n * nrp), kT, 0, st>>>(ws.U, ws.w, ws.S, L.B64, n, nr, nrp);
  LK_CHECK_LAUNCH();
  const int sq_grid = (int)std::min<int64_t>(kMaxBlocks, ((int64_t)nr * nr + kT * 4 - 1) / (kT * 4));
  sq_init_kernel<<<sq_grid, kT, 0, st>>>(ws.C, ws.w, ws.S, ws.Y, ws.Zm, nr, ws.bpart);
  LK_CHECK_LAUNCH();
  sq_scale_kernel<<<ew_grid((int64_t)nr * nr), kT, 0, st>>>(ws.Y, ws.S, 0, nr * nr);
  LK_CHECK_LAUNCH();
  {
    double* yc = ws.Y;
    double* zc = ws.Zm;
    double* y2 = ws.Zi;
    double* z2 = ws.M;
    double* pt = ws.Yi;
    int nsq = gemm_pick_split(nr, nr, nr, ws.part_cap);
    if (nsq > 4) nsq = 4;
    double prev_change = 1e300;
    for (int it = 0; it < 100; ++it) {
      LK_TRY(gemm_f64(nr, nr, nr, zc, nr, 1, yc, nr, 1, pt, nr, 1.0, nullptr, 0.0, ws.part, nsq, st));
      sq_t_kernel<<<sq_grid, kT, 0, st>>>(pt, ws.S, nr, ws.bpart);
      LK_CHECK_LAUNCH();
      LK_TRY(gemm_f64(nr, nr, nr, yc, nr, 1, pt, nr, 1, y2, nr, 1.0, nullptr, 0.0, ws.part, nsq, st));
      LK_TRY(gemm_f64(nr, nr, nr, pt, nr, 1, zc, nr, 1, z2, nr, 1.0, nullptr, 0.0, ws.part, nsq, st));
      std::swap(yc, y2);
      std::swap(zc, z2);
      LK_TRY(hipMemcpyAsync(&hs, ws.S, sizeof(hs), hipMemcpyDeviceToHost, st));
      LK_TRY(hipStreamSynchronize(st));
      if (!(hs.db_change == hs.db_change)) return LAKER_EBREAKDOWN;
      // quadratic convergence to rounding level, or stagnation there
      if (hs.db_change <= 1e-14) break;
      if (hs.db_change <= 1e-10 && hs.db_change >= 0.5 * prev_change) break;
      prev_change = hs.db_change;
    }
    // R^{1/2} = sqrt(c) Y into ws.Y, R^{-1/2} = Z / sqrt(c) into ws.Zm
    const size_t mb = (size_t)nr * nr * sizeof(double);
    if (yc != ws.Y) LK_TRY(hipMemcpyAsync(ws.Y, yc, mb, hipMemcpyDeviceToDevice, st));
    if (zc != ws.Zm) LK_TRY(hipMemcpyAsync(ws.Zm, zc, mb, hipMemcpyDeviceToDevice, st));
    sq_scale_kernel<<<ew_grid((int64_t)nr * nr), kT, 0, st>>>(ws.Y, ws.S, 1, nr * nr);
    LK_CHECK_LAUNCH();
    sq_scale_kernel<<<ew_grid((int64_t)nr * nr), kT, 0, st>>>(ws.Zm, ws.S, 2, nr * nr);
    LK_CHECK_LAUNCH();
  }
  // 7. Gs = -b^{-1/2} Zm (sqrt(b) I + Y)^{-1}
  add_sqrtb_diag_kernel<<<ew_grid((int64_t)nr * nr), kT, 0, st>>>(ws.Y, ws.S, ws.M, nr);
  LK_CHECK_LAUNCH();
  LK_TRY(inverse(1, ws.M, nullptr, &ws.S->ld_y, nullptr));
  write_header_kernel<<<1, 64, 0, st>>>(ws.S, L.hdr);
  LK_CHECK_LAUNCH();
  {
    int ns = gemm_pick_split(nr, nr, nr, ws.part_cap);
    LK_TRY(gemm_f64(nr, nr, nr, ws.Zm, nr, 1, ws.M, nr, 1, ws.Gs, nr, -1.0, L.hdr, 0.0, ws.part, ns, st));
  }
  // 8. Bt = B Gs; float32 copies
  {
    int ns = gemm_pick_split(n, nr, nr, ws.part_cap);
    LK_TRY(hipMemsetAsync(L.Bt64, 0, sizeof(double) * n * nrp, st));
    LK_TRY(gemm_f64(n, nr, nr, L.B64, nrp, 1, ws.Gs, nr, 1, L.Bt64, nrp, 1.0, nullptr, 0.0, ws.part, ns, st));
  }
  to_f32_kernel<<<ew_grid(n * nrp), kT, 0, st>>>(L.B64, L.B32, n * nrp);
  LK_CHECK_LAUNCH();
  to_f32_kernel<<<ew_grid(n * nrp), kT, 0, st>>>(L.Bt64, L.Bt32, n * nrp);
  LK_CHECK_LAUNCH();
  LK_TRY(hipMemcpyAsync(&hs, ws.S, sizeof(hs), hipMemcpyDeviceToHost, st));
  LK_TRY(hipStreamSynchronize(st));
  if (hs.gjflag) return LAKER_EBREAKDOWN;
  return LAKER_OK;   // a CCCP iterate stopped at max_iter still gives an SPD preconditioner
}

laker_status fit_jacobi(const Problem& pb, const PrecondLayout& L, hipStream_t st) {
  jacobi_kernel<<<ew_grid(pb.n), kT, 0, st>>>(pb.E, pb.n, pb.d, pb.scale, pb.lambda, L.dinv64);
  LK_CHECK_LAUNCH();
  return LAKER_OK;
}

}  // namespace lk
