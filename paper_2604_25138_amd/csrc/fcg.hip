// Flexible conjugate gradients in float64 around a reduced-precision inner PCG.
//
// The method's solve (Alg. 1) runs inside: each outer step takes the inner
// PCG's approximate solution z of (lambda I + G) z = r, computed with bfloat16
// or float32 score tiles, as its preconditioned residual.  Because the inner
// solve changes from step to step, the direction is made conjugate to the
// previous one explicitly (flexible CG with one stored direction):
//     beta = -(z^T q_prev) / (p_prev^T q_prev),   p = z + beta p_prev,
//     q = (lambda I + G) p   (float64 product),
//     gamma = p^T r / p^T q,  alpha += gamma p,  r -= gamma q.
// Compared with plain refinement (alpha += z), the float64 outer Krylov
// recurrence also resolves the directions where the reduced-precision product
// is no longer accurate (lambda far below its rounding relative to ||G||),
// where refinement stalls or diverges.
#include <math.h>

#include "internal.hpp"
#include "pcg.hpp"

namespace lk {

namespace {

constexpr int kT = 256;

inline int blocks_for(int64_t n) {
  int64_t g = (n + kT - 1) / kT;
  if (g > kMaxBlocks) g = kMaxBlocks;
  return (int)(g < 1 ? 1 : g);
}

// out[0] = a1^T b1, out[1] = a2^T b2 (fixed-order reduction, last block finishes)
__global__ __launch_bounds__(kT) void dot2_kernel(const double* __restrict__ a1, const double* __restrict__ b1,
                                                  const double* __restrict__ a2, const double* __restrict__ b2,
                                                  int64_t n, double* __restrict__ part, unsigned* cnt,
                                                  double* __restrict__ out) {
  __shared__ double sh[16];
  double s1 = 0.0, s2 = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    s1 = fma(a1[i], b1[i], s1);
    s2 = fma(a2[i], b2[i], s2);
  }
  s1 = block_sum(s1, sh);
  s2 = block_sum(s2, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s1;
    part[kMaxBlocks + blockIdx.x] = s2;
  }
  if (last_block_arrived(cnt)) {
    const double t1 = ordered_sum(part, gridDim.x, sh);
    const double t2 = ordered_sum(part + kMaxBlocks, gridDim.x, sh);
    if (threadIdx.x == 0) {
      out[0] = t1;
      out[1] = t2;
      *cnt = 0;
    }
  }
}

// The outer scalars stay on the device, s = 4 doubles: s[0], s[1] the last
// dot2 results, s[2] = p_prev^T q_prev, s[3] = 1 after a breakdown.  The host
// reads them once per outer step, with ||r||^2.

// Truncated flexible CG keeps the last m directions: the new direction is z
// made A-conjugate to each of them,
//   p = z - sum_i (z^T q_i) / (p_i^T q_i) p_i,
// with the pairs (p_i, q_i = A p_i) in a ring of kFcgHist slots and
// p_i^T q_i in pq[slot].  dz[i] = z^T q_(slot i) for the c slots listed.
struct FcgSlots {
  int c;
  int slot[kFcgHist];
};

__global__ __launch_bounds__(kT) void mdot_kernel(const double* __restrict__ z, const double* __restrict__ Qr,
                                                  FcgSlots sl, int64_t n, double* __restrict__ part, unsigned* cnt,
                                                  double* __restrict__ dz) {
  __shared__ double sh[16];
  double acc[kFcgHist];
#pragma unroll
  for (int i = 0; i < kFcgHist; ++i) acc[i] = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < n; j += (int64_t)gridDim.x * kT) {
    const double zj = z[j];
#pragma unroll
    for (int i = 0; i < kFcgHist; ++i)
      if (i < sl.c) acc[i] = fma(zj, Qr[(int64_t)sl.slot[i] * n + j], acc[i]);
  }
#pragma unroll
  for (int i = 0; i < kFcgHist; ++i) {
    if (i < sl.c) {
      const double v = block_sum(acc[i], sh);
      if (threadIdx.x == 0) part[(int64_t)i * kMaxBlocks + blockIdx.x] = v;
    }
  }
  if (last_block_arrived(cnt)) {
    for (int i = 0; i < sl.c; ++i) {
      const double t = ordered_sum(part + (int64_t)i * kMaxBlocks, gridDim.x, sh);
      if (threadIdx.x == 0) dz[i] = t;
    }
    if (threadIdx.x == 0) *cnt = 0;
  }
}

// p = z - sum_i dz[i] / pq[slot i] p_(slot i)
__global__ void pdir_m_kernel(const double* __restrict__ z, const double* __restrict__ Pr, FcgSlots sl,
                              const double* __restrict__ dz, const double* __restrict__ pq, double* __restrict__ p,
                              int64_t n) {
  double cf[kFcgHist];
#pragma unroll
  for (int i = 0; i < kFcgHist; ++i) cf[i] = i < sl.c ? dz[i] / pq[sl.slot[i]] : 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < n; j += (int64_t)gridDim.x * kT) {
    double v = z[j];
#pragma unroll
    for (int i = 0; i < kFcgHist; ++i)
      if (i < sl.c) v = fma(-cf[i], Pr[(int64_t)sl.slot[i] * n + j], v);
    p[j] = v;
  }
}

__global__ void store_pq_kernel(const double* __restrict__ s, double* __restrict__ pq, int slot) {
  if (threadIdx.x == 0 && blockIdx.x == 0 && s[3] == 0.0) pq[slot] = s[2];
}

// p = z + beta p, beta = -(z^T q_prev) / (p_prev^T q_prev) = -s[0] / s[2]
__global__ void pdir_kernel(const double* __restrict__ z, double* __restrict__ p, const double* __restrict__ s,
                            int64_t n) {
  const double beta = -s[0] / s[2];
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT)
    p[i] = fma(beta, p[i], z[i]);
}

// gamma = p^T r / p^T q (s[1] / s[0]); alpha += gamma p; r -= gamma q; s[2] =
// p^T q.  p^T q <= 0 or a non-finite p^T r: nothing is updated and s[3] = 1.
__global__ void step_kernel(double* __restrict__ alpha, double* __restrict__ r, const double* __restrict__ p,
                            const double* __restrict__ q, double* __restrict__ s, int64_t n) {
  const double pq = s[0], pr = s[1];
  if (!(pq > 0.0) || !isfinite(pr)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) s[3] = 1.0;
    return;
  }
  const double gamma = pr / pq;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
    alpha[i] = fma(gamma, p[i], alpha[i]);
    r[i] = fma(-gamma, q[i], r[i]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) s[2] = pq;
}

}  // namespace

laker_status fcg_run(const Problem& pb, const SolveWs& W, const PrecondView& P, const double* y, double* alpha,
                     const laker_pcg_opts& o, int check, laker_stats* sp, hipStream_t st) {
  const int64_t n = pb.n;
  const int g = blocks_for(n);
  double* r = W.rout;
  double* z = W.dalpha;
  double* p = W.fp;
  double* q = W.fq;
  double* s = W.misc + 8;
  auto dots_dev = [&](const double* a1, const double* b1, const double* a2, const double* b2) -> hipError_t {
    dot2_kernel<<<g, kT, 0, st>>>(a1, b1, a2, b2, n, W.bpart, W.cnt, s);
    return hipGetLastError();
  };
  auto dots = [&](const double* a1, const double* b1, const double* a2, const double* b2, double* h) -> hipError_t {
    hipError_t e = dots_dev(a1, b1, a2, b2);
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(h, s, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  };
  // q = (lambda I + G) p in float64
  const KmvPlan pl = kmv_plan_square(n, pb.dp, LAKER_F64);
  auto product = [&](const double* v, double* out) -> hipError_t {
    KmvArgs A = kmv_args(W.e64, n, W.e64, n, v, W);
    A.lam = pb.lambda;
    A.pself = v;
    A.out = out;
    return kmv_run(LAKER_F64, pb.dp, pl, A, st);
  };

  // directions kept by the truncated flexible CG (1: the previous one only)
  int hist = o.outer_history > 0 ? o.outer_history : 1;
  if (hist > kFcgHist) hist = kFcgHist;
  if (!o.warm_start) LK_TRY(hipMemsetAsync(alpha, 0, sizeof(double) * n, st));
  double rel = 0.0;
  laker_status e = true_residual(pb, W, y, alpha, r, &rel, o.warm_start != 0, st);
  if (e != LAKER_OK) return e;
  double h[4];
  LK_TRY(hipMemsetAsync(s, 0, 4 * sizeof(double), st));
  LK_TRY(dots(y, y, y, y, h));
  const double ynorm = sqrt(h[0]);
  sp->ir_relres[0] = rel;
  sp->relres_true = rel;
  sp->relres = rel;
  sp->ir_steps = 0;
  if (rel <= o.tol) return LAKER_OK;
  int used = 0;
  const int inner_cap = o.inner_max_iter > 0 ? o.inner_max_iter : o.max_iter;
  StallTest stall;
  stall.window = o.stall_window;
  (void)stall.stalled(0, rel);
  // Inner arithmetic: the requested precision; with o.escalate made finer
  // (bfloat16 -> float32 -> float64) when the outer residual has not halved
  // over the last kEscalateSteps outer steps.  Near the float64 floor of the reduced
  // product, the inner solves no longer resolve the directions where its
  // rounding exceeds lambda, and only finer inner products make progress.
  constexpr int kEscalateSteps = 40;
  int prec_now = o.precision;
  StallTest slow;
  slow.window = kEscalateSteps;
  (void)slow.stalled(0, rel);
  for (int k = 0; k < o.ir_max; ++k) {
    if (used >= o.max_iter) break;
    // z = inner solve of A z = r; a reduced-precision breakdown or cap keeps
    // the z it has
    laker_stats inner{};
    int cap = o.max_iter - used;
    if (cap > inner_cap) cap = inner_cap;
    const double itol = fmax(o.inner_tol, 0.5 * o.tol / rel);
    // (a single chunk is only enqueued; its iteration count is read with the
    // step's scalars below, saving a host round trip per outer step)
    const bool defer = check >= cap && !o.graph && !o.profile;
    laker_status ri = pcg_run(pb, W, P, r, z, false, itol, cap, check, prec_now, o.graph != 0, o.profile != 0,
                              &inner, st, defer);
    if (ri == LAKER_EHIP || ri == LAKER_EINVAL) return ri;
    if (!defer) {
      used += inner.iters;
      sp->iters = used;
    }
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
    // p = z + beta p_prev, beta = -(z^T q_prev) / (p_prev^T q_prev)
    // (beta, gamma and the breakdown test on the device: one host read per step)
    double* pk = p;
    double* qk = q;
    if (hist == 1) {
      if (k == 0) {
        LK_TRY(hipMemcpyAsync(p, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      } else {
        LK_TRY(dots_dev(z, q, z, q));
        pdir_kernel<<<g, kT, 0, st>>>(z, p, s, n);
        LK_CHECK_LAUNCH();
      }
    } else {
      // the last min(k, hist) directions, oldest first, from the ring
      const int slot = k % hist;
      pk = W.fring + (int64_t)slot * n;
      qk = W.fring + (int64_t)(kFcgHist + slot) * n;
      FcgSlots sl{};
      sl.c = k < hist ? k : hist;
      for (int i = 0; i < sl.c; ++i) sl.slot[i] = (k - sl.c + i) % hist;
      if (sl.c == 0) {
        LK_TRY(hipMemcpyAsync(pk, z, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      } else {
        mdot_kernel<<<g, kT, 0, st>>>(z, W.fring + (int64_t)kFcgHist * n, sl, n, W.fpart, W.cnt, W.fdz);
        LK_CHECK_LAUNCH();
        pdir_m_kernel<<<g, kT, 0, st>>>(z, W.fring, sl, W.fdz, W.fpq, pk, n);
        LK_CHECK_LAUNCH();
      }
    }
    LK_TRY(product(pk, qk));
    LK_TRY(dots_dev(pk, qk, pk, r));
    step_kernel<<<g, kT, 0, st>>>(alpha, r, pk, qk, s, n);
    LK_CHECK_LAUNCH();
    if (hist > 1) {
      store_pq_kernel<<<1, 64, 0, st>>>(s, W.fpq, k % hist);
      LK_CHECK_LAUNCH();
    }
    // ||r||^2, the scalars and (deferred inner solve) its iteration count in one host read
    int inner_iters = 0;
    LK_TRY(dots_dev(r, r, r, r));
    if (defer) LK_TRY(hipMemcpyAsync(&inner_iters, &W.S->iters, sizeof(int), hipMemcpyDeviceToHost, st));
    LK_TRY(hipMemcpyAsync(h, s, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
    LK_TRY(hipStreamSynchronize(st));
    if (defer) {
      used += inner_iters;
      sp->iters = used;
    }
    if (h[3] != 0.0) return LAKER_EBREAKDOWN;
    rel = ynorm > 0.0 ? sqrt(h[0]) / ynorm : 0.0;
    if (k + 1 < 64) sp->ir_relres[k + 1] = rel;
    sp->ir_steps = k + 1;
    sp->relres = rel;
    if (rel <= o.tol) {
      // confirm on the true residual (and continue from it if the recursion drifted)
      double rt = 0.0;
      e = true_residual(pb, W, y, alpha, r, &rt, true, st);
      if (e != LAKER_OK) return e;
      sp->relres_true = rt;
      rel = rt;
      if (rt <= o.tol) return LAKER_OK;
    }
    sp->relres_true = rel;
    if (stall.stalled(used, rel)) return LAKER_ESTALL;
    if (o.escalate && slow.stalled(k + 1, rel) && prec_now != LAKER_F64) {
      prec_now = prec_now == LAKER_BF16 ? LAKER_F32 : LAKER_F64;
      sp->escalations += 1;
      if (prec_now == LAKER_F32) LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, LAKER_F32, W.e32, st));
      slow.n = 0;
      (void)slow.stalled(k + 1, rel);
    }
  }
  double rt = 0.0;
  e = true_residual(pb, W, y, alpha, nullptr, &rt, true, st);
  if (e != LAKER_OK) return e;
  sp->relres_true = rt;
  return rt <= o.tol ? LAKER_OK : LAKER_ENOCONV;
}

}  // namespace lk
