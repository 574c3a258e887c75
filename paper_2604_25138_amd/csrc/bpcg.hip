// Batched PCG: many independent maps of uneven size solved together.
//
// Every pass of an iteration is one launch for the whole batch: the kernel
// products of all maps run as one grid of (map, row block, column range) tiles
// from a table (tiles in a fixed order, optionally arranged so that each XCD
// works through its own contiguous stretch of the table and keeps the key rows
// of its column ranges in its own L2), and the vector passes run on a grid
// whose row y is the map.  Each map keeps its own scalars; a map that has
// converged (or retired from the outer refinement) makes every later pass of
// its row return at once, so maps retire at their own tolerance.  The chunk of
// iterations between host checks can be captured into a HIP graph and
// replayed.  The per-block bodies are the ones of the single-map solver, with
// the same block counts, so a map gives bitwise the same iterates in a batch as
// alone when the product uses the single-map column ranges.
#include "bpcg.hpp"

#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "pcg_body.hpp"

namespace lk {

namespace {

using namespace pcgk;

// ---- batched passes (grid: x = blocks of the largest map, y = entry of the map
// list R: the maps a pass works on) ----

__global__ __launch_bounds__(kThreads) void b_zero_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if (!d.active) return;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * kThreads)
    d.x[i] = 0.0;
}

__global__ __launch_bounds__(kThreads) void b_init_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if (!d.active || (int)blockIdx.x >= d.g) return;
  pcg_init_body(blockIdx.x, d.g, d.rhs, nullptr, d.r, d.p, d.n, d.yyp, d.rrp);
}

__global__ __launch_bounds__(kThreads) void b_start_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if (!d.active) return;
  pcg_start_body(0, 1, d.S, d.yyp, d.rrp, d.g, d.tol, d.max_iter);
}

// (maps with a symmetric product skip this pass: their product kernel forms
// p^T A p and the step update adds the partials, as in the single solver)
__global__ __launch_bounds__(kThreads) void b_ap_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if ((int)blockIdx.x >= d.g || d.ps.sym) return;
  const PartSum ps = d.ps;
  pcg_ap_body(blockIdx.x, d.g, d.p, d.part, ps, d.Ap, d.n, d.lam, d.papp, d.S);
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void b_update_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if ((int)blockIdx.x >= d.g) return;
  const PartSum ps = d.ps;
  pcg_update_body<KIND>(blockIdx.x, d.g, d.x, d.r, d.p, ps.sym ? nullptr : d.Ap, d.part, ps, d.lam, d.dinv, d.th, d.n,
                        d.S, d.papp, ps.sym ? ps.sp.grid : d.g, d.rrp, d.rzp);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void b_update_t_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if ((int)blockIdx.x >= d.nbt) return;
  const PartSum ps = d.ps;
  pcg_update_t_body<MT>(blockIdx.x, d.nbt, d.x, d.r, d.p, ps.sym ? d.th : nullptr, ps.sym ? nullptr : d.Ap, d.part, ps,
                        d.lam, (const MT*)d.B, d.nrp, d.n, d.S, d.papp, ps.sym ? ps.sp.grid : d.g, d.rrp, d.tpart);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void b_lr_t_partial_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if (!d.active || (int)blockIdx.x >= d.nbt) return;
  lr_t_partial_body<MT>(blockIdx.x, d.nbt, (const MT*)d.B, d.r, d.n, d.nrp, d.tpart, d.S);
}

__global__ __launch_bounds__(kThreads) void b_lr_t_finish_kernel(const BDesc* __restrict__ D, const int* __restrict__ R, int decide, int masked) {
  const BDesc& d = D[R[blockIdx.y]];
  const int nb = (d.nrp + 15) / 16;
  if ((masked && !d.active) || (int)blockIdx.x >= nb) return;
  if (lr_fused_t(d.n, d.nrp)) {
    // t in the single solver's fused order, by one block (see lr_t_finish_fused_order_body)
    if (blockIdx.x == 0) lr_t_finish_fused_order_body(d.tpart, d.nbt, d.nrp, d.t, d.S, decide ? d.rrp : nullptr, d.nbt);
    return;
  }
  lr_t_finish_body(blockIdx.x, nb, d.tpart, d.nbt, d.nrp, d.t, d.S, decide ? d.rrp : nullptr, d.nbt);
}

template <typename MT>
__global__ __launch_bounds__(kThreads) void b_lr_apply_kernel(const BDesc* __restrict__ D, const int* __restrict__ R, int masked,
                                                              int decide) {
  const BDesc& d = D[R[blockIdx.y]];
  if ((masked && !d.active) || (int)blockIdx.x >= d.ga) return;
  // (rows and r^T theta partials as the single solver's fused apply, t from the
  // preceding pass in the same order: the iterates stay bitwise equal)
  if (lr_fused_t(d.n, d.nrp))
    lr_apply_t_body<MT>(blockIdx.x, d.tpart, d.nbt, (const MT*)d.Bt, d.r, d.th, d.n, d.nrp, d.c0p, d.dinv, d.S,
                        nullptr, 0, d.rzp, d.t);
  else
    lr_apply_body<MT>(blockIdx.x, d.ga, (const MT*)d.Bt, d.t, d.r, d.th, d.n, d.nrp, d.c0p, d.dinv, d.S, d.rzp);
}

__global__ __launch_bounds__(kThreads) void b_jacobi_apply_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if (!d.active || (int)blockIdx.x >= d.g) return;
  jacobi_apply_body(blockIdx.x, d.g, d.r, d.dinv, d.th, d.n, d.S, d.rzp);
}

template <int KIND>
__global__ __launch_bounds__(kThreads) void b_pupdate_kernel(const BDesc* __restrict__ D, const int* __restrict__ R, int init, int masked) {
  const BDesc& d = D[R[blockIdx.y]];
  if ((masked && !d.active) || (int)blockIdx.x >= d.g) return;
  // low-rank maps with a symmetric product conjugate inside the product kernel
  if (KIND == LAKER_PRECOND_CCCP && d.ps.sym) return;
  const double* src = KIND == LAKER_PRECOND_NONE ? d.r : d.th;
  const int grz = KIND == LAKER_PRECOND_CCCP ? d.ga : d.g;
  pcg_pupdate_body<KIND>(blockIdx.x, d.g, init, src, d.p, d.n, d.S, d.rrp, d.g, d.rzp, grz);
}

__global__ __launch_bounds__(kThreads) void b_resid_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if (!d.active || (int)blockIdx.x >= d.g) return;
  resid_body(blockIdx.x, d.g, d.y, d.have_alpha ? d.w64 : nullptr, d.rout, d.n, d.bpart, d.cnt, d.misc);
}

__global__ __launch_bounds__(kThreads) void b_axpy_kernel(const BDesc* __restrict__ D, const int* __restrict__ R) {
  const BDesc& d = D[R[blockIdx.y]];
  if (!d.active || (int)blockIdx.x >= d.g) return;
  axpy_body(blockIdx.x, d.g, d.alpha, d.x, d.n);
}

// scalars of every map, and the outer residual norms, gathered for one copy
__global__ void b_gather_kernel(const BDesc* __restrict__ D, int count, PcgScalars* __restrict__ hs,
                                double* __restrict__ misc) {
  for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < count; b += gridDim.x * blockDim.x) {
    hs[b] = *D[b].S;
    misc[2 * b] = D[b].misc[0];
    misc[2 * b + 1] = D[b].misc[1];
  }
}

// ---- host helpers ----

struct Plan1 {
  int rowblocks;
  int nsplit;
  int64_t cps;
};

Plan1 plan_for(int64_t n, int prec, int cps) {
  Plan1 p;
  const int rpb = kmv_rows_per_block(prec);
  p.rowblocks = (int)((n + rpb - 1) / rpb);
  if (cps <= 0) {
    KmvPlan k = kmv_plan(n, n, prec);
    p.nsplit = k.nsplit;
    p.cps = k.cols_per_split;
  } else {
    p.cps = cps;
    p.nsplit = (int)((n + cps - 1) / cps);
  }
  return p;
}

// Tiles (map, row block, column range), map-major then column range then row
// block; with xcd, block b takes entry (b % 8) * (T / 8) + b / 8 of that list
// (T padded to a multiple of 8 with empty tiles), so the blocks an XCD receives
// (every 8th block id) walk one contiguous stretch of the list.
std::vector<int> build_tiles(int count, const std::vector<Plan1>& pl, const std::vector<int>& use, bool xcd) {
  std::vector<int> L;
  for (int b = 0; b < count; ++b) {
    if (!use[b]) continue;
    for (int sp = 0; sp < pl[b].nsplit; ++sp)
      for (int rb = 0; rb < pl[b].rowblocks; ++rb) {
        L.push_back(b);
        L.push_back(rb);
        L.push_back(sp);
      }
  }
  if (!xcd) return L;
  const int64_t T = (int64_t)L.size() / 3;
  const int64_t T8 = (T + 7) / 8 * 8;
  const int64_t per = T8 / 8;
  std::vector<int> out((size_t)T8 * 3, -1);
  for (int64_t blk = 0; blk < T8; ++blk) {
    const int64_t src = (blk % 8) * per + blk / 8;
    if (src < T) {
      out[3 * blk + 0] = L[3 * src + 0];
      out[3 * blk + 1] = L[3 * src + 1];
      out[3 * blk + 2] = L[3 * src + 2];
    }
  }
  return out;
}

int max_of(const std::vector<BDesc>& h, int BDesc::*f) {
  int m = 1;
  for (const BDesc& d : h) m = std::max(m, d.*f);
  return m;
}

// Autotuned column-range length per (precision, dp, size class, maps in the
// class); chosen by timing one product sweep of the class for each candidate.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int64_t>, int> g_tuned;

}  // namespace

size_t plan_batch_ws(int count, const int64_t* n, int d, size_t* offsets, void* base, BatchWs* out) {
  WsCarver c(base);
  for (int b = 0; b < count; ++b) {
    const size_t bytes = plan_solve_ws(nullptr, n[b], d, 0).total;
    unsigned char* p = c.take<unsigned char>(bytes);
    if (offsets) offsets[b] = base ? (size_t)(p - (unsigned char*)base) : 0;
  }
  BatchWs w{};
  int64_t tiles = 0;
  for (int b = 0; b < count; ++b) {
    // the most tiles a map can produce: float32/bfloat16 rows of 128, float64
    // rows of 64, at most kMaxSplit column ranges
    tiles += ((n[b] + 63) / 64) * kMaxSplit;
  }
  tiles += 32;
  w.desc = c.take<BDesc>(count);
  w.inner = c.take<KmvArgs>(count);
  w.outer = c.take<KmvArgs>(count);
  w.tiles_in = c.take<int>((size_t)tiles * 3);
  w.tiles_out = c.take<int>((size_t)tiles * 3);
  w.run_it = c.take<int>(count);
  w.run_op = c.take<int>(count);
  w.hs = c.take<PcgScalars>(count);
  w.misc = c.take<double>((size_t)2 * count);
  w.plans = c.take<SymPlan>(count);
  w.sym_list = c.take<int>(count);
  w.total = c.bytes();
  if (out) *out = w;
  return w.total;
}

laker_status pcg_batch(int count, const Problem* pbs, const SolveWs* wss, const PrecondView* Ps,
                       const double* const* y, double* const* alpha, const laker_pcg_opts& o, const BatchOpts& bo,
                       const BatchWs& bw, laker_stats* stats, int* cps_used, hipStream_t st) {
  const int prec = o.precision;
  const int kind = Ps[0].kind;
  const int f32 = Ps[0].f32;
  const int dp = pbs[0].dp;
  const bool lowrank = kind == LAKER_PRECOND_CCCP || kind == LAKER_PRECOND_LEARNED;
  const bool xcd = bo.xcd_order != 0;
  const int check = o.check_every > 0 ? o.check_every : 16;

  // per-map descriptors
  std::vector<BDesc> hd(count);
  int64_t max_n = 1;
  for (int b = 0; b < count; ++b) {
    const Problem& pb = pbs[b];
    const SolveWs& w = wss[b];
    BDesc& d = hd[b];
    d = BDesc{};
    d.n = pb.n;
    d.lam = pb.lambda;
    d.g = red_blocks(pb.n);
    // blocks of the preconditioner apply (one r^T theta partial each)
    d.ga = lowrank && lr_fused_t(pb.n, Ps[b].nrp) ? (int)((pb.n + kTRows - 1) / kTRows) : apply_blocks(pb.n);
    d.nbt = (int)((pb.n + kTRows - 1) / kTRows);
    d.S = w.S;
    d.r = w.r;
    d.p = w.p;
    d.Ap = w.ap;
    d.th = w.theta;
    d.part = w.part;
    d.yyp = w.yyp;
    d.rrp = w.rrp;
    d.rzp = w.rzp;
    d.papp = w.papp;
    d.tpart = w.tpart;
    d.t = w.t;
    d.B = Ps[b].B;
    d.Bt = Ps[b].Bt;
    d.c0p = Ps[b].c0p;
    d.dinv = (const double*)Ps[b].dinv;
    d.nrp = lowrank ? Ps[b].nrp : 4;
    d.y = y[b];
    d.alpha = alpha[b];
    d.rout = w.rout;
    d.w64 = w.w64;
    d.bpart = w.bpart;
    d.cnt = w.cnt;
    d.misc = w.misc;
    d.active = 1;
    max_n = std::max<int64_t>(max_n, pb.n);
    LK_TRY(hipMemsetAsync(w.S, 0, sizeof(PcgScalars), st));
    LK_TRY(hipMemsetAsync(w.cnt, 0, 16 * sizeof(unsigned), st));
    LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, LAKER_F64, w.e64, st));
    if (w.kmat64 != nullptr) LK_TRY(kmat_build(pb.dp, w.e64, pb.n, LAKER_F64, w.kmat64, st));
    if (prec != LAKER_F64)
      LK_TRY(prep_embed(pb.E, pb.n, pb.d, pb.dp, pb.scale, prec, prec == LAKER_F32 ? (void*)w.e32 : (void*)w.e16, st));
  }

  // column ranges of the inner products: the single-map plan, a given length,
  // or autotuned per size class (maps with the same floor(log2 n)): the product
  // of the class's largest map is timed for each candidate length
  std::vector<KmvArgs> hin(count), hout(count);
  std::vector<int> cps_map(count, bo.cps > 0 ? bo.cps : 0);
  if (bo.cps < 0) {
    std::map<int, std::vector<int>> classes;
    for (int b = 0; b < count; ++b) {
      int c = 0;
      while ((int64_t(1) << (c + 1)) <= pbs[b].n) ++c;
      classes[c].push_back(b);
    }
    hipEvent_t e0, e1;
    LK_TRY(hipEventCreate(&e0));
    LK_TRY(hipEventCreate(&e1));
    for (auto& kv : classes) {
      const std::vector<int>& members = kv.second;
      const auto key = std::make_tuple(prec, dp, kv.first, (int64_t)members.size());
      {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
          for (int b : members) cps_map[b] = it->second;
          continue;
        }
      }
      const int cands[] = {0, 512, 1024, 2048, 4096};
      float best = 1e30f;
      int best_c = 0;
      for (int cand : cands) {
        bool ok = true;
        for (int b : members)
          if (cand > 0 && (pbs[b].n + cand - 1) / cand > kMaxSplit) ok = false;
        if (!ok) continue;
        // timed on the class's largest map alone: the refinement's tail, where
        // a few large maps run by themselves, is where the batch spends its time
        int big = members[0];
        for (int b : members)
          if (pbs[b].n > pbs[big].n) big = b;
        std::vector<Plan1> pl(count);
        std::vector<int> use(count, 0);
        for (int b : {big}) {
          use[b] = 1;
          pl[b] = plan_for(pbs[b].n, prec, cand);
          KmvArgs A = kmv_args(prepared(wss[b], prec), pbs[b].n, prepared(wss[b], prec), pbs[b].n, wss[b].p,
                               wss[b]);
          A.kmat = nullptr;   // the inner products recompute G
          A.mode = 0;
          A.cps = pl[b].cps;
          A.nsplit = pl[b].nsplit;
          hin[b] = A;   // no scalars: nothing skips
        }
        std::vector<int> tl = build_tiles(count, pl, use, xcd);
        const int nt = (int)(tl.size() / 3);
        LK_TRY(hipMemcpyAsync(bw.inner, hin.data(), sizeof(KmvArgs) * count, hipMemcpyHostToDevice, st));
        LK_TRY(hipMemcpyAsync(bw.tiles_in, tl.data(), sizeof(int) * tl.size(), hipMemcpyHostToDevice, st));
        LK_TRY(kmv_run_batch(prec, dp, count, bw.inner, bw.tiles_in, nt, false, max_n, st));
        LK_TRY(hipEventRecord(e0, st));
        for (int rep = 0; rep < 2; ++rep)
          LK_TRY(kmv_run_batch(prec, dp, count, bw.inner, bw.tiles_in, nt, false, max_n, st));
        LK_TRY(hipEventRecord(e1, st));
        LK_TRY(hipEventSynchronize(e1));
        float ms = 0.f;
        LK_TRY(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
          best = ms;
          best_c = cand;
        }
      }
      for (int b : members) cps_map[b] = best_c;
      std::lock_guard<std::mutex> lock(g_tune_mu);
      g_tuned[key] = best_c;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  if (cps_used) {
    int big = 0;
    for (int b = 0; b < count; ++b)
      if (pbs[b].n > pbs[big].n) big = b;
    *cps_used = cps_map[big];
  }

  // per-map inner arithmetic (refinement can make it finer per map) and the
  // product tiles grouped by arithmetic: group q holds the maps computing in
  // precision kPrecOrder[q]
  const int kPrecOrder[3] = {LAKER_BF16, LAKER_F32, LAKER_F64};
  std::vector<int> pm(count, prec);
  int grp_off[3] = {0, 0, 0}, grp_nt[3] = {0, 0, 0};
  // maps whose square product takes the symmetric schedule run the single
  // solver's kernel and plan: the bfloat16 ones of dp = 32, 64 all in one
  // launch (grid row = map), the others one map at a time; the other maps
  // share the tile table
  std::vector<int> sym_in[3];
  std::vector<KmvPlan> sq_in(count);
  std::vector<SymPlan> sym_plans(count);
  const bool sym_batch = kmv_sym16(dp, LAKER_BF16);
  // arguments of every map; tiles only for the maps in `members`
  auto rebuild_inner = [&](const std::vector<int>& members) -> laker_status {
    std::vector<int> in_list(count, 0);
    for (int b : members) in_list[b] = 1;
    std::vector<int> tl_all;
    for (int q = 0; q < 3; ++q) {
      const int pq = kPrecOrder[q];
      std::vector<Plan1> pl(count);
      std::vector<int> use(count, 0);
      sym_in[q].clear();
      for (int b = 0; b < count; ++b) {
        if (pm[b] != pq) continue;
        KmvArgs A = kmv_args(prepared(wss[b], pq), pbs[b].n, prepared(wss[b], pq), pbs[b].n, wss[b].p, wss[b]);
        A.kmat = nullptr;   // the inner products recompute G (a stored G serves the outer residuals)
        A.mode = 0;
        A.S = wss[b].S;
        A.pcg_step = 1;
        sq_in[b] = kmv_plan_square(pbs[b].n, dp, pq);
        if (sq_in[b].sym) {
          if (in_list[b]) sym_in[q].push_back(b);
          hd[b].ps = part_sum(sq_in[b]);
          // (the fields kmv_run fills in, for the batched launch)
          A.cps = sq_in[b].cols_per_split;
          A.nsplit = sq_in[b].nsplit;
          A.ps = part_sum(sq_in[b]);
          sym_plans[b] = sq_in[b].sp;
          A.pap = wss[b].papp;
          A.lam = pbs[b].lambda;
          if (lowrank) {
            A.theta = wss[b].theta;
            A.rzp = wss[b].rzp;
            A.grz = hd[b].ga;
          }
        } else {
          use[b] = in_list[b];
          pl[b] = plan_for(pbs[b].n, pq, pq == prec ? cps_map[b] : 0);
          A.cps = pl[b].cps;
          A.nsplit = pl[b].nsplit;
          hd[b].ps = PartSum{};
          hd[b].ps.nsplit = pl[b].nsplit;
        }
        hin[b] = A;
      }
      std::vector<int> tl = build_tiles(count, pl, use, xcd);
      grp_off[q] = (int)(tl_all.size() / 3);
      grp_nt[q] = (int)(tl.size() / 3);
      tl_all.insert(tl_all.end(), tl.begin(), tl.end());
    }
    LK_TRY(hipMemcpyAsync(bw.inner, hin.data(), sizeof(KmvArgs) * count, hipMemcpyHostToDevice, st));
    if (sym_batch && !sym_in[0].empty()) {
      LK_TRY(hipMemcpyAsync(bw.plans, sym_plans.data(), sizeof(SymPlan) * count, hipMemcpyHostToDevice, st));
      LK_TRY(hipMemcpyAsync(bw.sym_list, sym_in[0].data(), sizeof(int) * sym_in[0].size(), hipMemcpyHostToDevice,
                            st));
    }
    if (!tl_all.empty())
      LK_TRY(hipMemcpyAsync(bw.tiles_in, tl_all.data(), sizeof(int) * tl_all.size(), hipMemcpyHostToDevice, st));
    return LAKER_OK;
  };

  // float64 products of the outer residual: single-map plans
  std::vector<Plan1> pl_out(count);
  std::vector<KmvPlan> sq_out(count);
  for (int b = 0; b < count; ++b) {
    pl_out[b] = plan_for(pbs[b].n, LAKER_F64, 0);
    sq_out[b] = kmv_plan_square(pbs[b].n, dp, LAKER_F64);
    KmvArgs A = kmv_args(wss[b].e64, pbs[b].n, wss[b].e64, pbs[b].n, alpha[b], wss[b]);
    A.lam = pbs[b].lambda;
    A.pself = alpha[b];
    A.out = wss[b].w64;
    A.cps = pl_out[b].cps;
    A.nsplit = pl_out[b].nsplit;
    hout[b] = A;
  }

  const int gx = max_of(hd, &BDesc::g);
  const int gax = max_of(hd, &BDesc::ga);
  const int gtx = max_of(hd, &BDesc::nbt);
  int gfx = 1;
  for (const BDesc& d : hd) gfx = std::max(gfx, (d.nrp + 15) / 16);
  // map lists: the maps the iteration passes work on (inner solve running)
  // and the maps of the current host-side operation (restart, correction,
  // residual)
  std::vector<int> it_list, op_list;
  unsigned nit = 0, nop = 0;
  auto set_it_list = [&](const std::vector<int>& l) -> hipError_t {
    it_list = l;
    nit = (unsigned)l.size();
    return l.empty() ? hipSuccess : hipMemcpyAsync(bw.run_it, l.data(), sizeof(int) * l.size(), hipMemcpyHostToDevice, st);
  };
  auto set_op_list = [&]() -> hipError_t {
    op_list.clear();
    for (int b = 0; b < count; ++b)
      if (hd[b].active) op_list.push_back(b);
    nop = (unsigned)op_list.size();
    return op_list.empty() ? hipSuccess
                           : hipMemcpyAsync(bw.run_op, op_list.data(), sizeof(int) * op_list.size(), hipMemcpyHostToDevice, st);
  };

  auto upload_desc = [&]() -> hipError_t {
    return hipMemcpyAsync(bw.desc, hd.data(), sizeof(BDesc) * count, hipMemcpyHostToDevice, st);
  };

  // one inner iteration for the whole batch (maps whose inner solve is over
  // return at once in every pass)
  auto enqueue_iteration = [&](hipStream_t s2) -> laker_status {
    if (nit == 0) return LAKER_OK;
    for (int q = 0; q < 3; ++q) {
      if (grp_nt[q] > 0)
        LK_TRY(kmv_run_batch(kPrecOrder[q], dp, count, bw.inner, bw.tiles_in + 3 * (int64_t)grp_off[q], grp_nt[q],
                             false, max_n, s2));
      if (q == 0 && sym_batch)
        LK_TRY(kmv_run_sym16_batch(dp, (int)sym_in[0].size(), bw.inner, bw.plans, bw.sym_list, s2));
      else
        for (int b : sym_in[q]) LK_TRY(kmv_run(kPrecOrder[q], dp, sq_in[b], hin[b], s2));
    }
    b_ap_kernel<<<dim3(gx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it);
    LK_CHECK_LAUNCH();
    if (lowrank) {
      if (f32) b_update_t_kernel<float><<<dim3(gtx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it);
      else b_update_t_kernel<double><<<dim3(gtx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it);
      LK_CHECK_LAUNCH();
      b_lr_t_finish_kernel<<<dim3(gfx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it, 1, 0);
      LK_CHECK_LAUNCH();
      if (f32) b_lr_apply_kernel<float><<<dim3(gax, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it, 0, 1);
      else b_lr_apply_kernel<double><<<dim3(gax, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it, 0, 1);
      LK_CHECK_LAUNCH();
      b_pupdate_kernel<LAKER_PRECOND_CCCP><<<dim3(gx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it, 0, 0);
    } else if (kind == LAKER_PRECOND_JACOBI) {
      b_update_kernel<LAKER_PRECOND_JACOBI><<<dim3(gx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it);
      LK_CHECK_LAUNCH();
      b_pupdate_kernel<LAKER_PRECOND_JACOBI><<<dim3(gx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it, 0, 0);
    } else {
      b_update_kernel<LAKER_PRECOND_NONE><<<dim3(gx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it);
      LK_CHECK_LAUNCH();
      b_pupdate_kernel<LAKER_PRECOND_NONE><<<dim3(gx, nit), kThreads, 0, s2>>>(bw.desc, bw.run_it, 0, 0);
    }
    LK_CHECK_LAUNCH();
    return LAKER_OK;
  };

  // (re)start the inner PCG of the maps marked active, from x = 0; the other
  // maps are not touched
  auto restart = [&]() -> laker_status {
    LK_TRY(upload_desc());
    LK_TRY(set_op_list());
    if (nop == 0) return LAKER_OK;
    b_zero_kernel<<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
    LK_CHECK_LAUNCH();
    b_init_kernel<<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
    LK_CHECK_LAUNCH();
    b_start_kernel<<<dim3(1, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
    LK_CHECK_LAUNCH();
    if (lowrank) {
      if (f32) b_lr_t_partial_kernel<float><<<dim3(gtx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
      else b_lr_t_partial_kernel<double><<<dim3(gtx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
      LK_CHECK_LAUNCH();
      b_lr_t_finish_kernel<<<dim3(gfx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op, 0, 1);
      LK_CHECK_LAUNCH();
      if (f32) b_lr_apply_kernel<float><<<dim3(gax, nop), kThreads, 0, st>>>(bw.desc, bw.run_op, 1, 0);
      else b_lr_apply_kernel<double><<<dim3(gax, nop), kThreads, 0, st>>>(bw.desc, bw.run_op, 1, 0);
      LK_CHECK_LAUNCH();
      b_pupdate_kernel<LAKER_PRECOND_CCCP><<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op, 1, 1);
    } else if (kind == LAKER_PRECOND_JACOBI) {
      b_jacobi_apply_kernel<<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
      LK_CHECK_LAUNCH();
      b_pupdate_kernel<LAKER_PRECOND_JACOBI><<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op, 1, 1);
    } else {
      b_pupdate_kernel<LAKER_PRECOND_NONE><<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op, 1, 1);
    }
    LK_CHECK_LAUNCH();
    return LAKER_OK;
  };

  hipGraphExec_t gexec = nullptr;
  auto drop_graph = [&]() {
    if (gexec != nullptr) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
  };
  auto capture = [&]() -> laker_status {
    drop_graph();
    if (!o.graph) return LAKER_OK;
    hipStream_t cs = pcg_capture_stream();
    hipGraph_t graph = nullptr;
    bool ok = cs != nullptr && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      laker_status e = LAKER_OK;
      for (int c = 0; c < check && e == LAKER_OK; ++c) e = enqueue_iteration(cs);
      ok = hipStreamEndCapture(cs, &graph) == hipSuccess && e == LAKER_OK;
      if (ok) ok = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0) == hipSuccess;
      if (graph != nullptr) (void)hipGraphDestroy(graph);
    }
    if (!ok) {
      (void)hipGetLastError();
      drop_graph();
      return LAKER_EHIP;
    }
    return LAKER_OK;
  };
  // one chunk of iterations, then the scalars of every map on the host
  std::vector<PcgScalars> hs(count);
  auto run_chunk = [&]() -> laker_status {
    if (gexec != nullptr) {
      LK_TRY(hipGraphLaunch(gexec, st));
    } else {
      for (int c = 0; c < check; ++c) {
        laker_status e = enqueue_iteration(st);
        if (e != LAKER_OK) return e;
      }
    }
    b_gather_kernel<<<(count + 63) / 64, 64, 0, st>>>(bw.desc, count, bw.hs, bw.misc);
    LK_CHECK_LAUNCH();
    LK_TRY(hipMemcpyAsync(hs.data(), bw.hs, sizeof(PcgScalars) * count, hipMemcpyDeviceToHost, st));
    LK_TRY(hipStreamSynchronize(st));
    return LAKER_OK;
  };

  // outer residual y - A alpha (float64) of the maps marked active
  std::vector<double> rel(count, 0.0);
  auto outer_residual = [&](bool have_alpha) -> laker_status {
    std::vector<int> act(count);
    for (int b = 0; b < count; ++b) {
      act[b] = hd[b].active;
      hd[b].have_alpha = have_alpha ? 1 : 0;
      hout[b].mode = hd[b].active ? 1 : 2;
    }
    LK_TRY(upload_desc());
    LK_TRY(set_op_list());
    if (nop == 0) return LAKER_OK;
    if (have_alpha) {
      // symmetric-schedule maps: the single solver's product, one launch each
      std::vector<int> act_tiles = act;
      for (int b = 0; b < count; ++b)
        if (act[b] && sq_out[b].sym) {
          act_tiles[b] = 0;
          LK_TRY(kmv_run(LAKER_F64, dp, sq_out[b], hout[b], st));
          hout[b].mode = 2;   // finished: the tile pass below leaves it alone
        }
      std::vector<int> tl = build_tiles(count, pl_out, act_tiles, xcd);
      LK_TRY(hipMemcpyAsync(bw.outer, hout.data(), sizeof(KmvArgs) * count, hipMemcpyHostToDevice, st));
      if (!tl.empty())
        LK_TRY(hipMemcpyAsync(bw.tiles_out, tl.data(), sizeof(int) * tl.size(), hipMemcpyHostToDevice, st));
      LK_TRY(kmv_run_batch(LAKER_F64, dp, count, bw.outer, bw.tiles_out, (int)(tl.size() / 3), true, max_n, st));
    }
    b_resid_kernel<<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
    LK_CHECK_LAUNCH();
    std::vector<double> h(2 * count);
    b_gather_kernel<<<(count + 63) / 64, 64, 0, st>>>(bw.desc, count, bw.hs, bw.misc);
    LK_CHECK_LAUNCH();
    LK_TRY(hipMemcpyAsync(h.data(), bw.misc, sizeof(double) * 2 * count, hipMemcpyDeviceToHost, st));
    LK_TRY(hipStreamSynchronize(st));
    for (int b = 0; b < count; ++b)
      if (hd[b].active) rel[b] = h[2 * b + 1] > 0 ? sqrt(h[2 * b] / h[2 * b + 1]) : 0.0;
    return LAKER_OK;
  };

  std::vector<laker_status> res(count, LAKER_ENOCONV);
  for (int b = 0; b < count; ++b) stats[b] = laker_stats{};
  laker_status status = LAKER_OK;

  if (!o.refine) {
    // PCG on y directly, every map at once
    for (int b = 0; b < count; ++b) {
      hd[b].rhs = y[b];
      hd[b].x = alpha[b];
      hd[b].tol = o.tol;
      hd[b].max_iter = o.max_iter;
      hd[b].active = 1;
    }
    std::vector<int> everyone(count);
    for (int b = 0; b < count; ++b) everyone[b] = b;
    status = set_it_list(everyone) == hipSuccess ? rebuild_inner(everyone) : LAKER_EHIP;
    if (status == LAKER_OK) status = restart();
    if (status == LAKER_OK) status = capture();
    for (int k = 0; status == LAKER_OK;) {
      status = run_chunk();
      k += check;
      bool all = true;
      for (int b = 0; b < count; ++b)
        if (hs[b].done == 0) all = false;
      if (all || k >= o.max_iter + check) break;
    }
    drop_graph();
    if (status != LAKER_OK) return status;
    for (int b = 0; b < count; ++b) {
      stats[b].iters = hs[b].iters;
      stats[b].relres = hs[b].yy > 0 ? sqrt(hs[b].rr / hs[b].yy) : 0.0;
      res[b] = hs[b].done == 1 ? LAKER_OK : (hs[b].done == 2 ? LAKER_EBREAKDOWN : LAKER_ENOCONV);
    }
    status = outer_residual(true);
    if (status != LAKER_OK) return status;
    for (int b = 0; b < count; ++b) stats[b].relres_true = rel[b];
  } else {
    // Refinement with every map on its own schedule: when a map's inner PCG
    // ends, its correction is added, its float64 residual formed and its next
    // inner PCG started at the following check, while the other maps keep
    // iterating.
    std::vector<int> step(count, 0), used(count, 0), running(count, 0);
    for (int b = 0; b < count; ++b) {
      LK_TRY(hipMemsetAsync(alpha[b], 0, sizeof(double) * pbs[b].n, st));
      hd[b].rhs = wss[b].rout;
      hd[b].x = wss[b].dalpha;
      hd[b].active = 1;
    }
    // decide, for the maps marked active whose residual was just formed:
    // finished, or the next inner solve (finer arithmetic after two steps
    // without progress)
    bool tables_changed = false;
    auto decide = [&]() {
      for (int b = 0; b < count; ++b) {
        if (!hd[b].active) continue;
        const int s = step[b];
        if (s < 64) stats[b].ir_relres[s] = rel[b];
        stats[b].relres_true = rel[b];
        stats[b].relres = rel[b];
        stats[b].ir_steps = s;
        bool go = true;
        if (rel[b] <= o.tol) {
          res[b] = LAKER_OK;
          go = false;
        } else if (s >= o.ir_max || used[b] >= o.max_iter || res[b] == LAKER_EBREAKDOWN) {
          go = false;
        }
        if (!go) {
          hd[b].active = 0;
          running[b] = 0;
          continue;
        }
        if (s >= 2 && rel[b] >= stats[b].ir_relres[s - 2] && pm[b] != LAKER_F64) {
          pm[b] = pm[b] == LAKER_BF16 ? LAKER_F32 : LAKER_F64;
          stats[b].escalations += 1;
          tables_changed = true;
        }
        hd[b].tol = std::max(o.inner_tol, 0.5 * o.tol / rel[b]);
        hd[b].max_iter = o.max_iter - used[b];
        running[b] = 1;
      }
    };
    status = outer_residual(false);
    if (status != LAKER_OK) return status;
    decide();
    auto prepare_escalated = [&]() -> laker_status {
      for (int b = 0; b < count; ++b)
        if (hd[b].active && pm[b] == LAKER_F32)
          LK_TRY(prep_embed(pbs[b].E, pbs[b].n, pbs[b].d, pbs[b].dp, pbs[b].scale, LAKER_F32, wss[b].e32, st));
      return LAKER_OK;
    };
    auto running_list = [&]() {
      std::vector<int> l;
      for (int b = 0; b < count; ++b)
        if (running[b]) l.push_back(b);
      return l;
    };
    status = prepare_escalated();
    if (status == LAKER_OK) status = set_it_list(running_list()) == hipSuccess ? LAKER_OK : LAKER_EHIP;
    if (status == LAKER_OK) status = rebuild_inner(it_list);
    tables_changed = false;
    if (status == LAKER_OK) status = restart();
    if (status == LAKER_OK) status = capture();
    int64_t chunks = 0;
    const int64_t max_chunks = ((int64_t)o.max_iter + check - 1) / check + 2 * (int64_t)(o.ir_max + 1);
    while (status == LAKER_OK) {
      bool any = false;
      for (int b = 0; b < count; ++b)
        if (running[b]) any = true;
      if (!any) break;
      status = run_chunk();
      if (status != LAKER_OK) break;
      if (++chunks > max_chunks) break;
      // maps whose inner solve ended in this chunk
      bool ended = false;
      for (int b = 0; b < count; ++b) {
        hd[b].active = 0;
        if (!running[b] || hs[b].done == 0) continue;
        hd[b].active = 1;
        ended = true;
        used[b] += hs[b].iters;
        stats[b].iters = used[b];
        // an inner breakdown ends that inner solve; only in float64 is it final
        if (hs[b].done == 2 && pm[b] == LAKER_F64) res[b] = LAKER_EBREAKDOWN;
      }
      if (!ended) continue;
      status = (upload_desc() == hipSuccess && set_op_list() == hipSuccess) ? LAKER_OK : LAKER_EHIP;
      if (status != LAKER_OK) break;
      b_axpy_kernel<<<dim3(gx, nop), kThreads, 0, st>>>(bw.desc, bw.run_op);
      if (hipGetLastError() != hipSuccess) {
        status = LAKER_EHIP;
        break;
      }
      for (int b = 0; b < count; ++b)
        if (hd[b].active) step[b] += 1;
      status = outer_residual(true);
      if (status != LAKER_OK) break;
      decide();
      const std::vector<int> now = running_list();
      if (tables_changed || now != it_list) {
        status = prepare_escalated();
        if (status == LAKER_OK) status = set_it_list(now) == hipSuccess ? LAKER_OK : LAKER_EHIP;
        if (status == LAKER_OK) status = rebuild_inner(it_list);
        if (status == LAKER_OK) status = capture();
        tables_changed = false;
        if (status != LAKER_OK) break;
      }
      status = restart();
    }
    drop_graph();
    if (status != LAKER_OK) return status;
  }
  LK_TRY(hipStreamSynchronize(st));
  laker_status worst = LAKER_OK;
  for (int b = 0; b < count; ++b) {
    stats[b].status = res[b];
    if (res[b] == LAKER_EBREAKDOWN) worst = LAKER_EBREAKDOWN;
    else if (res[b] == LAKER_ENOCONV && worst == LAKER_OK) worst = LAKER_ENOCONV;
  }
  return worst;
}

}  // namespace lk
