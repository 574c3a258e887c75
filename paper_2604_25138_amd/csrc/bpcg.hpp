// Batched PCG over many independent maps (bpcg.hip).
#pragma once

#include "internal.hpp"
#include "pcg.hpp"

namespace lk {

// Per-problem state of a batched solve, read by the batched kernels from
// device memory (one entry per problem; grid row blockIdx.y = problem).
struct BDesc {
  int64_t n;
  double lam;
  int g, ga, nbt;        // block counts of the reduction, apply and row-slab passes
  PartSum ps;            // layout of the product's partial sums
  int active;            // 0: the problem is finished and every batched pass skips it
  int nrp;
  PcgScalars* S;
  const double* rhs;     // right-hand side of the inner PCG
  double* x;             // its solution
  double* r;
  double* p;
  double* Ap;
  double* th;
  double* part;
  double* yyp;
  double* rrp;
  double* rzp;
  double* papp;
  double* tpart;
  double* t;
  const void* B;
  const void* Bt;
  const double* c0p;
  const double* dinv;
  const double* y;       // outer right-hand side
  double* alpha;         // outer solution
  double* rout;          // outer residual y - A alpha (float64)
  double* w64;           // float64 product output
  double* bpart;
  unsigned* cnt;
  double* misc;          // [0] ||y - A alpha||^2, [1] ||y||^2
  double tol;            // inner tolerance
  int max_iter;          // inner iteration cap
  int have_alpha;        // outer residual: 0 when alpha = 0 (r = y)
};

// Device arrays of a batched solve carved from the caller's workspace.
struct BatchWs {
  BDesc* desc;
  KmvArgs* inner;        // product arguments of the inner PCG (mode 0)
  KmvArgs* outer;        // float64 products of the outer residual (mode 1)
  int* tiles_in;         // 3 ints per tile
  int* tiles_out;
  int* run_it;           // maps of the iteration passes
  int* run_op;           // maps of the current host-side operation
  PcgScalars* hs;        // gathered scalars of every map
  double* misc;          // gathered outer residual norms (2 per map)
  SymPlan* plans;        // square plans of the inner products (one per map)
  int* sym_list;         // maps whose inner products share the symmetric batched launch
  size_t total;
};

// Workspace: per-problem solver workspaces (plan_solve_ws) followed by the batch
// arrays.  `offsets[b]` receives the byte offset of problem b's workspace.
size_t plan_batch_ws(int count, const int64_t* n, int d, size_t* offsets, void* base, BatchWs* out);

struct BatchOpts {
  int cps;               // -1: autotune; 0: the single-problem plan; > 0: columns per range
  int xcd_order;         // 1: XCD-aware tile order
};

laker_status pcg_batch(int count, const Problem* pbs, const SolveWs* wss, const PrecondView* Ps,
                       const double* const* y, double* const* alpha, const laker_pcg_opts& o, const BatchOpts& bo,
                       const BatchWs& bw, laker_stats* stats, int* cps_used, hipStream_t st);

}  // namespace lk
