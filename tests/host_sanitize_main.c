/* Host-side checks of the library's argument validation and workspace sizing,
 * built with AddressSanitizer and UndefinedBehaviorSanitizer on the host code
 * (tests/test_host_sanitizers.py).  No call here reaches a device: every one
 * is rejected, or answered, before the first HIP call. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "laker.h"

static int failures = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      fprintf(stderr, "line %d: %s\n", __LINE__, #cond);          \
      ++failures;                                                 \
    }                                                             \
  } while (0)

int main(void) {
  /* size queries over a range of shapes, including ones far beyond memory */
  const int64_t ns[] = {1, 2, 63, 64, 65, 255, 257, 4096, 9999, 16384, 65536, 131072, (int64_t)1 << 24};
  const int ds[] = {1, 3, 16, 17, 64, 100, 128};
  for (size_t a = 0; a < sizeof(ns) / sizeof(ns[0]); ++a) {
    for (size_t b = 0; b < sizeof(ds) / sizeof(ds[0]); ++b) {
      const int64_t n = ns[a];
      const int d = ds[b];
      EXPECT(laker_solve_workspace_bytes(n, d, 0) > 0);
      EXPECT(laker_solve_workspace_bytes(n, d, 2025) >= laker_solve_workspace_bytes(n, d, 0));
      EXPECT(laker_multi_workspace_bytes(n, d, 8) > 0);
      EXPECT(laker_learned_workspace_bytes(n, d, 0) > 0);
      (void)laker_kmat_bytes(n, d, LAKER_F64);
      (void)laker_kmat_bytes(n, d, LAKER_F32);
      if (n >= 64) EXPECT(laker_fit_workspace_bytes(n, d, 64) > 0);
    }
    EXPECT(laker_precond_bytes(ns[a], 64) > 0);
    EXPECT(laker_precond_apply_workspace_bytes(ns[a], 512) > 0);
    EXPECT(laker_online_state_bytes(ns[a], 96) > 0);
  }
  EXPECT(laker_solve_workspace_bytes(0, 4, 0) == 0);
  EXPECT(laker_solve_workspace_bytes(16, 0, 0) == 0);
  EXPECT(laker_solve_workspace_bytes(16, 129, 0) == 0);
  EXPECT(laker_fit_workspace_bytes(512, 200, 91) == 0);
  EXPECT(laker_multi_workspace_bytes(100, 8, 9) == 0);
  EXPECT(laker_online_state_bytes(100, 0) == 0);
  int64_t nb[3] = {1000, 0, 5};
  EXPECT(laker_batch_workspace_bytes(3, nb, 16) == 0);
  nb[1] = 2000;
  EXPECT(laker_batch_workspace_bytes(3, nb, 16) > 0);

  /* invalid arguments: rejected before any launch */
  double dummy[16];
  laker_problem bad = {16, 4, 0, NULL, 1e-2, 0.5};
  laker_problem good = {16, 4, 0, dummy, 1e-2, 0.5};
  laker_pcg_opts po = {0};
  po.tol = 1e-8;
  po.max_iter = 10;
  po.check_every = 16;
  laker_stats st;
  EXPECT(laker_pcg_solve(&bad, NULL, dummy, dummy, &po, dummy, 1 << 30, &st, NULL) == LAKER_EINVAL);
  EXPECT(laker_pcg_solve(&good, NULL, dummy, dummy, NULL, dummy, 1 << 30, &st, NULL) == LAKER_EINVAL);
  po.refine = 3;
  EXPECT(laker_pcg_solve(&good, NULL, dummy, dummy, &po, dummy, 1 << 30, &st, NULL) == LAKER_EINVAL);
  po.refine = 0;
  po.outer_history = 9;
  EXPECT(laker_pcg_solve(&good, NULL, dummy, dummy, &po, dummy, 1 << 30, &st, NULL) == LAKER_EINVAL);
  po.outer_history = 0;
  EXPECT(laker_pcg_solve(&good, NULL, dummy, dummy, &po, dummy, 8, &st, NULL) == LAKER_ENOMEM);
  laker_problem neg = {16, 4, 0, dummy, -1.0, 0.5};
  EXPECT(laker_kernel_matvec(&neg, dummy, dummy, 0, dummy, 1 << 30, NULL) == LAKER_EINVAL);
  EXPECT(laker_kernel_matvec_noalloc(&neg, dummy, dummy, 0, NULL) == LAKER_EINVAL);
  laker_problem huge = {(int64_t)1 << 20, 64, 0, dummy, 1e-2, 0.5};
  EXPECT(laker_kernel_matvec_noalloc(&huge, dummy, dummy, LAKER_BF16, NULL) == LAKER_ENOMEM);
  EXPECT(laker_predict(&good, dummy, 0, dummy, dummy, 0, dummy, 1 << 30, NULL) == LAKER_EINVAL);
  laker_cccp_opts co = {64, 300, 0.1, 0.0, 1e-10, 1e-8, LAKER_F64, 0};
  laker_precond pc = {0, 0, 16, dummy, sizeof(dummy)};
  co.n_r = 17; /* more directions than sites */
  EXPECT(laker_fit_precond(&good, dummy, &co, &pc, dummy, 1 << 30, &st, NULL) == LAKER_EINVAL);
  co.n_r = 4;
  co.rho = 2.0;
  EXPECT(laker_fit_precond(&good, dummy, &co, &pc, dummy, 1 << 30, &st, NULL) == LAKER_EINVAL);
  co.rho = 0.0;
  co.precision = LAKER_BF16; /* the online state holds float64 directions */
  EXPECT(laker_fit_precond_online(&good, 0, dummy, &co, dummy, 1 << 30, &pc, dummy, 1 << 30, &st, NULL) ==
         LAKER_EINVAL);
  co.precision = LAKER_F64;
  EXPECT(laker_fit_precond_online(&good, 17, dummy, &co, dummy, 1 << 30, &pc, dummy, 1 << 30, &st, NULL) ==
         LAKER_EINVAL);
  EXPECT(laker_pcg_solve_multi(&good, NULL, 9, dummy, dummy, &po, dummy, 1 << 30, &st, NULL) == LAKER_EINVAL);
  laker_precond none = {LAKER_PRECOND_NONE, 0, 16, NULL, 0};
  EXPECT(laker_precond_apply(NULL, dummy, dummy, 0, dummy, 64, NULL) == LAKER_EINVAL);
  EXPECT(laker_precond_apply(&none, NULL, dummy, 0, dummy, 64, NULL) == LAKER_EINVAL);
  laker_mlp_layout lay;
  EXPECT(laker_mlp_layout_query(0, &lay) == LAKER_EINVAL);
  EXPECT(laker_mlp_layout_query(8, &lay) == LAKER_OK && lay.in_dim == 26);
  EXPECT(laker_pcg_solve_batched(0, &good, NULL, NULL, NULL, &po, NULL, dummy, 64, &st, NULL) == LAKER_EINVAL);
  for (int s = -7; s <= 1; ++s) EXPECT(laker_status_str(s) != NULL);

  if (failures) {
    fprintf(stderr, "%d host checks failed\n", failures);
    return 1;
  }
  printf("host checks passed\n");
  return 0;
}
