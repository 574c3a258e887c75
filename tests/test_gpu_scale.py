"""Full-size mixed precision: n = 65536 sites, d = 64, lambda = 1e-4, bfloat16
score tiles with the flexible float64 outer CG (refine = 2) to a true relative
residual of 1e-8 (CCCP preconditioner, gamma = 1e-3).  The library's float64
residual is checked on sampled rows that the oracle recomputes one by one in
float64.  (At lambda = 1e-5 the same path reaches a few 1e-9, the float64
floor of the product at this conditioning; plain refinement diverges there.)"""
import numpy as np
import pytest
import torch

from oracle import laker_oracle as O
from synth import default_n_r, make_directions, make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_flexible_outer_cg_at_65536_sites():
    from paper_2604_25138_amd import laker as L
    L.load()
    n, d = 65536, 64
    pr = make_problem(n, d, 1e-4, n_tx=4, seed=3)
    prob = L.Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)
    pc = L.fit_precond(prob, torch.tensor(make_directions(n, default_n_r(n), 3), device=DEV), gamma=1e-3,
                       precision="bf16")
    alpha, st = L.pcg_solve(prob, pr.y, pc, tol=1e-8, max_iter=30000, precision="bf16", refine=2, inner_tol=0.1,
                            ir_max=5000, check_every=32, inner_max_iter=50)
    assert st.status == 0 and st.relres_true <= 1e-8
    rows = np.random.default_rng(3).choice(n, size=32, replace=False)
    r = pr.y[rows] - O.matvec_rows(pr.E, pr.scale, pr.lam, alpha.cpu().numpy(), rows)
    assert np.abs(r).max() <= 1e-8 * np.linalg.norm(pr.y)


def test_flexible_outer_cg_at_65536_sites_lambda_1e5_stored():
    """lambda = 1e-5 (lambda / ||G|| about 1.5e-10, below the bfloat16 product's
    rounding): the flexible float64 outer CG around capped bfloat16 inner
    solves, its float64 products streaming the stored G (17.2 GB), reaches the
    float64 floor of the product at this conditioning (a few 1e-9); the
    per-step residuals are recorded and the final residual is checked on
    sampled rows against the oracle."""
    import time

    from paper_2604_25138_amd import laker as L
    L.load()
    n, d = 65536, 64
    pr = make_problem(n, d, 1e-5, n_tx=4, seed=5)
    prob = L.Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)
    pc = L.fit_precond(prob, torch.tensor(make_directions(n, default_n_r(n), 5), device=DEV), gamma=1e-3,
                       precision="bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    alpha, st = L.pcg_solve(prob, pr.y, pc, tol=5e-9, max_iter=60000, precision="bf16", refine=2, inner_tol=0.1,
                            ir_max=5000, check_every=30, inner_max_iter=30, materialized=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    steps = [st.ir_relres[k] for k in range(min(st.ir_steps + 1, 64))]
    print(f"n=65536 lambda=1e-5: {st.iters} inner iterations, {st.ir_steps} outer steps, {dt:.1f} s, "
          f"relres_true {st.relres_true:.3e}; first outer residuals {['%.2e' % v for v in steps[:12]]}")
    assert st.status == 0 and st.relres_true <= 5e-9
    assert all(np.isfinite(steps)) and steps[-1] < steps[0]
    rows = np.random.default_rng(5).choice(n, size=32, replace=False)
    r = pr.y[rows] - O.matvec_rows(pr.E, pr.scale, pr.lam, alpha.cpu().numpy(), rows)
    assert np.abs(r).max() <= 5e-9 * np.linalg.norm(pr.y)


def test_stopping_sum_covers_every_partial_beyond_65536_rows():
    """The stopping test of PCG adds one ||r||^2 partial per 64 rows; above
    65536 rows a thread's stripe holds more than the four partials it loads
    ahead, and every one of them must enter the sum.  After five float32 PCG
    iterations with a CCCP preconditioner (the separate t pass, as for any map
    above 16384 sites) the reported recursive residual must equal the float64
    true residual of the same iterate up to the float32 product's rounding;
    a sum that dropped partials would report about 0.7 of it at 131072 rows."""
    from paper_2604_25138_amd import laker as L
    L.load()
    n, d = 131072, 16
    pr = make_problem(n, d, 1e-2, n_tx=2, seed=17)
    prob = L.Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)
    pc = L.fit_precond(prob, torch.tensor(make_directions(n, 64, 17), device=DEV), gamma=0.1, precision="f32")
    alpha, st = L.pcg_solve(prob, pr.y, pc, tol=1e-12, max_iter=5, precision="f32", check_every=5,
                            allow_noconv=True)
    print(f"n={n}: {st.iters} iterations, recursive {st.relres:.6e}, true {st.relres_true:.6e}")
    assert st.status == L.LAKER_ENOCONV and st.iters == 5
    assert abs(st.relres / st.relres_true - 1.0) <= 1e-3
