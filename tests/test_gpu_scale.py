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
