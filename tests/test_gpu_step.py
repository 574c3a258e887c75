"""The timed step of the benchmark, checked against the oracle.

The step combines: the learned rank-64-plus-diagonal preconditioner (network
forward, Woodbury factors; up to 16384 sites its apply finishes t = B^T r
itself), the bfloat16 symmetric product that forms p^T A p and conjugates the
direction on the fly (from ~9900 sites), the flexible float64 outer CG around
inner PCG solves capped at 30 iterations, and G stored once in float64 for the
outer products.  The network is trained briefly on the method's own CCCP fits
of smaller maps.  Pass: the library reports a float64 true relative residual
<= 1e-6, and the residual rows y_i - ((lambda I + G) alpha)_i that the oracle
computes one by one in float64 on 64 sampled sites are each <= 1e-6 ||y||
(every entry of a residual is bounded by its norm)."""
import numpy as np
import pytest
import torch

from oracle import laker_oracle as O
from synth import default_n_r, make_directions, make_mlp_init, make_probes, make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
INNER_CAP = 30


def _trained_model(L, LR, d):
    exs = []
    rng = np.random.default_rng(99)
    for k in range(8):
        lam = float(10 ** rng.uniform(-5, -2))
        pr = make_problem(4096, d, lam, n_tx=int(rng.integers(1, 9)), seed=7000 + k)
        prob = L.Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)
        Zd = torch.tensor(make_directions(4096, default_n_r(4096), 7000 + k), device=DEV)
        exs.append(LR.make_example(prob, Zd, make_probes(4096, 64, 7000 + k), gamma=1e-3, precision="bf16"))
    model = L.MlpModel(d, DEV)
    model.set_params(make_mlp_init(L.mlp_layout(d).in_dim, L.MLP_HIDDEN, L.MLP_RANK + 1, 0))
    LR.train(model, exs, epochs=6, lr=1e-3, seed=0)
    return model


@pytest.mark.parametrize("n,lam,seed", [(16384, 1e-4, 0), (65536, 1e-5, 0)])
def test_bench_step_residual_against_oracle(n, lam, seed):
    from paper_2604_25138_amd import laker as L
    from paper_2604_25138_amd import learned as LR
    L.load()
    d = 64
    model = _trained_model(L, LR, d)
    pr = make_problem(n, d, lam, n_tx=4, seed=seed)
    prob = L.Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)
    pc = L.learned_precond(prob, model)
    print(f"bench step n={n} lambda={lam}", flush=True)
    alpha, st = L.pcg_solve(prob, pr.y, pc, tol=1e-6, max_iter=200000, precision="bf16", refine=2, inner_tol=0.1,
                            ir_max=5000, check_every=INNER_CAP, inner_max_iter=INNER_CAP, materialized=True)
    print(f"  {st.iters} inner iterations, {st.ir_steps} outer steps, true relres {st.relres_true:.3e}", flush=True)
    assert st.status == L.LAKER_OK and st.relres_true <= 1e-6
    rows = np.random.default_rng(seed + 1).choice(n, size=64, replace=False)
    a = alpha.cpu().numpy()
    r = pr.y[rows] - O.matvec_rows(pr.E, pr.scale, pr.lam, a, rows)
    ny = np.linalg.norm(pr.y)
    print(f"  sampled residual rows: max |r_i| / ||y|| = {np.abs(r).max() / ny:.3e}")
    assert np.abs(r).max() <= 1e-6 * ny
