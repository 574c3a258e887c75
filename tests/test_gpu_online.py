"""Measurements that arrive over time (the online setting the paper leaves to
future work, Sec. VI): sites appended to a fitted map.

The online fit extends the random directions (previous entries kept, new
rows drawn) and forms only the products with the new rows; CCCP starts from
the previous fit's weights.  Checks:
* the stored directions U = (lambda I + G) Z equal the oracle's for the
  enlarged problem, element by element (1e-13 relative to sum_j |G_ij Z_jk|
  + lambda |Z_ik|, the float64 product bound);
* (a, b) and P v equal the oracle's fit of the enlarged problem with the same
  directions (1e-7, the fit's bound), in no more CCCP iterations than a fit
  from Sigma_0 = I;
* PCG warm-started from [alpha_prev; 0] reaches the Cholesky solution of the
  enlarged system in no more iterations than from zero.
The float64 directions product itself (the fit's first step, on the f64 MFMA)
is also checked row by row against the oracle at several shapes, down to maps
smaller than one 16 x 16 tile.
"""
import numpy as np
import pytest
import torch

from oracle import laker_oracle as O
from synth import make_directions, make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def L():
    from paper_2604_25138_amd import laker
    laker.load()
    return laker


@pytest.mark.parametrize("n0,m,d,nr", [(3000, 200, 16, 96), (2000 + 13, 64 + 5, 32, 64)])
def test_appended_sites_extend_the_fit(n0, m, d, nr):
    n = n0 + m
    pr = make_problem(n, d, 1e-3, n_tx=2, seed=n0)
    Z = make_directions(n, nr, n0)
    E_all = torch.tensor(pr.E, device=DEV)
    prob0 = L().Problem(E_all[:n0].contiguous(), pr.lam, pr.scale)
    prob = L().Problem(E_all, pr.lam, pr.scale)
    state = L().OnlineFitState(n, nr, DEV)
    pc0 = state.fit(prob0, torch.tensor(Z[:n0], device=DEV), gamma=0.1)
    pc1 = state.fit(prob, torch.tensor(Z, device=DEV), gamma=0.1)
    # directions of the enlarged problem, against the oracle's
    U_ref, Ub = O.random_directions(pr.E, pr.scale, pr.lam, Z)
    U = state.directions().cpu().numpy()
    G = O.kernel_matrix(pr.E, pr.scale)
    mag = np.abs(G) @ np.abs(Z) + pr.lam * np.abs(Z)
    assert (np.abs(U - U_ref) / mag).max() <= 1e-13
    # the fit's fixed point, against the oracle and a fresh fit
    a, b, w, it = O.cccp_lowrank(Ub, 0.1, 0.0, 1e-10, 1e-8, 300)
    fresh = L().fit_precond(prob, torch.tensor(Z, device=DEV), gamma=0.1)
    h1, hf = pc1.header.numpy(), fresh.header.numpy()
    print(f"n0={n0} m={m}: warm CCCP {pc1.stats.cccp_iters} iterations, fresh {fresh.stats.cccp_iters}, "
          f"oracle {it}; a {h1[1]:.10e} / {a:.10e}")
    assert abs(h1[1] - a) <= 1e-7 * a and abs(h1[2] - b) <= 1e-7 * b
    assert pc1.stats.cccp_iters <= fresh.stats.cccp_iters
    v = np.random.default_rng(n).normal(size=n)
    Pv = L().precond_apply(pc1, torch.tensor(v, device=DEV), "f64").cpu().numpy()
    P = O.LowRankPrecond(Ub, a, b, w)
    assert np.linalg.norm(Pv - P.apply(v)) <= 1e-7 * np.linalg.norm(P.apply(v))
    # warm-started PCG from the previous solution, zero on the new sites
    a0, s0 = L().pcg_solve(prob0, pr.y[:n0], pc0, tol=1e-12, max_iter=20000)
    start = torch.cat([a0, torch.zeros(m, dtype=torch.float64, device=DEV)])
    a1, s1 = L().pcg_solve(prob, pr.y, pc1, tol=1e-12, max_iter=20000, alpha0=start)
    _, s2 = L().pcg_solve(prob, pr.y, pc1, tol=1e-12, max_iter=20000)
    print(f"  PCG warm {s1.iters} iterations, from zero {s2.iters}")
    ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    assert np.linalg.norm(a1.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    assert s1.iters <= s2.iters


@pytest.mark.parametrize("n,d,nr,seed", [(12288 + 37, 64, 200, 3), (3000 + 5, 100, 70, 4), (7, 3, 3, 5),
                                         (40, 16, 17, 6)])
def test_float64_directions_elementwise(n, d, nr, seed):
    """U = (lambda I + G) Z of a fresh float64 fit (eq. random_directions: the
    product every float64 fit starts from), on sampled rows -- the first and
    last of every 64-row block and up to 64 random ones -- against the
    oracle's one-row evaluation, 1e-13 relative to sum_j |G_ij Z_jk| +
    lambda |Z_ik|.  The sizes leave ragged row blocks and column tiles, d = 100
    runs the dp = 128 form, and the small maps have fewer rows and columns than
    one 16 x 16 tile."""
    pr = make_problem(n, d, 1e-3, n_tx=3, seed=seed)
    Z = make_directions(n, nr, seed)
    prob = L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)
    state = L().OnlineFitState(n, nr, DEV)
    state.fit(prob, torch.tensor(Z, device=DEV), gamma=0.1)
    U = state.directions().cpu().numpy()
    rng = np.random.default_rng(seed)
    rows = np.unique(np.r_[np.arange(0, n, 64), np.minimum(np.arange(63, n + 63, 64), n - 1),
                           rng.choice(n, min(n, 64), replace=False)])
    for i in rows:
        g = np.exp(pr.scale * (pr.E @ pr.E[i]))
        ref = g @ Z + pr.lam * Z[i]
        mag = g @ np.abs(Z) + pr.lam * np.abs(Z[i])
        assert (np.abs(U[i] - ref) / mag).max() <= 1e-13, i
