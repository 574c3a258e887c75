"""Preconditioner parity at the sizes the solves run, through the C ABI.

* The CCCP fit at N_r = 256 and 512 random directions (the bench map has 16384
  sites and 512 directions): (a, b), the iteration count and theta = P v from
  the library's own apply kernels (laker_precond_apply), element by element,
  against the oracle's low-rank CCCP and its P = Sigma^{-1/2} (same Z).
* The apply of every preconditioner kind against its definition: CCCP
  (float64 and float32 factors), the learned rank-64-plus-diagonal inverse
  (the apply that finishes t = B^T r itself on up to 16384 sites, and the
  separate t pass above), Jacobi, none.

Element-wise bounds are relative to mag_i = |c r_i| + sum_k |Bt_ik| |t_k|, the
magnitude of the terms of theta_i:
  * fit + apply against the oracle: 1e-7 (q_k comes from SPD solves with
    kappa(M) up to ~1e7 on either side, ~1e-9 each, amplified by at most
    1/(1 - rate) of the CCCP fixed-point map; P from Newton-Schulz against an
    eigendecomposition agrees to the same order); float32 factors add their
    rounding 2^-24 per entry: 3e-7;
  * the learned preconditioner against the float64 Woodbury oracle on the
    network's outputs: 1e-12 kappa(S) (float64 capacitance Cholesky and
    float64 apply);
  * Jacobi: a reciprocal, a product and the diagonal's exp, a few ulp.
"""
import numpy as np
import pytest
import torch

from oracle import laker_oracle as O
from oracle import learned_oracle as LO
from synth import make_directions, make_mlp_init, make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def L():
    from paper_2604_25138_amd import laker
    laker.load()
    return laker


def _gp(pr):
    return L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)


def _lowrank_mag(P: O.LowRankPrecond, r):
    t = P.Gs @ (P.B.T @ r)
    return np.abs(r) / np.sqrt(P.b) + np.abs(P.B) @ np.abs(t)


@pytest.mark.parametrize("n,d,nr,seed", [(8192 + 77, 32, 256, 31), (16384, 64, 512, 0)])
def test_cccp_fit_and_apply_match_oracle_at_full_rank(n, d, nr, seed):
    pr = make_problem(n, d, 1e-4, n_tx=4, seed=seed)
    Z = make_directions(n, nr, seed)
    prob = _gp(pr)
    print(f"cccp fit n={n} nr={nr}", flush=True)
    pc = L().fit_precond(prob, torch.tensor(Z, device=DEV), gamma=0.1, rho=0.0, tol=1e-8, max_iter=300)
    _, Ub = O.random_directions(pr.E, pr.scale, pr.lam, Z)
    a, b, w, it = O.cccp_lowrank(Ub, 0.1, 0.0, 1e-10, 1e-8, 300)
    hdr = pc.header.numpy()
    print(f"  a {hdr[1]:.6e} / {a:.6e}, b {hdr[2]:.6e} / {b:.6e}, iterations {pc.stats.cccp_iters} / {it}")
    assert abs(hdr[1] - a) <= 1e-7 * a and abs(hdr[2] - b) <= 1e-7 * b
    assert abs(pc.stats.cccp_iters - it) <= 2
    P = O.LowRankPrecond(Ub, a, b, w)
    rng = np.random.default_rng(seed)
    for prec, tol in (("f64", 1e-7), ("f32", 3e-7)):
        v = rng.normal(size=n)
        got = L().precond_apply(pc, torch.tensor(v, device=DEV), prec).cpu().numpy()
        ref = P.apply(v)
        err = np.abs(got - ref) / _lowrank_mag(P, v)
        print(f"  apply {prec}: max element error {err.max():.2e} of the term magnitude")
        assert err.max() <= tol, (prec, err.max(), int(err.argmax()))


def _learned_model(d, seed):
    p = make_mlp_init(LO.input_dim(d), LO.HIDDEN, LO.RANK + 1, seed, log_delta0=-2.0)
    for k in p:
        p[k] = p[k] * 0.5
    p["b3"][LO.RANK] = -2.0
    m = L().MlpModel(d, DEV)
    m.set_params(p)
    return m


@pytest.mark.parametrize("n,d", [(16384, 64), (20000 + 3, 32), (777, 16)])
def test_learned_apply_matches_woodbury_oracle(n, d):
    """Up to 16384 sites the apply finishes t = B^T r itself (one pass fewer
    per iteration); above, t has a pass of its own.  Both against the float64
    Woodbury oracle applied to the network's outputs (V, delta)."""
    pr = make_problem(n, d, 1e-4, n_tx=2, seed=n)
    prob = _gp(pr)
    model = _learned_model(d, n)
    out = L().learned_forward(prob, model).cpu().double().numpy()
    V, delta = out[:, :LO.RANK], np.exp(out[:, LO.RANK])
    pc = L().learned_precond(prob, model)
    Dinv = 1.0 / delta
    K = np.eye(LO.RANK) + V.T @ (Dinv[:, None] * V)
    kev = np.linalg.eigvalsh(K)
    kappa = kev[-1] / kev[0] * Dinv.max() / Dinv.min()
    rng = np.random.default_rng(n)
    for prec in ("f64", "bf16"):
        r = rng.normal(size=n)
        got = L().precond_apply(pc, torch.tensor(r, device=DEV), prec).cpu().numpy()
        ref = LO.woodbury_solve(V, delta, r)
        # terms of theta_i: D^{-1}_i r_i and the rank-64 correction D^{-1}_i v_i^T K^{-1} V^T D^{-1} r
        t = np.linalg.solve(K, V.T @ (Dinv * r))
        mag = Dinv * np.abs(r) + Dinv * (np.abs(V) @ np.abs(t))
        err = np.abs(got - ref) / mag
        print(f"learned apply n={n} {prec}: max element error {err.max():.2e}, kappa {kappa:.2e}", flush=True)
        assert err.max() <= 1e-12 * kappa, (prec, err.max(), int(err.argmax()))


def test_jacobi_and_identity_apply():
    n, d = 5000 + 11, 16
    pr = make_problem(n, d, 1e-3, seed=5)
    prob = _gp(pr)
    r = np.random.default_rng(5).normal(size=n)
    pj = L().jacobi_precond(prob)
    got = L().precond_apply(pj, torch.tensor(r, device=DEV), "f64").cpu().numpy()
    diag = O.jacobi_diag(pr.E, pr.scale, pr.lam)
    # the library divides by its float64 diagonal once per fit and multiplies
    # per apply; exp of the squared norm within an ulp or two on either side
    assert np.all(np.abs(got - r / diag) <= 1e-15 * np.abs(r / diag))
    pn = L().none_precond(n)
    got = L().precond_apply(pn, torch.tensor(r, device=DEV), "f64").cpu().numpy()
    assert np.array_equal(got, r)
