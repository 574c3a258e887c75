"""Pins of the learned-preconditioner oracle (CPU, float64).

The network, its loss and their gradients have no printed values to match;
they are pinned by mathematics: central finite differences of the loss (a
dropped term, a wrong sign or a transposed weight anywhere in the backward
pass fails these), the Woodbury solve and the loss against dense solves, the
closed-form first Adam step, SPD-ness of S for arbitrary weights, and
Sigma^{1/2} Z against a dense eigendecomposition of the fitted Sigma.
"""
import math

import numpy as np
import pytest

from oracle import laker_oracle as O
from oracle import learned_oracle as LO
from synth import make_directions, make_mlp_init, make_probes, make_problem


def _setup(n=40, d=4, m=6, seed=0, scale=1.0):
    pr = make_problem(n, d, 1e-2, seed=seed)
    X = LO.features(pr.E, pr.lam)
    p = make_mlp_init(X.shape[1], LO.HIDDEN, LO.RANK + 1, seed, log_delta0=-1.0)
    for k in p:
        p[k] = p[k] * scale
    p["b3"][LO.RANK] = -1.0
    Z = make_probes(n, m, seed)
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(n, n))
    U = (A @ A.T / n + np.eye(n)) @ Z
    return p, X, Z, U


def test_woodbury_matches_dense_solve():
    rng = np.random.default_rng(1)
    n, r = 90, LO.RANK
    V = rng.normal(size=(n, r)) * 0.3
    delta = np.exp(rng.uniform(-4, 1, size=n))
    X = rng.normal(size=(n, 5))
    S = LO.learned_dense(V, delta)
    ref = np.linalg.solve(S, X)
    got = LO.woodbury_solve(V, delta, X)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
    assert np.allclose(LO.woodbury_solve(V, delta, X[:, 0]), got[:, 0], rtol=0, atol=1e-14 * np.abs(ref).max())


def test_s_is_spd_for_arbitrary_weights():
    p, X, Z, U = _setup(scale=3.0, seed=2)
    O_, _ = LO.mlp_forward(p, X)
    V, delta = LO.split_output(O_)
    ev = np.linalg.eigvalsh(LO.learned_dense(V, delta))
    assert ev.min() > 0.0 and ev.min() >= 0.999 * delta.min()


def test_loss_matches_dense_definition():
    p, X, Z, U = _setup(seed=3)
    O_, _ = LO.mlp_forward(p, X)
    V, delta = LO.split_output(O_)
    S = LO.learned_dense(V, delta)
    ref = ((Z - np.linalg.solve(S, U)) ** 2).sum() / Z.size
    assert abs(LO.loss(p, X, Z, U) - ref) <= 1e-12 * ref


@pytest.mark.parametrize("seed", [4, 5])
def test_gradient_matches_finite_differences(seed):
    p, X, Z, U = _setup(seed=seed)
    L0, g, dO = LO.loss_and_grad(p, X, Z, U)
    rng = np.random.default_rng(seed)
    h = 1e-6
    for key in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[key].reshape(-1)
        idx = rng.choice(flat.size, size=min(6, flat.size), replace=False)
        if key == "b3":
            idx = np.unique(np.concatenate([idx, [LO.RANK]]))   # the log-diagonal output
        if key == "W3":
            idx = np.unique(np.concatenate([idx, [5 * (LO.RANK + 1) + LO.RANK]]))
        for i in idx:
            old = flat[i]
            flat[i] = old + h
            lp = LO.loss(p, X, Z, U)
            flat[i] = old - h
            lm = LO.loss(p, X, Z, U)
            flat[i] = old
            fd = (lp - lm) / (2 * h)
            an = g[key].reshape(-1)[i]
            scale = max(abs(fd), 1e-3 * np.abs(g[key]).max(), 1e-12)
            assert abs(an - fd) <= 1e-6 * scale + 1e-10, (key, i, an, fd)


def test_first_adam_step_closed_form():
    p, X, Z, U = _setup(seed=6)
    _, g, _ = LO.loss_and_grad(p, X, Z, U)
    p0 = {k: v.copy() for k, v in p.items()}
    st = {}
    LO.adam_step(p, g, st, lr=1e-3, t=1)
    for k in p:
        # m_hat = g, v_hat = g^2  =>  step = lr g / (|g| + eps)
        assert np.allclose(p[k], p0[k] - 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=0, atol=1e-15)


def test_sigma_half_apply_matches_dense_square_root():
    pr = make_problem(300, 8, 1e-3, seed=7)
    Z = make_directions(pr.n, 40, 7)
    P, _ = O.fit_precond(pr.E, pr.scale, pr.lam, Z, gamma=1e-3)
    Sigma = P.b * np.eye(pr.n) + P.B @ P.B.T
    ev, Vv = np.linalg.eigh(Sigma)
    root = (Vv * np.sqrt(ev)) @ Vv.T
    probes = make_probes(pr.n, 5, 7)
    got = LO.sigma_half_apply(P.b, P.B, P.apply, probes)
    ref = root @ probes
    # Sigma (P z) multiplies the rounding error of P z by up to ||Sigma||: the
    # bound scales with the condition number of Sigma (3e6 here)
    tol = 1e-13 * ev[-1] / ev[0]
    assert np.abs(got - ref).max() <= tol * np.abs(ref).max()
    # and P really is its inverse: Sigma^{1/2} P z = z
    assert np.abs(root @ np.column_stack([P.apply(probes[:, k]) for k in range(5)]) - probes).max() <= tol
