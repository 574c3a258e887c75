"""Pins of the learned-preconditioner oracle (CPU, float64).

The network, its loss and their gradients have no printed values to match;
they are pinned by mathematics: central finite differences of the loss (a
dropped term, a wrong sign or a transposed weight anywhere in the backward
pass fails these), the Woodbury solve and the loss against dense solves, the
closed-form first Adam step, SPD-ness of S for arbitrary weights,
Sigma^{1/2} Z against a dense eigendecomposition of the fitted Sigma, and the
forward pass itself through closed forms of the logistic function (SiLU at 0,
1 and ln 3; a width-1 network whose output is exactly 4) and hand-written
feature rows.
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


def test_silu_closed_forms():
    """SiLU z * logistic(z): logistic(0) = 1/2, logistic(1) = e / (e + 1),
    logistic(ln 3) = 3/4; silu(z) - silu(-z) = z (logistic(z) + logistic(-z) = 1);
    the derivative is 1/2 at 0 and tends to 1 and 0 far out."""
    z = np.array([0.0, 1.0, math.log(3.0), -math.log(3.0), 40.0, -40.0])
    s = LO.silu(z)
    assert s[0] == 0.0
    assert s[1] == pytest.approx(math.e / (math.e + 1.0), rel=1e-15)
    assert s[2] == pytest.approx(0.75 * math.log(3.0), rel=1e-15)
    assert s[3] == pytest.approx(-0.25 * math.log(3.0), rel=1e-15)
    assert s[4] == pytest.approx(40.0, rel=1e-15) and abs(s[5]) < 1e-15
    w = np.linspace(-6.0, 6.0, 25)
    assert np.allclose(LO.silu(w) - LO.silu(-w), w, rtol=0, atol=1e-15)
    g = LO.silu_grad(np.array([0.0, 40.0, -40.0]))
    assert g[0] == 0.5 and g[1] == pytest.approx(1.0, abs=1e-14) and abs(g[2]) < 1e-14


def test_features_hand_computed_rows():
    """x_i = [e_i, log lambda, log(n)/10, column means of e, column means of e^2]
    for a 2 x 2 embedding written out by hand."""
    E = np.array([[1.0, 2.0], [3.0, 4.0]])
    X = LO.features(E, math.exp(-2.0))
    g = [-2.0, math.log(2.0) / 10.0, 2.0, 3.0, 5.0, 10.0]
    assert X.shape == (2, LO.input_dim(2))
    assert np.allclose(X[0], [1.0, 2.0] + g, rtol=1e-15, atol=1e-15)
    assert np.allclose(X[1], [3.0, 4.0] + g, rtol=1e-15, atol=1e-15)


def test_network_forward_exact_through_logistic_of_ln3():
    """A width-1 network whose pre-activations are both ln 3, where the
    logistic function is exactly 3/4: o = (4 / ln 3) * (3/4) ln 3 + 1 = 4, for
    two inputs that reach ln 3 through different input weights; the second
    output column reads the hidden unit with weight 0 and bias -7."""
    L3 = math.log(3.0)
    # biases enter before each activation: (L3 + 1) - 1 = L3 and 2 (3/4 L3) / (3/4) - L3 = L3
    params = {"W1": np.array([[L3 + 1.0], [5.0]]), "b1": np.array([-1.0]),
              "W2": np.array([[2.0 / 0.75]]), "b2": np.array([-L3]),
              "W3": np.array([[4.0 / L3, 0.0]]), "b3": np.array([1.0, -7.0])}
    X = np.array([[1.0, 0.0], [0.0, (L3 + 1.0) / 5.0]])
    out, _ = LO.mlp_forward(params, X)
    assert out.shape == (2, 2)
    assert out[0, 0] == pytest.approx(4.0, rel=1e-14) and out[0, 1] == -7.0
    assert out[1, 0] == pytest.approx(4.0, rel=1e-14) and out[1, 1] == -7.0


def test_adam_constant_gradient_every_step_closed_form():
    """With a constant gradient g, m_t = (1 - beta1^t) g and v_t = (1 - beta2^t) g^2,
    so the bias-corrected moments are exactly g and g^2 at every t (Kingma & Ba):
    each of three steps moves the weights by lr g / (|g| + eps).  A missing or
    wrong bias correction (e.g. beta^1 instead of beta^t) fails at t >= 2."""
    rng = np.random.default_rng(31)
    g = {"W": rng.normal(size=(3, 4)), "b": np.array([2.0, -0.5, 1e-3])}
    p = {k: rng.normal(size=v.shape) for k, v in g.items()}
    st = {}
    lr, eps = 1e-2, 1e-8
    for t in (1, 2, 3):
        before = {k: v.copy() for k, v in p.items()}
        LO.adam_step(p, g, st, lr=lr, t=t, eps=eps)
        for k in p:
            assert np.allclose(p[k] - before[k], -lr * g[k] / (np.abs(g[k]) + eps), rtol=1e-12, atol=1e-17)


def test_adam_sign_flip_two_steps_hand_computed():
    """g at t = 1, then -g at t = 2 (beta1 = 0.9, beta2 = 0.999), worked with exact
    fractions: m_2 = 0.9 * 0.1 g - 0.1 g = -0.01 g, v_2 = 0.999 * 0.001 g^2 + 0.001 g^2
    = 0.001999 g^2; m_hat = -0.01 g / 0.19, v_hat = 0.001999 g^2 / (1 - 0.999^2) = g^2.
    The second step is therefore +lr (1/19) g / (|g| + eps) (eps = 0 here)."""
    from fractions import Fraction as Fr
    g = 3.0
    p = {"x": np.array([1.0])}
    st = {}
    lr = 0.1
    LO.adam_step(p, {"x": np.array([g])}, st, lr=lr, t=1, eps=0.0)
    x1 = 1.0 - lr                      # first step: lr g / |g|
    assert p["x"][0] == pytest.approx(x1, rel=1e-15)
    LO.adam_step(p, {"x": np.array([-g])}, st, lr=lr, t=2, eps=0.0)
    b1, b2 = Fr(9, 10), Fr(999, 1000)
    G = Fr(3)
    m2 = b1 * (1 - b1) * G - (1 - b1) * G
    v2 = b2 * (1 - b2) * G * G + (1 - b2) * G * G
    mh = m2 / (1 - b1 ** 2)
    vh = v2 / (1 - b2 ** 2)
    assert mh == Fr(-3, 19) and vh == 9
    x2 = Fr(x1) - Fr(1, 10) * mh / 3    # sqrt(v_hat) = 3 exactly
    assert p["x"][0] == pytest.approx(float(x2), rel=1e-14)
    assert st["m_x"][0] == pytest.approx(float(m2), rel=1e-14)
    assert st["v_x"][0] == pytest.approx(float(v2), rel=1e-14)
