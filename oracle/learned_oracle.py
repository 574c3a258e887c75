"""Oracle of the learned rank-64-plus-diagonal preconditioner.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls or
links this module; only the tests and the benchmark's CPU-baseline leg do.  It
shares no code with the HIP path.

The paper's preconditioner is P = Sigma_star^{-1/2}, obtained by shrinkage
CCCP (Sec. IV, Alg. 1).  The learned variant replaces the fit by a per-point
network whose output defines a surrogate of Sigma_star^{1/2}:

    o_i = f_theta(x_i)  (a 3-layer MLP with SiLU activations),
    v_i = o_i[0:R],  delta_i = exp(o_i[R]),   S = diag(delta) + V V^T,

with x_i = [e_i, log lambda, log(n)/10, mean_j e_j, mean_j e_j^2].  S is SPD
for every theta, and the preconditioner is P_theta = S^{-1} (Woodbury).  It is
trained on preconditioners the method itself fits: with Gaussian probes Z and
U = Sigma_star^{1/2} Z (computed from the CCCP fit), the loss is

    L(theta) = ||Z - S^{-1} U||_F^2 / (n m),

which is small exactly when S^{-1} Sigma_star^{1/2} is close to the identity
on the probes, i.e. when P_theta acts like the CCCP preconditioner
Sigma_star^{-1/2}.  Its gradient, with Y = S^{-1} U, G = -2 (Z - Y) / (n m),
H = S^{-1} G:
    dL/d delta_i = -sum_k H_ik Y_ik,    dL/dV = -(H (Y^T V) + Y (H^T V)).

Everything here is float64 numpy; the network is evaluated exactly as written
(no fusion).  Pins: finite differences of the loss (central, h = 1e-6), the
Woodbury solve against a dense solve, the loss against its dense definition,
and Sigma^{1/2} Z against a dense eigendecomposition of Sigma.
"""
from __future__ import annotations

import math

import numpy as np

RANK = 64          # rank of the learned low-rank part
HIDDEN = 256       # width of the two hidden layers


def input_dim(d: int) -> int:
    return 3 * d + 2


def features(E: np.ndarray, lam: float) -> np.ndarray:
    """Per-point network inputs x_i = [e_i, log lambda, log(n)/10, mean e, mean e^2]."""
    n, d = E.shape
    m1 = E.mean(axis=0)
    m2 = (E * E).mean(axis=0)
    g = np.concatenate([[math.log(lam), math.log(n) / 10.0], m1, m2])
    return np.concatenate([E, np.repeat(g[None, :], n, axis=0)], axis=1)


def silu(z: np.ndarray) -> np.ndarray:
    return z / (1.0 + np.exp(-z))


def silu_grad(z: np.ndarray) -> np.ndarray:
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def mlp_forward(params: dict, X: np.ndarray):
    """o = W3^T silu(W2^T silu(W1^T x + b1) + b2) + b3 per row; weights stored
    (fan_in x fan_out).  Returns (o, cache)."""
    Z1 = X @ params["W1"] + params["b1"]
    H1 = silu(Z1)
    Z2 = H1 @ params["W2"] + params["b2"]
    H2 = silu(Z2)
    O = H2 @ params["W3"] + params["b3"]
    return O, (X, Z1, H1, Z2, H2)


def mlp_backward(params: dict, cache, dO: np.ndarray) -> dict:
    X, Z1, H1, Z2, H2 = cache
    g = {}
    g["W3"] = H2.T @ dO
    g["b3"] = dO.sum(axis=0)
    dZ2 = (dO @ params["W3"].T) * silu_grad(Z2)
    g["W2"] = H1.T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ params["W2"].T) * silu_grad(Z1)
    g["W1"] = X.T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return g


def split_output(O: np.ndarray):
    """V (n x R) and delta (n) from the network output."""
    return O[:, :RANK], np.exp(O[:, RANK])


def woodbury_solve(V: np.ndarray, delta: np.ndarray, X: np.ndarray) -> np.ndarray:
    """(diag(delta) + V V^T)^{-1} X by the Woodbury identity with the R x R
    capacitance matrix K = I + V^T D^{-1} V."""
    Di = 1.0 / delta
    K = np.eye(V.shape[1]) + V.T @ (Di[:, None] * V)
    X2 = X if X.ndim == 2 else X[:, None]
    T = Di[:, None] * X2
    out = T - Di[:, None] * (V @ np.linalg.solve(K, V.T @ T))
    return out if X.ndim == 2 else out[:, 0]


def learned_dense(V: np.ndarray, delta: np.ndarray) -> np.ndarray:
    """S = diag(delta) + V V^T (dense; for pins)."""
    return np.diag(delta) + V @ V.T


def loss(params: dict, X: np.ndarray, Z: np.ndarray, U: np.ndarray) -> float:
    O, _ = mlp_forward(params, X)
    V, delta = split_output(O)
    Y = woodbury_solve(V, delta, U)
    n, m = Z.shape
    return float(((Z - Y) ** 2).sum() / (n * m))


def loss_and_grad(params: dict, X: np.ndarray, Z: np.ndarray, U: np.ndarray):
    """L and dL/dtheta (same keys as params), plus dL/dO for checks."""
    O, cache = mlp_forward(params, X)
    V, delta = split_output(O)
    n, m = Z.shape
    Y = woodbury_solve(V, delta, U)
    R = Z - Y
    L = float((R * R).sum() / (n * m))
    G = -2.0 * R / (n * m)
    H = woodbury_solve(V, delta, G)
    d_delta = -(H * Y).sum(axis=1)
    dV = -(H @ (Y.T @ V) + Y @ (H.T @ V))
    dO = np.zeros_like(O)
    dO[:, :RANK] = dV
    dO[:, RANK] = d_delta * delta
    return L, mlp_backward(params, cache, dO), dO


def sigma_half_apply(b: float, B: np.ndarray, P_apply, Z: np.ndarray) -> np.ndarray:
    """Sigma^{1/2} Z for Sigma = b I + B B^T, computed as Sigma (Sigma^{-1/2} Z)
    with the fitted P = Sigma^{-1/2} (Sec. IV, Alg. 1 preconditioner)."""
    PZ = np.column_stack([P_apply(Z[:, k]) for k in range(Z.shape[1])])
    return b * PZ + B @ (B.T @ PZ)


def adam_step(params: dict, grads: dict, state: dict, lr: float, t: int,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam update (Kingma & Ba), in place; state holds m and v per key."""
    for k in params:
        m = state.setdefault("m_" + k, np.zeros_like(params[k]))
        v = state.setdefault("v_" + k, np.zeros_like(params[k]))
        m[...] = beta1 * m + (1 - beta1) * grads[k]
        v[...] = beta2 * v + (1 - beta2) * grads[k] ** 2
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        params[k] = params[k] - lr * mh / (np.sqrt(vh) + eps)
