"""LAKER oracle -- plain, slow, FP64 CPU reference of the solve path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, calls or
links this module; only the tests, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP path; its only common
dependency is the seeded input generator in ``synth`` (which holds none of the
method's arithmetic).

Everything is float64 numpy.  Library primitives (matrix products, Cholesky,
symmetric eigendecomposition) serve as steps; there is no blocking, fusion or
reordering beyond what the paper's definitions state.  Section, equation and
algorithm references are to Tao & Tan, "Accelerating Regularized Attention
Kernel Regression for Spectrum Cartography".

Parity status per function (what pins it) is listed in tests/test_oracle_*.py;
functions with no independent pin say "parity unpinned" in their docstring.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

LN2 = math.log(2.0)


# ---------------------------------------------------------------------------
# Kernel construction (Sec. III-A, eq. sc-exp-kernel; Alg. 1 "Kernel Construction")
# ---------------------------------------------------------------------------

def kernel_matrix(E: np.ndarray, scale: float = 1.0, Eq: np.ndarray | None = None) -> np.ndarray:
    """Exponential attention kernel G_ij = exp(scale * <e_i, e_j>).

    The paper's kernel (eq. sc-exp-kernel) has scale 1; scale 1/sqrt(d) is the
    same kernel applied to embeddings multiplied by scale^(1/2).  With ``Eq``
    the rectangular query-by-site kernel G(x, x_i) of eq.
    sc-radio-map-reconstruction is returned.  The square kernel is made
    bitwise symmetric by computing the upper triangle and mirroring it.
    """
    E = np.asarray(E, dtype=np.float64)
    if Eq is None:
        S = E @ E.T
        S = np.triu(S) + np.triu(S, 1).T
    else:
        S = np.asarray(Eq, dtype=np.float64) @ E.T
    return np.exp(scale * S)


def system_matrix(E: np.ndarray, scale: float, lam: float) -> np.ndarray:
    """A = lambda I + G, the SPD matrix of the normal equations (eq. sc-final)."""
    n = E.shape[0]
    return kernel_matrix(E, scale) + lam * np.eye(n)


def matvec(E: np.ndarray, scale: float, lam: float, p: np.ndarray) -> np.ndarray:
    """(lambda I + G) p for a vector or an (n, k) block of vectors (Alg. 1,
    step size and residual update; the remark after eq. kernel_shrinkage_cccp_normalization
    notes only such products are needed)."""
    return system_matrix(E, scale, lam) @ p


def matvec_rows(E: np.ndarray, scale: float, lam: float, p: np.ndarray, rows) -> np.ndarray:
    """Selected entries of (lambda I + G) p, each computed on its own from row i
    of G -- usable at sizes where forming G is too large."""
    E = np.asarray(E, dtype=np.float64)
    out = []
    for i in rows:
        g = np.exp(scale * (E @ E[i]))
        out.append(g @ p + lam * p[i])
    return np.asarray(out)


def jacobi_diag(E: np.ndarray, scale: float, lam: float) -> np.ndarray:
    """Diagonal of lambda I + G; its inverse is the Jacobi preconditioner
    P_J = diag(lambda I + G)^{-1} of the numerical-layer baseline (Sec. V-A)."""
    return lam + np.exp(scale * np.einsum("ij,ij->i", E, E))


# ---------------------------------------------------------------------------
# Direct reference solution (replaces the convex-solver reference, Sec. V-A)
# ---------------------------------------------------------------------------

def solve_direct(A: np.ndarray, y: np.ndarray) -> np.ndarray:
    """alpha* = A^{-1} y by dense Cholesky; A is SPD for any lambda > 0
    (discussion after eq. sc-final).  The minimiser of R(alpha) is unique."""
    cf = sla.cho_factor(A, lower=True)
    return sla.cho_solve(cf, y)


# ---------------------------------------------------------------------------
# Random directions (eq. random_directions; Alg. 1, first two steps of learning)
# ---------------------------------------------------------------------------

def random_directions(E: np.ndarray, scale: float, lam: float, Z: np.ndarray):
    """u_k = (lambda I + G) z_k and u_bar_k = u_k / ||u_k||_2.

    Z is (n, N_r) with column k equal to z_k ~ N(0, I_n); the draws are inputs.
    Returns (U, Ubar), both (n, N_r).
    """
    U = matvec(E, scale, lam, Z)
    Ubar = U / np.linalg.norm(U, axis=0)[None, :]
    return U, Ubar


# ---------------------------------------------------------------------------
# Shrinkage-regularised CCCP (Sec. IV-C/D: eqs. kernel_shrinkage_cccp_F,
# kernel_shrinkage_cccp_Sigma, kernel_shrinkage_cccp_normalization; Alg. 1)
# ---------------------------------------------------------------------------

def cccp_F(Sigma: np.ndarray, Ubar: np.ndarray, gamma: float, eps: float) -> np.ndarray:
    """F_gamma(Sigma) = (1/(1+gamma/n)) ((n/N_r) sum_k u_k u_k^T / (u_k^T Sigma^{-1} u_k + eps) + gamma I)
    (eq. kernel_shrinkage_cccp_F)."""
    n, nr = Ubar.shape
    X = sla.cho_solve(sla.cho_factor(Sigma, lower=True), Ubar)     # Sigma^{-1} u_k
    q = np.einsum("ik,ik->k", Ubar, X)                              # u_k^T Sigma^{-1} u_k
    S = (Ubar / (q + eps)[None, :]) @ Ubar.T
    return (1.0 / (1.0 + gamma / n)) * ((n / nr) * S + gamma * np.eye(n))


def cccp_T(Sigma: np.ndarray, Ubar: np.ndarray, gamma: float, rho: float, eps: float,
           normalize: bool = True) -> np.ndarray:
    """One shrinkage-CCCP step: Sigma_tilde = (1-rho) F + rho I
    (eq. kernel_shrinkage_cccp_Sigma), then Sigma_tilde / (tr(Sigma_tilde)/n)
    (eq. kernel_shrinkage_cccp_normalization); the map T of Theorem 1."""
    n = Sigma.shape[0]
    St = (1.0 - rho) * cccp_F(Sigma, Ubar, gamma, eps) + rho * np.eye(n)
    if normalize:
        St = St / (np.trace(St) / n)
    return St


def _fixed_point(T, X0: np.ndarray, tol: float, max_iter: int, record: bool):
    """Repeat X <- T(X) from X0 until the relative Frobenius change of one
    application is at most tol, or max_iter applications.  Returns
    (X, applications, iterates or None)."""
    X = X0
    seen = [X0] if record else None
    count = 0
    while count < max_iter:
        X_next = T(X)
        count += 1
        moved = np.linalg.norm(X_next - X) / np.linalg.norm(X)
        X = X_next
        if record:
            seen.append(X)
        if moved <= tol:
            break
    return X, count, seen


def cccp_dense(Ubar: np.ndarray, gamma: float = 0.1, rho: float = 0.0, eps: float = 1e-10,
               tol: float = 1e-8, max_iter: int = 300, normalize: bool = True,
               record: bool = False):
    """Sigma_star as the fixed point of the shrinkage-CCCP map T of Theorem 1
    (eqs. kernel_shrinkage_cccp_F/Sigma/normalization), reached by applying T to
    dense n x n matrices from Sigma = I until one application changes Sigma by
    at most tol in relative Frobenius norm, or max_iter applications (the
    preconditioner-learning part of Algorithm 1).

    Returns (Sigma_star, applications of T, iterates when ``record`` is set).
    """
    n = Ubar.shape[0]
    return _fixed_point(lambda S: cccp_T(S, Ubar, gamma, rho, eps, normalize), np.eye(n), tol, max_iter, record)


def mle_objective(Theta: np.ndarray, Ubar: np.ndarray, gamma: float, eps: float = 0.0) -> float:
    """L(Theta) = -(1+gamma/n) logdet Theta + (n/N_r) sum_k log(u_k^T Theta u_k + eps)
    + gamma tr(Theta), the objective of eq. kernel-mle-theta with Theta = Sigma^{-1}
    (the nuclear norm of an SPD matrix is its trace, remark after eq. prob:kernel-mle).
    With eps > 0 this is the objective whose CCCP linearisation gives eq.
    kernel_shrinkage_cccp_F."""
    n, nr = Ubar.shape
    sign, logdet = np.linalg.slogdet(Theta)
    if sign <= 0:
        return float("inf")
    quad = np.einsum("ik,ij,jk->k", Ubar, Theta, Ubar)
    return float(-(1.0 + gamma / n) * logdet + (n / nr) * np.sum(np.log(quad + eps))
                 + gamma * np.trace(Theta))


def cccp_lowrank(Ubar: np.ndarray, gamma: float = 0.1, rho: float = 0.0, eps: float = 1e-10,
                 tol: float = 1e-8, max_iter: int = 300):
    """The same shrinkage-CCCP iteration carried in exact low-rank coordinates.

    From Sigma_0 = I every iterate of eqs. kernel_shrinkage_cccp_F/Sigma/normalization
    has the form Sigma_t = b_t I + a_t Ubar diag(w) Ubar^T with
        w_k    = 1 / (q_k + eps),  q_k = u_k^T Sigma_{t-1}^{-1} u_k,
        tau    = tr(Sigma_tilde)/n = (1-rho) c (sum_k w_k ||u_k||^2 / N_r + gamma) + rho,
        a_t    = (1-rho) c n / (N_r tau),   b_t = ((1-rho) c gamma + rho) / tau,
    c = 1/(1+gamma/n).  By Woodbury, with C = Ubar^T Ubar and
    M = (b/a) diag(1/w) + C,  q_k = (M^{-1} C)_kk / (a w_k).
    The stopping rule is the dense one, ||Sigma_{t+1}-Sigma_t||_F/||Sigma_t||_F,
    evaluated exactly through C.

    Returns (a, b, w, iterations).
    """
    n, nr = Ubar.shape
    C = Ubar.T @ Ubar
    cdiag = np.diag(C).copy()
    c = 1.0 / (1.0 + gamma / n)
    a, b, w = 0.0, 1.0, np.zeros(nr)
    it = 0
    for it in range(1, max_iter + 1):
        if a == 0.0:
            q = cdiag.copy()                          # Sigma_0 = I
        else:
            M = (b / a) * np.diag(1.0 / w) + C
            q = np.diag(np.linalg.solve(M, C)) / (a * w)
        w_new = 1.0 / (q + eps)
        tau = (1.0 - rho) * c * (np.dot(w_new, cdiag) / nr + gamma) + rho
        a_new = (1.0 - rho) * c * n / (nr * tau)
        b_new = ((1.0 - rho) * c * gamma + rho) / tau
        change = _lowrank_frob_change(C, n, a, b, w, a_new, b_new, w_new)
        a, b, w = a_new, b_new, w_new
        if change <= tol:
            break
    return a, b, w, it


def _lowrank_frob_change(C, n, a0, b0, w0, a1, b1, w1) -> float:
    """||S1 - S0||_F / ||S0||_F for S = b I + a Ubar diag(w) Ubar^T, through C."""
    def frob2(db, D):
        # ||db I + Ubar D Ubar^T||_F^2 = n db^2 + 2 db sum_k D_k C_kk + sum_kl D_k D_l C_kl^2
        return n * db * db + 2.0 * db * np.dot(D, np.diag(C)) + D @ (C * C) @ D
    num = frob2(b1 - b0, a1 * w1 - a0 * w0)
    den = frob2(b0, a0 * w0)
    return math.sqrt(max(num, 0.0) / den)


def lowrank_sigma(Ubar: np.ndarray, a: float, b: float, w: np.ndarray) -> np.ndarray:
    """Dense b I + a Ubar diag(w) Ubar^T (for comparing with the dense iteration)."""
    n = Ubar.shape[0]
    return b * np.eye(n) + a * (Ubar * w[None, :]) @ Ubar.T


# ---------------------------------------------------------------------------
# Preconditioner P = Sigma_star^{-1/2} (eq. preconditioner-Sigmma; Alg. 1)
# ---------------------------------------------------------------------------

def precond_dense(Sigma: np.ndarray) -> np.ndarray:
    """P = Sigma^{-1/2} from the symmetric eigendecomposition of Sigma."""
    lam, V = np.linalg.eigh(Sigma)
    return (V * (lam ** -0.5)[None, :]) @ V.T


class LowRankPrecond:
    """P = Sigma^{-1/2} for Sigma = b I + B B^T, B = sqrt(a) Ubar diag(sqrt(w)).

    With K = B^T B = V diag(Lambda) V^T,
        P = b^{-1/2} I + B V diag(g) V^T B^T,
        g_j = -1 / (sqrt(b + Lambda_j) sqrt(b) (sqrt(b + Lambda_j) + sqrt(b))),
    which equals ((b+Lambda_j)^{-1/2} - b^{-1/2}) / Lambda_j without cancellation:
    on range(B) P acts as (b+Lambda)^{-1/2}, on its complement as b^{-1/2}.
    """

    def __init__(self, Ubar: np.ndarray, a: float, b: float, w: np.ndarray):
        self.b = float(b)
        self.B = math.sqrt(a) * Ubar * np.sqrt(w)[None, :]
        K = self.B.T @ self.B
        K = 0.5 * (K + K.T)
        Lam, V = np.linalg.eigh(K)
        Lam = np.maximum(Lam, 0.0)
        sb = math.sqrt(b)
        sl = np.sqrt(b + Lam)
        self.g = -1.0 / (sl * sb * (sl + sb))
        self.Gs = (V * self.g[None, :]) @ V.T           # V diag(g) V^T
        self.Lam = Lam

    def apply(self, r: np.ndarray) -> np.ndarray:
        return r / math.sqrt(self.b) + self.B @ (self.Gs @ (self.B.T @ r))

    def dense(self) -> np.ndarray:
        n = self.B.shape[0]
        return np.eye(n) / math.sqrt(self.b) + self.B @ self.Gs @ self.B.T


def fit_precond(E: np.ndarray, scale: float, lam: float, Z: np.ndarray, gamma: float = 0.1,
                rho: float = 0.0, eps: float = 1e-10, tol: float = 1e-8, max_iter: int = 300):
    """Alg. 1, preconditioner learning: random directions, low-rank shrinkage
    CCCP, P = Sigma_star^{-1/2}.  Returns (LowRankPrecond, cccp_iterations)."""
    _, Ubar = random_directions(E, scale, lam, Z)
    a, b, w, it = cccp_lowrank(Ubar, gamma, rho, eps, tol, max_iter)
    return LowRankPrecond(Ubar, a, b, w), it


# ---------------------------------------------------------------------------
# Preconditioned conjugate gradient (Sec. IV-E; Alg. 1 "Preconditioned Conjugate Gradient")
# ---------------------------------------------------------------------------

def pcg(apply_A, apply_P, y: np.ndarray, tol: float, max_iter: int,
        alpha0: np.ndarray | None = None):
    """Preconditioned conjugate gradients for (lambda I + G) alpha = y with an
    SPD preconditioner P (Sec. IV-E; Algorithm 1), written from the two
    conditions that define CG:

    * the step t along the search direction d minimises the A-norm of the
      error on the line alpha + t d; with the residual r = y - A alpha this is
      t = <r, P r> / <d, A d>;
    * the next direction is P r (for the updated r) made A-conjugate to d,
      which in CG takes only the multiple <r, P r>_new / <r, P r>_old of d.

    The residual is carried recursively (r <- r - t A d), and the method stops
    as soon as ||r|| / ||y|| <= tol on that recursive residual, before P is
    applied again.  Starts from alpha = 0 (r = y) or from alpha0.

    Returns (alpha, iterations, residual_history); iterations counts the
    products with A made inside the loop.
    """
    ynorm = float(np.linalg.norm(y))
    if alpha0 is None:
        x = np.zeros(y.shape[0])
        res = y.copy()
    else:
        x = alpha0.copy()
        res = y - apply_A(alpha0)
    z = apply_P(res)
    d = z.copy()
    rz = float(res @ z)
    history = []
    steps = 0
    while steps < max_iter:
        Ad = apply_A(d)
        steps += 1
        t = rz / float(d @ Ad)
        x = x + t * d
        res = res - t * Ad
        history.append(float(np.linalg.norm(res)) / ynorm)
        if history[-1] <= tol:
            break
        z = apply_P(res)
        rz_prev, rz = rz, float(res @ z)
        d = z + (rz / rz_prev) * d
    return x, steps, history


# ---------------------------------------------------------------------------
# Reconstruction and metrics (eq. sc-radio-map-reconstruction; Sec. V-A metrics)
# ---------------------------------------------------------------------------

def predict(Eq: np.ndarray, E: np.ndarray, scale: float, alpha: np.ndarray) -> np.ndarray:
    """r_hat(x) = sum_i G(x, x_i) alpha_i (eq. sc-radio-map-reconstruction)."""
    return kernel_matrix(E, scale, Eq=Eq) @ alpha


def predict_rows(Eq: np.ndarray, E: np.ndarray, scale: float, alpha: np.ndarray, rows) -> np.ndarray:
    """Selected query outputs of ``predict``, each from its own kernel row."""
    return np.asarray([np.exp(scale * (E @ Eq[j])) @ alpha for j in rows])


def relative_residual(A: np.ndarray, alpha: np.ndarray, y: np.ndarray) -> float:
    """Res. = ||(lambda I + G) alpha - y|| / ||y|| (eq. residual)."""
    return float(np.linalg.norm(A @ alpha - y) / np.linalg.norm(y))


def objective(G: np.ndarray, lam: float, alpha: np.ndarray, y: np.ndarray) -> float:
    """R(alpha) = ||G alpha - y||^2 + lambda alpha^T G alpha (eq. simu-R-definition)."""
    Ga = G @ alpha
    return float(np.dot(Ga - y, Ga - y) + lam * np.dot(alpha, Ga))


def objective_gap(G, lam, alpha, alpha_ref, y) -> float:
    """|R(alpha) - R(alpha_ref)| / |R(alpha_ref)| (eq. objective-gap)."""
    R0 = objective(G, lam, alpha_ref, y)
    return abs(objective(G, lam, alpha, y) - R0) / abs(R0)


def prediction_discrepancy(Gq: np.ndarray, alpha: np.ndarray, alpha_ref: np.ndarray) -> float:
    """||G alpha - G alpha_ref|| / ||G alpha_ref|| (eq. prediction-discrepancy)."""
    return float(np.linalg.norm(Gq @ alpha - Gq @ alpha_ref) / np.linalg.norm(Gq @ alpha_ref))


def rmse(r_hat: np.ndarray, r_true: np.ndarray) -> float:
    """eq. rmse."""
    return float(np.sqrt(np.mean((r_hat - r_true) ** 2)))


def nmse(r_hat: np.ndarray, r_true: np.ndarray) -> float:
    """eq. nmse."""
    return float(np.sum((r_hat - r_true) ** 2) / np.sum(r_true ** 2))


def condition_number(M: np.ndarray) -> float:
    """lambda_max / lambda_min of a matrix with real positive spectrum
    (eq. attention-kernel-objective); P A is similar to P^{1/2} A P^{1/2}."""
    ev = np.linalg.eigvals(M).real
    return float(ev.max() / ev.min())
