"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these compares the oracle with itself: each pin is a printed value of
the paper's worked example, a closed form, an invariant of the method, a
special case with a textbook answer, or a brute-force evaluation on tiny
inputs.  A dropped term, a wrong sign or index, or a transposed operand in the
oracle fails at least one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import laker_oracle as O
from synth import make_problem, make_directions

HERE = os.path.dirname(os.path.abspath(__file__))


def _example1():
    with open(os.path.join(HERE, "golden", "example1.json")) as f:
        return json.load(f)


# --- Example 1 (Sec. IV-E): printed values -----------------------------------------

def test_example1_kernel_matches_printed():
    ex = _example1()
    E = np.array(ex["E"])
    # embeddings are printed to 3 decimals: |de| <= 5e-4 per entry moves each
    # <e_i,e_j> by <= 2 * 5e-4 * max|e| ~ 4.5e-4, G by ~ 1.3x that, plus 5e-4
    # print rounding of G itself  ->  1.5e-3 bound
    G = O.kernel_matrix(E, 1.0)
    assert np.abs(G - np.array(ex["G"])).max() <= 1.5e-3
    A = O.system_matrix(E, 1.0, ex["lambda"])
    assert np.abs(A - np.array(ex["A"])).max() <= 1.5e-3
    gq = O.kernel_matrix(E, 1.0, Eq=np.array([ex["e_query"]]))[0]
    assert np.abs(gq - np.array(ex["g_query"])).max() <= 1.5e-3


def test_example1_solution_matches_printed():
    ex = _example1()
    E, y = np.array(ex["E"]), np.array(ex["y"])
    A = O.system_matrix(E, 1.0, ex["lambda"])
    alpha = O.solve_direct(A, y)
    a_pr = np.array(ex["alpha"])
    # printed alpha solves the system built from unrounded embeddings; the
    # rounding of e (cond(A) ~ 29) moves alpha by ~6e-4 relative
    assert np.linalg.norm(alpha - a_pr) / np.linalg.norm(a_pr) <= 1e-3
    assert O.relative_residual(A, a_pr, y) <= 2e-4
    # and the PCG of Alg. 1 with P = I reaches the same alpha
    a_cg, it, _ = O.pcg(lambda v: A @ v, lambda v: v, y, 1e-13, 50)
    assert it <= 3 + 1
    assert np.linalg.norm(a_cg - alpha) / np.linalg.norm(alpha) <= 1e-10


def test_example1_prediction_matches_printed():
    ex = _example1()
    E, y = np.array(ex["E"]), np.array(ex["y"])
    alpha = O.solve_direct(O.system_matrix(E, 1.0, ex["lambda"]), y)
    r = O.predict(np.array([ex["e_query"]]), E, 1.0, alpha)[0]
    assert abs(r - ex["r_hat_query"]) <= 0.05      # printed to one decimal


# --- brute force on tiny inputs ----------------------------------------------------

def _tiny(n, d, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.5, (n, d)), rng.normal(0, 1, n)


def test_kernel_and_matvec_bruteforce():
    E, p = _tiny(7, 3, 1)
    s, lam = 0.7, 0.3
    G = O.kernel_matrix(E, s)
    Av = O.matvec(E, s, lam, p)
    for i in range(7):
        acc = 0.0
        for j in range(7):
            dot = sum(E[i][k] * E[j][k] for k in range(3))
            gij = math.exp(s * dot)
            assert abs(G[i, j] - gij) <= 1e-15 * gij
            acc += gij * p[j]
        acc += lam * p[i]
        assert abs(Av[i] - acc) <= 1e-14 * (1 + abs(acc))
    rows = [0, 3, 6]
    assert np.allclose(O.matvec_rows(E, s, lam, p, rows), Av[rows], rtol=1e-14, atol=1e-14)
    # Jacobi diagonal
    assert np.allclose(O.jacobi_diag(E, s, lam), np.diag(G) + lam, rtol=1e-15)
    # rectangular kernel
    Eq = _tiny(4, 3, 2)[0]
    Gq = O.kernel_matrix(E, s, Eq=Eq)
    for a in range(4):
        for j in range(7):
            assert abs(Gq[a, j] - math.exp(s * sum(Eq[a][k] * E[j][k] for k in range(3)))) <= 1e-15 * Gq[a, j]


def _exact_solve(A, y):
    """Gaussian elimination in exact rationals on the float entries."""
    n = len(y)
    M = [[Fraction(float(A[i, j])) for j in range(n)] + [Fraction(float(y[i]))] for i in range(n)]
    for k in range(n):
        piv = max(range(k, n), key=lambda r: abs(M[r][k]))
        M[k], M[piv] = M[piv], M[k]
        for r in range(n):
            if r != k and M[r][k] != 0:
                f = M[r][k] / M[k][k]
                M[r] = [a - f * b for a, b in zip(M[r], M[k])]
    return np.array([float(M[i][n] / M[i][i]) for i in range(n)])


def test_direct_solve_exact_rational():
    for seed in range(3):
        E, y = _tiny(4, 2, 10 + seed)
        A = O.system_matrix(E, 1.0, 0.2)
        ex = _exact_solve(A, y)
        al = O.solve_direct(A, y)
        assert np.linalg.norm(al - ex) <= 1e-12 * np.linalg.norm(ex)


# --- closed forms ------------------------------------------------------------------

def test_zero_embeddings_closed_form():
    """E = 0 gives G = 1 1^T exactly; Sherman-Morrison gives
    alpha = y/lam - (1^T y / (lam (lam + n))) 1; the spectrum of A is {lam, lam + n}
    so CG ends in 2 steps."""
    n, lam = 50, 0.5
    E = np.zeros((n, 4))
    y = np.random.default_rng(0).normal(-80, 10, n)
    G = O.kernel_matrix(E, 0.25)
    assert np.array_equal(G, np.ones((n, n)))
    A = O.system_matrix(E, 0.25, lam)
    al = O.solve_direct(A, y)
    closed = y / lam - (y.sum() / (lam * (lam + n))) * np.ones(n)
    assert np.linalg.norm(al - closed) <= 1e-13 * np.linalg.norm(closed)
    a_cg, it, _ = O.pcg(lambda v: O.matvec(E, 0.25, lam, v), lambda v: v, y, 1e-12, 100)
    assert it <= 2
    assert np.linalg.norm(a_cg - closed) <= 1e-11 * np.linalg.norm(closed)


def _cluster_problem(n, Q, cval):
    E = np.zeros((n, Q))
    for i in range(n):
        E[i, i % Q] = cval
    return E


def test_cluster_spectrum_closed_form():
    """One-hot cluster embeddings e_i = c u_{cl(i)}, Q clusters of size q:
    G = 1 1^T + (e^{c^2} - 1) blockdiag(1_q 1_q^T), so A has exactly the
    eigenvalues lam (n - Q times), lam + (e^{c^2}-1) q (Q - 1 times) and
    lam + (e^{c^2}-1) q + n (once); CG ends in 3 steps.  This is the exact form
    of the clustered model of Sec. III-B."""
    n, Q, cval, lam = 60, 4, 1.1, 0.2
    q = n // Q
    E = _cluster_problem(n, Q, cval)
    A = O.system_matrix(E, 1.0, lam)
    ev = np.sort(np.linalg.eigvalsh(A))
    m = math.expm1(cval * cval) * q
    expect = np.sort(np.r_[np.full(n - Q, lam), np.full(Q - 1, lam + m), [lam + m + n]])
    assert np.allclose(ev, expect, rtol=1e-12, atol=1e-11)
    # kappa = 1 + (n + (e^{c^2}-1) q)/lam, the clustered estimate 1 + n/(Q lam) up to the constant block
    y = np.random.default_rng(1).normal(-70, 5, n)
    _, it, _ = O.pcg(lambda v: A @ v, lambda v: v, y, 1e-12, 100)
    assert it <= 3


def test_kernel_is_spd_schur_product():
    """G = exp o (s E E^T) = sum_m s^m (E E^T)^{o m} / m! is PSD (Schur product
    theorem); the square kernel is bitwise symmetric."""
    pr = make_problem(300, 16, 1e-3, seed=3)
    G = O.kernel_matrix(pr.E, pr.scale)
    assert np.array_equal(G, G.T)
    ev = np.linalg.eigvalsh(G)
    assert ev.min() >= -300 * np.finfo(float).eps * ev.max()
    np.linalg.cholesky(G + pr.lam * np.eye(300))


def test_objective_at_solution_closed_form():
    """At alpha*, G alpha* = y - lam alpha* (eq. sc-final) so
    R(alpha*) = lam y^T alpha* (eq. simu-R-definition)."""
    pr = make_problem(200, 8, 1e-2, seed=4)
    G = O.kernel_matrix(pr.E, pr.scale)
    A = G + pr.lam * np.eye(pr.n)
    al = O.solve_direct(A, pr.y)
    R = O.objective(G, pr.lam, al, pr.y)
    assert abs(R - pr.lam * pr.y @ al) <= 1e-8 * abs(R)
    assert O.objective_gap(G, pr.lam, al, al, pr.y) == 0.0


def test_prediction_at_training_sites():
    """r_hat(x_i) = (G alpha*)_i = y_i - lam alpha*_i (eqs. sc-final and
    sc-radio-map-reconstruction)."""
    pr = make_problem(150, 8, 1e-2, seed=5)
    A = O.system_matrix(pr.E, pr.scale, pr.lam)
    al = O.solve_direct(A, pr.y)
    r = O.predict(pr.E, pr.E, pr.scale, al)
    assert np.allclose(r, pr.y - pr.lam * al, rtol=0, atol=1e-9 * np.abs(pr.y).max())
    rows = [0, 7, 149]
    assert np.allclose(O.predict_rows(pr.E, pr.E, pr.scale, al, rows), r[rows], rtol=1e-13)


def test_metrics_definitions():
    r_true = np.array([1.0, 2.0, 3.0, 4.0])
    r_hat = np.array([1.0, 2.5, 2.0, 4.0])
    assert O.rmse(r_hat, r_true) == pytest.approx(math.sqrt((0.25 + 1.0) / 4))
    assert O.nmse(r_hat, r_true) == pytest.approx(1.25 / 30.0)


# --- PCG --------------------------------------------------------------------------

def test_pcg_finite_termination_tiny():
    """CG on an n x n SPD system ends within n steps in exact arithmetic; in FP64
    the residual after step n is at rounding level (kappa(A) <= 40 here)."""
    for n in range(2, 9):
        E, y = _tiny(n, 3, 100 + n)
        A = O.system_matrix(E, 1.0, 1.0)
        al, it, hist = O.pcg(lambda v: A @ v, lambda v: v, y, 1e-12, 10 * n)
        assert it <= n + 1
        assert hist[n - 1] <= 1e-8
        assert all(h > 1e-6 for h in hist[: n - 1]) or n < 3
        assert np.linalg.norm(al - _exact_solve(A, y)) <= 1e-10 * np.linalg.norm(al)


def test_pcg_with_exact_inverse_is_one_step():
    E, y = _tiny(20, 4, 7)
    A = O.system_matrix(E, 1.0, 0.1)
    Ainv = np.linalg.inv(A)
    al, it, _ = O.pcg(lambda v: A @ v, lambda v: Ainv @ v, y, 1e-10, 10)
    assert it == 1


def test_pcg_matches_direct_at_small_config():
    """n = 512, d = 16, lam = 1e-3, s = 1/4: PCG run to 1e-12 recovers the
    Cholesky alpha* to 1e-10 (relative), with P = I and with Jacobi."""
    pr = make_problem(512, 16, 1e-3, seed=0)
    A = O.system_matrix(pr.E, pr.scale, pr.lam)
    ref = O.solve_direct(A, pr.y)
    jd = O.jacobi_diag(pr.E, pr.scale, pr.lam)
    for P in (lambda v: v, lambda v: v / jd):
        al, it, hist = O.pcg(lambda v: A @ v, P, pr.y, 1e-12, 5000)
        assert hist[-1] <= 1e-12
        assert np.linalg.norm(al - ref) / np.linalg.norm(ref) <= 1e-10
        assert O.relative_residual(A, al, pr.y) <= 1e-11


def test_pcg_warm_start_residual():
    pr = make_problem(100, 8, 1e-2, seed=8)
    A = O.system_matrix(pr.E, pr.scale, pr.lam)
    ref = O.solve_direct(A, pr.y)
    al, it, _ = O.pcg(lambda v: A @ v, lambda v: v, pr.y, 1e-12, 5000, alpha0=ref)
    assert it == 1 or np.linalg.norm(al - ref) <= 1e-9 * np.linalg.norm(ref)


# --- random directions and CCCP -----------------------------------------------------

def test_random_directions_normalised():
    E, _ = _tiny(6, 2, 3)
    Z = make_directions(6, 4, 0)
    U, Ub = O.random_directions(E, 1.0, 0.5, Z)
    assert np.allclose(np.linalg.norm(Ub, axis=0), 1.0, rtol=1e-15, atol=1e-15)
    for k in range(4):
        for i in range(6):
            acc = 0.5 * Z[i, k]
            for j in range(6):
                acc += math.exp(sum(E[i][m] * E[j][m] for m in range(2))) * Z[j, k]
            assert abs(U[i, k] - acc) <= 1e-13 * (1 + abs(acc))


def _directions(n, nr, seed, lam=1e-2, d=8):
    pr = make_problem(n, d, lam, seed=seed)
    Z = make_directions(n, nr, seed)
    _, Ub = O.random_directions(pr.E, pr.scale, pr.lam, Z)
    return pr, Ub


def test_cccp_invariants_theorem1():
    """Every iterate has tr(Sigma_t) = n and Sigma_t >= ((1-rho) c gamma + rho)/tau I > 0;
    the limit is a fixed point of T with tr = n (Theorem 1)."""
    n, nr, gamma, rho, eps = 120, 40, 0.1, 0.05, 1e-10
    pr, Ub = _directions(n, nr, 11)
    Sig, it, hist = O.cccp_dense(Ub, gamma, rho, eps, 1e-12, 500, record=True)
    assert it < 500
    for S in hist:
        assert abs(np.trace(S) - n) <= 1e-10 * n
        assert np.linalg.eigvalsh(S).min() > 0
    # lower bound from the shrinkage term: Sigma_{t+1} >= rho / tau I with tau <= (1-rho) c (max_k n/(N_r) ... ) bound
    # checked in its plain form: smallest eigenvalue at least rho * n / tr(Sigma_tilde) > 0
    T = O.cccp_T(Sig, Ub, gamma, rho, eps)
    assert np.linalg.norm(T - Sig) / np.linalg.norm(Sig) <= 1e-10
    # independent evaluation of the fixed-point equation, direction by direction
    Sinv = np.linalg.inv(Sig)
    c = 1.0 / (1.0 + gamma / n)
    F = np.zeros((n, n))
    for k in range(nr):
        u = Ub[:, k]
        F += np.outer(u, u) / (u @ Sinv @ u + eps)
    F = c * ((n / nr) * F + gamma * np.eye(n))
    St = (1 - rho) * F + rho * np.eye(n)
    assert np.linalg.norm(n * St / np.trace(St) - Sig) / np.linalg.norm(Sig) <= 1e-9


def test_cccp_is_majorize_minimize():
    """Without shrinkage and normalisation the update is the CCCP step of
    L(Theta) = l(Theta) + g(Theta) with the concave g linearised (Sec. IV-C), so
    L(Sigma_t^{-1}) never increases.  Unnormalised, the scale drifts (Sec. IV-C):
    the largest eigenvalue grows ~2x per step, so only the first 10 steps are
    taken, where Sigma^{-1} is still computed accurately."""
    n, nr, gamma, eps = 60, 30, 0.1, 1e-10
    _, Ub = _directions(n, nr, 12)
    _, _, hist = O.cccp_dense(Ub, gamma, 0.0, eps, 1e-14, 10, normalize=False, record=True)
    L = [O.mle_objective(np.linalg.inv(S), Ub, gamma, eps) for S in hist]
    for a, b in zip(L, L[1:]):
        assert b <= a + 1e-9 * abs(a)
    assert L[-1] < L[0] - 1e-3


def test_tyler_limit_recovers_inverse():
    """gamma = rho = 0 is Tyler's fixed point (eq. tyler-fixed-point); as N_r grows
    Sigma_star -> n A^2 / tr(A^2) (u_k ~ N(0, A^2)), so kappa(P A) -> 1."""
    rng = np.random.default_rng(5)
    n = 8
    E = rng.normal(0, 0.6, (n, 3))
    A = O.system_matrix(E, 1.0, 0.05)
    kA = O.condition_number(A)
    ks = []
    for nr in (64, 512, 4096):
        Z = rng.standard_normal((n, nr))
        _, Ub = O.random_directions(E, 1.0, 0.05, Z)
        Sig, _, _ = O.cccp_dense(Ub, 0.0, 0.0, 1e-14, 1e-12, 2000)
        P = O.precond_dense(Sig)
        ks.append(O.condition_number(P @ A))
    assert kA > 20
    assert ks[0] > ks[1] > ks[2]
    assert ks[2] < 1.15


def test_lowrank_cccp_equals_dense():
    n, nr, gamma, rho = 200, 30, 0.1, 0.05
    _, Ub = _directions(n, nr, 13)
    Sd, itd, _ = O.cccp_dense(Ub, gamma, rho, 1e-10, 1e-10, 300)
    a, b, w, itl = O.cccp_lowrank(Ub, gamma, rho, 1e-10, 1e-10, 300)
    Sl = O.lowrank_sigma(Ub, a, b, w)
    assert abs(itd - itl) <= 1
    assert np.linalg.norm(Sl - Sd) / np.linalg.norm(Sd) <= 1e-9
    assert abs(np.trace(Sl) - n) <= 1e-10 * n


def test_preconditioner_is_inverse_square_root():
    """P = Sigma^{-1/2}: P Sigma P = I, P symmetric positive definite; the
    low-rank closed form equals the dense one."""
    n, nr, gamma, rho = 150, 25, 0.1, 0.02
    _, Ub = _directions(n, nr, 14)
    a, b, w, _ = O.cccp_lowrank(Ub, gamma, rho, 1e-10, 1e-10, 300)
    Sig = O.lowrank_sigma(Ub, a, b, w)
    Pd = O.precond_dense(Sig)
    assert np.linalg.norm(Pd @ Sig @ Pd - np.eye(n)) <= 1e-9
    lr = O.LowRankPrecond(Ub, a, b, w)
    Pl = lr.dense()
    assert np.abs(Pl - Pl.T).max() <= 1e-12 * np.abs(Pl).max()
    assert np.linalg.eigvalsh(Pl).min() > 0
    assert np.linalg.norm(Pl @ Sig @ Pl - np.eye(n)) <= 1e-9
    assert np.linalg.norm(Pl - Pd) / np.linalg.norm(Pd) <= 1e-10
    v = np.random.default_rng(0).normal(size=n)
    assert np.allclose(lr.apply(v), Pd @ v, rtol=1e-9, atol=1e-9 * np.abs(Pd @ v).max())


def test_laker_pcg_solves_and_preconditions():
    """End to end at a paper-like regime (scale 1, lam = 1e-2, 10-d embeddings):
    LAKER-PCG reaches the direct alpha*, and the preconditioned system is better
    conditioned than A.  The paper's own kappa / iteration numbers depend on its
    unspecified embedding and schedules: parity unpinned for those values."""
    n = 400
    pr = make_problem(n, 10, 1e-2, seed=21, scale=1.0)
    A = O.system_matrix(pr.E, pr.scale, pr.lam)
    ref = O.solve_direct(A, pr.y)
    Z = make_directions(n, 80, 21)
    P, _ = O.fit_precond(pr.E, pr.scale, pr.lam, Z, gamma=0.1, rho=0.0)
    al, it, _ = O.pcg(lambda v: A @ v, P.apply, pr.y, 1e-11, 5000)
    assert np.linalg.norm(al - ref) / np.linalg.norm(ref) <= 1e-8
    _, it_cg, _ = O.pcg(lambda v: A @ v, lambda v: v, pr.y, 1e-11, 5000)
    assert O.condition_number(P.dense() @ A) < O.condition_number(A)
    assert it < it_cg


# --- metrics with hand-computed values ------------------------------------------------

def test_prediction_discrepancy_hand_computed():
    """||Gq a - Gq a_ref|| / ||Gq a_ref|| (Sec. V-A, prediction discrepancy) on a
    2 x 2 case worked by hand: Gq a = (3, 7), Gq a_ref = (1, 3), difference
    (2, 4): sqrt(20) / sqrt(10) = sqrt(2).  Normalising by ||Gq a|| instead
    would give sqrt(20/58); dropping Gq, ||a - a_ref|| / ||a_ref|| = 1."""
    Gq = np.array([[1.0, 2.0], [3.0, 4.0]])
    a, a_ref = np.array([1.0, 1.0]), np.array([1.0, 0.0])
    assert O.prediction_discrepancy(Gq, a, a_ref) == pytest.approx(math.sqrt(2.0), rel=1e-15)
    # a transposed Gq gives (4, 6) and (1, 2), difference (3, 4): 5 / sqrt(5) -- not sqrt(2)
    assert O.prediction_discrepancy(Gq.T, a, a_ref) == pytest.approx(math.sqrt(5.0), rel=1e-15)
    assert O.prediction_discrepancy(Gq, a_ref, a_ref) == 0.0


def test_objective_gap_hand_computed():
    """R(a) = ||G a - y||^2 + lam a^T G a (Sec. V-A) and the relative gap on a
    diagonal 2 x 2 case: G = diag(2, 1), lam = 1, y = (2, 1), a_ref = (1, 0):
    R(a_ref) = 1 + 2 = 3; a = (0, 1): G a - y = (-2, 0), R = 4 + 1 = 5; gap 2/3."""
    G = np.diag([2.0, 1.0])
    y = np.array([2.0, 1.0])
    assert O.objective(G, 1.0, np.array([1.0, 0.0]), y) == pytest.approx(3.0, rel=1e-15)
    assert O.objective(G, 1.0, np.array([0.0, 1.0]), y) == pytest.approx(5.0, rel=1e-15)
    assert O.objective_gap(G, 1.0, np.array([0.0, 1.0]), np.array([1.0, 0.0]), y) == pytest.approx(2.0 / 3.0,
                                                                                                    rel=1e-15)


def test_condition_number_known_spectra():
    """kappa = lambda_max / lambda_min of the (real, positive) eigenvalues.
    * a diagonal matrix: the ratio of its extreme entries;
    * a non-normal triangular matrix: its diagonal entries are its eigenvalues
      (ratio 4), while its singular values have ratio ~ 1e4 -- a singular-value
      definition fails here;
    * P A with P = A^{-1/2} for the clustered system, whose spectrum is known
      in closed form: eigenvalues lam, lam + (e^{c^2}-1) q and
      lam + (e^{c^2}-1) q + n, so kappa(A) = (lam + (e^{c^2}-1) q + n) / lam and
      kappa(A^{-1/2} A) = sqrt(kappa(A)); P = A^{-1} gives 1."""
    assert O.condition_number(np.diag([2.0, 5.0, 10.0])) == pytest.approx(5.0, rel=1e-14)
    M = np.array([[1.0, 100.0], [0.0, 4.0]])
    assert O.condition_number(M) == pytest.approx(4.0, rel=1e-13)
    sv = np.linalg.svd(M, compute_uv=False)
    assert sv[0] / sv[-1] > 1000.0
    nq, q, cc, lam = 6, 5, 0.8, 0.5
    n = nq * q
    E = np.zeros((n, nq))
    for i in range(n):
        E[i, i // q] = cc
    A = O.system_matrix(E, 1.0, lam)
    kA = (lam + (math.exp(cc * cc) - 1.0) * q + n) / lam
    assert O.condition_number(A) == pytest.approx(kA, rel=1e-12)
    ev, V = np.linalg.eigh(A)
    Ph = (V * ev ** -0.5) @ V.T
    assert O.condition_number(Ph @ A) == pytest.approx(math.sqrt(kA), rel=1e-12)
    assert O.condition_number(np.linalg.inv(A) @ A) == pytest.approx(1.0, rel=1e-12)


# --- CCCP with orthonormal directions: scalar closed form -------------------------------

def _orthonormal(n, nr, seed):
    Q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(n, nr)))
    return Q


def _two_level(n, nr, gamma, rho, eps, s1):
    """One step of eqs. kernel_shrinkage_cccp_F/Sigma/normalization worked by hand for
    Sigma = s1 on span(U_bar), s0 elsewhere, with U_bar orthonormal (C = I):
    every q_k = 1/s1, so F = c((n/N_r) s1/(1 + eps s1) U U^T + gamma I) and
    Sigma_tilde has eigenvalue (1-rho) c ((n/N_r) h + gamma) + rho on span(U)
    (h = s1/(1 + eps s1)) and (1-rho) c gamma + rho elsewhere; the trace
    normalisation divides both by tau = (1-rho) c (h + gamma) + rho."""
    c = 1.0 / (1.0 + gamma / n)
    h = s1 / (1.0 + eps * s1)
    tau = (1 - rho) * c * (h + gamma) + rho
    return ((1 - rho) * c * ((n / nr) * h + gamma) + rho) / tau, ((1 - rho) * c * gamma + rho) / tau


def test_cccp_step_orthonormal_directions_closed_form():
    """From Sigma_0 = I (s1 = 1), three steps of the oracle's map T equal the
    hand-worked two-level recursion: N_r eigenvalues s1 on span(U_bar) and
    n - N_r eigenvalues s0.  gamma = 5 with n = 40 makes c = 1/(1 + gamma/n) = 0.889
    and rho = 0.2 keeps it from cancelling in the normalisation; eps = 1e-3
    enters through h = s1/(1 + eps s1)."""
    n, nr, gamma, rho, eps = 40, 6, 5.0, 0.2, 1e-3
    U = _orthonormal(n, nr, 1)
    S = np.eye(n)
    s1 = 1.0
    for _ in range(3):
        S = O.cccp_T(S, U, gamma, rho, eps)
        s1, s0 = _two_level(n, nr, gamma, rho, eps, s1)
        ref = s0 * np.eye(n) + (s1 - s0) * U @ U.T
        assert np.abs(S - ref).max() <= 1e-12 * s1
        assert nr * s1 + (n - nr) * s0 == pytest.approx(n, rel=1e-13)


def test_cccp_fixed_point_orthonormal_directions_closed_form():
    """With eps = 0 the fixed point s1 of the two-level recursion solves
    k s1^2 + (K - k n/N_r) s1 - K = 0 with k = (1-rho) c and K = (1-rho) c gamma + rho
    (clear the denominator tau = k (s1 + gamma) + rho); s0 = K / (k s1 + K).
    The dense iteration must converge to s1 I on span(U_bar) and s0 elsewhere,
    and its low-rank form to the same matrix.  The second case has rho = 0,
    where c cancels: the same roots with k = 1, K = gamma."""
    n, nr = 48, 8
    for gamma, rho in ((6.0, 0.3), (2.0, 0.0)):
        c = 1.0 / (1.0 + gamma / n)
        k = (1 - rho) * c
        K = (1 - rho) * c * gamma + rho
        bq = K - k * n / nr
        s1 = (-bq + math.sqrt(bq * bq + 4.0 * k * K)) / (2.0 * k)
        s0 = K / (k * s1 + K)
        U = _orthonormal(n, nr, 2)
        Sig, it, _ = O.cccp_dense(U, gamma, rho, 0.0, 1e-14, 2000)
        assert it < 2000
        ev = np.sort(np.linalg.eigvalsh(Sig))
        assert np.allclose(ev[:n - nr], s0, rtol=1e-11, atol=0)
        assert np.allclose(ev[n - nr:], s1, rtol=1e-11, atol=0)
        a, b, w, _ = O.cccp_lowrank(U, gamma, rho, 0.0, 1e-14, 2000)
        assert np.abs(O.lowrank_sigma(U, a, b, w) - Sig).max() <= 1e-10 * s1


def test_cccp_smallest_eigenvalue_bound():
    """Every iterate satisfies lambda_min(Sigma_{t+1}) >= ((1-rho) c gamma + rho) / tau_t
    with tau_t = tr(Sigma_tilde_t) / n (the shrinkage and gamma terms add that
    multiple of I to a PSD sum before normalising); tau_t is evaluated here
    directly from the definition of Sigma_tilde, direction by direction."""
    n, nr, gamma, rho, eps = 90, 30, 0.1, 0.05, 1e-10
    _, Ub = _directions(n, nr, 19)
    _, _, hist = O.cccp_dense(Ub, gamma, rho, eps, 1e-12, 60, record=True)
    c = 1.0 / (1.0 + gamma / n)
    for S0, S1 in zip(hist, hist[1:]):
        Sinv = np.linalg.inv(S0)
        tr_sum = 0.0
        for kk in range(nr):
            u = Ub[:, kk]
            tr_sum += (u @ u) / (u @ Sinv @ u + eps)
        tau = ((1 - rho) * c * ((n / nr) * tr_sum + gamma * n) + rho * n) / n
        bound = ((1 - rho) * c * gamma + rho) / tau
        lmin = np.linalg.eigvalsh(S1).min()
        assert lmin >= bound * (1.0 - 1e-10)
        # the bound is attained on the complement of span(U_bar) (N_r < n)
        assert lmin <= bound * (1.0 + 1e-8)
