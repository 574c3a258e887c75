"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Sizes span several tiles and a ragged tail; the full-size checks (n = 16384, d = 64) use
sampled rows the oracle computes one by one.  Tolerances:
  * float64 products: 1e-13 relative to sum_j |G_ij p_j| + lam |p_i| (FP64
    rounding of d-term dot products, exp and n-term sums);
  * float32 products: 2e-6 relative to the same magnitude (float32 inputs
    rounded once, a d-term float32 MFMA dot product of the pre-scaled rows,
    exp2 within 2 ulp; the exp(.) p_j products of one stage, 4 per lane and
    row, are summed in float32 with weights rounded to float32, 4 u relative,
    then accumulated in float64);
  * bfloat16 products: compared with the oracle evaluated on the same
    bfloat16-rounded pre-scaled rows (G_ij = 2^{<e^_i, e^_j>}), 2e-6 relative
    (bfloat16 products are exact in float32; float32 MFMA accumulation over d
    terms and exp2 as above; the square products of dp = 32, 64 store their
    partial sums in float32, one rounding of each, 2^-24 of the magnitude at
    most in all);
  * float64 solves: alpha within 1e-10 (relative) of the Cholesky solution when
    PCG is run to 1e-12.
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


def _gp(pr):
    return L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)


def _mag(E, s, lam, p):
    G = O.kernel_matrix(E, s)
    return np.abs(G) @ np.abs(p) + lam * np.abs(p)


@pytest.mark.parametrize("n,d", [(1, 4), (3, 2), (64, 16), (777, 10), (2048 + 37, 64), (1500, 128)])
def test_matvec_f64_parity(n, d):
    pr = make_problem(n, d, 1e-3, seed=n)
    p = np.random.default_rng(n).normal(size=n)
    w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), "f64").cpu().numpy()
    ref = O.matvec(pr.E, pr.scale, pr.lam, p)
    err = np.abs(w - ref) / _mag(pr.E, pr.scale, pr.lam, p)
    assert err.max() <= 1e-13, (n, d, err.max())


@pytest.mark.parametrize("n,d", [(3, 2), (777, 10), (2048 + 37, 64)])
def test_matvec_f32_parity(n, d):
    pr = make_problem(n, d, 1e-3, seed=n)
    p = np.random.default_rng(n).normal(size=n)
    w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), "f32").cpu().numpy()
    ref = O.matvec(pr.E, pr.scale, pr.lam, p)
    err = np.abs(w - ref) / _mag(pr.E, pr.scale, pr.lam, p)
    assert err.max() <= 2e-6, (n, d, err.max())


def _bf16_rows(E, s):
    """fp64 -> fp32 (round to nearest) -> bfloat16 (round to nearest even) of
    sqrt(s log2 e) e, the rows the bfloat16 product works on."""
    c = np.sqrt(s * np.log2(np.e))
    u = (c * E).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


@pytest.mark.parametrize("n,d", [(3, 2), (777, 10), (2048 + 37, 64), (1500, 128)])
def test_matvec_bf16_parity(n, d):
    pr = make_problem(n, d, 1e-3, seed=n)
    p = np.random.default_rng(n).normal(size=n)
    w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), "bf16").cpu().numpy()
    Eb = _bf16_rows(pr.E, pr.scale)
    ref = O.matvec(Eb, np.log(2.0), pr.lam, p)
    err = np.abs(w - ref) / _mag(Eb, np.log(2.0), pr.lam, p)
    assert err.max() <= 2e-6, (n, d, err.max())
    # and the bfloat16 kernel is within its rounding of the exact kernel
    ref64 = O.matvec(pr.E, pr.scale, pr.lam, p)
    assert (np.abs(w - ref64) / _mag(pr.E, pr.scale, pr.lam, p)).max() <= 2e-2


@pytest.mark.parametrize("n,d,prec", [(6000, 64, "f32"), (7000 + 37, 32, "f32"), (6000, 16, "f64"),
                                      (7000 + 37, 64, "f64"), (5800, 32, "f64")])
def test_matvec_symmetric_schedule_parity(n, d, prec):
    """float32 / float64 products of n >= 5700 take the symmetric schedule
    (each off-diagonal tile formed once, used for its rows and its columns);
    ragged n leaves a partial last row block and column stage.  Same
    tolerances as the rectangular schedule: the float32 / bfloat16 column sums
    add 16 products per lane in float32 (four of four, then pairwise), then
    the 16 lane halves in float64; the float64 kernel sums in float64."""
    pr = make_problem(n, d, 1e-3, seed=n + d)
    p = np.random.default_rng(n).normal(size=n)
    w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), prec).cpu().numpy()
    if prec == "f64":
        ref = O.matvec(pr.E, pr.scale, pr.lam, p)
        err = np.abs(w - ref) / _mag(pr.E, pr.scale, pr.lam, p)
        assert err.max() <= 1e-13, (n, d, prec, err.max())
        return
    if prec == "f32":
        ref = O.matvec(pr.E, pr.scale, pr.lam, p)
        err = np.abs(w - ref) / _mag(pr.E, pr.scale, pr.lam, p)
    else:
        Eb = _bf16_rows(pr.E, pr.scale)
        ref = O.matvec(Eb, np.log(2.0), pr.lam, p)
        err = np.abs(w - ref) / _mag(Eb, np.log(2.0), pr.lam, p)
    assert err.max() <= 2e-6, (n, d, prec, err.max())


@pytest.mark.parametrize("n,d", [(10000 + 37, 16), (14000 + 37, 64), (15000, 32)])
def test_matvec_symmetric_schedule_bf16_sampled_rows(n, d):
    """bfloat16 products take the symmetric schedule from n >= 9900: sampled
    rows of every row block (its first and last row among them) against the
    oracle's one-row evaluation on the same bfloat16-rounded rows."""
    pr = make_problem(n, d, 1e-4, n_tx=3, seed=n)
    p = np.random.default_rng(n).normal(size=n)
    w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), "bf16").cpu().numpy()
    rng = np.random.default_rng(n + 1)
    rows = np.unique(np.r_[np.arange(0, n, 256), np.minimum(np.arange(255, n + 255, 256), n - 1),
                           rng.choice(n, 64, replace=False)])
    Eb = _bf16_rows(pr.E, pr.scale)
    refb = O.matvec_rows(Eb, np.log(2.0), pr.lam, p, rows)
    magb = np.array([np.exp2(Eb @ Eb[i]) @ np.abs(p) + pr.lam * abs(p[i]) for i in rows])
    assert (np.abs(w[rows] - refb) / magb).max() <= 2e-6


def test_matvec_symmetric_schedule_bf16_full_size():
    """The bench's map size (65536 sites, d = 64, lambda = 1e-5) plus a ragged
    row block: the four-wave bfloat16 kernel with float32 partials, first and
    last row of every row block and 64 random rows against the oracle's
    one-row evaluation on the same bfloat16-rounded rows."""
    n, d = 65536 + 77, 64
    pr = make_problem(n, d, 1e-5, n_tx=4, seed=5)
    p = np.random.default_rng(7).normal(size=n)
    w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), "bf16").cpu().numpy()
    rng = np.random.default_rng(8)
    rows = np.unique(np.r_[np.arange(0, n, 256), np.minimum(np.arange(255, n + 255, 256), n - 1),
                           rng.choice(n, 64, replace=False)])
    Eb = _bf16_rows(pr.E, pr.scale)
    refb = O.matvec_rows(Eb, np.log(2.0), pr.lam, p, rows)
    magb = np.array([np.exp2(Eb @ Eb[i]) @ np.abs(p) + pr.lam * abs(p[i]) for i in rows])
    assert (np.abs(w[rows] - refb) / magb).max() <= 2e-6


def test_matvec_symmetric_schedule_zero_embeddings():
    """E = 0 on the symmetric schedule (every precision at this size):
    w = lam p + (sum p) 1 within a few float32 units of sum |p|."""
    n = 14400
    E = np.zeros((n, 8))
    p = np.random.default_rng(5).normal(size=n)
    prob = L().Problem(torch.tensor(E, device=DEV), 0.25, 1.0)
    for prec, tol in (("f64", 1e-13), ("f32", 3e-7), ("bf16", 3e-7)):
        w = L().kernel_matvec(prob, torch.tensor(p, device=DEV), prec).cpu().numpy()
        ref = 0.25 * p + p.sum()
        assert np.abs(w - ref).max() <= tol * (np.abs(p).sum() + 1), prec


def test_matvec_zero_embeddings_exact():
    """E = 0: G = 1 1^T exactly in every precision (exp2(0) = 1), so
    w = lam p + (sum p) 1 up to summation rounding: float64 to 1e-13; the
    float32 / bfloat16 kernels round the weights p_j and the per-stage sums to
    float32 (at most a few float32 units, 3e-7, relative to sum |p|)."""
    n = 1000
    E = np.zeros((n, 8))
    p = np.random.default_rng(0).normal(size=n)
    prob = L().Problem(torch.tensor(E, device=DEV), 0.25, 1.0)
    for prec, tol in (("f64", 1e-13), ("f32", 3e-7), ("bf16", 3e-7)):
        w = L().kernel_matvec(prob, torch.tensor(p, device=DEV), prec).cpu().numpy()
        ref = 0.25 * p + p.sum()
        assert np.abs(w - ref).max() <= tol * (np.abs(p).sum() + 1), prec


def test_matvec_full_size_sampled_rows():
    """n = 16384, d = 64 (the at-scale configuration): sampled rows against
    the oracle's one-row evaluation."""
    pr = make_problem(16384, 64, 1e-4, n_tx=4, seed=0)
    p = np.random.default_rng(1).normal(size=pr.n)
    rows = np.random.default_rng(2).choice(pr.n, 64, replace=False)
    rows = np.r_[rows, [0, pr.n - 1]]
    ref = O.matvec_rows(pr.E, pr.scale, pr.lam, p, rows)
    mag = np.array([np.exp(pr.scale * (pr.E @ pr.E[i])) @ np.abs(p) + pr.lam * abs(p[i]) for i in rows])
    for prec, tol in (("f64", 1e-13), ("f32", 2e-6)):
        w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), prec).cpu().numpy()
        assert (np.abs(w[rows] - ref) / mag).max() <= tol, prec
    Eb = _bf16_rows(pr.E, pr.scale)
    refb = O.matvec_rows(Eb, np.log(2.0), pr.lam, p, rows)
    magb = np.array([np.exp2(Eb @ Eb[i]) @ np.abs(p) + pr.lam * abs(p[i]) for i in rows])
    w = L().kernel_matvec(_gp(pr), torch.tensor(p, device=DEV), "bf16").cpu().numpy()
    assert (np.abs(w[rows] - refb) / magb).max() <= 2e-6


def test_predict_parity_and_example1():
    pr = make_problem(900, 16, 1e-3, seed=3)
    alpha = np.random.default_rng(3).normal(size=pr.n)
    rh = L().predict(_gp(pr), torch.tensor(alpha, device=DEV), pr.Eq, "f64").cpu().numpy()
    ref = O.predict(pr.Eq, pr.E, pr.scale, alpha)
    mag = np.abs(O.kernel_matrix(pr.E, pr.scale, Eq=pr.Eq)) @ np.abs(alpha)
    assert (np.abs(rh - ref) / mag).max() <= 1e-13
    rh32 = L().predict(_gp(pr), torch.tensor(alpha, device=DEV), pr.Eq, "f32").cpu().numpy()
    assert (np.abs(rh32 - ref) / mag).max() <= 2e-6
    Eb, Eqb = _bf16_rows(pr.E, pr.scale), _bf16_rows(pr.Eq, pr.scale)
    refb = O.predict(Eqb, Eb, np.log(2.0), alpha)
    magb = np.abs(O.kernel_matrix(Eb, np.log(2.0), Eq=Eqb)) @ np.abs(alpha)
    rhb = L().predict(_gp(pr), torch.tensor(alpha, device=DEV), pr.Eq, "bf16").cpu().numpy()
    assert (np.abs(rhb - refb) / magb).max() <= 2e-6


def test_example1_solve_and_predict():
    import json, os
    ex = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "example1.json")))
    E, y = np.array(ex["E"]), np.array(ex["y"])
    prob = L().Problem(torch.tensor(E, device=DEV), ex["lambda"], 1.0)
    alpha, st = L().pcg_solve(prob, y, None, tol=1e-13, max_iter=50)
    ref = O.solve_direct(O.system_matrix(E, 1.0, ex["lambda"]), y)
    assert np.linalg.norm(alpha.cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)
    r = L().predict(prob, alpha, np.array([ex["e_query"]]))
    assert abs(r.item() - ex["r_hat_query"]) <= 0.05


@pytest.mark.parametrize("kind", ["none", "jacobi"])
def test_pcg_f64_small_config(kind):
    """n = 512, d = 16, lam = 1e-3, s = 1/4: alpha within 1e-10 of Cholesky."""
    pr = make_problem(512, 16, 1e-3, seed=0)
    prob = _gp(pr)
    pc = None if kind == "none" else L().jacobi_precond(prob)
    alpha, st = L().pcg_solve(prob, pr.y, pc, tol=1e-12, max_iter=5000, precision="f64")
    ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    err = np.linalg.norm(alpha.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= 1e-10, err
    assert st.relres <= 1e-12 and st.relres_true <= 1e-11
    # iteration count of the oracle's PCG on the same system (same arithmetic up to rounding)
    A = O.system_matrix(pr.E, pr.scale, pr.lam)
    Pj = (lambda v: v) if kind == "none" else (lambda v: v / O.jacobi_diag(pr.E, pr.scale, pr.lam))
    _, it_o, _ = O.pcg(lambda v: A @ v, Pj, pr.y, 1e-12, 5000)
    assert abs(st.iters - it_o) <= max(3, it_o // 20)


def test_pcg_closed_forms():
    """E = 0: 2 iterations, Sherman-Morrison alpha; one-hot clusters: 3 iterations."""
    n, lam = 300, 0.5
    y = np.random.default_rng(0).normal(-80, 10, n)
    prob = L().Problem(torch.zeros((n, 4), dtype=torch.float64, device=DEV), lam, 0.25)
    alpha, st = L().pcg_solve(prob, y, None, tol=1e-12, max_iter=100)
    closed = y / lam - (y.sum() / (lam * (lam + n))) * np.ones(n)
    assert st.iters <= 2
    assert np.linalg.norm(alpha.cpu().numpy() - closed) <= 1e-11 * np.linalg.norm(closed)
    Q, cval = 5, 1.1
    E = np.zeros((n, Q))
    E[np.arange(n), np.arange(n) % Q] = cval
    prob = L().Problem(torch.tensor(E, device=DEV), 0.2, 1.0)
    alpha, st = L().pcg_solve(prob, y, None, tol=1e-12, max_iter=100)
    assert st.iters <= 3


def test_cccp_fit_matches_oracle():
    """Same directions Z: the fitted (a, b), the CCCP iteration count and the
    operator P = Sigma^{-1/2} agree with the oracle's low-rank CCCP.

    Tolerance: q_k comes from an SPD solve with kappa(M) up to ~1e7, so each
    side's q carries ~kappa(M) u ~ 1e-9 relative rounding (LU in the oracle,
    Gauss-Jordan on the GPU); the fixed-point map amplifies a perturbation by
    at most 1/(1 - rate) with rate <= 0.99 here, hence 1e-7 on (a, b) and on P v."""
    pr = make_problem(700, 16, 1e-3, seed=7)
    nr = 64
    Z = make_directions(pr.n, nr, 7)
    prob = _gp(pr)
    pc = L().fit_precond(prob, torch.tensor(Z, device=DEV), gamma=0.1, rho=0.02, eps=1e-10, tol=1e-9,
                         max_iter=300)
    _, Ub = O.random_directions(pr.E, pr.scale, pr.lam, Z)
    a, b, w, it = O.cccp_lowrank(Ub, 0.1, 0.02, 1e-10, 1e-9, 300)
    hdr = pc.header.numpy()
    assert abs(hdr[1] - a) <= 1e-7 * a and abs(hdr[2] - b) <= 1e-7 * b
    assert abs(pc.stats.cccp_iters - it) <= 2
    P = O.LowRankPrecond(Ub, a, b, w)
    parts = L().precond_parts(pc)
    v = np.random.default_rng(1).normal(size=pr.n)
    vt = torch.tensor(v, device=DEV)
    Pv = (parts["hdr"][0] * vt + parts["Bt64"] @ (parts["B64"].T @ vt)).cpu().numpy()
    ref = P.apply(v)
    assert np.linalg.norm(Pv - ref) <= 1e-7 * np.linalg.norm(ref)
    # trace normalisation of Sigma_star: tr = n b + a sum_k w_k ||u_k||^2
    assert abs(pr.n * hdr[2] + hdr[1] * np.sum(w * np.sum(Ub * Ub, axis=0)) - pr.n) <= 1e-8 * pr.n


@pytest.mark.parametrize("prec,tol_ab,tol_p", [("f32", 1e-4, 1e-3), ("bf16", 3e-2, 1e-1)])
def test_cccp_fit_reduced_precision_directions(prec, tol_ab, tol_p):
    """Directions u_k = (lam I + G) z_k formed on the matrix cores in float32 /
    bfloat16: the fit lands near the oracle's (same Z).  The directions carry
    relative errors ~1e-6 (f32) / ~4e-3 (bf16); the CCCP fixed point moves by
    that times its sensitivity (up to ~10 here), hence the tolerances on (a, b)
    and on P v.  PCG with the resulting P still reaches the float64 solution."""
    pr = make_problem(700, 16, 1e-3, seed=7)
    nr = 64
    Z = make_directions(pr.n, nr, 7)
    prob = _gp(pr)
    pc = L().fit_precond(prob, torch.tensor(Z, device=DEV), gamma=0.1, rho=0.02, eps=1e-10, tol=1e-9,
                         max_iter=300, precision=prec)
    _, Ub = O.random_directions(pr.E, pr.scale, pr.lam, Z)
    a, b, w, it = O.cccp_lowrank(Ub, 0.1, 0.02, 1e-10, 1e-9, 300)
    hdr = pc.header.numpy()
    assert abs(hdr[1] - a) <= tol_ab * a and abs(hdr[2] - b) <= tol_ab * b, (hdr[1], a, hdr[2], b)
    parts = L().precond_parts(pc)
    v = np.random.default_rng(1).normal(size=pr.n)
    vt = torch.tensor(v, device=DEV)
    Pv = (parts["hdr"][0] * vt + parts["Bt64"] @ (parts["B64"].T @ vt)).cpu().numpy()
    ref = O.LowRankPrecond(Ub, a, b, w).apply(v)
    assert np.linalg.norm(Pv - ref) <= tol_p * np.linalg.norm(ref)
    alpha, st = L().pcg_solve(prob, pr.y, pc, tol=1e-12, max_iter=5000)
    sol = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    assert np.linalg.norm(alpha.cpu().numpy() - sol) / np.linalg.norm(sol) <= 1e-10


def test_laker_pcg_f64_matches_direct():
    """Full method at n = 512: CCCP fit + PCG to 1e-12, alpha within 1e-10."""
    pr = make_problem(512, 16, 1e-3, seed=0)
    Z = make_directions(pr.n, 91, 0)
    prob = _gp(pr)
    pc = L().fit_precond(prob, torch.tensor(Z, device=DEV), gamma=0.1, rho=0.0)
    alpha, st = L().pcg_solve(prob, pr.y, pc, tol=1e-12, max_iter=5000)
    ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    assert np.linalg.norm(alpha.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-10
    # oracle PCG with the oracle preconditioner on the same Z
    Po, _ = O.fit_precond(pr.E, pr.scale, pr.lam, Z, gamma=0.1, rho=0.0)
    A = O.system_matrix(pr.E, pr.scale, pr.lam)
    _, it_o, _ = O.pcg(lambda v: A @ v, Po.apply, pr.y, 1e-12, 5000)
    assert abs(st.iters - it_o) <= max(3, it_o // 20)


@pytest.mark.parametrize("prec,inner", [("f32", 1e-2), ("bf16", 1e-1)])
def test_refinement_reaches_f64_accuracy(prec, inner):
    """Reduced-precision products inside float64 iterative refinement: the
    float64 true residual reaches 1e-11 and alpha the Cholesky solution."""
    pr = make_problem(1000, 16, 1e-3, seed=5)
    prob = _gp(pr)
    alpha, st = L().pcg_solve(prob, pr.y, None, tol=1e-11, max_iter=20000, precision=prec, refine=True,
                              inner_tol=inner, ir_max=60)
    ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    assert st.relres_true <= 1e-11
    assert np.linalg.norm(alpha.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8
    hist = [st.ir_relres[i] for i in range(st.ir_steps + 1)]
    assert hist[-1] <= 1e-11
    if prec == "f32":   # float32 products: every refinement step contracts the residual
        assert all(b < a for a, b in zip(hist, hist[1:]))


def test_solves_are_deterministic():
    pr = make_problem(600, 16, 1e-3, seed=9)
    prob = _gp(pr)
    a1, s1 = L().pcg_solve(prob, pr.y, None, tol=1e-10, max_iter=5000)
    a2, s2 = L().pcg_solve(prob, pr.y, None, tol=1e-10, max_iter=5000)
    assert torch.equal(a1, a2) and s1.iters == s2.iters


@pytest.mark.parametrize("kind", ["none", "jacobi", "cccp"])
def test_graph_replay_matches_eager(kind):
    """Chunks of PCG iterations replayed from a captured HIP graph (many
    replays, with host synchronisation and other eager work in between) give
    bitwise the same iterate as the eagerly enqueued kernels."""
    pr = make_problem(900, 16, 1e-3, seed=11)
    prob = _gp(pr)
    if kind == "none":
        pc = None
    elif kind == "jacobi":
        pc = L().jacobi_precond(prob)
    else:
        pc = L().fit_precond(prob, torch.tensor(make_directions(pr.n, 48, 11), device=DEV))
    a1, s1 = L().pcg_solve(prob, pr.y, pc, tol=1e-11, max_iter=5000, check_every=8, graph=True)
    _ = L().kernel_matvec(prob, torch.ones(pr.n, dtype=torch.float64, device=DEV))   # eager work in between
    a2, s2 = L().pcg_solve(prob, pr.y, pc, tol=1e-11, max_iter=5000, check_every=8, graph=False)
    assert s1.iters == s2.iters and s1.iters > 16
    assert torch.equal(a1, a2)
    b1, t1 = L().pcg_solve(prob, pr.y, pc, tol=1e-11, max_iter=5000, precision="bf16", refine=True,
                           inner_tol=1e-1, check_every=8, graph=True)
    b2, t2 = L().pcg_solve(prob, pr.y, pc, tol=1e-11, max_iter=5000, precision="bf16", refine=True,
                           inner_tol=1e-1, check_every=8, graph=False)
    assert t1.iters == t2.iters and torch.equal(b1, b2)


def test_iteration_cap_returns_enoconv():
    pr = make_problem(512, 16, 1e-3, seed=0)
    alpha, st = L().pcg_solve(_gp(pr), pr.y, None, tol=1e-12, max_iter=5, allow_noconv=True)
    assert st.iters == 5 and st.status == L().LAKER_ENOCONV


def test_profiled_solve_matches_and_counts_products():
    """Timing every product with events changes nothing in the result; one
    timed product per iteration that ran, plus the launches that returned at
    entry after convergence."""
    pr = make_problem(900, 16, 1e-3, seed=12)
    prob = _gp(pr)
    pc = L().fit_precond(prob, torch.tensor(make_directions(pr.n, 48, 12), device=DEV))
    a1, s1 = L().pcg_solve(prob, pr.y, pc, tol=1e-11, max_iter=5000, check_every=8, profile=True)
    a2, s2 = L().pcg_solve(prob, pr.y, pc, tol=1e-11, max_iter=5000, check_every=8)
    assert torch.equal(a1, a2) and s1.iters == s2.iters
    assert s1.kmv_count == s1.iters and s1.kmv_ms > 0.0
    assert s1.iters <= s1.kmv_launches < s1.iters + 8 and s1.kmv_launch_ms > 0.0
    assert s2.kmv_count == 0
    b1, t1 = L().pcg_solve(prob, pr.y, pc, tol=1e-11, max_iter=5000, precision="bf16", refine=True,
                           inner_tol=1e-1, check_every=8, profile=True)
    assert t1.kmv_count == t1.iters and t1.kmv_launches >= t1.iters


def test_profiled_flexible_cg_counts_inner_products():
    """The flexible outer CG passes the profiling request to its inner solves:
    one timed product per inner iteration, the same iterate as unprofiled."""
    pr = make_problem(900, 16, 1e-4, seed=13)
    prob = _gp(pr)
    kw = dict(tol=1e-9, max_iter=20000, precision="bf16", refine=2, inner_tol=1e-1, ir_max=500, check_every=8,
              inner_max_iter=20)
    a1, s1 = L().pcg_solve(prob, pr.y, None, profile=True, **kw)
    a2, s2 = L().pcg_solve(prob, pr.y, None, **kw)
    assert s1.status == 0 and torch.equal(a1, a2) and s1.iters == s2.iters
    assert s1.kmv_count == s1.iters and s1.kmv_ms > 0.0 and s2.kmv_count == 0


# ---- PCG whose products take the symmetric schedule: the product kernel also
# forms p^T A p, and with a low-rank preconditioner conjugates the direction
# itself (the step update adds each row's partials and stores the direction)

_SYM = {}


def _sym_case(n):
    """Problem, Cholesky solution and CCCP directions of one symmetric-path size."""
    if n not in _SYM:
        pr = make_problem(n, 16, 1e-3, seed=21)
        A = O.system_matrix(pr.E, pr.scale, pr.lam)
        _SYM[n] = (pr, A, O.solve_direct(A, pr.y), make_directions(pr.n, 256, 21))
    return _SYM[n]


def _sym_precond(kind, prob, Z):
    if kind == "none":
        return None
    if kind == "jacobi":
        return L().jacobi_precond(prob)
    return L().fit_precond(prob, torch.tensor(Z, device=DEV), gamma=0.1, rho=0.0)


@pytest.mark.parametrize("kind", ["none", "jacobi", "cccp"])
def test_pcg_f64_on_symmetric_schedule(kind):
    """n = 6000, float64 products on the symmetric schedule: alpha within 1e-8 of
    the Cholesky solution at tol 1e-10, and (P = I, CCCP) the iteration count of
    the oracle's PCG with the same preconditioner within 10%: at tol 1e-10 and
    kappa(P A) ~ 1e4 the count moves with rounding (the oracle's own PCG takes
    396 to 422 iterations when its products are perturbed by 1e-16 to 1e-14
    relative or its CCCP tolerance changes from 1e-8 to 1e-12)."""
    pr, A, ref, Z = _sym_case(6000)
    prob = _gp(pr)
    pc = _sym_precond(kind, prob, Z)
    alpha, st = L().pcg_solve(prob, pr.y, pc, tol=1e-10, max_iter=20000)
    assert st.status == 0
    assert np.linalg.norm(alpha.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8
    assert st.relres_true <= 2e-10
    if kind != "jacobi":
        if kind == "none":
            apply_p = lambda r: r
        else:
            Po, _ = O.fit_precond(pr.E, pr.scale, pr.lam, Z, gamma=0.1, rho=0.0)
            apply_p = Po.apply
        _, it_o, _ = O.pcg(lambda v: A @ v, apply_p, pr.y, 1e-10, 20000)
        assert abs(st.iters - it_o) <= max(3, it_o // 10)


@pytest.mark.parametrize("prec,n,kind", [("f32", 6000, "none"), ("f32", 6000, "cccp"), ("bf16", 10037, "none"),
                                         ("bf16", 10037, "cccp")])
def test_reduced_precision_pcg_on_symmetric_schedule(prec, n, kind):
    """float32 (n = 6000) and bfloat16 (n = 10037) inner products on the symmetric
    schedule inside the float64 flexible outer CG: the float64 true residual
    reaches 1e-10 and alpha the Cholesky solution to 1e-8."""
    pr, A, ref, Z = _sym_case(n)
    prob = _gp(pr)
    pc = _sym_precond(kind, prob, Z)
    alpha, st = L().pcg_solve(prob, pr.y, pc, tol=1e-10, max_iter=50000, precision=prec, refine=2,
                              inner_tol=1e-1, ir_max=1000, check_every=30, inner_max_iter=30)
    assert st.status == 0 and st.relres_true <= 1e-10
    assert np.linalg.norm(alpha.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8
    assert O.relative_residual(A, alpha.cpu().numpy(), pr.y) <= 1e-10


def test_graph_replay_matches_eager_on_symmetric_schedule():
    """The conjugating product kernel inside captured chunks of iterations:
    bitwise the same iterate as the eagerly enqueued launches."""
    pr, A, ref, Z = _sym_case(6000)
    prob = _gp(pr)
    pc = _sym_precond("cccp", prob, Z)
    kw = dict(tol=1e-10, max_iter=20000, precision="f32", refine=True, inner_tol=1e-1, check_every=8)
    a1, s1 = L().pcg_solve(prob, pr.y, pc, graph=True, **kw)
    _ = L().kernel_matvec(prob, torch.ones(pr.n, dtype=torch.float64, device=DEV))   # eager work in between
    a2, s2 = L().pcg_solve(prob, pr.y, pc, graph=False, **kw)
    assert s1.iters == s2.iters and s1.iters > 16 and torch.equal(a1, a2)


# ---- stored G (materialized): formed once per solve as float64 (and float32)
# tiles of the symmetric schedule and streamed by the products


@pytest.mark.parametrize("n,d", [(6000, 16), (5837, 64)])
def test_stored_kernel_matrix_f64_pcg(n, d):
    """Float64 PCG whose products stream the stored float64 G: alpha within
    1e-10 of the Cholesky solution at tol 1e-12, the iteration count of the
    recomputing products (same entries, other summation order) within 1%, and
    the reported float64 true residual at the float64 floor with the oracle's
    (both ~1e-11 here: their difference is rounding of the residual itself)."""
    pr = make_problem(n, d, 1e-3, seed=31)
    A = O.system_matrix(pr.E, pr.scale, pr.lam)
    ref = O.solve_direct(A, pr.y)
    prob = _gp(pr)
    a1, s1 = L().pcg_solve(prob, pr.y, None, tol=1e-12, max_iter=20000, materialized=True)
    a2, s2 = L().pcg_solve(prob, pr.y, None, tol=1e-12, max_iter=20000)
    a1n = a1.cpu().numpy()
    assert s1.status == 0
    assert np.linalg.norm(a1n - ref) / np.linalg.norm(ref) <= 1e-10
    assert abs(s1.iters - s2.iters) <= max(2, s2.iters // 100)
    rt = O.relative_residual(A, a1n, pr.y)
    assert s1.relres_true <= 5e-11 and rt <= 5e-11
    assert abs(s1.relres_true - rt) <= 0.5 * rt + 1e-12


@pytest.mark.parametrize("prec,kind", [("f32", "cccp"), ("bf16", "cccp"), ("f32", "none")])
def test_stored_kernel_matrix_mixed_precision(prec, kind):
    """Flexible outer CG with the stored G: its float64 products (and with
    float32 inner products, those too) stream the stored tiles; the float64
    true residual reaches 1e-10 and alpha the Cholesky solution to 1e-8."""
    pr, A, ref, Z = _sym_case(6000)
    prob = _gp(pr)
    pc = _sym_precond(kind, prob, Z)
    alpha, st = L().pcg_solve(prob, pr.y, pc, tol=1e-10, max_iter=50000, precision=prec, refine=2,
                              inner_tol=1e-1, ir_max=1000, check_every=30, inner_max_iter=30, materialized=True)
    assert st.status == 0 and st.relres_true <= 1e-10
    assert np.linalg.norm(alpha.cpu().numpy() - ref) / np.linalg.norm(ref) <= 1e-8
    assert O.relative_residual(A, alpha.cpu().numpy(), pr.y) <= 1e-10


def test_stored_kernel_matrix_below_threshold_is_ignored():
    """Below the symmetric schedule's size nothing is stored and the solve is
    the recomputing one, bitwise."""
    pr = make_problem(900, 16, 1e-3, seed=12)
    prob = _gp(pr)
    a1, s1 = L().pcg_solve(prob, pr.y, None, tol=1e-11, max_iter=5000, materialized=True)
    a2, s2 = L().pcg_solve(prob, pr.y, None, tol=1e-11, max_iter=5000)
    assert s1.iters == s2.iters and torch.equal(a1, a2)


def test_flexible_cg_deferred_inner_solves_match():
    """An inner solve that fits one chunk is enqueued without a host round trip
    (its iteration count read with the outer step's scalars); the iterate and
    the counts equal those of the waiting form (profiling waits) bit for bit."""
    pr, A, ref, Z = _sym_case(6000)
    prob = _gp(pr)
    pc = _sym_precond("cccp", prob, Z)
    kw = dict(tol=1e-10, max_iter=50000, precision="bf16", refine=2, inner_tol=1e-1, ir_max=1000, check_every=30,
              inner_max_iter=30)
    a1, s1 = L().pcg_solve(prob, pr.y, pc, **kw)
    a2, s2 = L().pcg_solve(prob, pr.y, pc, profile=True, **kw)
    assert s1.status == 0 and s2.status == 0
    assert s1.iters == s2.iters and s1.ir_steps == s2.ir_steps and torch.equal(a1, a2)
    assert s2.kmv_count == s2.iters
