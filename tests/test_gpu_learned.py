"""GPU parity of the learned preconditioner against its FP64 oracle, through the C ABI.

Tolerances:
  * network output and gradients: the library multiplies bfloat16-rounded
    operands (8-bit significands, relative rounding 2^-9) with float32
    accumulation; the oracle is exact float64.  Three stacked layers give a
    norm-wise relative error of a few 2^-9; the bound used is 2e-2 per tensor
    for outputs and gradients;
  * Sigma^{1/2} Z, the Woodbury preconditioner and the solves are float64:
    bounds scale with the conditioning as stated in each test.
"""
import math

import numpy as np
import pytest
import torch

from oracle import laker_oracle as O
from oracle import learned_oracle as LO
from synth import make_directions, make_mlp_init, make_probes, make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def L():
    from paper_2604_25138_amd import laker
    laker.load()
    return laker


def _gp(pr):
    return L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)


def _model(d, seed, log_delta0=-1.0, scale=1.0):
    p = make_mlp_init(LO.input_dim(d), LO.HIDDEN, LO.RANK + 1, seed, log_delta0=log_delta0)
    for k in p:
        p[k] = p[k] * scale
    p["b3"][LO.RANK] = log_delta0
    m = L().MlpModel(d, DEV)
    m.set_params(p)
    return m, m.params()     # the float32 weights the library holds, back in float64


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300))


def test_sigma_half_matches_dense_root_of_fitted_sigma():
    pr = make_problem(300, 8, 1e-3, seed=7)
    prob = _gp(pr)
    Z = make_directions(pr.n, 40, 7)
    pc = L().fit_precond(prob, torch.tensor(Z, device=DEV), gamma=1e-3)
    parts = L().precond_parts(pc)
    B = parts["B64"].cpu().numpy()
    b = float(parts["hdr"][2].cpu())
    Sigma = b * np.eye(pr.n) + B @ B.T
    ev, V = np.linalg.eigh(Sigma)
    probes = make_probes(pr.n, 6, 7)
    U = L().sigma_half(pc, torch.tensor(probes, device=DEV)).cpu().numpy()
    ref = (V * np.sqrt(ev)) @ V.T @ probes
    assert np.abs(U - ref).max() <= 1e-13 * (ev[-1] / ev[0]) * np.abs(ref).max()


@pytest.mark.parametrize("n,d", [(300, 8), (1000, 16), (77, 4)])
def test_network_forward_matches_oracle(n, d):
    pr = make_problem(n, d, 1e-3, seed=n)
    model, params = _model(d, n)
    O_gpu = L().learned_forward(_gp(pr), model).cpu().double().numpy()
    X = LO.features(pr.E, pr.lam)
    O_ref, _ = LO.mlp_forward(params, X)
    assert O_gpu.shape == O_ref.shape
    assert _rel(O_gpu, O_ref) <= 2e-2
    # the float32 inputs the library builds are the oracle's features
    assert np.isfinite(O_gpu).all()


def test_gradient_matches_oracle():
    n, d, m = 400, 8, 12
    pr = make_problem(n, d, 1e-3, seed=21)
    model, params = _model(d, 21)
    Zd = make_directions(n, 48, 21)
    P, _ = O.fit_precond(pr.E, pr.scale, pr.lam, Zd, gamma=1e-3)
    probes = make_probes(n, m, 21)
    U = LO.sigma_half_apply(P.b, P.B, P.apply, probes)
    loss, g = L().learned_train_step(_gp(pr), model, torch.tensor(probes, device=DEV), torch.tensor(U, device=DEV),
                                     update=False, want_grad=True)
    X = LO.features(pr.E, pr.lam)
    Lref, gref, _ = LO.loss_and_grad(params, X, probes, U)
    assert abs(loss - Lref) <= 2e-2 * Lref
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        assert _rel(g[k].cpu().double().numpy(), gref[k]) <= 2e-2, k


def test_first_adam_step_closed_form():
    n, d, m = 256, 8, 8
    pr = make_problem(n, d, 1e-3, seed=22)
    model, params = _model(d, 22)
    probes = make_probes(n, m, 22)
    U = probes * 2.0
    lr = 1e-3
    _, g = L().learned_train_step(_gp(pr), model, torch.tensor(probes, device=DEV), torch.tensor(U, device=DEV),
                                  lr=lr, update=True, want_grad=True)
    new = model.params()
    for k in params:
        gk = g[k].cpu().double().numpy()
        expect = params[k] - lr * gk / (np.abs(gk) + 1e-8)
        assert np.abs(new[k] - expect).max() <= 1e-6 * max(1.0, np.abs(params[k]).max()), k


def test_learned_preconditioner_is_inverse_of_s():
    n, d = 500, 8
    pr = make_problem(n, d, 1e-3, seed=23)
    prob = _gp(pr)
    model, _ = _model(d, 23, log_delta0=-2.0, scale=0.5)
    out = L().learned_forward(prob, model).cpu().double().numpy()
    pc = L().learned_precond(prob, model)
    parts = L().precond_parts(pc)
    B = parts["B64"].cpu().numpy()
    Bt = parts["Bt64"].cpu().numpy()
    dinv = parts["dinv64"].cpu().numpy()
    V, delta = out[:, :LO.RANK], np.exp(out[:, LO.RANK])
    S = LO.learned_dense(V, delta)
    Pd = np.diag(dinv) + Bt @ B.T
    ev = np.linalg.eigvalsh(S)
    err = np.abs(Pd @ S - np.eye(n)).max()
    assert err <= 1e-13 * ev[-1] / ev[0]
    assert np.abs(Pd - Pd.T).max() <= 1e-12 * np.abs(Pd).max()


def test_pcg_with_learned_preconditioner_reaches_cholesky_solution():
    n, d = 512, 16
    pr = make_problem(n, d, 1e-3, seed=24)
    prob = _gp(pr)
    model, _ = _model(d, 24, log_delta0=-3.0, scale=0.3)
    pc = L().learned_precond(prob, model)
    alpha, st = L().pcg_solve(prob, pr.y, pc, tol=1e-12, max_iter=20000)
    ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    assert np.linalg.norm(alpha.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)
    # mixed precision with refinement uses the same preconditioner
    a2, st2 = L().pcg_solve(prob, pr.y, pc, tol=1e-10, max_iter=20000, precision="bf16", refine=True,
                            inner_tol=0.1)
    assert st2.relres_true <= 1e-10


def test_training_gains_over_plain_cg_and_fallback():
    """A/B: a network trained on CCCP fits of small maps needs far fewer PCG
    iterations than plain CG on larger held-out maps."""
    from paper_2604_25138_amd import learned as LR
    d, m = 16, 64
    rng = np.random.default_rng(0)
    exs = []
    for k in range(12):
        lam = float(10 ** rng.uniform(-4, -2))
        pr = make_problem(1024, d, lam, n_tx=int(rng.integers(1, 5)), seed=100 + k)
        prob = _gp(pr)
        exs.append(LR.make_example(prob, torch.tensor(make_directions(pr.n, 128, 100 + k), device=DEV),
                                   make_probes(pr.n, m, 100 + k), gamma=1e-3, precision="f64"))
    model = L().MlpModel(d, DEV)
    model.set_params(make_mlp_init(LO.input_dim(d), LO.HIDDEN, LO.RANK + 1, 0))
    hist = LR.train(model, exs, epochs=25, lr=1e-3)
    assert hist[-1] < 0.5 * hist[0]
    gains = []
    for k in range(2):
        pr = make_problem(2048, d, 3e-4, n_tx=2, seed=900 + k)
        prob = _gp(pr)
        _, s_cg = L().pcg_solve(prob, pr.y, None, tol=1e-6, max_iter=50000)
        _, s_lr = L().pcg_solve(prob, pr.y, L().learned_precond(prob, model), tol=1e-6, max_iter=50000)
        gains.append(s_lr.iters / s_cg.iters)
    assert max(gains) <= 0.7, gains


@pytest.mark.parametrize("refine", [0, 2])
def test_stalled_learned_solve_falls_back_to_cccp_in_the_library(refine):
    """An untrained network (random weights) gives a preconditioner under which
    PCG makes little progress at lambda = 1e-5; the library's stall test (less
    than 2x residual reduction over 60 iterations) stops that solve, fits CCCP
    (Alg. 1) with the given directions, continues from the learned solve's
    iterate and reaches the float64 Cholesky solution."""
    n, d = 1500, 16
    pr = make_problem(n, d, 1e-5, n_tx=2, seed=960)
    prob = _gp(pr)
    model, _ = _model(d, 960, log_delta0=-7.0)
    Zd = torch.tensor(make_directions(n, 128, 960), device=DEV)
    window, check = 60, 10
    if refine == 0:
        alpha, st, pc = L().learned_solve(prob, pr.y, model, Zd, tol=1e-12, max_iter=20000, precision="f64",
                                          refine=0, check_every=check, stall_window=window)
    else:
        alpha, st, pc = L().learned_solve(prob, pr.y, model, Zd, tol=1e-11, max_iter=40000, precision="bf16",
                                          refine=2, inner_tol=0.1, check_every=10, inner_max_iter=10,
                                          stall_window=window)
    print(f"refine={refine}: fell_back={st.fell_back} learned_iters={st.learned_iters} iters={st.iters} "
          f"cccp_iters={st.cccp_iters} relres_true={st.relres_true:.2e}")
    assert st.status == L().LAKER_OK
    assert st.fell_back == 1 and pc.kind == L().PRECOND_CCCP
    # the stall is detected at the first read-back at least `window` iterations
    # after one that the residual has not halved since
    assert window <= st.learned_iters <= window + 4 * check
    ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    err = np.linalg.norm(alpha.cpu().numpy() - ref) / np.linalg.norm(ref)
    # kappa(A) ~ 1e8 here: the Cholesky reference itself is good to ~kappa u
    assert st.relres_true <= 1e-10 and err <= 1e-8, err


def test_learned_solve_without_stall_keeps_the_learned_preconditioner():
    n, d = 1024, 16
    pr = make_problem(n, d, 1e-2, n_tx=1, seed=961)
    prob = _gp(pr)
    model, _ = _model(d, 961, log_delta0=-1.0, scale=0.5)
    Zd = torch.tensor(make_directions(n, 64, 961), device=DEV)
    alpha, st, pc = L().learned_solve(prob, pr.y, model, Zd, tol=1e-12, max_iter=20000, precision="f64", refine=0,
                                      check_every=16, stall_window=0)
    assert st.status == L().LAKER_OK and st.fell_back == 0 and pc.kind == L().PRECOND_LEARNED
    assert st.learned_iters == st.iters
    ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
    assert np.linalg.norm(alpha.cpu().numpy() - ref) <= 1e-10 * np.linalg.norm(ref)


def _bf16(x):
    """Round float64 values through float32 to bfloat16 (nearest even), the
    operands the network's matrix products multiply."""
    u = np.asarray(x, dtype=np.float64).astype(np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def _emulated_forward(params, X):
    """The oracle's forward pass on the operands the library multiplies:
    inputs, weights and hidden activations rounded to bfloat16 before each
    product, everything else (sums, bias, SiLU) in float64."""
    W1, W2, W3 = (_bf16(params[k]) for k in ("W1", "W2", "W3"))
    Z1 = _bf16(X) @ W1 + params["b1"]
    H1 = LO.silu(Z1)
    Z2 = _bf16(H1) @ W2 + params["b2"]
    H2 = LO.silu(Z2)
    O = _bf16(H2) @ W3 + params["b3"]
    mags = (np.abs(_bf16(X)) @ np.abs(W1) + np.abs(params["b1"]),
            np.abs(_bf16(H1)) @ np.abs(W2) + np.abs(params["b2"]),
            np.abs(_bf16(H2)) @ np.abs(W3) + np.abs(params["b3"]))
    return O, (Z1, H1, Z2, H2), mags


@pytest.mark.parametrize("n,d", [(300, 8), (1000 + 3, 16), (700, 64)])
def test_network_forward_elementwise(n, d):
    """Every output element against the oracle evaluated on bfloat16-rounded
    operands (same weights), relative to the magnitude of its terms
    mag_ik = sum_j |h_ij| |W3_jk| + |b3_k|: float32 sums and SiLU give ~1e-6;
    where a hidden value lies within that of a bfloat16 rounding boundary the
    two sides round it to neighbouring values (2^-8 apart), which moves the
    outputs it feeds by a small part of 2^-8 of their magnitude (measured:
    at most 3.1e-4, 99% below 6.1e-7, median 4e-9 over 700-1003 points).
    Bound: 2^-9 for every element, 1e-5 for 99% of them."""
    pr = make_problem(n, d, 1e-3, seed=n)
    model, params = _model(d, n)
    O_gpu = L().learned_forward(_gp(pr), model).cpu().double().numpy()
    X = LO.features(pr.E, pr.lam)
    O_ref, _, mags = _emulated_forward(params, X)
    r = np.abs(O_gpu - O_ref) / mags[2]
    print(f"n={n} d={d}: output error / magnitude: max {r.max():.2e}, 99% {np.quantile(r, 0.99):.2e}, "
          f"median {np.median(r):.2e}")
    assert r.max() <= 2.0 ** -9
    assert np.quantile(r, 0.99) <= 1e-5


def test_network_gradient_elementwise():
    """Every gradient element against the oracle's backward pass on bfloat16
    operands (inputs, weights, activations and output gradients rounded before
    each product, as the library multiplies them), relative to the magnitude
    of its terms (e.g. sum_i |h2_ij| |dO_ik| for W3): the output gradient
    inherits the forward rounding through the Woodbury solves and is rounded
    to bfloat16 itself (measured: at most 4.6e-4 (W1), 99% below 2.6e-4).
    Bound: 2^-9 for every element and 2^-10 for 99% of them."""
    n, d, m = 400, 8, 12
    pr = make_problem(n, d, 1e-3, seed=21)
    model, params = _model(d, 21)
    Zd = make_directions(n, 48, 21)
    P, _ = O.fit_precond(pr.E, pr.scale, pr.lam, Zd, gamma=1e-3)
    probes = make_probes(n, m, 21)
    U = LO.sigma_half_apply(P.b, P.B, P.apply, probes)
    _, g = L().learned_train_step(_gp(pr), model, torch.tensor(probes, device=DEV), torch.tensor(U, device=DEV),
                                  update=False, want_grad=True)
    X = LO.features(pr.E, pr.lam)
    O_ref, (Z1, H1, Z2, H2), _ = _emulated_forward(params, X)
    V, delta = LO.split_output(O_ref)
    # loss gradient with respect to the outputs (float64, as the oracle's)
    Y = LO.woodbury_solve(V, delta, U)
    G = -2.0 * (probes - Y) / (n * m)
    Hm = LO.woodbury_solve(V, delta, G)
    dO = np.zeros_like(O_ref)
    dO[:, :LO.RANK] = -(Hm @ (Y.T @ V) + Y @ (Hm.T @ V))
    dO[:, LO.RANK] = -(Hm * Y).sum(axis=1) * delta
    W2, W3 = _bf16(params["W2"]), _bf16(params["W3"])
    b = {k: _bf16(v) for k, v in (("X", X), ("H1", H1), ("H2", H2), ("dO", dO))}
    ref, mag = {}, {}
    ref["W3"], mag["W3"] = b["H2"].T @ b["dO"], np.abs(b["H2"]).T @ np.abs(b["dO"])
    ref["b3"], mag["b3"] = b["dO"].sum(axis=0), np.abs(b["dO"]).sum(axis=0)
    dZ2 = (b["dO"] @ W3.T) * LO.silu_grad(Z2)
    bz2 = _bf16(dZ2)
    ref["W2"], mag["W2"] = b["H1"].T @ bz2, np.abs(b["H1"]).T @ np.abs(bz2)
    ref["b2"], mag["b2"] = bz2.sum(axis=0), np.abs(bz2).sum(axis=0)
    dZ1 = (bz2 @ W2.T) * LO.silu_grad(Z1)
    bz1 = _bf16(dZ1)
    ref["W1"], mag["W1"] = b["X"].T @ bz1, np.abs(b["X"]).T @ np.abs(bz1)
    ref["b1"], mag["b1"] = bz1.sum(axis=0), np.abs(bz1).sum(axis=0)
    for k in ("W3", "b3", "W2", "b2", "W1", "b1"):
        gk = g[k].cpu().double().numpy()
        r = np.abs(gk - ref[k]) / np.maximum(mag[k], 1e-300)
        print(f"{k}: error / magnitude max {r.max():.2e}, 99% {np.quantile(r, 0.99):.2e}, median {np.median(r):.2e}")
        assert r.max() <= 2.0 ** -9, k
        assert np.quantile(r, 0.99) <= 2.0 ** -10, k
