"""Batched PCG over maps of uneven size, through the C ABI.

With each map's own (single-map) column ranges the batched passes run the
same per-block arithmetic as laker_pcg_solve, so the iterates must be bitwise
equal to solving the maps one by one; with other column ranges (autotuned or
XCD-ordered tiles) the products add their partials in another order and the
check is the float64 true residual and the distance to the Cholesky solution.
"""
import numpy as np
import pytest
import torch

from oracle import laker_oracle as O
from synth import make_directions, make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SIZES = [(300, 1e-3, 1), (1000, 1e-4, 3), (2085, 1e-3, 2), (64, 1e-2, 1), (777, 1e-5, 4), (1500, 3e-4, 2)]


def L():
    from paper_2604_25138_amd import laker
    laker.load()
    return laker


def _maps(d=16, seed=0):
    out = []
    for k, (n, lam, ntx) in enumerate(SIZES):
        pr = make_problem(n, d, lam, n_tx=ntx, seed=seed + k)
        out.append((pr, L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)))
    return out


def _precs(maps, kind):
    if kind == "none":
        return None
    if kind == "jacobi":
        return [L().jacobi_precond(p) for _, p in maps]
    return [L().fit_precond(p, torch.tensor(make_directions(pr.n, min(48, pr.n), 7), device=DEV)) for pr, p in maps]


@pytest.mark.parametrize("kind", ["none", "jacobi", "cccp"])
def test_batched_f64_is_bitwise_equal_to_single_solves(kind):
    maps = _maps()
    precs = _precs(maps, kind)
    alphas, stats, used = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], precs, tol=1e-10,
                                                max_iter=20000, check_every=8)
    assert used == 0
    for b, (pr, p) in enumerate(maps):
        a1, s1 = L().pcg_solve(p, pr.y, None if precs is None else precs[b], tol=1e-10, max_iter=20000,
                               check_every=8)
        assert stats[b].iters == s1.iters, b
        assert torch.equal(alphas[b], a1), b
        assert stats[b].relres_true <= 1e-9


def test_batched_mixed_refinement_matches_single_and_graph():
    maps = _maps(seed=10)
    precs = _precs(maps, "cccp")
    kw = dict(tol=1e-10, max_iter=40000, precision="bf16", refine=True, inner_tol=0.1, check_every=8)
    alphas, stats, _ = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], precs, **kw)
    ga, gstats, _ = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], precs, graph=True, **kw)
    for b, (pr, p) in enumerate(maps):
        a1, s1 = L().pcg_solve(p, pr.y, precs[b], **kw)
        assert stats[b].iters == s1.iters and stats[b].ir_steps == s1.ir_steps, b
        assert torch.equal(alphas[b], a1), b
        assert torch.equal(ga[b], a1), b
        assert stats[b].relres_true <= 1e-10


@pytest.mark.parametrize("cps,xcd", [(-1, False), (512, True), (0, True)])
def test_batched_other_tilings_reach_cholesky_solution(cps, xcd):
    maps = _maps(seed=20)
    precs = _precs(maps, "cccp")
    alphas, stats, used = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], precs, tol=1e-12,
                                                max_iter=40000, cols_per_split=cps, xcd_order=xcd, check_every=8)
    if cps > 0:
        assert used == cps
    for b, (pr, p) in enumerate(maps):
        ref = O.solve_direct(O.system_matrix(pr.E, pr.scale, pr.lam), pr.y)
        assert np.linalg.norm(alphas[b].cpu().numpy() - ref) <= 1e-9 * np.linalg.norm(ref), b


def test_batched_rejects_mixed_dimensions():
    pr1 = make_problem(100, 8, 1e-3, seed=1)
    pr2 = make_problem(100, 16, 1e-3, seed=2)
    ps = [L().Problem(torch.tensor(x.E, device=DEV), x.lam, x.scale) for x in (pr1, pr2)]
    with pytest.raises(L().LakerError):
        L().pcg_solve_batched(ps, [pr1.y, pr2.y])


def test_refinement_escalates_and_converges_on_hard_maps():
    """Small lambda at the largest sizes of the batch: bfloat16 corrections stop
    contracting the float64 residual, the map moves to finer inner products and
    still reaches the tolerance; the batch and the single solves agree bit for
    bit."""
    specs = [(4096, 1e-6, 3), (2048, 3e-6, 5), (1024, 1e-2, 1), (3000, 1e-5, 8)]
    maps = []
    for k, (n, lam, ntx) in enumerate(specs):
        pr = make_problem(n, 32, lam, n_tx=ntx, seed=40 + k)
        maps.append((pr, L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)))
    kw = dict(tol=1e-8, max_iter=200000, precision="bf16", refine=True, inner_tol=0.1, check_every=16)
    alphas, stats, _ = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], None, **kw)
    for b, (pr, p) in enumerate(maps):
        assert stats[b].status == 0 and stats[b].relres_true <= 1e-8, (b, stats[b].relres_true)
        a1, s1 = L().pcg_solve(p, pr.y, None, **kw)
        assert s1.escalations == stats[b].escalations and torch.equal(alphas[b], a1), b


def test_batch_with_symmetric_maps_is_bitwise_equal_to_single_solves():
    """Maps large enough for the symmetric product schedule run it inside the
    batch too (the single solver's kernel and plan, the small maps sharing the
    tile table), so
    the batch still reproduces the single solves bit for bit: the 14500-site
    map in its bf16 inner products and float64 outer residuals, the 6000-site
    map in its float64 outer residuals."""
    specs = [(14500, 1e-3, 3, 77), (1500, 1e-3, 2, 78), (6000, 1e-4, 4, 79)]
    maps = []
    for n, lam, ntx, seed in specs:
        pr = make_problem(n, 32, lam, n_tx=ntx, seed=seed)
        maps.append((pr, L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)))
    kw = dict(tol=1e-9, max_iter=100000, precision="bf16", refine=True, inner_tol=0.1, check_every=16)
    alphas, stats, _ = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], None, **kw)
    for b, (pr, p) in enumerate(maps):
        a1, s1 = L().pcg_solve(p, pr.y, None, **kw)
        assert stats[b].status == 0 and stats[b].relres_true <= 1e-9, b
        assert stats[b].iters == s1.iters and torch.equal(alphas[b], a1), b


@pytest.mark.parametrize("kind,graph", [("none", False), ("cccp", False), ("cccp", True)])
def test_batch_with_several_symmetric_maps_is_bitwise_equal_to_single_solves(kind, graph):
    """Three symmetric-size maps of different sizes (different stage lists per
    grid row) share one launch of the bf16 symmetric product in the batch; with
    a CCCP preconditioner the launch also conjugates each map's direction with
    its own beta; with graph the iterations between host checks replay a HIP
    graph (re-captured whenever maps retire).  Every map reproduces its single
    solve bit for bit."""
    specs = [(14500, 1e-3, 3, 81), (10300, 1e-3, 2, 82), (12288 + 5, 1e-4, 4, 83), (1500, 1e-3, 2, 84)]
    maps = []
    for n, lam, ntx, seed in specs:
        pr = make_problem(n, 32, lam, n_tx=ntx, seed=seed)
        maps.append((pr, L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)))
    precs = _precs(maps, kind)
    kw = dict(tol=1e-9, max_iter=100000, precision="bf16", refine=True, inner_tol=0.1, check_every=16)
    alphas, stats, _ = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], precs, graph=graph,
                                             **kw)
    for b, (pr, p) in enumerate(maps):
        a1, s1 = L().pcg_solve(p, pr.y, None if precs is None else precs[b], **kw)
        assert stats[b].status == 0 and stats[b].relres_true <= 1e-9, b
        assert stats[b].iters == s1.iters and torch.equal(alphas[b], a1), b


def test_batch_with_stored_kernel_matrices_matches_single_solves():
    """materialized: the 14500- and 6000-site maps' float64 outer residuals
    stream a G stored once per call, in the batch as in the single solver, so
    the batch reproduces the single solves with the same option bit for bit
    (no map here moves its inner products to float64, where the single solver
    would also stream the stored G); the results agree with the recomputing
    batch to the solve's tolerance."""
    specs = [(14500, 1e-3, 3, 77), (1500, 1e-3, 2, 78), (6000, 1e-4, 4, 79)]
    maps = []
    for n, lam, ntx, seed in specs:
        pr = make_problem(n, 32, lam, n_tx=ntx, seed=seed)
        maps.append((pr, L().Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)))
    kw = dict(tol=1e-9, max_iter=100000, precision="bf16", refine=True, inner_tol=0.1, check_every=16)
    alphas, stats, _ = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], None,
                                             materialized=True, **kw)
    ref, _, _ = L().pcg_solve_batched([p for _, p in maps], [pr.y for pr, _ in maps], None, **kw)
    for b, (pr, p) in enumerate(maps):
        a1, s1 = L().pcg_solve(p, pr.y, None, materialized=True, **kw)
        assert stats[b].status == 0 and stats[b].relres_true <= 1e-9, b
        assert s1.escalations < 2, b
        assert stats[b].iters == s1.iters and torch.equal(alphas[b], a1), b
        err = float((alphas[b] - ref[b]).norm() / ref[b].norm())
        A = O.system_matrix(pr.E, pr.scale, pr.lam) if pr.n <= 6000 else None
        if A is not None:
            assert O.relative_residual(A, alphas[b].cpu().numpy(), pr.y) <= 2e-9, b
        assert err <= 1e-6, (b, err)
