"""Training and use of the learned rank-64-plus-diagonal preconditioner.

Orchestration only: every numerical step (the CCCP fits that provide the
targets, Sigma_star^{1/2} Z, the network's forward and backward passes, the
Adam update, the Woodbury preconditioner and the PCG solves) runs in the HIP
library through the bindings of ``laker``.

Targets: for each training problem the CCCP preconditioner P = Sigma_star^{-1/2}
is fitted (Alg. 1, preconditioner learning) and U = Sigma_star^{1/2} Z is formed
for Gaussian probes Z; the network learns S with S^{-1} U close to Z.
At solve time the learned P = S^{-1} replaces the fit; when PCG stalls (its
residual falls by less than 2x over a window of iterations), breaks down or
runs out of its budget, the library falls back to a CCCP fit and continues
from the learned solve's iterate (laker_learned_solve).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import torch

from . import laker as L


@dataclass
class Example:
    prob: L.Problem
    Z: torch.Tensor      # probes, n x m (device float64)
    U: torch.Tensor      # Sigma_star^{1/2} Z


def make_example(prob: L.Problem, directions, probes, gamma: float = 1e-3, precision: str = "bf16") -> Example:
    """Fit CCCP on the problem and form its training pair (Z, Sigma_star^{1/2} Z)."""
    pc = L.fit_precond(prob, directions, gamma=gamma, rho=0.0, precision=precision)
    Z = L._dev_f64(probes, prob.device)
    return Example(prob, Z, L.sigma_half(pc, Z))


def train(model: L.MlpModel, examples: list, epochs: int, lr: float = 1e-3, seed: int = 0,
          log_every: int = 0) -> list:
    """Adam over the examples in a seeded random order each epoch; returns the
    mean loss per epoch."""
    rng = np.random.default_rng(seed)
    hist = []
    for ep in range(epochs):
        order = rng.permutation(len(examples))
        tot = 0.0
        for i in order:
            ex = examples[i]
            loss, _ = L.learned_train_step(ex.prob, model, ex.Z, ex.U, lr=lr, update=True, want_loss=True)
            tot += loss
        hist.append(tot / len(examples))
        if log_every and (ep % log_every == 0 or ep == epochs - 1):
            print(f"epoch {ep}: mean loss {hist[-1]:.4e}", flush=True)
    return hist


@dataclass
class LearnedSolve:
    alpha: torch.Tensor
    stats: L.laker_stats
    fell_back: int           # 0 none, 1 the learned solve stalled / hit its cap, 2 it broke down
    learned_iters: int
    precond: L.Precond       # the preconditioner used last


def solve_with_fallback(prob: L.Problem, y, model: L.MlpModel, fallback_directions, tol: float = 1e-6,
                        budget: int = 200000, precision: str = "bf16", refine=2, inner_tol: float = 0.1,
                        gamma: float = 0.1, check_every: int = 30, inner_max_iter: int = 30,
                        materialized: bool = False, stall_window: int = 2000,
                        outer_history: int = 0) -> LearnedSolve:
    """PCG with the learned preconditioner; when it stalls (the residual falls by
    less than 2x over stall_window iterations), breaks down or exhausts the
    budget, the library fits CCCP with the fallback directions and continues
    from the current iterate (laker_learned_solve).  refine: 0, 1 (iterative
    refinement) or 2 (flexible float64 outer CG, inner solves capped at
    inner_max_iter iterations).  materialized: the float64 products stream a G
    stored once per solve."""
    ir_max = 20000 if refine == 2 else 64
    alpha, st, pc = L.learned_solve(prob, y, model, fallback_directions, tol=tol, max_iter=budget, precision=precision,
                                    refine=int(refine), inner_tol=inner_tol, ir_max=ir_max, check_every=check_every,
                                    inner_max_iter=inner_max_iter, materialized=materialized,
                                    stall_window=stall_window, gamma=gamma, outer_history=outer_history)
    return LearnedSolve(alpha, st, st.fell_back, st.learned_iters, pc)
