"""Benchmark of the LAKER solve path on one MI355X.

A step is one full pass of the production path over one synthetic map (by
default the largest single-map configuration: 65536 sites, d = 64, 4
transmitters, lambda = 1e-5): the learned rank-64-plus-diagonal preconditioner
(network inference and the Woodbury factors), the solve to a float64 true
relative residual of 1e-6 by a flexible float64 outer CG around bfloat16 inner
PCG solves (falling back to a CCCP fit if PCG stalls), and reconstruction on the
45 x 45 grid.  Inputs are resident in HBM before the timed region.  The network
is trained beforehand (outside the timed region, reported) on CCCP fits of
smaller maps drawn from the same generator with random lambda and transmitter
counts.

Beside the timed path the run reports: the same map solved entirely in float64
with the paper's CCCP preconditioner (FP64 CCCP-PCG, the metric's comparison),
CCCP with the timed step's mixed-precision solver at gamma = 0.1 and 1e-3, the
roofline position of the dominant kernel (the fused kernel product, timed with
HIP events around every product of the solve on the library's stream), the
16384-site map (learned step; float32 products with G stored against
recomputed), a batched leg (maps of uneven size solved together vs one after
the other), and the FP64 CPU oracle timed on a bounded sample of the same
workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "solves/s to rel-res 1e-6 (learned+mixed vs FP64 CCCP-PCG); matvec % roofline"

WORKLOADS = {
    # the largest single-map configuration: 65536 sites, 64-d RFF embeddings,
    # 4 transmitters, lambda = 1e-5 (lambda / ||G|| ~ 1.5e-10), solved to a
    # float64 relative residual of 1e-6
    "n65536_d64": dict(n=65536, d=64, n_tx=4, lam=1e-5, tol=1e-6, seed=0, history=8),
    # the at-scale float32 configuration: 16384 sites, 64-d RFF embeddings,
    # 4 transmitters, lambda = 1e-4, PCG to relative residual 1e-6
    "n16384_d64": dict(n=16384, d=64, n_tx=4, lam=1e-4, tol=1e-6, seed=0, history=1),
    # small float64 configuration: 512 sites, 16-d embeddings, lambda = 1e-3
    "n512_d16": dict(n=512, d=16, n_tx=1, lam=1e-3, tol=1e-6, seed=0, history=1),
}

# the solve: flexible float64 outer CG around bf16 inner PCG solves of at most
# INNER_CAP iterations each (a sweep of the cap on the n16384_d64 map:
# 15 -> 110 ms, 20 -> 96, 25 -> 96, 30 -> 85, 40 -> 90; iterative refinement
# with inner tolerance 0.1: 100 ms; on the n65536_d64 map with the trained
# network: 20 / 25 / 30 / 40 / 50 -> 2.30 / 2.30 / 2.18 / 2.21 / 2.24 s, and
# the held-out leg's learned solves 1.05 / 1.12 / 1.06 / 1.17 / 1.24 s); the
# inner solves check for convergence every INNER_CAP iterations, so no
# launches are enqueued past the cap
INNER_CAP = 30
# directions the flexible outer CG keeps (per workload, `history`): at 65536
# sites keeping 8 took 2.74 / 2.80 s per solve on two maps against 3.51 / 3.27 s
# with 1 (cap 30; cap 20: 2.85 / 2.70 against 3.31 / 3.14); at 16384 sites it
# makes no difference (0.061-0.064 s)
# the learned solve falls back to CCCP when its residual falls by less than 2x
# over this many inner iterations (the bench maps fall by ~1.3 decades in it)
STALL_WINDOW = 2000

# training set of the learned preconditioner: maps of TRAIN_N sites with
# lambda log-uniform in [1e-5, 1e-2] and 1..8 transmitters, CCCP targets at
# gamma = 1e-3.  Chosen on the held-out leg (8 maps of 32768 sites, d = 32,
# mean inner iterations against CCCP's 1091): 192 maps of 2048 sites for 30 /
# 60 / 90 / 120 / 180 epochs 775 / 768 / 740 / 836 / 1019; 60 epochs of 4096
# sites 842, 384 maps of 2048 sites 929; targets at gamma 1e-2 / 1e-4 785 /
# 813.  The 65536-site map's inner iterations follow (3850 / 3801 / 3662 /
# 3981 / 3879; 4166 with 4096-site maps; of 8192 sites 4680, of 512 a fallback)
TRAIN_N, TRAIN_MAPS, TRAIN_EPOCHS, TRAIN_PROBES = 2048, 192, 90, 128

# vector ALU issue rate: 256 CUs x 64 lanes x 2.4 GHz unpacked float32
# multiply-adds, one slot each.  The library is built without packed float32
# instructions, and the 157.3 TFLOP/s fp32 vector figure counts them (128
# lanes' worth); 64 lanes is the issue width of the 78.6 TFLOP/s fp64 vector
# figure.  exp2 (v_exp_f32) issues at half that rate and takes 2 slots.  Both
# were measured by calib/valu_rates.hip: 57-58 lane-FMA and 28-30 lane-exp2 per
# CU per nominal clock at 8 waves per SIMD, exp2 + 2 FMA at 15.3-15.5 (the two
# do not overlap); all ~11% under 64 / 32, the clock the busy chip holds.
PEAK_VALU_TOPS = 256 * 64 * 2.4e9 / 1e12
EXP2_SLOTS = 2.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="n65536_d64", choices=sorted(WORKLOADS))
    ap.add_argument("--no-c2", action="store_true", help="skip the 16384-site leg")
    ap.add_argument("--no-paper", action="store_true", help="skip the sweep of the paper's own regime")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-right-hand-side and online legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--counters", action="store_true",
                    help="only 20 bfloat16 products of the workload, a 20-iteration float64 PCG streaming the "
                         "stored G, and 5 copies of a 256 MiB buffer (the calibration), for hardware counter runs")
    ap.add_argument("--no-f64", action="store_true", help="skip the float64 comparison leg")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle work in the CPU sample")
    ap.add_argument("--train-maps", type=int, default=TRAIN_MAPS)
    ap.add_argument("--train-epochs", type=int, default=TRAIN_EPOCHS)
    ap.add_argument("--batch-maps", type=int, default=256,
                    help="maps in the batched leg (n ~ U[1024, 16384], d = 32); 0 skips it")
    ap.add_argument("--learned-eval", type=int, default=8,
                    help="held-out maps of 32768 sites (d = 32) on which the learned preconditioner is compared "
                         "with a CCCP fit under the same solver options; 0 skips the leg")
    return ap.parse_args()


def train_model(L, LR, d, dev, n_maps, epochs):
    """Untimed: CCCP fits of n_maps training maps, then Adam epochs."""
    import numpy as np
    import torch

    from synth import default_n_r, make_directions, make_mlp_init, make_probes, make_problem
    rng = np.random.default_rng(12345)
    t0 = time.perf_counter()
    exs = []
    for k in range(n_maps):
        lam = float(10 ** rng.uniform(-5, -2))
        ntx = int(rng.integers(1, 9))
        pr = make_problem(TRAIN_N, d, lam, n_tx=ntx, seed=1000 + k)
        prob = L.Problem(torch.tensor(pr.E, device=dev), pr.lam, pr.scale)
        Zd = torch.tensor(make_directions(TRAIN_N, default_n_r(TRAIN_N), 1000 + k), device=dev)
        exs.append(LR.make_example(prob, Zd, make_probes(TRAIN_N, TRAIN_PROBES, 1000 + k), gamma=1e-3,
                                   precision="bf16"))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    in_dim = L.mlp_layout(d).in_dim
    model = L.MlpModel(d, dev)
    model.set_params(make_mlp_init(in_dim, L.MLP_HIDDEN, L.MLP_RANK + 1, 0))
    hist = LR.train(model, exs, epochs=epochs, lr=1e-3, seed=0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    info = {"maps": n_maps, "n": TRAIN_N, "epochs": epochs, "probes": TRAIN_PROBES,
            "targets_s": t1 - t0, "train_s": t2 - t1, "ms_per_step": (t2 - t1) * 1e3 / (epochs * n_maps),
            "loss_first_epoch": hist[0], "loss_last_epoch": hist[-1]}
    return model, info


def _note(msg):
    """Progress of the legs on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def batched_leg(L, LR, dev, count, train_maps, train_epochs):
    """Maps of uneven size (n ~ U[1024, 16384], d = 32, lambda log-uniform in
    [1e-5, 1e-2], 1..8 transmitters) solved together to float64 relative
    residual 1e-6 with learned preconditioners, against the same maps solved
    one after the other with the same kernels."""
    import torch

    from synth import make_batch_specs, make_problem
    model, _ = train_model(L, LR, 32, dev, max(16, train_maps // 2), train_epochs)
    probs, ys = [], []
    for (n, lam, ntx, seed) in make_batch_specs(count, 1024, 16384, 1e-5, 1e-2, 1, 8, seed=4):
        pr = make_problem(n, 32, lam, n_tx=ntx, seed=seed)
        probs.append(L.Problem(torch.tensor(pr.E, device=dev), pr.lam, pr.scale))
        ys.append(torch.tensor(pr.y, device=dev))
    kw = dict(tol=1e-6, max_iter=200000, precision="bf16", refine=True, inner_tol=0.1, ir_max=64, check_every=32,
              materialized=True)
    # autotune once (cached per size class), then time without and with the
    # iteration chunks captured into HIP graphs
    precs = [L.learned_precond(p, model) for p in probs]
    L.pcg_solve_batched(probs, ys, precs, cols_per_split=-1, xcd_order=False, allow_noconv=True, **kw)
    torch.cuda.synchronize()
    timed = {}
    for graph in (False, True):
        a = time.perf_counter()
        precs = [L.learned_precond(p, model) for p in probs]
        _, st_g, used = L.pcg_solve_batched(probs, ys, precs, cols_per_split=-1, xcd_order=False, allow_noconv=True,
                                            graph=graph, **kw)
        torch.cuda.synchronize()
        timed[graph] = (time.perf_counter() - a, st_g)
    use_graph = timed[True][0] < timed[False][0]
    b_s, st = timed[use_graph]
    _note(f"batched leg: {count} maps together in {b_s:.2f} s (graphs {'on' if use_graph else 'off'}); "
          "now one after the other")
    b = time.perf_counter()
    a = b - b_s
    its_serial = []
    for p, y in zip(probs, ys):
        pc = L.learned_precond(p, model)
        _, s1 = L.pcg_solve(p, y, pc, allow_noconv=True, **kw)
        its_serial.append(s1.iters)
    torch.cuda.synchronize()
    c = time.perf_counter()
    return {"maps": count, "pairs_per_sweep": float(sum(p.n * p.n for p in probs)),
            "batched_s": b - a, "maps_per_s": count / (b - a), "serial_s": c - b, "serial_maps_per_s": count / (c - b),
            "batched_s_graphs_off": timed[False][0], "batched_s_graphs_on": timed[True][0], "graphs": use_graph,
            "speedup_vs_serial": (c - b) / (b - a), "converged": sum(1 for x in st if x.status == 0),
            "worst_relres_true": max(x.relres_true for x in st), "escalations": sum(x.escalations for x in st),
            "max_iters": max(x.iters for x in st), "cols_per_split_largest": used}


def learned_eval_leg(L, LR, dev, count, train_maps, train_epochs):
    """Held-out maps of 32768 sites (d = 32, lambda log-uniform in [1e-5, 1e-2],
    1..8 transmitters, seeds outside the training set): time to float64
    relative residual 1e-6 and inner iterations with the learned preconditioner
    (built per map; CCCP fallback on a stall) against a CCCP fit and solve,
    both by the flexible float64 outer CG around bf16 inner PCG."""
    import numpy as np
    import torch

    from synth import default_n_r, make_directions, make_problem
    model, _ = train_model(L, LR, 32, dev, train_maps, train_epochs)
    rng = np.random.default_rng(777)
    n = 32768
    kw = dict(tol=1e-6, precision="bf16", refine=2, inner_tol=0.1, check_every=INNER_CAP, inner_max_iter=INNER_CAP,
              materialized=True)
    rows = []
    for k in range(count):
        lam = float(10 ** rng.uniform(-5, -2))
        ntx = int(rng.integers(1, 9))
        pr = make_problem(n, 32, lam, n_tx=ntx, seed=50000 + k)
        prob = L.Problem(torch.tensor(pr.E, device=dev), pr.lam, pr.scale)
        y = torch.tensor(pr.y, device=dev)
        Zd = torch.tensor(make_directions(n, default_n_r(n), 50000 + k), device=dev)
        torch.cuda.synchronize()
        a = time.perf_counter()
        res = LR.solve_with_fallback(prob, y, model, Zd, budget=100000, gamma=0.1, stall_window=STALL_WINDOW, **kw)
        torch.cuda.synchronize()
        b = time.perf_counter()
        pc = L.fit_precond(prob, Zd, gamma=0.1, rho=0.0, precision="bf16")
        _, st = L.pcg_solve(prob, y, pc, max_iter=100000, ir_max=1000, allow_noconv=True, **kw)
        torch.cuda.synchronize()
        c = time.perf_counter()
        its = res.stats.iters
        rows.append((its, b - a, res.fell_back, res.stats.status == 0, st.iters, c - b, st.status == 0))
        if (k + 1) % 8 == 0:
            _note(f"learned evaluation: {k + 1} of {count} maps")
    it_l = np.array([r[0] for r in rows], dtype=float)
    it_c = np.array([r[4] for r in rows], dtype=float)
    t_l = sum(r[1] for r in rows)
    t_c = sum(r[5] for r in rows)
    return {"maps": count, "n": n, "d": 32, "train_maps": train_maps,
            "learned_iters_mean": float(it_l.mean()), "cccp_iters_mean": float(it_c.mean()),
            "learned_fewer_iters_maps": int((it_l < it_c).sum()),
            "learned_s": t_l, "cccp_s": t_c, "learned_speedup": t_c / t_l,
            "fallbacks": sum(1 for r in rows if r[2]),
            "converged_learned": sum(1 for r in rows if r[3]), "converged_cccp": sum(1 for r in rows if r[6])}


def solve_cost(L, prob, y, pc, kw):
    """Time of one solve with the given preconditioner (seconds) and its stats."""
    import torch
    torch.cuda.synchronize()
    a = time.perf_counter()
    _, st = L.pcg_solve(prob, y, pc, allow_noconv=True, **kw)
    torch.cuda.synchronize()
    return time.perf_counter() - a, st


def cccp_mixed_leg(L, prob, y, Zd, Eq, tol, gamma, hist):
    """CCCP fit (bfloat16 directions) + the same solver as the timed step
    (flexible float64 outer CG around capped bf16 inner PCG, stored G for the
    outer products) + predict: the learned preconditioner's comparison with
    identical solver options."""
    import torch
    torch.cuda.synchronize()
    a = time.perf_counter()
    pc = L.fit_precond(prob, Zd, gamma=gamma, rho=0.0, precision="bf16")
    torch.cuda.synchronize()
    b = time.perf_counter()
    alc, stc = L.pcg_solve(prob, y, pc, tol=tol, max_iter=400000, precision="bf16", refine=2, inner_tol=0.1,
                           ir_max=20000, check_every=INNER_CAP, inner_max_iter=INNER_CAP, materialized=True,
                           allow_noconv=True, outer_history=hist)
    torch.cuda.synchronize()
    c = time.perf_counter()
    L.predict(prob, alc, Eq, precision="f64")
    torch.cuda.synchronize()
    d_ = time.perf_counter()
    return {"gamma": gamma, "fit_ms": (b - a) * 1e3, "solve_ms": (c - b) * 1e3, "predict_ms": (d_ - c) * 1e3,
            "solves_per_s": 1.0 / (d_ - a), "pcg_iters": stc.iters, "outer_steps": stc.ir_steps,
            "relres_true": stc.relres_true, "converged": stc.status == 0, "cccp_iters": pc.stats.cccp_iters}, pc


# the paper's Table II (Sec. V-B), for direction and order of magnitude only
# (its embedding map is unspecified; hardware not stated)
PAPER_TABLE2 = {50: (5.05e3, 1.33e2, 16, 21), 200: (2.02e4, 1.95e2, 21, 32), 500: (5.04e4, 2.07e2, 25, 42),
                1000: (1.01e5, 1.79e2, 28, 47), 2000: (2.02e5, 2.09e2, 30, 59)}


def paper_regime_leg(L, dev):
    """The paper's numerical layer (Sec. V-A): G = exp(E E^T), d_e = 10,
    lambda = 1e-2, gamma = 0.1, rho by the undersampling rule, N_r by the
    schedule, n in {50, 200, 500, 1000, 2000}.  Per n: kappa(lambda I + G),
    kappa(P (lambda I + G)) and kappa(P_J (lambda I + G)) estimated from the
    PCG coefficients (Lanczos), iterations to an objective gap of 1e-3 for
    LAKER, Jacobi PCG and CG, LAKER's time (fit + PCG to 1e-10), final
    residual, objective gap and map RMSE, beside the paper's Table II."""
    import torch

    from synth import default_n_r, make_directions, make_paper_problem, paper_rho
    rows = {}
    for n in (50, 200, 500, 1000, 2000):
        pr = make_paper_problem(n, seed=n)
        prob = L.Problem(torch.tensor(pr.E, device=dev), pr.lam, pr.scale)
        y = torch.tensor(pr.y, device=dev)
        nr = default_n_r(n)
        rho = paper_rho(n, nr, 0.1)
        Zd = torch.tensor(make_directions(n, nr, n), device=dev)
        # warm-up of the kernels at this size, then LAKER timed: fit + PCG to 1e-10
        pc = L.fit_precond(prob, Zd, gamma=0.1, rho=rho)
        L.pcg_solve(prob, y, pc, tol=1e-10, max_iter=20000, precision="f64", allow_noconv=True)
        torch.cuda.synchronize()
        a = time.perf_counter()
        pc = L.fit_precond(prob, Zd, gamma=0.1, rho=rho)
        al, st = L.pcg_solve(prob, y, pc, tol=1e-10, max_iter=20000, precision="f64", lanczos=True)
        torch.cuda.synchronize()
        t_laker = time.perf_counter() - a
        jac = L.jacobi_precond(prob)
        torch.cuda.synchronize()
        a = time.perf_counter()
        _, sj = L.pcg_solve(prob, y, jac, tol=1e-10, max_iter=20000, precision="f64", lanczos=True,
                            allow_noconv=True)
        torch.cuda.synchronize()
        t_jac = time.perf_counter() - a
        _, sc = L.pcg_solve(prob, y, None, tol=1e-10, max_iter=20000, precision="f64", lanczos=True,
                            allow_noconv=True)
        a_star, _ = L.pcg_solve(prob, y, pc, tol=1e-13, max_iter=20000, precision="f64", allow_noconv=True)

        def R(v):
            g = L.kernel_matvec(prob, v, "f64") - pr.lam * v
            return float(torch.sum((g - y) ** 2) + pr.lam * torch.dot(v, g))
        rs = R(a_star)

        def iters_to_gap(q):
            for k in range(1, 600):
                v, _ = L.pcg_solve(prob, y, q, tol=1e-30, max_iter=k, precision="f64", check_every=k,
                                   allow_noconv=True)
                if abs(R(v) - rs) <= 1e-3 * abs(rs):
                    return k
            return None
        rhat = L.predict(prob, al, torch.tensor(pr.Eq, device=dev), precision="f64").cpu()
        ref = PAPER_TABLE2[n]
        rows[str(n)] = {
            "n_r": nr, "rho": rho, "cccp_iters": pc.stats.cccp_iters,
            "kappa_A": sc.cond_est, "kappa_PA": st.cond_est, "kappa_PJA": sj.cond_est,
            "iters_to_gap_1e-3": {"laker": iters_to_gap(pc), "jacobi": iters_to_gap(jac), "cg": iters_to_gap(None)},
            "pcg_iters_to_1e-10": {"laker": st.iters, "jacobi": sj.iters, "cg": sc.iters},
            "laker_ms": t_laker * 1e3, "jacobi_pcg_ms": t_jac * 1e3, "relres_true": st.relres_true,
            "obj_gap": abs(R(al) - rs) / abs(rs),
            "rmse_db": float(torch.sqrt(torch.mean((rhat - torch.tensor(pr.r_true)) ** 2))),
            "paper": {"kappa_A": ref[0], "kappa_PA": ref[1], "iters_laker": ref[2], "iters_jacobi": ref[3]}}
    return rows


def multi_rhs_leg(L, dev, k=8):
    """Several right-hand sides on one map (k bands or snapshots measured at the
    same 16384 sites, d = 64, lambda = 1e-3): the k columns solved together
    (one product launch per iteration for all columns, float64) against the
    same k solves one after the other (float64 products recomputed, and with G
    stored once per solve), CCCP preconditioner, PCG to 1e-6."""
    import numpy as np
    import torch

    from synth import default_n_r, make_directions, make_problem
    n, d, lam = 16384, 64, 1e-3
    pr = make_problem(n, d, lam, n_tx=4, seed=11)
    prob = L.Problem(torch.tensor(pr.E, device=dev), pr.lam, pr.scale)
    rng = np.random.default_rng(11)
    # band-to-band variation of the measured field
    Y = pr.y[:, None] + rng.normal(0.0, 3.0, size=(n, k))
    Yd = torch.tensor(Y, device=dev)
    pc = L.fit_precond(prob, torch.tensor(make_directions(n, default_n_r(n), 11), device=dev), gamma=0.1)
    kw = dict(tol=1e-6, max_iter=20000, precision="f64", check_every=32)
    L.pcg_solve_multi(prob, Yd[:, :2], pc, **kw)
    torch.cuda.synchronize()
    a = time.perf_counter()
    _, st = L.pcg_solve_multi(prob, Yd, pc, **kw)
    torch.cuda.synchronize()
    t_multi = time.perf_counter() - a
    out = {"n": n, "d": d, "lambda": lam, "k": k, "multi_s": t_multi,
           "multi_iters": [s.iters for s in st], "multi_worst_relres_true": max(s.relres_true for s in st)}
    for mat in (False, True):
        torch.cuda.synchronize()
        a = time.perf_counter()
        its = []
        for q in range(k):
            _, s1 = L.pcg_solve(prob, Yd[:, q], pc, materialized=mat, **kw)
            its.append(s1.iters)
        torch.cuda.synchronize()
        key = "serial_stored_g" if mat else "serial_recomputed"
        out[key + "_s"] = time.perf_counter() - a
        out[key + "_iters"] = its
    out["speedup_vs_serial_recomputed"] = out["serial_recomputed_s"] / t_multi
    out["speedup_vs_serial_stored_g"] = out["serial_stored_g_s"] / t_multi
    return out


def online_leg(L, dev):
    """Sites appended to a fitted map (16384 sites, 1024 of them arriving after
    the first 15360 were fitted and solved; d = 64, lambda = 1e-3): the
    extended fit (products with the new rows only, CCCP from the previous
    weights) and PCG from the previous solution, against a fresh fit and a
    solve from zero; float64, PCG to 1e-6."""
    import torch

    from synth import default_n_r, make_directions, make_problem
    n, m, d, lam = 16384, 1024, 64, 1e-3
    n0 = n - m
    pr = make_problem(n, d, lam, n_tx=4, seed=12)
    nr = default_n_r(n)
    Z = torch.tensor(make_directions(n, nr, 12), device=dev)
    E = torch.tensor(pr.E, device=dev)
    prob0 = L.Problem(E[:n0].contiguous(), pr.lam, pr.scale)
    prob = L.Problem(E, pr.lam, pr.scale)
    y = torch.tensor(pr.y, device=dev)
    kw = dict(tol=1e-6, max_iter=20000, precision="f64", check_every=32, materialized=True)
    state = L.OnlineFitState(n, nr, dev)
    pc0 = state.fit(prob0, Z[:n0].contiguous(), gamma=0.1)
    a0, _ = L.pcg_solve(prob0, y[:n0], pc0, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pc1 = state.fit(prob, Z, gamma=0.1)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    start = torch.cat([a0, torch.zeros(m, dtype=torch.float64, device=dev)])
    _, s1 = L.pcg_solve(prob, y, pc1, alpha0=start, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    pcf = L.fit_precond(prob, Z, gamma=0.1)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    _, s2 = L.pcg_solve(prob, y, pcf, **kw)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    return {"n_prev": n0, "appended": m, "n_r": nr,
            "online_fit_ms": (t1 - t0) * 1e3, "online_cccp_iters": pc1.stats.cccp_iters,
            "warm_pcg_ms": (t2 - t1) * 1e3, "warm_pcg_iters": s1.iters,
            "fresh_fit_ms": (t3 - t2) * 1e3, "fresh_cccp_iters": pcf.stats.cccp_iters,
            "cold_pcg_ms": (t4 - t3) * 1e3, "cold_pcg_iters": s2.iters,
            "speedup": (t4 - t2) / (t2 - t0)}


def c2_leg(L, LR, model, dev):
    """The 16384-site map (d = 64, 4 transmitters, lambda = 1e-4): the learned
    step as timed above, and float32 CCCP-PCG with G stored once (float32
    tiles streamed from HBM) against G recomputed in every product."""
    import torch

    from synth import default_n_r, make_directions, make_problem
    wl = WORKLOADS["n16384_d64"]
    pr = make_problem(wl["n"], wl["d"], wl["lam"], n_tx=wl["n_tx"], seed=wl["seed"])
    prob = L.Problem(torch.tensor(pr.E, device=dev), pr.lam, pr.scale)
    y = torch.tensor(pr.y, device=dev)
    Zd = torch.tensor(make_directions(pr.n, default_n_r(pr.n), wl["seed"]), device=dev)
    Eq = torch.tensor(pr.Eq, device=dev)
    tol = wl["tol"]

    def step():
        res = LR.solve_with_fallback(prob, y, model, Zd, tol=tol, budget=200000, precision="bf16", refine=2,
                                     inner_tol=0.1, gamma=0.1, check_every=INNER_CAP, inner_max_iter=INNER_CAP,
                                     materialized=True, stall_window=STALL_WINDOW)
        L.predict(prob, res.alpha, Eq, precision="f64")
        return res

    step()
    torch.cuda.synchronize()
    a = time.perf_counter()
    reps = 5
    for _ in range(reps):
        res = step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - a) * 1e3 / reps
    out = {"workload": "n=16384 d=64 n_tx=4 lambda=1e-4 tol=1e-6", "learned_step_ms": ms,
           "learned_solves_per_s": 1e3 / ms, "learned_pcg_iters": res.stats.iters,
           "learned_relres_true": res.stats.relres_true}
    pc = L.fit_precond(prob, Zd, gamma=0.1, rho=0.0, precision="bf16")
    f32c = {}
    for mat in (False, True):
        kw32 = dict(tol=tol, max_iter=100000, precision="f32", refine=True, inner_tol=0.1, ir_max=64,
                    check_every=32, materialized=mat)
        dt, s32 = solve_cost(L, prob, y, pc, kw32)
        _, s32p = L.pcg_solve(prob, y, pc, profile=True, **kw32)
        f32c["stored" if mat else "recomputed"] = {
            "ms_per_solve": dt * 1e3, "pcg_iters": s32.iters, "ir_steps": s32.ir_steps,
            "relres_true": s32.relres_true, "us_per_product": s32p.kmv_ms * 1e3}
    sb32 = L.load().laker_kmat_bytes(pr.n, pr.d, L.F32)
    f32c["stored"]["gb_per_s"] = sb32 / (f32c["stored"]["us_per_product"] * 1e-6) / 1e9
    f32c["stored"]["frac_of_hbm_peak"] = f32c["stored"]["gb_per_s"] / PEAK_HBM_GBS
    f32c["stored_bytes"] = sb32
    us32 = f32c["recomputed"]["us_per_product"] * 1e-6
    dist = pr.n * (pr.n + 1) / 2.0
    f32c["recomputed"]["frac_of_alu_peak"] = (EXP2_SLOTS * dist + float(pr.n) * pr.n) / us32 / 1e12 / PEAK_VALU_TOPS
    f32c["recomputed"]["frac_of_fp32_mfma_peak"] = 2.0 * pr.d * dist / us32 / 1e12 / PEAK_FP32_MFMA_TFLOPS
    out["f32_stored_vs_recomputed"] = f32c
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    from paper_2604_25138_amd import laker as L
    from paper_2604_25138_amd import learned as LR
    from synth import default_n_r, make_directions, make_problem

    L.load()
    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    pr = make_problem(wl["n"], wl["d"], wl["lam"], n_tx=wl["n_tx"], seed=wl["seed"])
    nr = default_n_r(pr.n)
    Z = make_directions(pr.n, nr, wl["seed"])
    prob = L.Problem(torch.tensor(pr.E, device=dev), pr.lam, pr.scale)
    y = torch.tensor(pr.y, device=dev)
    Zd = torch.tensor(Z, device=dev)
    Eq = torch.tensor(pr.Eq, device=dev)
    tol = wl["tol"]
    hist = wl["history"]
    budget = 400000

    if args.counters:
        # the product kernel alone, then a plain copy of known size whose
        # counter readings calibrate FETCH_SIZE / WRITE_SIZE
        p1 = torch.ones(pr.n, dtype=torch.float64, device=dev)
        for _ in range(20):
            L.kernel_matvec(prob, p1, "bf16")
        # float64 products streaming the stored G: a 20-iteration float64 PCG
        L.pcg_solve(prob, y, None, tol=1e-30, max_iter=20, precision="f64", check_every=32, allow_noconv=True,
                    materialized=True)
        a = torch.empty(64 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"counters": "done", "products": 20, "stored_g_products": 21, "copy_bytes": 4 * (64 << 20)}))
        return

    model, train_info = train_model(L, LR, pr.d, dev, args.train_maps, args.train_epochs)
    _note("preconditioner network trained")

    def step():
        res = LR.solve_with_fallback(prob, y, model, Zd, tol=tol, budget=budget, precision="bf16", refine=2,
                                     inner_tol=0.1, gamma=0.1, check_every=INNER_CAP, inner_max_iter=INNER_CAP,
                                     materialized=True, stall_window=STALL_WINDOW, outer_history=hist)
        rhat = L.predict(prob, res.alpha, Eq, precision="f64")
        return res, rhat

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    runs = []
    for k in range(args.steps):
        res, rhat = step()
        runs.append(res)
        if pr.n >= 32768:
            torch.cuda.synchronize()
            _note(f"timed step {k + 1} of {args.steps}")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = 1e3 / ms_per_step
    rmse = float(torch.sqrt(torch.mean((rhat.cpu() - torch.tensor(pr.r_true)) ** 2)))
    last = runs[-1]
    extra = {
        "pcg_iters": last.stats.iters, "outer_steps": last.stats.ir_steps, "relres_true": last.stats.relres_true,
        "fell_back": max(r.fell_back for r in runs), "learned_iters": last.learned_iters,
        "map_rmse_db": rmse, "training": train_info,
    }
    torch.cuda.synchronize()
    a = time.perf_counter()
    L.learned_precond(prob, model)
    torch.cuda.synchronize()
    extra["learned_precond_ms"] = (time.perf_counter() - a) * 1e3
    _note("timed step done")

    # CCCP + mixed precision on the same map with the same solver, at the
    # paper's gamma = 0.1 and at the gamma of the network's training targets
    extra["cccp_mixed"] = {}
    pc = None
    for g in (0.1, 1e-3):
        leg, pcg_ = cccp_mixed_leg(L, prob, y, Zd, Eq, tol, g, hist)
        extra["cccp_mixed"][f"gamma_{g:g}"] = leg
        if pc is None:
            pc = pcg_
    extra["cccp_mixed"]["n_r"] = nr
    _note("CCCP + mixed precision legs done")

    # float64 CCCP-PCG on the same map (the method with every product in float64)
    if not args.no_f64:
        torch.cuda.synchronize()
        a = time.perf_counter()
        pc64 = L.fit_precond(prob, Zd, gamma=0.1, rho=0.0)
        torch.cuda.synchronize()
        fa = time.perf_counter()
        al64, st64 = L.pcg_solve(prob, y, pc64, tol=tol, max_iter=100000, precision="f64", check_every=32,
                                 materialized=True)
        L.predict(prob, al64, Eq, precision="f64")
        torch.cuda.synchronize()
        b = time.perf_counter()
        extra["f64_cccp_pcg"] = {"solves_per_s": 1.0 / (b - a), "ms_per_solve": (b - a) * 1e3,
                                 "fit_ms": (fa - a) * 1e3, "cccp_iters": pc64.stats.cccp_iters,
                                 "pcg_iters": st64.iters, "relres_true": st64.relres_true}
        extra["speedup_vs_f64_cccp_pcg"] = (b - a) * 1e3 / ms_per_step
        _note("float64 CCCP-PCG leg done")

    # roofline of the dominant kernel: the fused product exp2(<e_i, e_j>) p of
    # the solve, timed by the library with HIP events on the stream it launches
    # on (one pair of events around every product of the loop)
    pcl = L.learned_precond(prob, model)
    _, stp = L.pcg_solve(prob, y, pcl, tol=tol, max_iter=budget, precision="bf16", refine=2, inner_tol=0.1,
                         ir_max=20000, check_every=INNER_CAP, inner_max_iter=INNER_CAP, profile=True,
                         materialized=True, outer_history=hist)
    kms = stp.kmv_ms
    pairs = float(pr.n) * pr.n
    # the symmetric product forms each of the n (n + 1) / 2 distinct kernel
    # entries once (one exp2) and uses it for both of its ordered pairs (one
    # multiply-add each); its score tiles cost 2 d flops per distinct entry
    distinct = pr.n * (pr.n + 1) / 2.0
    slots = EXP2_SLOTS * distinct + pairs
    achieved = slots / (kms * 1e-3) / 1e12
    mfma_flops = 2.0 * pr.d * distinct
    traffic = measured_traffic(args.workload)
    roofline = {"kernel": "kmvsym16_kernel<64> (fused exp2(<e_i,e_j>) p product over the symmetric tile "
                          "schedule, bf16 16x16x32 score tiles on MFMA, 64 rows per wave)",
                "bound": "alu", "achieved": achieved, "peak": PEAK_VALU_TOPS, "unit": "TOP/s",
                "frac": achieved / PEAK_VALU_TOPS, "traffic": traffic,
                "per_launch": {"pairs": pairs, "distinct_entries": distinct, "valu_slot_ops": slots,
                               "mfma_flops": mfma_flops, "ms": kms, "products_timed": stp.kmv_count,
                               "launches": stp.kmv_launches, "ms_all_launches": stp.kmv_launch_ms},
                "mfma": {"achieved": mfma_flops / (kms * 1e-3) / 1e12, "peak": PEAK_BF16_MFMA_TFLOPS,
                         "unit": "TFLOP/s"}}
    roofline["mfma"]["frac"] = roofline["mfma"]["achieved"] / roofline["mfma"]["peak"]

    # stand-alone products of the three precisions (one product + its finishing
    # reduction per call), for reference
    p = torch.randn(pr.n, dtype=torch.float64, device=dev)

    def time_kmv(pname, reps=10):
        for _ in range(2):
            L.kernel_matvec(prob, p, pname)
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            L.kernel_matvec(prob, p, pname)
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    standalone = {q: time_kmv(q) for q in ("bf16", "f32", "f64")}
    extra["kmv_standalone_ms"] = standalone
    extra["kmv_standalone_gpairs_per_s"] = {q: pairs / (v * 1e-3) / 1e9 for q, v in standalone.items()}
    _note("roofline and stand-alone products done")

    if not args.no_paper:
        extra["paper_regime"] = paper_regime_leg(L, dev)
        _note("paper regime sweep done")
    if not args.no_multi:
        extra["multi_rhs"] = multi_rhs_leg(L, dev)
        extra["online"] = online_leg(L, dev)
        _note("multi-right-hand-side and online legs done")

    if args.workload != "n16384_d64" and not args.no_c2:
        extra["n16384_d64"] = c2_leg(L, LR, model, dev)
        _note("16384-site leg done")

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "bf16+f64", "data": "synthetic",
        "config": {"workload": f"{args.workload}: n={pr.n} d={pr.d} n_tx={wl['n_tx']} lambda={pr.lam} "
                               f"scale=1/sqrt(d) tol={tol}",
                   "path": "learned rank-64+diag preconditioner (BF16 MLP) + flexible f64 outer CG (its float64 "
                           "products stream G stored once per solve) around bf16 "
                           f"inner PCG (<= {INNER_CAP} iterations each; {hist} outer directions kept; CCCP "
                           f"fallback in the library when the "
                           f"residual falls less than 2x over {STALL_WINDOW} iterations) + predict 45x45",
                   "training": f"{args.train_maps} maps n={TRAIN_N} lambda~logU[1e-5,1e-2] n_tx~U{{1..8}}, "
                               f"{args.train_epochs} epochs, CCCP targets gamma=1e-3"},
        "roofline": roofline,
        "extra": extra,
    }

    if args.learned_eval > 0:
        extra["learned_eval"] = learned_eval_leg(L, LR, dev, args.learned_eval, args.train_maps, args.train_epochs)
    if args.batch_maps > 0:
        extra["batched"] = batched_leg(L, LR, dev, args.batch_maps, args.train_maps, args.train_epochs)
        _note("batched leg done")

    if not args.no_cpu:
        _note("CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(pr, Z, tol, extra.get("f64_cccp_pcg", {}).get("pcg_iters"),
                                           args.cpu_budget)
    print(json.dumps(out))


KMV_SOURCE = os.path.join(ROOT, "paper_2604_25138_amd", "csrc", "kmv.hip")


def measured_traffic(workload):
    """HBM bytes per launch of the product kernel from the committed counter
    runs (FETCH_SIZE and WRITE_SIZE, scaled by the same counters' reading for a
    plain copy), or None when the kernel source has changed since they were
    taken (the summary records the source's SHA-256)."""
    import hashlib
    summary = os.path.join(ROOT, "profiles", f"kmvsym_bf16_{workload}_pmc.json")
    try:
        with open(summary) as f:
            m = json.load(f)
        with open(KMV_SOURCE, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if m.get("kmv_source_sha256") != sha:
        return None
    return m.get("traffic_bytes_per_launch")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _threads():
    threads = os.cpu_count()
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 0) for i in threadpool_info()), default=threads) or threads
    except Exception:
        pass
    return threads


def cpu_baseline(pr, Z, tol, iters_hint, budget):
    """The FP64 oracle on the host cores.  Up to 16384 sites: the kernel
    matrix and the CCCP fit measured in full, PCG iterations measured on a
    bounded sample and scaled to the iteration count of the float64 GPU solve.
    Above, where the dense float64 matrix alone is n^2 8 bytes (34 GB at 65536
    sites): every stage timed on a block of rows and extrapolated (the oracle's
    cost is linear in the rows it forms): kernel matrix rows, the product of
    those rows with a vector (one PCG iteration's product), the random
    directions U = A Z on those rows, and the low-rank CCCP iteration on the
    full N_r x N_r system; the solve scaled to the float64 GPU solve's
    iteration count."""
    import numpy as np

    from oracle import laker_oracle as O
    threads = _threads()
    cpu = _cpu_model()
    iters_default = iters_hint if iters_hint else 1000
    if pr.n <= 16384:
        t0 = time.perf_counter()
        A = O.system_matrix(pr.E, pr.scale, pr.lam)
        t1 = time.perf_counter()
        P, _ = O.fit_precond(pr.E, pr.scale, pr.lam, Z, gamma=0.1, rho=0.0)
        t2 = time.perf_counter()
        remaining = max(1.0, budget - (t2 - t0))
        tm = time.perf_counter()
        _ = A @ P.apply(pr.y)
        per_it = time.perf_counter() - tm
        k = int(max(3, min(200, remaining / max(per_it, 1e-6))))
        _, it_done, _ = O.pcg(lambda v: A @ v, P.apply, pr.y, tol, k)
        t3 = time.perf_counter()
        per_iter = (t3 - t2) / max(it_done, 1)
        iters = iters_hint if iters_hint else it_done
        solve_s = (t1 - t0) + (t2 - t1) + per_iter * iters
        return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": threads, "cpu": cpu, "kind": "oracle",
                "sample": f"oracle FP64 CCCP-PCG on n={pr.n}: kernel matrix {t1 - t0:.1f}s + CCCP fit "
                          f"{t2 - t1:.1f}s (measured) + {it_done} PCG iterations measured at "
                          f"{per_iter * 1e3:.1f} ms each, scaled to {iters} iterations",
                "seconds_measured": t3 - t0}
    n, nr = pr.n, Z.shape[1]
    rows = np.arange(min(n, 2048))
    frac = n / len(rows)
    t0 = time.perf_counter()
    Gb = O.kernel_matrix(pr.E, pr.scale, Eq=pr.E[rows])
    t1 = time.perf_counter()
    v = np.random.default_rng(0).normal(size=n)
    reps = 5
    for _ in range(reps):
        _ = Gb @ v + pr.lam * v[rows]
    t2 = time.perf_counter()
    _ = Gb @ Z
    t3 = time.perf_counter()
    # the CCCP iteration on the full-size low-rank system: its cost does not
    # depend on the values of the directions, so normalised Gaussian columns
    # stand in for them
    Ub = Z / np.linalg.norm(Z, axis=0)[None, :]
    _, _, _, cit = O.cccp_lowrank(Ub, 0.1, 0.0, 1e-10, 1e-8, 40)
    t4 = time.perf_counter()
    P = O.LowRankPrecond(Ub, 0.5, 0.5, np.ones(nr))
    t5 = time.perf_counter()
    for _ in range(reps):
        _ = P.apply(v)
    t6 = time.perf_counter()
    form_s = (t1 - t0) * frac
    matvec_s = (t2 - t1) / reps * frac
    dirs_s = (t3 - t2) * frac
    cccp_s = (t4 - t3) / max(cit, 1) * 300 + (t5 - t4)
    apply_s = (t6 - t5) / reps
    iters = iters_default
    solve_s = form_s + dirs_s + cccp_s + iters * (matvec_s + apply_s)
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": threads, "cpu": cpu, "kind": "oracle",
            "extrapolated": True,
            "sample": f"oracle FP64 CCCP-PCG on n={n}, extrapolated from a block of {len(rows)} rows "
                      f"(x{frac:.0f}): kernel matrix {form_s:.1f}s, directions U = A Z {dirs_s:.1f}s, "
                      f"CCCP (300 iterations, {cit} timed) {cccp_s:.1f}s, then {iters} PCG iterations at "
                      f"{(matvec_s + apply_s) * 1e3:.0f} ms each (product {matvec_s * 1e3:.0f} ms, apply "
                      f"{apply_s * 1e3:.1f} ms)",
            "seconds_measured": t6 - t0}


if __name__ == "__main__":
    main()
