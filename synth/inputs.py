"""Synthetic path-loss fields and location embeddings.

The paper evaluates on a synthetic radio field built from several transmitters
with distance-decaying power and log-normal shadowing, measured at sites drawn
uniformly over a square region (Sec. V-A "Problem Setup"), and maps each site to
an embedding through an unspecified position-driven map.  The recipe here is a
concrete instance of that description:

* region [0, L]^2 with L = 1000 m, sites and transmitters uniform in it;
* per-transmitter received power RSS_t(x) = -30 - 30 log10(max(|x - t|, 1 m)) dBm
  plus i.i.d. N(0, sigma^2) shadowing per (site, transmitter), sigma = 6 dB;
  powers of several transmitters are summed in mW;
* embeddings e(x) = sqrt(2/d) cos(x W + phi), W ~ N(0, 0.1^2 m^-2) entrywise,
  phi ~ U[0, 2 pi) -- random Fourier features of location (the paper cites
  random features as the scalable kernel approximation of this family);
* the map truth used for RMSE is the shadowing-free field on a 45 x 45 grid
  (Sec. V-A, evaluation grid).

Everything is drawn from numpy's PCG64 with an explicit seed.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

REGION_M = 1000.0
SHADOW_DB = 6.0
RFF_FREQ_STD = 0.1
GRID = 45


@dataclass
class Problem:
    n: int
    d: int
    lam: float
    scale: float
    E: np.ndarray            # (n, d) float64 embeddings of the measurement sites
    y: np.ndarray            # (n,) float64 measurements in dBm
    sites: np.ndarray        # (n, 2) metres
    tx: np.ndarray           # (n_tx, 2) metres
    Eq: np.ndarray           # (m, d) embeddings of the query grid
    r_true: np.ndarray       # (m,) shadowing-free field on the query grid, dBm
    seed: int = 0
    meta: dict = field(default_factory=dict)


def _field_dbm(points: np.ndarray, tx: np.ndarray, shadow: np.ndarray | None) -> np.ndarray:
    dist = np.sqrt(((points[:, None, :] - tx[None, :, :]) ** 2).sum(axis=2))
    dist = np.maximum(dist, 1.0)
    rss = -30.0 - 30.0 * np.log10(dist)
    if shadow is not None:
        rss = rss + shadow
    if tx.shape[0] == 1:
        return rss[:, 0]
    return 10.0 * np.log10(np.sum(10.0 ** (rss / 10.0), axis=1))


def _rff(points: np.ndarray, W: np.ndarray, phase: np.ndarray) -> np.ndarray:
    d = W.shape[1]
    return math.sqrt(2.0 / d) * np.cos(points @ W + phase[None, :])


def make_problem(n: int, d: int, lam: float, n_tx: int = 1, seed: int = 0,
                 scale: float | None = None, grid: int = GRID) -> Problem:
    """Draw one regression problem: sites, field samples y and embeddings E.

    scale defaults to 1/sqrt(d); the paper's own kernel has scale 1.
    """
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, REGION_M, size=(n, 2))
    tx = rng.uniform(0.0, REGION_M, size=(n_tx, 2))
    shadow = rng.normal(0.0, SHADOW_DB, size=(n, n_tx))
    y = _field_dbm(sites, tx, shadow)
    W = rng.normal(0.0, RFF_FREQ_STD, size=(2, d))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=d)
    E = _rff(sites, W, phase)
    g = np.linspace(0.0, REGION_M, grid)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    qpts = np.stack([gx.ravel(), gy.ravel()], axis=1)
    Eq = _rff(qpts, W, phase)
    r_true = _field_dbm(qpts, tx, None)
    s = (1.0 / math.sqrt(d)) if scale is None else float(scale)
    return Problem(n=n, d=d, lam=float(lam), scale=s, E=np.ascontiguousarray(E),
                   y=np.ascontiguousarray(y), sites=sites, tx=tx,
                   Eq=np.ascontiguousarray(Eq), r_true=r_true, seed=seed,
                   meta={"n_tx": n_tx})


# The paper's own numerical-layer regime (Sec. V-A, Table I): a 100 m x 100 m
# region, d_e = 10, G = exp(E E^T) (scale 1), lambda = 1e-2, measurement noise
# 1.5 dB.  Its position-to-embedding map is unspecified; random Fourier
# features with frequencies N(0, 0.05^2 m^-2) put kappa(lambda I + G) within
# 1.5x of the values Table II lists for n = 50 ... 2000.
PAPER_REGION_M = 100.0
PAPER_D = 10
PAPER_LAMBDA = 1e-2
PAPER_NOISE_DB = 1.5
PAPER_FREQ_STD = 0.05
PAPER_TX = 3


def make_paper_problem(n: int, seed: int = 0, grid: int = GRID) -> Problem:
    """One problem of the paper's sweep: n sites uniform in [0, 100]^2 m, the
    field a superposition of PAPER_TX transmitters' path loss (as make_problem,
    without shadowing), y = field + N(0, 1.5^2) dB, random Fourier feature
    embeddings of dimension 10, kernel scale 1, lambda = 1e-2; the map truth is
    the field on the 45 x 45 grid."""
    rng = np.random.default_rng(seed)
    sites = rng.uniform(0.0, PAPER_REGION_M, size=(n, 2))
    tx = rng.uniform(0.0, PAPER_REGION_M, size=(PAPER_TX, 2))
    y = _field_dbm(sites, tx, None) + rng.normal(0.0, PAPER_NOISE_DB, size=n)
    W = rng.normal(0.0, PAPER_FREQ_STD, size=(2, PAPER_D))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=PAPER_D)
    E = _rff(sites, W, phase)
    g = np.linspace(0.0, PAPER_REGION_M, grid)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    qpts = np.stack([gx.ravel(), gy.ravel()], axis=1)
    return Problem(n=n, d=PAPER_D, lam=PAPER_LAMBDA, scale=1.0, E=np.ascontiguousarray(E),
                   y=np.ascontiguousarray(y), sites=sites, tx=tx, Eq=np.ascontiguousarray(_rff(qpts, W, phase)),
                   r_true=_field_dbm(qpts, tx, None), seed=seed, meta={"n_tx": PAPER_TX, "paper_regime": True})


def paper_rho(n: int, n_r: int, gamma: float, eps_rho: float = 1e-3) -> float:
    """Shrinkage for the paper's sweep (Sec. V-A): a small fixed eps_rho when the
    directions are not undersampled (N_r >= n), otherwise growing with the
    undersampling 1 - N_r / n, scaled by gamma (capped at 1/2)."""
    if n_r >= n:
        return eps_rho
    return min(0.5, eps_rho + gamma * (1.0 - n_r / n))


def default_n_r(n: int) -> int:
    """Number of random directions: grows like sqrt(n) for small n, linearly
    for large n (Sec. V-A "Preconditioner Construction"), capped at 512.

    N_r = min(n, 512, max(ceil(4 sqrt(n)), ceil(n / 32))).
    """
    return int(min(n, 512, max(math.ceil(4.0 * math.sqrt(n)), math.ceil(n / 32.0))))


def make_directions(n: int, n_r: int, seed: int) -> np.ndarray:
    """z_k ~ N(0, I_n) for k = 1..N_r (eq. random_directions), returned as an
    (n, N_r) row-major float64 array: column k is z_k."""
    rng = np.random.default_rng(seed + 1_000_000)
    return np.ascontiguousarray(rng.standard_normal(size=(n, n_r)))


def make_batch_specs(count: int, n_lo: int, n_hi: int, lam_lo: float, lam_hi: float,
                     tx_lo: int, tx_hi: int, seed: int):
    """Sizes, regularisation weights and transmitter counts of a batch of
    independent maps: n ~ U[n_lo, n_hi], lambda log-uniform, n_tx ~ U{tx_lo..tx_hi}."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    lams = np.exp(rng.uniform(math.log(lam_lo), math.log(lam_hi), size=count))
    txs = rng.integers(tx_lo, tx_hi + 1, size=count)
    return [(int(a), float(b), int(c), seed * 100003 + i) for i, (a, b, c) in enumerate(zip(ns, lams, txs))]


def make_probes(n: int, m: int, seed: int) -> np.ndarray:
    """Gaussian probe vectors (n, m) for training the learned preconditioner."""
    rng = np.random.default_rng(seed + 2_000_000)
    return np.ascontiguousarray(rng.standard_normal(size=(n, m)))


def make_mlp_init(in_dim: int, hidden: int, out_dim: int, seed: int, log_delta0: float = -7.0) -> dict:
    """Initial weights of the 3-layer network (stored fan_in x fan_out), each
    entry uniform in +-1/sqrt(fan_in); the last output's bias (the log of the
    diagonal) starts at log_delta0."""
    rng = np.random.default_rng(seed + 3_000_000)
    dims = [(in_dim, hidden), (hidden, hidden), (hidden, out_dim)]
    p = {}
    for i, (a, b) in enumerate(dims, start=1):
        bound = 1.0 / math.sqrt(a)
        p[f"W{i}"] = rng.uniform(-bound, bound, size=(a, b))
        p[f"b{i}"] = rng.uniform(-bound, bound, size=b)
    p["b3"][out_dim - 1] = log_delta0
    return p
