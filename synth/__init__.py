"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only draws inputs: measurement sites, transmitters, the received
signal strength field, random-Fourier-feature embeddings of locations, query
grids, the Gaussian random directions z_k, training probes and the initial
weights of the learned preconditioner's network.  It holds none of the method's
arithmetic (no kernel, no solve, no preconditioner).
"""
from .inputs import (  # noqa: F401
    Problem, make_problem, make_directions, make_batch_specs, default_n_r, make_probes, make_mlp_init,
    make_paper_problem, paper_rho,
)
