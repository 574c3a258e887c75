"""The allocation-free kernel product (laker_kernel_matvec_noalloc) against
laker_kernel_matvec, through the C ABI.

Both run the same kernels with the same plan and the same order of the partial
sums, so the results must be bitwise equal.  Two calls in a row share the
library's device scratch: the second, on a smaller problem, must not see
anything of the first.  Each result is also checked against the float64
oracle (float64: 1e-13 relative to sum_j |G_ij p_j| + lam |p_i|, the bound of
the product's parity tests)."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import laker_oracle as O
from synth import make_problem

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _lib():
    from paper_2604_25138_amd import laker as L
    lib = L.load()
    f = lib.laker_kernel_matvec_noalloc
    f.argtypes = [C.POINTER(L.laker_problem), C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]
    f.restype = C.c_int32
    return L, lib


def _noalloc(L, lib, prob, p, prec):
    w = torch.full_like(p, float("nan"))
    s = lib.laker_kernel_matvec_noalloc(C.byref(prob.c), C.c_void_p(p.data_ptr()), C.c_void_p(w.data_ptr()),
                                        L._PREC[prec], L._stream())
    assert s == L.LAKER_OK, L.status_str(s)
    return w


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_noalloc_matches_workspace_product_twice(prec):
    L, lib = _lib()
    # first a product large enough for the symmetric schedule (bf16 from ~9900
    # sites), then a smaller one with a ragged tail
    for n, d, seed in ((12000, 64, 1), (2048 + 37, 32, 2)):
        pr = make_problem(n, d, 1e-3, seed=seed)
        prob = L.Problem(torch.tensor(pr.E, device=DEV), pr.lam, pr.scale)
        p = torch.tensor(np.random.default_rng(seed).normal(size=n), device=DEV)
        ref = L.kernel_matvec(prob, p, prec)
        got = _noalloc(L, lib, prob, p, prec)
        torch.cuda.synchronize()
        print(f"noalloc {prec} n={n} d={d}", flush=True)
        assert torch.equal(got, ref), (prec, n, (got - ref).abs().max().item())
        if prec == "f64":
            rows = np.random.default_rng(seed).choice(n, size=64, replace=False)
            pv = p.cpu().numpy()
            want = O.matvec_rows(pr.E, pr.scale, pr.lam, pv, rows)
            G = np.exp(pr.scale * (pr.E[rows] @ pr.E.T))
            mag = np.abs(G) @ np.abs(pv) + pr.lam * np.abs(pv[rows])
            assert (np.abs(got.cpu().numpy()[rows] - want) / mag).max() <= 1e-13


def test_noalloc_rejects_problems_beyond_its_scratch():
    L, lib = _lib()
    n = 65536
    E = torch.zeros(n, 64, dtype=torch.float64, device=DEV)
    prob = L.Problem(E, 1e-3, 0.125)
    p = torch.ones(n, dtype=torch.float64, device=DEV)
    w = torch.zeros_like(p)
    s = lib.laker_kernel_matvec_noalloc(C.byref(prob.c), C.c_void_p(p.data_ptr()), C.c_void_p(w.data_ptr()),
                                        L.BF16, L._stream())
    torch.cuda.synchronize()
    assert s == L.LAKER_ENOMEM
    assert torch.count_nonzero(w).item() == 0
