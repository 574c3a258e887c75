"""Host-side checks of the C ABI: the built library loads without a GPU and
exports every entry point that include/laker.h declares; size queries and
argument validation need no device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "laker.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(laker_[a-z0-9_]+)\s*\(", src)))


def _lib():
    from paper_2604_25138_amd import laker
    if not os.path.exists(laker.LIB_PATH):
        pytest.skip("liblaker.so not built")
    return laker, laker.load()


def test_header_declarations_match_binding():
    from paper_2604_25138_amd import laker
    assert _declared() == sorted(laker.EXPORTS)


def test_library_exports_every_declared_symbol():
    laker, lib = _lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_size_queries_and_status_strings():
    laker, lib = _lib()
    assert lib.laker_precond_bytes(16384, 512) >= 16384 * 512 * 24
    assert lib.laker_precond_bytes(0, 4) == 0
    assert lib.laker_fit_workspace_bytes(512, 16, 91) > 0
    assert lib.laker_fit_workspace_bytes(512, 200, 91) == 0        # d above the supported maximum
    assert lib.laker_solve_workspace_bytes(1000, 10, 2025) > lib.laker_solve_workspace_bytes(1000, 10, 0)
    assert laker.status_str(0) == "ok"
    assert "invalid" in laker.status_str(-1)


def test_invalid_arguments_rejected_before_any_launch():
    """Validation happens on the host; null or inconsistent arguments return
    LAKER_EINVAL without touching the device."""
    laker, lib = _lib()
    prob = laker.laker_problem(16, 4, 0, None, 1e-2, 0.5)          # E = NULL
    opts = laker.laker_pcg_opts(1e-8, 10, 0, 0, 1, 1e-2, 0, 16)
    st = laker.laker_stats()
    r = lib.laker_pcg_solve(C.byref(prob), None, C.c_void_p(8), C.c_void_p(8), C.byref(opts), C.c_void_p(8),
                            1 << 30, C.byref(st), None)
    assert r == laker.LAKER_EINVAL
    prob = laker.laker_problem(16, 4, 0, 8, -1.0, 0.5)              # lambda <= 0
    r = lib.laker_kernel_matvec(C.byref(prob), C.c_void_p(8), C.c_void_p(8), 0, C.c_void_p(8), 1 << 30, None)
    assert r == laker.LAKER_EINVAL
    prob = laker.laker_problem(16, 4, 0, 8, 1e-2, 0.5)
    co = laker.laker_cccp_opts(32, 10, 0.1, 0.0, 1e-10, 1e-8, 0, 0)   # n_r > n
    pc = laker.laker_precond(2, 32, 16, 8, 1 << 30)
    r = lib.laker_fit_precond(C.byref(prob), C.c_void_p(8), C.byref(co), C.byref(pc), C.c_void_p(8), 1 << 30,
                              C.byref(st), None)
    assert r == laker.LAKER_EINVAL
    co = laker.laker_cccp_opts(8, 10, 0.1, 1.5, 1e-10, 1e-8, 0, 0)    # rho outside [0, 1]
    r = lib.laker_fit_precond(C.byref(prob), C.c_void_p(8), C.byref(co), C.byref(pc), C.c_void_p(8), 1 << 30,
                              C.byref(st), None)
    assert r == laker.LAKER_EINVAL
    opts = laker.laker_pcg_opts(1e-8, 10, 0, 0, 1, 1e-2, 0, 16)
    r = lib.laker_pcg_solve(C.byref(prob), None, C.c_void_p(8), C.c_void_p(8), C.byref(opts), C.c_void_p(8),
                            16, C.byref(st), None)                  # workspace too small
    assert r == laker.LAKER_ENOMEM


def _sym_stages(n):
    """Stages of the symmetric schedule (256-row blocks against 128-column
    stages on or right of the block diagonal), counted by brute force."""
    nrb, ncs = -(-n // 256), -(-n // 128)
    return sum(1 for I in range(nrb) for J in range(ncs) if J >= 2 * I)


def test_stored_kernel_matrix_size_query():
    """laker_kmat_bytes: one 256 x 128 tile per stage of the symmetric schedule
    (float64 or float32 entries), 0 below the schedule's threshold (2 stages per
    block of 256), for bfloat16 and for unsupported d."""
    laker, lib = _lib()
    for n, d in [(6000, 16), (5837, 64), (16384, 64), (65536, 32)]:
        T = _sym_stages(n)
        assert T >= 2 * 256
        assert lib.laker_kmat_bytes(n, d, laker.F64) == T * 256 * 128 * 8
        assert lib.laker_kmat_bytes(n, d, laker.F32) == T * 256 * 128 * 4
        assert lib.laker_kmat_bytes(n, d, laker.BF16) == 0
    assert _sym_stages(16384) == 4160 and lib.laker_kmat_bytes(16384, 64, laker.F64) == 4160 * 262144
    assert lib.laker_kmat_bytes(4096, 16, laker.F64) == 0          # fewer than 2 stages per block
    assert lib.laker_kmat_bytes(6000, 128, laker.F64) == 0         # dp above the schedule's 64
    assert lib.laker_kmat_bytes(6000, 200, laker.F64) == 0


def test_stored_kernel_matrix_options_validated_on_the_host():
    """materialized outside {0, 1} is rejected, and a workspace without room
    for the stored G is LAKER_ENOMEM, both before any device work."""
    laker, lib = _lib()
    n, d = 6000, 16
    prob = laker.laker_problem(n, d, 0, 8, 1e-2, 0.5)
    st = laker.laker_stats()
    ws = lib.laker_solve_workspace_bytes(n, d, 0)
    opts = laker.laker_pcg_opts(1e-8, 10, 0, 0, 1, 1e-2, 0, 16, 0, 0, 0, 2)
    r = lib.laker_pcg_solve(C.byref(prob), None, C.c_void_p(8), C.c_void_p(8), C.byref(opts), C.c_void_p(8),
                            ws, C.byref(st), None)
    assert r == laker.LAKER_EINVAL
    opts = laker.laker_pcg_opts(1e-8, 10, 0, 0, 1, 1e-2, 0, 16, 0, 0, 0, 1)
    r = lib.laker_pcg_solve(C.byref(prob), None, C.c_void_p(8), C.c_void_p(8), C.byref(opts), C.c_void_p(8),
                            ws + lib.laker_kmat_bytes(n, d, laker.F64) // 2, C.byref(st), None)
    assert r == laker.LAKER_ENOMEM


def test_empty_inputs_rejected_on_the_host():
    """Degenerate sizes have no device work to do and are invalid calls: a
    problem with no sites, a prediction with no query points, a batch with no
    maps, and a batch holding one empty map all return LAKER_EINVAL (and the
    size queries 0) before any launch."""
    laker, lib = _lib()
    st = laker.laker_stats()
    empty = laker.laker_problem(0, 4, 0, 8, 1e-2, 0.5)
    r = lib.laker_kernel_matvec(C.byref(empty), C.c_void_p(8), C.c_void_p(8), 0, C.c_void_p(8), 1 << 30, None)
    assert r == laker.LAKER_EINVAL
    opts = laker.laker_pcg_opts(1e-8, 10, 0, 0, 1, 1e-2, 0, 16)
    r = lib.laker_pcg_solve(C.byref(empty), None, C.c_void_p(8), C.c_void_p(8), C.byref(opts), C.c_void_p(8),
                            1 << 30, C.byref(st), None)
    assert r == laker.LAKER_EINVAL
    r = lib.laker_predict(C.byref(empty), C.c_void_p(8), 4, C.c_void_p(8), C.c_void_p(8), 0, C.c_void_p(8), 1 << 30,
                          None)
    assert r == laker.LAKER_EINVAL
    prob = laker.laker_problem(16, 4, 0, 8, 1e-2, 0.5)
    r = lib.laker_predict(C.byref(prob), C.c_void_p(8), 0, C.c_void_p(8), C.c_void_p(8), 0, C.c_void_p(8), 1 << 30,
                          None)                                         # m = 0 query points
    assert r == laker.LAKER_EINVAL
    assert lib.laker_solve_workspace_bytes(0, 4, 0) == 0
    assert lib.laker_kmat_bytes(0, 4, 0) == 0

    probs = (laker.laker_problem * 2)(prob, empty)
    ptrs = (C.c_void_p * 2)(8, 8)
    sts = (laker.laker_stats * 2)()
    bo = laker.laker_batch_opts(0, 0, 0, 0)
    for count in (0, 2):                                                # no maps; an empty map
        r = lib.laker_pcg_solve_batched(count, probs, None, ptrs, ptrs, C.byref(opts), C.byref(bo), C.c_void_p(8),
                                        1 << 30, sts, None)
        assert r == laker.LAKER_EINVAL, count
    ns = (C.c_int64 * 2)(16, 0)
    assert lib.laker_batch_workspace_bytes(2, ns, 4) == 0


def test_missing_library_fails_loudly_and_product_never_imports_the_oracle():
    """Without the built library the binding raises (there is no CPU fallback),
    and no module of the package imports the oracle."""
    import subprocess
    import sys
    code = ("from paper_2604_25138_amd import laker\n"
            "try:\n    laker.load('/nonexistent/liblaker.so')\nexcept ImportError as e:\n    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("raised"), (r.stdout, r.stderr[-2000:])
    pkg = os.path.join(ROOT, "paper_2604_25138_amd")
    for f in sorted(os.listdir(pkg)):
        if f.endswith(".py"):
            src = open(os.path.join(pkg, f)).read()
            assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f


def test_model_save_load_round_trip(tmp_path):
    """The network's weights, Adam moments and step count survive a save/load
    (host memory; the layout comes from the library's size query)."""
    import numpy as np
    laker, _ = _lib()
    from synth import make_mlp_init
    d = 8
    m = laker.MlpModel(d, "cpu")
    lay = laker.mlp_layout(d)
    m.set_params(make_mlp_init(lay.in_dim, laker.MLP_HIDDEN, laker.MLP_RANK + 1, 3))
    for blk in (1, 2):
        for k, t in m.tensor_views(blk).items():
            t.copy_(torch_rand_like(t, blk))
    m.step = 17
    f = tmp_path / "model.npz"
    m.save(str(f))
    m2 = laker.MlpModel.load(str(f), "cpu")
    assert m2.d == d and m2.step == 17
    assert np.array_equal(m.buf.numpy(), m2.buf.numpy())


def torch_rand_like(t, seed):
    import torch
    g = torch.Generator().manual_seed(seed)
    return torch.rand(t.shape, generator=g, dtype=t.dtype)
