"""Python binding of the LAKER C ABI (include/laker.h).

Argument marshalling only: every step of the method runs in the HIP library
``liblaker.so``.  torch provides device memory and the current stream.  The
library must be built (``python -m paper_2604_25138_amd.build_lib``); there is
no fallback path.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
from dataclasses import dataclass, field

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblaker.so")

LAKER_OK, LAKER_EINVAL, LAKER_ENOMEM, LAKER_EHIP, LAKER_EBREAKDOWN, LAKER_ENOCONV, LAKER_ESTALL = 0, -1, -2, -3, -4, -5, -6
F64, F32, BF16 = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI, PRECOND_CCCP, PRECOND_LEARNED = 0, 1, 2, 3
_PREC = {"f64": F64, "f32": F32, "bf16": BF16, F64: F64, F32: F32, BF16: BF16}

# every symbol declared in include/laker.h
EXPORTS = (
    "laker_precond_bytes", "laker_fit_workspace_bytes", "laker_solve_workspace_bytes",
    "laker_kernel_matvec", "laker_fit_precond", "laker_jacobi_precond", "laker_pcg_solve",
    "laker_predict", "laker_status_str", "laker_mlp_layout_query", "laker_learned_workspace_bytes",
    "laker_learned_forward", "laker_learned_train_step", "laker_learned_precond",
    "laker_sigma_half_workspace_bytes", "laker_precond_sigma_half", "laker_batch_workspace_bytes",
    "laker_pcg_solve_batched", "laker_kmat_bytes", "laker_precond_apply_workspace_bytes", "laker_precond_apply",
    "laker_learned_solve_workspace_bytes", "laker_learned_solve", "laker_kernel_matvec_noalloc",
    "laker_multi_workspace_bytes", "laker_kernel_matvec_multi", "laker_pcg_solve_multi",
    "laker_online_state_bytes", "laker_fit_precond_online",
)
MLP_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")
MLP_HIDDEN, MLP_RANK = 256, 64


class laker_problem(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("reserved", C.c_int32), ("E", C.c_void_p),
                ("lambda_", C.c_double), ("scale", C.c_double)]


class laker_cccp_opts(C.Structure):
    _fields_ = [("n_r", C.c_int32), ("max_iter", C.c_int32), ("gamma", C.c_double), ("rho", C.c_double),
                ("eps", C.c_double), ("tol", C.c_double), ("precision", C.c_int32), ("reserved", C.c_int32)]


class laker_precond(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_r", C.c_int32), ("n", C.c_int64), ("data", C.c_void_p),
                ("bytes", C.c_size_t)]


class laker_pcg_opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("precision", C.c_int32), ("refine", C.c_int32),
                ("ir_max", C.c_int32), ("inner_tol", C.c_double), ("warm_start", C.c_int32),
                ("check_every", C.c_int32), ("graph", C.c_int32), ("profile", C.c_int32),
                ("inner_max_iter", C.c_int32), ("materialized", C.c_int32), ("stall_window", C.c_int32),
                ("outer_history", C.c_int32), ("escalate", C.c_int32), ("lanczos", C.c_int32)]


class laker_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("ir_steps", C.c_int32), ("cccp_iters", C.c_int32), ("status", C.c_int32),
                ("relres", C.c_double), ("relres_true", C.c_double), ("ir_relres", C.c_double * 64),
                ("kmv_ms", C.c_double), ("kmv_count", C.c_int32), ("kmv_launches", C.c_int32),
                ("kmv_launch_ms", C.c_double), ("escalations", C.c_int32), ("fell_back", C.c_int32),
                ("learned_iters", C.c_int32), ("lanczos_steps", C.c_int32), ("reserved", C.c_int32),
                ("eig_min", C.c_double), ("eig_max", C.c_double), ("cond_est", C.c_double)]


class laker_mlp_layout(C.Structure):
    _fields_ = [("d", C.c_int32), ("in_dim", C.c_int32), ("count", C.c_int64), ("off", C.c_int64 * 6),
                ("block_bytes", C.c_size_t), ("bytes", C.c_size_t)]


class laker_train_opts(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double), ("eps", C.c_double),
                ("step", C.c_int32), ("update", C.c_int32)]


class laker_batch_opts(C.Structure):
    _fields_ = [("cols_per_split", C.c_int32), ("xcd_order", C.c_int32), ("cols_used", C.c_int32),
                ("reserved", C.c_int32)]


class LakerError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} ({status})")


_lib = None


def load(path: str = LIB_PATH):
    """Load liblaker.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2604_25138_amd.build_lib`")
    lib = C.CDLL(path)
    vp, sz, i32, i64 = C.c_void_p, C.c_size_t, C.c_int32, C.c_int64
    P = C.POINTER
    lib.laker_precond_bytes.argtypes = [i64, i32]
    lib.laker_precond_bytes.restype = sz
    lib.laker_fit_workspace_bytes.argtypes = [i64, i32, i32]
    lib.laker_fit_workspace_bytes.restype = sz
    lib.laker_solve_workspace_bytes.argtypes = [i64, i32, i64]
    lib.laker_solve_workspace_bytes.restype = sz
    lib.laker_kmat_bytes.argtypes = [i64, i32, i32]
    lib.laker_kmat_bytes.restype = sz
    lib.laker_kernel_matvec.argtypes = [P(laker_problem), vp, vp, i32, vp, sz, vp]
    lib.laker_kernel_matvec.restype = i32
    lib.laker_fit_precond.argtypes = [P(laker_problem), vp, P(laker_cccp_opts), P(laker_precond), vp, sz,
                                      P(laker_stats), vp]
    lib.laker_fit_precond.restype = i32
    lib.laker_precond_apply_workspace_bytes.argtypes = [i64, i32]
    lib.laker_precond_apply_workspace_bytes.restype = sz
    lib.laker_precond_apply.argtypes = [P(laker_precond), vp, vp, i32, vp, sz, vp]
    lib.laker_precond_apply.restype = i32
    lib.laker_online_state_bytes.argtypes = [i64, i32]
    lib.laker_online_state_bytes.restype = sz
    lib.laker_fit_precond_online.argtypes = [P(laker_problem), i64, vp, P(laker_cccp_opts), vp, sz, P(laker_precond),
                                             vp, sz, P(laker_stats), vp]
    lib.laker_fit_precond_online.restype = i32
    lib.laker_jacobi_precond.argtypes = [P(laker_problem), P(laker_precond), vp]
    lib.laker_jacobi_precond.restype = i32
    lib.laker_pcg_solve.argtypes = [P(laker_problem), P(laker_precond), vp, vp, P(laker_pcg_opts), vp, sz,
                                    P(laker_stats), vp]
    lib.laker_pcg_solve.restype = i32
    lib.laker_predict.argtypes = [P(laker_problem), vp, i64, vp, vp, i32, vp, sz, vp]
    lib.laker_predict.restype = i32
    lib.laker_status_str.argtypes = [i32]
    lib.laker_status_str.restype = C.c_char_p
    lib.laker_mlp_layout_query.argtypes = [i32, P(laker_mlp_layout)]
    lib.laker_mlp_layout_query.restype = i32
    lib.laker_learned_workspace_bytes.argtypes = [i64, i32, i32]
    lib.laker_learned_workspace_bytes.restype = sz
    lib.laker_learned_forward.argtypes = [P(laker_problem), vp, vp, vp, sz, vp]
    lib.laker_learned_forward.restype = i32
    lib.laker_learned_train_step.argtypes = [P(laker_problem), vp, i32, vp, vp, P(laker_train_opts), vp,
                                             P(C.c_double), vp, sz, vp]
    lib.laker_learned_train_step.restype = i32
    lib.laker_learned_precond.argtypes = [P(laker_problem), vp, P(laker_precond), vp, sz, vp]
    lib.laker_learned_precond.restype = i32
    lib.laker_learned_solve_workspace_bytes.argtypes = [i64, i32, i32, i32, i32]
    lib.laker_learned_solve_workspace_bytes.restype = sz
    lib.laker_learned_solve.argtypes = [P(laker_problem), vp, vp, P(laker_cccp_opts), vp, vp, P(laker_pcg_opts),
                                        P(laker_precond), vp, sz, P(laker_stats), vp]
    lib.laker_learned_solve.restype = i32
    lib.laker_multi_workspace_bytes.argtypes = [i64, i32, i32]
    lib.laker_multi_workspace_bytes.restype = sz
    lib.laker_kernel_matvec_multi.argtypes = [P(laker_problem), i32, vp, vp, i32, vp, sz, vp]
    lib.laker_kernel_matvec_multi.restype = i32
    lib.laker_pcg_solve_multi.argtypes = [P(laker_problem), P(laker_precond), i32, vp, vp, P(laker_pcg_opts), vp, sz,
                                          P(laker_stats), vp]
    lib.laker_pcg_solve_multi.restype = i32
    lib.laker_sigma_half_workspace_bytes.argtypes = [i64, i32, i32]
    lib.laker_sigma_half_workspace_bytes.restype = sz
    lib.laker_precond_sigma_half.argtypes = [P(laker_precond), i32, vp, vp, vp, sz, vp]
    lib.laker_precond_sigma_half.restype = i32
    lib.laker_batch_workspace_bytes.argtypes = [i32, P(i64), i32]
    lib.laker_batch_workspace_bytes.restype = sz
    lib.laker_pcg_solve_batched.argtypes = [i32, P(laker_problem), P(laker_precond), P(vp), P(vp),
                                            P(laker_pcg_opts), P(laker_batch_opts), vp, sz, P(laker_stats), vp]
    lib.laker_pcg_solve_batched.restype = i32
    _lib = lib
    return lib


def status_str(s: int) -> str:
    return load().laker_status_str(int(s)).decode()


def _check(s: int, where: str, allow=(LAKER_OK,)):
    if s not in allow:
        raise LakerError(s, where)
    return s


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor | None):
    return C.c_void_p(0 if t is None else t.data_ptr())


def _dev_f64(x, device) -> torch.Tensor:
    t = torch.as_tensor(x, dtype=torch.float64)
    return t.to(device).contiguous()


_ws: dict = {}


def release() -> None:
    """Drop the cached device workspaces (registered to run at interpreter exit,
    so that they are freed while torch's allocator is still alive)."""
    if _ws:
        try:
            torch.cuda.synchronize()
        except Exception:
            pass
        _ws.clear()


atexit.register(release)


def _workspace(name: str, nbytes: int, device) -> torch.Tensor:
    """Grow-only cached workspace per (device, name)."""
    key = (str(device), name)
    t = _ws.get(key)
    if t is None or t.numel() < nbytes:
        t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws[key] = t
    return t


@dataclass
class Problem:
    """(lambda I + G) alpha = y with G_ij = exp(scale <e_i, e_j>); E on the device."""
    E: torch.Tensor
    lam: float
    scale: float
    c: laker_problem = field(init=False)

    def __post_init__(self):
        on_gpu = isinstance(self.E, torch.Tensor) and self.E.is_cuda
        self.E = _dev_f64(self.E, self.E.device if on_gpu else torch.device("cuda"))
        n, d = self.E.shape
        self.c = laker_problem(n, d, 0, self.E.data_ptr(), float(self.lam), float(self.scale))

    @property
    def n(self):
        return self.E.shape[0]

    @property
    def d(self):
        return self.E.shape[1]

    @property
    def device(self):
        return self.E.device


@dataclass
class Precond:
    kind: int
    n: int
    n_r: int
    data: torch.Tensor | None
    c: laker_precond
    stats: laker_stats | None = None

    @property
    def header(self) -> torch.Tensor:
        """Scalars written by the fit: [b^{-1/2}, a, b, cccp_iters, change, db_iters, db_change]."""
        return self.data[:256].view(torch.float64)[:7].cpu()


def none_precond(n: int) -> Precond:
    return Precond(PRECOND_NONE, n, 0, None, laker_precond(PRECOND_NONE, 0, n, None, 0))


def kernel_matvec(prob: Problem, p: torch.Tensor, precision="f64") -> torch.Tensor:
    lib = load()
    p = _dev_f64(p, prob.device)
    w = torch.empty_like(p)
    nb = lib.laker_solve_workspace_bytes(prob.n, prob.d, 0)
    ws = _workspace("solve", nb, prob.device)
    s = lib.laker_kernel_matvec(C.byref(prob.c), _ptr(p), _ptr(w), _PREC[precision], _ptr(ws), ws.numel(), _stream())
    _check(s, "laker_kernel_matvec")
    return w


def fit_precond(prob: Problem, Z: torch.Tensor, n_r: int | None = None, gamma: float = 0.1, rho: float = 0.0,
                eps: float = 1e-10, tol: float = 1e-8, max_iter: int = 300, precision="f64") -> Precond:
    lib = load()
    Z = _dev_f64(Z, prob.device)
    nr = Z.shape[1] if n_r is None else n_r
    pbytes = lib.laker_precond_bytes(prob.n, nr)
    data = torch.empty(pbytes, dtype=torch.uint8, device=prob.device)
    pc = laker_precond(PRECOND_CCCP, nr, prob.n, data.data_ptr(), pbytes)
    opts = laker_cccp_opts(nr, max_iter, gamma, rho, eps, tol, _PREC[precision], 0)
    nb = lib.laker_fit_workspace_bytes(prob.n, prob.d, nr)
    ws = _workspace("fit", nb, prob.device)
    st = laker_stats()
    s = lib.laker_fit_precond(C.byref(prob.c), _ptr(Z), C.byref(opts), C.byref(pc), _ptr(ws), ws.numel(),
                              C.byref(st), _stream())
    _check(s, "laker_fit_precond")
    return Precond(pc.kind, prob.n, nr, data, pc, st)


class OnlineFitState:
    """Device state of a fit that later fits extend with appended sites
    (laker_fit_precond_online): directions of the sites so far and the CCCP
    weights, for up to n_cap sites and n_r directions."""

    def __init__(self, n_cap: int, n_r: int, device="cuda"):
        lib = load()
        self.n_cap, self.n_r = int(n_cap), int(n_r)
        self.buf = torch.zeros(lib.laker_online_state_bytes(self.n_cap, self.n_r), dtype=torch.uint8, device=device)
        self.n = 0     # sites fitted so far

    def fit(self, prob: Problem, Z, gamma: float = 0.1, rho: float = 0.0, eps: float = 1e-10, tol: float = 1e-8,
            max_iter: int = 300) -> Precond:
        """Fit the preconditioner of prob (its first self.n sites are those of
        the previous fit, in the same order; Z has the previous rows first)."""
        lib = load()
        Z = _dev_f64(Z, prob.device)
        nr = self.n_r
        pbytes = lib.laker_precond_bytes(prob.n, nr)
        data = torch.empty(pbytes, dtype=torch.uint8, device=prob.device)
        pc = laker_precond(PRECOND_CCCP, nr, prob.n, data.data_ptr(), pbytes)
        opts = laker_cccp_opts(nr, max_iter, gamma, rho, eps, tol, F64, 0)
        nb = lib.laker_fit_workspace_bytes(prob.n, prob.d, nr)
        ws = _workspace("fit", nb, prob.device)
        st = laker_stats()
        s = lib.laker_fit_precond_online(C.byref(prob.c), self.n, _ptr(Z), C.byref(opts), _ptr(self.buf),
                                         self.buf.numel(), C.byref(pc), _ptr(ws), ws.numel(), C.byref(st), _stream())
        _check(s, "laker_fit_precond_online")
        self.n = prob.n
        return Precond(pc.kind, prob.n, nr, data, pc, st)

    def directions(self) -> torch.Tensor:
        """The stored unscaled directions U = (lambda I + G) Z (n x n_r view)."""
        off = load().laker_online_state_bytes(1, self.n_r) - 8 * self.n_r
        return self.buf[off:off + 8 * self.n * self.n_r].view(torch.float64).view(self.n, self.n_r)


def jacobi_precond(prob: Problem) -> Precond:
    lib = load()
    pbytes = lib.laker_precond_bytes(prob.n, 0)
    data = torch.empty(pbytes, dtype=torch.uint8, device=prob.device)
    pc = laker_precond(PRECOND_JACOBI, 0, prob.n, data.data_ptr(), pbytes)
    _check(lib.laker_jacobi_precond(C.byref(prob.c), C.byref(pc), _stream()), "laker_jacobi_precond")
    return Precond(pc.kind, prob.n, 0, data, pc)


def precond_apply(pc: Precond, r, precision="f64") -> torch.Tensor:
    """theta = P r with the solver's preconditioner kernels."""
    lib = load()
    dev = pc.data.device if pc.data is not None else torch.device("cuda")
    r = _dev_f64(r, dev)
    theta = torch.empty_like(r)
    nb = lib.laker_precond_apply_workspace_bytes(pc.n, pc.n_r)
    ws = _workspace("apply", nb, dev)
    s = lib.laker_precond_apply(C.byref(pc.c), _ptr(r), _ptr(theta), _PREC[precision], _ptr(ws), ws.numel(),
                                _stream())
    _check(s, "laker_precond_apply")
    return theta


def pcg_solve(prob: Problem, y, precond: Precond | None = None, tol: float = 1e-10, max_iter: int = 10000,
              precision="f64", refine: bool = False, inner_tol: float = 1e-2, ir_max: int = 64,
              alpha0: torch.Tensor | None = None, check_every: int = 16, allow_noconv: bool = False,
              graph: bool = False, profile: bool = False, inner_max_iter: int = 0, materialized: bool = False,
              stall_window: int = 0, lanczos: bool = False, outer_history: int = 0, escalate: bool = False):
    """Returns (alpha, stats).  materialized: store G once per call and stream it
    in the float64 (and float32) products; stall_window: LAKER_ESTALL when the
    residual falls by less than 2x over that many iterations; lanczos: estimate
    kappa(P A) from the PCG coefficients (stats.eig_min, eig_max, cond_est);
    outer_history: directions the flexible outer CG (refine=2) keeps; escalate:
    finer inner products when its outer residual stalls."""
    lib = load()
    y = _dev_f64(y, prob.device)
    if alpha0 is not None:
        alpha = _dev_f64(alpha0, prob.device).clone()
    else:
        alpha = torch.empty_like(y)
    opts = laker_pcg_opts(tol, max_iter, _PREC[precision], int(refine), ir_max, inner_tol,
                          1 if alpha0 is not None else 0, check_every, 1 if graph else 0, 1 if profile else 0,
                          inner_max_iter, 1 if materialized else 0, int(stall_window), int(outer_history),
                          1 if escalate else 0, 1 if lanczos else 0)
    nb = lib.laker_solve_workspace_bytes(prob.n, prob.d, 0)
    if materialized:
        nb += 256 + lib.laker_kmat_bytes(prob.n, prob.d, F64)
        if _PREC[precision] == F32:
            nb += 256 + lib.laker_kmat_bytes(prob.n, prob.d, F32)
    ws = _workspace("solve", nb, prob.device)
    st = laker_stats()
    pc = None if precond is None else C.byref(precond.c)
    s = lib.laker_pcg_solve(C.byref(prob.c), pc, _ptr(y), _ptr(alpha), C.byref(opts), _ptr(ws), ws.numel(),
                            C.byref(st), _stream())
    _check(s, "laker_pcg_solve", (LAKER_OK, LAKER_ENOCONV, LAKER_ESTALL) if allow_noconv else (LAKER_OK,))
    return alpha, st


def predict(prob: Problem, alpha: torch.Tensor, Eq, precision="f64") -> torch.Tensor:
    lib = load()
    Eq = _dev_f64(Eq, prob.device)
    alpha = _dev_f64(alpha, prob.device)
    m = Eq.shape[0]
    rhat = torch.empty(m, dtype=torch.float64, device=prob.device)
    nb = lib.laker_solve_workspace_bytes(prob.n, prob.d, m)
    ws = _workspace("predict", nb, prob.device)
    s = lib.laker_predict(C.byref(prob.c), _ptr(alpha), m, _ptr(Eq), _ptr(rhat), _PREC[precision], _ptr(ws),
                          ws.numel(), _stream())
    _check(s, "laker_predict")
    return rhat


def precond_parts(pc: Precond) -> dict:
    """Device views of a fitted preconditioner buffer (layout of the library:
    256-byte aligned header of 32 doubles, then B, Bt in float64, B, Bt in
    float32, then the Jacobi diagonal)."""
    def al(x):
        return (x + 255) & ~255
    n, nr = pc.n, pc.n_r
    nrp = (nr + 3) & ~3          # row stride: N_r rounded up to a multiple of 4
    off = 0
    out = {}
    for name, count, dt, es in (("hdr", 32, torch.float64, 8), ("B64", n * nrp, torch.float64, 8),
                                ("Bt64", n * nrp, torch.float64, 8), ("B32", n * nrp, torch.float32, 4),
                                ("Bt32", n * nrp, torch.float32, 4), ("dinv64", n, torch.float64, 8)):
        off = al(off)
        out[name] = pc.data[off:off + count * es].view(dt)
        off += count * es
    for name in ("B64", "Bt64", "B32", "Bt32"):
        out[name] = out[name].view(n, nrp)[:, :nr]
    return out


# ---------------------------------------------------------------------------
# learned rank-64-plus-diagonal preconditioner
# ---------------------------------------------------------------------------

def mlp_layout(d: int) -> laker_mlp_layout:
    L = laker_mlp_layout()
    _check(load().laker_mlp_layout_query(int(d), C.byref(L)), "laker_mlp_layout_query")
    return L


class MlpModel:
    """Device buffer of the network: weights, Adam moments (library layout)."""

    def __init__(self, d: int, device="cuda"):
        self.d = int(d)
        self.layout = mlp_layout(d)
        self.buf = torch.zeros(self.layout.bytes, dtype=torch.uint8, device=device)
        self.step = 0

    @property
    def device(self):
        return self.buf.device

    def _block(self, k: int) -> torch.Tensor:
        L = self.layout
        return self.buf[k * L.block_bytes:k * L.block_bytes + 4 * L.count].view(torch.float32)

    def _shapes(self):
        i, h, r = self.layout.in_dim, MLP_HIDDEN, MLP_RANK + 1
        return {"W1": (i, h), "b1": (h,), "W2": (h, h), "b2": (h,), "W3": (h, r), "b3": (r,)}

    def tensor_views(self, block: int = 0) -> dict:
        th = self._block(block)
        out = {}
        for t, (k, shp) in enumerate(self._shapes().items()):
            o = self.layout.off[t]
            cnt = 1
            for x in shp:
                cnt *= x
            out[k] = th[o:o + cnt].view(*shp)
        return out

    def set_params(self, params: dict) -> None:
        """Write weights (numpy or torch, fan_in x fan_out) and zero the Adam moments."""
        self.buf.zero_()
        views = self.tensor_views(0)
        for k in MLP_KEYS:
            views[k].copy_(torch.as_tensor(params[k], dtype=torch.float32))
        self.step = 0

    def params(self) -> dict:
        return {k: v.detach().cpu().double().numpy() for k, v in self.tensor_views(0).items()}

    def save(self, path: str) -> None:
        """Write the float32 weights, the Adam moments and the step count to an
        .npz file (plain arrays, no pickled objects)."""
        import numpy as np
        arrays = {"d": np.array([self.d]), "step": np.array([self.step])}
        for blk, tag in ((0, "w"), (1, "m"), (2, "v")):
            for k, t in self.tensor_views(blk).items():
                arrays[f"{tag}_{k}"] = t.detach().cpu().numpy()
        np.savez(path, **arrays)

    @classmethod
    def load(cls, path: str, device="cuda") -> "MlpModel":
        """Read a model written by save (the layout is rebuilt for its d)."""
        import numpy as np
        with np.load(path, allow_pickle=False) as z:
            model = cls(int(z["d"][0]), device)
            for blk, tag in ((0, "w"), (1, "m"), (2, "v")):
                views = model.tensor_views(blk)
                for k in MLP_KEYS:
                    views[k].copy_(torch.as_tensor(z[f"{tag}_{k}"], dtype=torch.float32))
            model.step = int(z["step"][0])
        return model

    def grad_views(self, flat: torch.Tensor) -> dict:
        out = {}
        for t, (k, shp) in enumerate(self._shapes().items()):
            o = self.layout.off[t]
            cnt = 1
            for x in shp:
                cnt *= x
            out[k] = flat[o:o + cnt].view(*shp)
        return out


def learned_forward(prob: Problem, model: MlpModel) -> torch.Tensor:
    lib = load()
    out = torch.empty(prob.n, MLP_RANK + 1, dtype=torch.float32, device=prob.device)
    nb = lib.laker_learned_workspace_bytes(prob.n, prob.d, 0)
    ws = _workspace("learned", nb, prob.device)
    s = lib.laker_learned_forward(C.byref(prob.c), _ptr(model.buf), _ptr(out), _ptr(ws), ws.numel(), _stream())
    _check(s, "laker_learned_forward")
    return out


def learned_train_step(prob: Problem, model: MlpModel, Z: torch.Tensor, U: torch.Tensor, lr: float = 1e-3,
                       update: bool = True, want_grad: bool = False, want_loss: bool = True,
                       beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step on one problem; returns (loss or None, gradient dict or None)."""
    lib = load()
    m = Z.shape[1]
    if update:
        model.step += 1
    opts = laker_train_opts(lr, beta1, beta2, eps, max(model.step, 1), 1 if update else 0)
    g = torch.empty(model.layout.count, dtype=torch.float32, device=prob.device) if want_grad else None
    loss = C.c_double(0.0)
    nb = lib.laker_learned_workspace_bytes(prob.n, prob.d, m)
    ws = _workspace("learned", nb, prob.device)
    s = lib.laker_learned_train_step(C.byref(prob.c), _ptr(model.buf), m, _ptr(Z), _ptr(U), C.byref(opts), _ptr(g),
                                     C.byref(loss) if want_loss else None, _ptr(ws), ws.numel(), _stream())
    _check(s, "laker_learned_train_step")
    return (loss.value if want_loss else None), (model.grad_views(g) if want_grad else None)


def learned_precond(prob: Problem, model: MlpModel) -> Precond:
    lib = load()
    pbytes = lib.laker_precond_bytes(prob.n, MLP_RANK)
    data = torch.empty(pbytes, dtype=torch.uint8, device=prob.device)
    pc = laker_precond(PRECOND_LEARNED, MLP_RANK, prob.n, data.data_ptr(), pbytes)
    nb = lib.laker_learned_workspace_bytes(prob.n, prob.d, 0)
    ws = _workspace("learned", nb, prob.device)
    s = lib.laker_learned_precond(C.byref(prob.c), _ptr(model.buf), C.byref(pc), _ptr(ws), ws.numel(), _stream())
    _check(s, "laker_learned_precond")
    return Precond(pc.kind, prob.n, MLP_RANK, data, pc)


def learned_solve(prob: Problem, y, model: MlpModel, Z, tol: float = 1e-6, max_iter: int = 200000,
                  precision="bf16", refine: int = 2, inner_tol: float = 0.1, ir_max: int = 20000,
                  check_every: int = 30, inner_max_iter: int = 30, materialized: bool = False,
                  stall_window: int = 0, gamma: float = 0.1, rho: float = 0.0, cccp_tol: float = 1e-8,
                  cccp_max_iter: int = 300, allow_noconv: bool = False, outer_history: int = 0):
    """Solve with the learned preconditioner, falling back to a CCCP fit with
    directions Z when that solve stalls or breaks down (laker_learned_solve).
    Returns (alpha, stats, precond used last)."""
    lib = load()
    y = _dev_f64(y, prob.device)
    Z = _dev_f64(Z, prob.device)
    nr = Z.shape[1]
    alpha = torch.empty_like(y)
    pbytes = lib.laker_precond_bytes(prob.n, max(MLP_RANK, nr))
    data = torch.empty(pbytes, dtype=torch.uint8, device=prob.device)
    pc = laker_precond(PRECOND_LEARNED, MLP_RANK, prob.n, data.data_ptr(), pbytes)
    copts = laker_cccp_opts(nr, cccp_max_iter, gamma, rho, 1e-10, cccp_tol, _PREC[precision], 0)
    opts = laker_pcg_opts(tol, max_iter, _PREC[precision], int(refine), ir_max, inner_tol, 0, check_every, 0, 0,
                          inner_max_iter, 1 if materialized else 0, int(stall_window), int(outer_history), 0, 0)
    nb = lib.laker_learned_solve_workspace_bytes(prob.n, prob.d, nr, _PREC[precision], 1 if materialized else 0)
    ws = _workspace("solve", nb, prob.device)
    st = laker_stats()
    s = lib.laker_learned_solve(C.byref(prob.c), _ptr(model.buf), _ptr(Z), C.byref(copts), _ptr(y), _ptr(alpha),
                                C.byref(opts), C.byref(pc), _ptr(ws), ws.numel(), C.byref(st), _stream())
    _check(s, "laker_learned_solve", (LAKER_OK, LAKER_ENOCONV, LAKER_ESTALL) if allow_noconv else (LAKER_OK,))
    return alpha, st, Precond(pc.kind, prob.n, pc.n_r, data, pc)


def sigma_half(pc: Precond, Z: torch.Tensor) -> torch.Tensor:
    """U = Sigma_star^{1/2} Z for a fitted CCCP preconditioner."""
    lib = load()
    Z = _dev_f64(Z, pc.data.device)
    m = Z.shape[1]
    U = torch.empty_like(Z)
    nb = lib.laker_sigma_half_workspace_bytes(pc.n, pc.n_r, m)
    ws = _workspace("sigma_half", nb, pc.data.device)
    s = lib.laker_precond_sigma_half(C.byref(pc.c), m, _ptr(Z), _ptr(U), _ptr(ws), ws.numel(), _stream())
    _check(s, "laker_precond_sigma_half")
    return U


# ---------------------------------------------------------------------------
# several right-hand sides on one map
# ---------------------------------------------------------------------------

def _columns(Y, device) -> torch.Tensor:
    """(n, k) input as k contiguous columns (the library's column-major layout)."""
    Y = torch.as_tensor(Y, dtype=torch.float64)
    if Y.dim() == 1:
        Y = Y[:, None]
    return Y.t().contiguous().to(device)


def kernel_matvec_multi(prob: Problem, P, precision="f64") -> torch.Tensor:
    """W = (lambda I + G) P for an (n, k) block P (k <= 8); returns (n, k)."""
    lib = load()
    Pc = _columns(P, prob.device)
    k = Pc.shape[0]
    W = torch.empty_like(Pc)
    nb = lib.laker_multi_workspace_bytes(prob.n, prob.d, k)
    ws = _workspace("multi", nb, prob.device)
    s = lib.laker_kernel_matvec_multi(C.byref(prob.c), k, _ptr(Pc), _ptr(W), _PREC[precision], _ptr(ws), ws.numel(),
                                      _stream())
    _check(s, "laker_kernel_matvec_multi")
    return W.t()


def pcg_solve_multi(prob: Problem, Y, precond: Precond | None = None, tol: float = 1e-10, max_iter: int = 10000,
                    precision="f64", check_every: int = 16, allow_noconv: bool = False):
    """Solve for the k <= 8 columns of Y (n, k) together; returns (alpha (n, k), stats list)."""
    lib = load()
    Yc = _columns(Y, prob.device)
    k = Yc.shape[0]
    A = torch.empty_like(Yc)
    opts = laker_pcg_opts(tol, max_iter, _PREC[precision], 0, 1, 1e-2, 0, check_every, 0, 0, 0, 0, 0, 0, 0, 0)
    nb = lib.laker_multi_workspace_bytes(prob.n, prob.d, k)
    ws = _workspace("multi", nb, prob.device)
    st = (laker_stats * k)()
    pc = None if precond is None else C.byref(precond.c)
    s = lib.laker_pcg_solve_multi(C.byref(prob.c), pc, k, _ptr(Yc), _ptr(A), C.byref(opts), _ptr(ws), ws.numel(), st,
                                  _stream())
    _check(s, "laker_pcg_solve_multi", (LAKER_OK, LAKER_ENOCONV) if allow_noconv else (LAKER_OK,))
    return A.t(), list(st)


# ---------------------------------------------------------------------------
# batched solve
# ---------------------------------------------------------------------------

def pcg_solve_batched(probs: list, ys: list, preconds: list | None = None, tol: float = 1e-10,
                      max_iter: int = 10000, precision="f64", refine: bool = False, inner_tol: float = 1e-2,
                      ir_max: int = 64, check_every: int = 16, graph: bool = False, cols_per_split: int = 0,
                      xcd_order: bool = False, allow_noconv: bool = False, materialized: bool = False):
    """Solve every problem of the batch; returns (alphas, stats list, columns per range used).
    materialized: the float64 outer residuals of the maps large enough stream a G
    stored once per call."""
    lib = load()
    count = len(probs)
    dev = probs[0].device
    ys = [_dev_f64(v, dev) for v in ys]
    alphas = [torch.empty_like(v) for v in ys]
    pa = (laker_problem * count)(*[p.c for p in probs])
    pc = None
    if preconds is not None:
        pc = (laker_precond * count)(*[q.c for q in preconds])
    yp = (C.c_void_p * count)(*[v.data_ptr() for v in ys])
    ap = (C.c_void_p * count)(*[v.data_ptr() for v in alphas])
    opts = laker_pcg_opts(tol, max_iter, _PREC[precision], 1 if refine else 0, ir_max, inner_tol, 0, check_every,
                          1 if graph else 0, 0, 0, 1 if materialized else 0)
    bo = laker_batch_opts(cols_per_split, 1 if xcd_order else 0, 0, 0)
    ns = (C.c_int64 * count)(*[p.n for p in probs])
    nb = lib.laker_batch_workspace_bytes(count, ns, probs[0].d)
    if materialized:
        nb += sum(256 + lib.laker_kmat_bytes(p.n, p.d, F64) for p in probs)
    ws = _workspace("batch", nb, dev)
    st = (laker_stats * count)()
    s = lib.laker_pcg_solve_batched(count, pa, pc, yp, ap, C.byref(opts), C.byref(bo), _ptr(ws), ws.numel(), st,
                                    _stream())
    _check(s, "laker_pcg_solve_batched", (LAKER_OK, LAKER_ENOCONV) if allow_noconv else (LAKER_OK,))
    return alphas, list(st), bo.cols_used
