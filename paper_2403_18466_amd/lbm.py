"""Thin ctypes binding of the C ABI in include/lbm.h.

Every function has the C name and only marshals arguments: torch tensors are
checked (device, dtype, contiguity, size) and passed as device pointers, the
stream defaults to torch's current stream.  All arithmetic runs in the HIP
library ``liblbm_hip.so``; there is no fallback: if the library is missing
or cannot be loaded every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm_hip.so")

LBM_OK, LBM_ERR_INVALID, LBM_ERR_UNSUPPORTED, LBM_ERR_HIP, LBM_ERR_WORKSPACE = range(5)
LBM_D2Q9, LBM_D3Q19 = 0, 1
LBM_MLP_FP32, LBM_MLP_BF16, LBM_MLP_FP16 = 1, 2, 3
LBM_FORCE_NONE, LBM_FORCE_KOLMOGOROV, LBM_FORCE_SINE3 = 0, 1, 2
LBM_NET_TANH, LBM_NET_LEAKY_300_300_100 = 0, 1
LBM_COLLISION_BGK, LBM_COLLISION_SMAGORINSKY = 0, 1

LATTICES = {"D2Q9": LBM_D2Q9, "D3Q19": LBM_D3Q19}
PRECISIONS = {"fp32": LBM_MLP_FP32, "bf16": LBM_MLP_BF16, "fp16": LBM_MLP_FP16}
NETS = {"tanh": LBM_NET_TANH, "paper": LBM_NET_LEAKY_300_300_100}
COLLISIONS = {"bgk": LBM_COLLISION_BGK, "smagorinsky": LBM_COLLISION_SMAGORINSKY}

# Every symbol include/lbm.h declares.
EXPORTS = (
    "lbm_create", "lbm_destroy", "lbm_state_elems", "lbm_param_elems", "lbm_workspace_bytes",
    "lbm_lattice_tables", "lbm_init", "lbm_step", "lbm_step_f64", "lbm_moments", "lbm_shift",
    "lbm_step_backward", "lbm_step_backward_static", "lbm_step_backward_seq", "lbm_loss_velocity_mse", "lbm_adam", "lbm_box_filter",
    "lbm_subsample", "lbm_loss_population_sse", "lbm_structure_functions_workspace_bytes",
    "lbm_structure_functions", "lbm_mrt_moment_sums", "lbm_status_str", "lbm_last_error",
)


class lbm_config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("force_kind", ctypes.c_int32), ("force_k", ctypes.c_int32),
        ("force_amp", ctypes.c_double),
        ("hidden", ctypes.c_int32), ("mlp_prec", ctypes.c_int32),
        ("out_scale", ctypes.c_double), ("net", ctypes.c_int32),
        ("collision", ctypes.c_int32), ("smag_cs", ctypes.c_double),
    ]


class LBMError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load liblbm_hip.so (built by ``python -m paper_2403_18466_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is not built; run "
                           "`python -m paper_2403_18466_amd.build` first")
    lib = ctypes.CDLL(path)
    vp, sz, i32, i64, dbl = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "lbm_create": ([ctypes.POINTER(lbm_config), ctypes.POINTER(vp)], ctypes.c_int),
        "lbm_destroy": ([vp], ctypes.c_int),
        "lbm_state_elems": ([vp], sz),
        "lbm_param_elems": ([vp], sz),
        "lbm_workspace_bytes": ([vp], sz),
        "lbm_lattice_tables": ([i32, ctypes.POINTER(i32), vp, vp], ctypes.c_int),
        "lbm_init": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "lbm_step": ([vp, vp, vp, vp, i32, vp], ctypes.c_int),
        "lbm_step_f64": ([vp, vp, vp, vp, i32, vp], ctypes.c_int),
        "lbm_moments": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "lbm_shift": ([vp, vp, vp, i32, vp], ctypes.c_int),
        "lbm_step_backward": ([vp, vp, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "lbm_step_backward_static": ([vp, vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "lbm_step_backward_seq": ([vp, vp, i32, vp, vp, vp, vp, vp, sz, vp], ctypes.c_int),
        "lbm_loss_velocity_mse": ([vp, vp, vp, vp, vp, vp], ctypes.c_int),
        "lbm_adam": ([vp, vp, vp, vp, i64, dbl, dbl, dbl, dbl, dbl, i32, vp], ctypes.c_int),
        "lbm_box_filter": ([vp, vp, i32, i32, i32, i32, i32, i32, vp], ctypes.c_int),
        "lbm_subsample": ([i32, vp, vp, i32, i32, i32, i32, i32, vp], ctypes.c_int),
        "lbm_loss_population_sse": ([vp, vp, vp, vp, i32, vp, vp, vp], ctypes.c_int),
        "lbm_structure_functions_workspace_bytes": ([vp, i32, i32], sz),
        "lbm_structure_functions": ([vp, vp, i32, i32, vp, vp, vp, sz, vp], ctypes.c_int),
        "lbm_mrt_moment_sums": ([vp, vp, vp, vp, vp], ctypes.c_int),
        "lbm_status_str": ([ctypes.c_int], ctypes.c_char_p),
        "lbm_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != LBM_OK:
        lib = load_library()
        raise LBMError(status, where, lib.lbm_last_error().decode())


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t, dtype, numel=None, name="array", allow_none=False):
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class Config:
    """Python mirror of lbm_config."""
    lattice: str = "D2Q9"
    nx: int = 64
    ny: int = 64
    nz: int = 1
    batch: int = 1
    tau: float = 0.6
    rho0: float = 1.0
    force_kind: int = LBM_FORCE_NONE
    force_k: int = 0
    force_amp: float = 0.0
    hidden: int = 0
    mlp_prec: str = "fp32"
    out_scale: float = 1.0
    net: str = "tanh"   # "tanh": Q-H-H-Q; "paper": Q-300-300-100-Q LeakyReLU (hidden=300)
    collision: str = "bgk"  # "bgk" or "smagorinsky" (hidden must be 0)
    smag_cs: float = 0.0

    @property
    def Q(self):
        return 9 if self.lattice == "D2Q9" else 19

    @property
    def D(self):
        return 2 if self.lattice == "D2Q9" else 3

    @property
    def state_shape(self):
        return (self.batch, self.Q, self.nz, self.ny, self.nx)

    def c_struct(self) -> lbm_config:
        return lbm_config(LATTICES[self.lattice], self.nx, self.ny, self.nz, self.batch,
                          float(self.tau), float(self.rho0), int(self.force_kind),
                          int(self.force_k), float(self.force_amp), int(self.hidden),
                          PRECISIONS[self.mlp_prec], float(self.out_scale), NETS[self.net],
                          COLLISIONS[self.collision], float(self.smag_cs))


# ----------------------------------------------------------------- C names
def lbm_create(cfg: Config) -> ctypes.c_void_p:
    lib = load_library()
    ctx = ctypes.c_void_p()
    c = cfg.c_struct()
    _check(lib.lbm_create(ctypes.byref(c), ctypes.byref(ctx)), "lbm_create")
    return ctx


def lbm_destroy(ctx):
    _check(load_library().lbm_destroy(ctx), "lbm_destroy")


def lbm_state_elems(ctx) -> int:
    return int(load_library().lbm_state_elems(ctx))


def lbm_param_elems(ctx) -> int:
    return int(load_library().lbm_param_elems(ctx))


def lbm_workspace_bytes(ctx) -> int:
    return int(load_library().lbm_workspace_bytes(ctx))


def lbm_lattice_tables(lattice: str):
    """(c [Q][3] list, w [Q] list) as the library holds them."""
    lib = load_library()
    q = ctypes.c_int32()
    c = (ctypes.c_int32 * 57)()
    w = (ctypes.c_double * 19)()
    _check(lib.lbm_lattice_tables(LATTICES[lattice], ctypes.byref(q), c, w), "lbm_lattice_tables")
    n = q.value
    return [[c[3 * i], c[3 * i + 1], c[3 * i + 2]] for i in range(n)], [w[i] for i in range(n)]


def lbm_init(ctx, cfg: Config, rho, u, A0, stream=None):
    n = cfg.batch * cfg.nx * cfg.ny * cfg.nz
    _check(load_library().lbm_init(ctx, _ptr(rho, torch.float32, n, "rho"),
                                   _ptr(u, torch.float32, n * cfg.D, "u"),
                                   _ptr(A0, torch.float32, lbm_state_elems(ctx), "A0"),
                                   _stream(stream)), "lbm_init")


def lbm_step(ctx, cfg: Config, A, B, theta, nsteps: int, stream=None):
    """Runs nsteps steps ping-ponging A -> B -> A ...; returns the buffer that
    holds the result (B for odd nsteps, A for even)."""
    n = lbm_state_elems(ctx)
    th = _ptr(theta, torch.float32, lbm_param_elems(ctx), "theta", allow_none=cfg.hidden == 0)
    _check(load_library().lbm_step(ctx, _ptr(A, torch.float32, n, "A"),
                                   _ptr(B, torch.float32, n, "B"), th, int(nsteps),
                                   _stream(stream)), "lbm_step")
    return B if nsteps % 2 == 1 else A


def lbm_step_f64(ctx, cfg: Config, A, B, theta, nsteps: int, stream=None):
    """The float64 reference step (A, B, theta float64 device tensors);
    returns the buffer that holds the result, as lbm_step."""
    n = lbm_state_elems(ctx)
    th = _ptr(theta, torch.float64, lbm_param_elems(ctx), "theta", allow_none=cfg.hidden == 0)
    _check(load_library().lbm_step_f64(ctx, _ptr(A, torch.float64, n, "A"),
                                       _ptr(B, torch.float64, n, "B"), th, int(nsteps),
                                       _stream(stream)), "lbm_step_f64")
    return B if nsteps % 2 == 1 else A


def lbm_moments(ctx, cfg: Config, A, rho=None, u=None, diag=None, stream=None):
    n = cfg.batch * cfg.nx * cfg.ny * cfg.nz
    _check(load_library().lbm_moments(
        ctx, _ptr(A, torch.float32, lbm_state_elems(ctx), "A"),
        _ptr(rho, torch.float32, n, "rho", allow_none=True),
        _ptr(u, torch.float32, n * cfg.D, "u", allow_none=True),
        _ptr(diag, torch.float64, 4 * cfg.batch, "diag", allow_none=True),
        _stream(stream)), "lbm_moments")


def lbm_shift(ctx, src, dst, direction: int, stream=None):
    n = lbm_state_elems(ctx)
    _check(load_library().lbm_shift(ctx, _ptr(src, torch.float32, n, "src"),
                                    _ptr(dst, torch.float32, n, "dst"), int(direction),
                                    _stream(stream)), "lbm_shift")


def lbm_step_backward(ctx, cfg: Config, A_n, theta, lam_n1, lam_n, dtheta, ws, stream=None):
    n = lbm_state_elems(ctx)
    npar = lbm_param_elems(ctx)
    nws = lbm_workspace_bytes(ctx)
    if ws is not None and (ws.device.type != "cuda" or not ws.is_contiguous()):
        raise ValueError("ws must be a contiguous device tensor")
    ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
    if cfg.hidden and ws_bytes < nws:
        raise ValueError(f"workspace of {ws_bytes} bytes, {nws} needed")
    _check(load_library().lbm_step_backward(
        ctx, _ptr(A_n, torch.float32, n, "A_n"),
        _ptr(theta, torch.float32, npar, "theta", allow_none=cfg.hidden == 0),
        _ptr(lam_n1, torch.float32, n, "lam_n1"), _ptr(lam_n, torch.float32, n, "lam_n"),
        _ptr(dtheta, torch.float32, npar, "dtheta", allow_none=cfg.hidden == 0),
        None if ws is None else ctypes.c_void_p(ws.data_ptr()), ws_bytes,
        _stream(stream)), "lbm_step_backward")


def lbm_step_backward_static(ctx, cfg: Config, A_n, theta, lam_n1, lam_n, dtheta, stream=None):
    """lbm_step_backward with the library's static scratch (no workspace,
    no allocation)."""
    n = lbm_state_elems(ctx)
    npar = lbm_param_elems(ctx)
    _check(load_library().lbm_step_backward_static(
        ctx, _ptr(A_n, torch.float32, n, "A_n"),
        _ptr(theta, torch.float32, npar, "theta", allow_none=cfg.hidden == 0),
        _ptr(lam_n1, torch.float32, n, "lam_n1"), _ptr(lam_n, torch.float32, n, "lam_n"),
        _ptr(dtheta, torch.float32, npar, "dtheta", allow_none=cfg.hidden == 0),
        _stream(stream)), "lbm_step_backward_static")


def lbm_step_backward_seq(ctx, cfg: Config, states, theta, lam_a, lam_b, dtheta, ws, stream=None):
    """Adjoint of len(states) consecutive steps, states[m] the state step m
    read; lam_a holds dL/dA after the last step.  Returns the buffer that holds
    dL/dA of states[0] (lam_b for an odd count, lam_a for even)."""
    n = lbm_state_elems(ctx)
    npar = lbm_param_elems(ctx)
    nws = lbm_workspace_bytes(ctx)
    if len(states) < 1:
        raise ValueError("states must hold at least one state")
    if ws is not None and (ws.device.type != "cuda" or not ws.is_contiguous()):
        raise ValueError("ws must be a contiguous device tensor")
    ws_bytes = 0 if ws is None else ws.numel() * ws.element_size()
    if cfg.hidden and ws_bytes < nws:
        raise ValueError(f"workspace of {ws_bytes} bytes, {nws} needed")
    arr = (ctypes.c_void_p * len(states))(
        *[_ptr(a, torch.float32, n, f"states[{m}]") for m, a in enumerate(states)])
    _check(load_library().lbm_step_backward_seq(
        ctx, arr, len(states),
        _ptr(theta, torch.float32, npar, "theta", allow_none=cfg.hidden == 0),
        _ptr(lam_a, torch.float32, n, "lam_a"), _ptr(lam_b, torch.float32, n, "lam_b"),
        _ptr(dtheta, torch.float32, npar, "dtheta", allow_none=cfg.hidden == 0),
        None if ws is None else ctypes.c_void_p(ws.data_ptr()), ws_bytes,
        _stream(stream)), "lbm_step_backward_seq")
    return lam_b if len(states) % 2 == 1 else lam_a


def lbm_loss_velocity_mse(ctx, cfg: Config, A, u_target, loss, dLdA=None, stream=None):
    n = cfg.batch * cfg.nx * cfg.ny * cfg.nz
    _check(load_library().lbm_loss_velocity_mse(
        ctx, _ptr(A, torch.float32, lbm_state_elems(ctx), "A"),
        _ptr(u_target, torch.float32, n * cfg.D, "u_target"),
        _ptr(loss, torch.float64, 1, "loss"),
        _ptr(dLdA, torch.float32, lbm_state_elems(ctx), "dLdA", allow_none=True),
        _stream(stream)), "lbm_loss_velocity_mse")


def lbm_adam(param, grad, m, v, lr, beta1, beta2, eps, weight_decay, t, stream=None):
    n = param.numel()
    _check(load_library().lbm_adam(
        _ptr(param, torch.float32, n, "param"), _ptr(grad, torch.float32, n, "grad"),
        _ptr(m, torch.float32, n, "m"), _ptr(v, torch.float32, n, "v"), n, float(lr),
        float(beta1), float(beta2), float(eps), float(weight_decay), int(t),
        _stream(stream)), "lbm_adam")


def lbm_box_filter(src, dst, batch, channels, nx, ny, nz, factor, stream=None):
    fz = factor if nz > 1 else 1
    _check(load_library().lbm_box_filter(
        _ptr(src, torch.float32, batch * channels * nx * ny * nz, "src"),
        _ptr(dst, torch.float32,
             batch * channels * (nx // factor) * (ny // factor) * (nz // fz), "dst"),
        batch, channels, nx, ny, nz, factor, _stream(stream)), "lbm_box_filter")


def lbm_subsample(lattice: str, src, dst, batch, nx, ny, nz, factor, stream=None):
    q = 9 if lattice == "D2Q9" else 19
    fz = factor if nz > 1 else 1
    _check(load_library().lbm_subsample(
        LATTICES[lattice], _ptr(src, torch.float32, batch * q * nx * ny * nz, "src"),
        _ptr(dst, torch.float32, batch * q * (nx // factor) * (ny // factor) * (nz // fz), "dst"),
        batch, nx, ny, nz, factor, _stream(stream)), "lbm_subsample")


def lbm_loss_population_sse(ctx, cfg: Config, A, target, nodes, loss, dLdA=None, stream=None):
    n = lbm_state_elems(ctx)
    if nodes.dtype != torch.int32 or nodes.device.type != "cuda" or not nodes.is_contiguous():
        raise ValueError("nodes must be a contiguous int32 device tensor")
    _check(load_library().lbm_loss_population_sse(
        ctx, _ptr(A, torch.float32, n, "A"), _ptr(target, torch.float32, n, "target"),
        ctypes.c_void_p(nodes.data_ptr()), int(nodes.numel()),
        _ptr(loss, torch.float64, 1, "loss"),
        _ptr(dLdA, torch.float32, n, "dLdA", allow_none=True), _stream(stream)),
        "lbm_loss_population_sse")


def lbm_structure_functions_workspace_bytes(ctx, lmax, pmax) -> int:
    return int(load_library().lbm_structure_functions_workspace_bytes(ctx, int(lmax), int(pmax)))


def lbm_structure_functions(ctx, cfg: Config, u, lmax, pmax, S, S_abs, ws, stream=None):
    n = cfg.batch * cfg.D * cfg.nx * cfg.ny * cfg.nz
    if ws is None or ws.device.type != "cuda" or not ws.is_contiguous():
        raise ValueError("ws must be a contiguous device tensor")
    _check(load_library().lbm_structure_functions(
        ctx, _ptr(u, torch.float32, n, "u"), int(lmax), int(pmax),
        _ptr(S, torch.float64, lmax * pmax, "S"), _ptr(S_abs, torch.float64, lmax * pmax, "S_abs"),
        ctypes.c_void_p(ws.data_ptr()), ws.numel() * ws.element_size(),
        _stream(stream)), "lbm_structure_functions")


def lbm_mrt_moment_sums(ctx, A_n, A_n1, stats, stream=None):
    n = lbm_state_elems(ctx)
    _check(load_library().lbm_mrt_moment_sums(
        ctx, _ptr(A_n, torch.float32, n, "A_n"), _ptr(A_n1, torch.float32, n, "A_n1"),
        _ptr(stats, torch.float64, 95, "stats"), _stream(stream)), "lbm_mrt_moment_sums")


# ------------------------------------------------------------ convenience
class Lattice:
    """A context plus the configuration, with tensor-allocating helpers."""

    def __init__(self, cfg: Config, device="cuda"):
        self.cfg = cfg
        self.device = torch.device(device)
        with torch.cuda.device(self.device):
            self.ctx = lbm_create(cfg)
        self.n_state = lbm_state_elems(self.ctx)
        self.n_param = lbm_param_elems(self.ctx)
        self._ws = None

    def close(self):
        if self.ctx is not None:
            lbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty_state(self):
        return torch.empty(self.cfg.state_shape, dtype=torch.float32, device=self.device)

    def init(self, rho, u):
        A = self.empty_state()
        lbm_init(self.ctx, self.cfg, rho, u, A)
        return A

    def step(self, A, theta=None, nsteps=1, out=None):
        """Advance nsteps; A is preserved.  Returns the new state tensor."""
        a = A.clone()
        b = self.empty_state() if out is None else out
        return lbm_step(self.ctx, self.cfg, a, b, theta, nsteps)

    def moments(self, A, want_fields=True):
        c = self.cfg
        rho = u = None
        if want_fields:
            rho = torch.empty((c.batch, c.nz, c.ny, c.nx), dtype=torch.float32, device=self.device)
            u = torch.empty((c.batch, c.D, c.nz, c.ny, c.nx), dtype=torch.float32, device=self.device)
        diag = torch.empty((c.batch, 4), dtype=torch.float64, device=self.device)
        lbm_moments(self.ctx, c, A, rho, u, diag)
        return rho, u, diag

    def shift(self, src, direction):
        dst = torch.empty_like(src)
        lbm_shift(self.ctx, src, dst, direction)
        return dst

    def workspace(self):
        if self._ws is None:
            nb = max(lbm_workspace_bytes(self.ctx), 4)
            self._ws = torch.empty(nb // 4 + 1, dtype=torch.float32, device=self.device)
        return self._ws

    def step_backward(self, A_n, theta, lam_n1, dtheta=None):
        lam_n = torch.empty_like(lam_n1)
        if self.cfg.hidden and dtheta is None:
            dtheta = torch.zeros(self.n_param, dtype=torch.float32, device=self.device)
        lbm_step_backward(self.ctx, self.cfg, A_n, theta, lam_n1, lam_n, dtheta,
                          self.workspace() if self.cfg.hidden else None)
        return lam_n, dtheta

    def loss_population_sse(self, A, target, nodes, want_grad=True):
        """eq. nn-loss on the node subset `nodes` (distinct flat indices);
        the gradient is zero outside the subset."""
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.zeros_like(A) if want_grad else None
        lbm_loss_population_sse(self.ctx, self.cfg, A, target, nodes, loss, g)
        return loss, g

    def loss_velocity_mse(self, A, u_target, want_grad=True):
        loss = torch.empty(1, dtype=torch.float64, device=self.device)
        g = torch.empty_like(A) if want_grad else None
        lbm_loss_velocity_mse(self.ctx, self.cfg, A, u_target, loss, g)
        return loss, g
