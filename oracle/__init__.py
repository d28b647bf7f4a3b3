"""FP64 serial CPU oracle of the learned-collision lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path never does.
It shares no code with the GPU library (``paper_2403_18466_amd``) and imports
nothing from it.

The arithmetic lives in ``lbm_oracle.c`` (plain C, double precision, node by
node); this module only compiles it with gcc and marshals numpy arrays.
State convention: canonical pre-collision deviations g_q = f_q - w_q rho0,
shape (B, Q, nz, ny, nx).

Paper: Ortali et al., "Kinetic data-driven approach to turbulence subgrid
modeling" (arXiv:2403.18466).  Each C function cites the passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

LATTICES = {"D2Q9": 0, "D3Q19": 1}
QUANT = {"none": 0, "bf16": 1, "fp16": 2}
NETS = {"tanh": 0, "paper": 1}
COLLISIONS = {"bgk": 0, "smagorinsky": 1}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
            "-fno-fast-math", "-fopenmp", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
        ("nz", ctypes.c_int32), ("batch", ctypes.c_int32),
        ("tau", ctypes.c_double), ("rho0", ctypes.c_double),
        ("force_kind", ctypes.c_int32), ("force_amp", ctypes.c_double),
        ("force_k", ctypes.c_int32), ("hidden", ctypes.c_int32),
        ("quant", ctypes.c_int32), ("out_scale", ctypes.c_double),
        ("net", ctypes.c_int32), ("collision", ctypes.c_int32), ("smag_cs", ctypes.c_double),
        ("quant_weights", ctypes.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(_Cfg)
        _lib.orc_tables.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int),
                                    ctypes.POINTER(ctypes.c_int), dp]
        _lib.orc_param_elems.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
        _lib.orc_param_elems.restype = ctypes.c_int64
        for name, args in [
            ("orc_step", [cp, dp, dp, dp]),
            ("orc_run", [cp, dp, dp, ctypes.c_int]),
            ("orc_collide", [cp, dp, dp, dp]),
            ("orc_init", [cp, dp, dp, dp]),
            ("orc_moments", [cp, dp, dp, dp, dp]),
            ("orc_step_adjoint", [cp, dp, dp, dp, dp, dp]),
            ("orc_loss_velocity_mse", [cp, dp, dp, dp, dp]),
            ("orc_subsample", [cp, dp, ctypes.c_int, dp]),
            ("orc_structure_functions", [cp, dp, ctypes.c_int, ctypes.c_int, dp, dp]),
            ("orc_mrt_moment_sums", [cp, dp, dp, dp]),
            ("orc_mrt_matrix", [ctypes.POINTER(ctypes.c_int32)]),
            ("orc_loss_population_sse", [cp, dp, dp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int,
                                         dp, dp]),
            ("orc_adam", [ctypes.c_int64, dp, dp, dp, dp, ctypes.c_double, ctypes.c_double,
                          ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int]),
            ("orc_box_filter", [ctypes.c_int] * 6 + [dp, dp]),
            ("orc_set_threads", [ctypes.c_int]),
        ]:
            f = getattr(_lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        _lib.orc_round_bf16.argtypes = [ctypes.c_double]
        _lib.orc_round_bf16.restype = ctypes.c_double
        _lib.orc_round_fp16.argtypes = [ctypes.c_double]
        _lib.orc_round_fp16.restype = ctypes.c_double
    return _lib


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Config:
    lattice: str = "D2Q9"
    nx: int = 64
    ny: int = 64
    nz: int = 1
    batch: int = 1
    tau: float = 0.6
    rho0: float = 1.0
    force_kind: int = 0
    force_amp: float = 0.0
    force_k: int = 0
    hidden: int = 0
    quant: str = "none"
    out_scale: float = 1.0
    net: str = "tanh"      # "tanh": Q-H-H-Q tanh; "paper": Q-300-300-100-Q LeakyReLU
    collision: str = "bgk"  # "bgk" or "smagorinsky" (BGK at the local tau_eff)
    smag_cs: float = 0.0
    # with quant != "none": round every weight to the format (True), or take
    # the weights as given (False: the caller passes the operand weights in
    # effect; only the input and the hidden activations are rounded)
    quant_weights: bool = True

    def _c(self) -> _Cfg:
        return _Cfg(LATTICES[self.lattice], self.nx, self.ny, self.nz, self.batch,
                    self.tau, self.rho0, self.force_kind, self.force_amp, self.force_k,
                    self.hidden, QUANT[self.quant], self.out_scale, NETS[self.net],
                    COLLISIONS[self.collision], self.smag_cs, int(bool(self.quant_weights)))

    @property
    def Q(self) -> int:
        return 9 if self.lattice == "D2Q9" else 19

    @property
    def D(self) -> int:
        return 2 if self.lattice == "D2Q9" else 3

    @property
    def state_shape(self):
        return (self.batch, self.Q, self.nz, self.ny, self.nx)

    @property
    def n_params(self) -> int:
        return int(_load().orc_param_elems(LATTICES[self.lattice], self.hidden, NETS[self.net]))


def tables(lattice: str):
    """(c [Q,3] int, w [Q] float64) as typed in the oracle."""
    lib = _load()
    Q = ctypes.c_int()
    D = ctypes.c_int()
    c = (ctypes.c_int * 57)()
    w = np.zeros(19, np.float64)
    rc = lib.orc_tables(LATTICES[lattice], ctypes.byref(Q), ctypes.byref(D), c, _ptr(w))
    assert rc == 0
    q = Q.value
    return np.array(c[: 3 * q], dtype=np.int64).reshape(q, 3), w[:q].copy()


def _theta(cfg: Config, theta):
    if cfg.hidden == 0:
        return None
    t = np.ascontiguousarray(theta, dtype=np.float64)
    if cfg.n_params == 0:
        raise ValueError(f"invalid network: hidden={cfg.hidden}, net={cfg.net!r}")
    assert t.size == cfg.n_params, (t.size, cfg.n_params)
    return t


def _check(rc, name):
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with code {rc}")


def step(cfg: Config, g, theta=None):
    """One collide+stream step of canonical pre-collision deviations."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == cfg.state_shape
    out = np.empty_like(g)
    c = cfg._c()
    _check(_load().orc_step(ctypes.byref(c), _ptr(_theta(cfg, theta)), _ptr(g), _ptr(out)), "step")
    return out


def run(cfg: Config, g, theta=None, nsteps: int = 1):
    g = np.array(g, dtype=np.float64, order="C", copy=True)
    assert g.shape == cfg.state_shape
    c = cfg._c()
    _check(_load().orc_run(ctypes.byref(c), _ptr(_theta(cfg, theta)), _ptr(g), nsteps), "run")
    return g


def collide(cfg: Config, g, theta=None):
    """Post-collision populations (no streaming)."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    out = np.empty_like(g)
    c = cfg._c()
    _check(_load().orc_collide(ctypes.byref(c), _ptr(_theta(cfg, theta)), _ptr(g), _ptr(out)), "collide")
    return out


def init_equilibrium(cfg: Config, rho, u):
    """g = f^eq(rho, u) - w rho0.  rho: (B,nz,ny,nx); u: (B,D,nz,ny,nx)."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert rho.shape == (cfg.batch, cfg.nz, cfg.ny, cfg.nx)
    assert u.shape == (cfg.batch, cfg.D, cfg.nz, cfg.ny, cfg.nx)
    g = np.empty(cfg.state_shape, np.float64)
    c = cfg._c()
    _check(_load().orc_init(ctypes.byref(c), _ptr(rho), _ptr(u), _ptr(g)), "init")
    return g


def moments(cfg: Config, g):
    """(rho, u, diag) with u = (j + F/2)/rho and diag[b] = [mass, KE, nonfinite, 0]."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    rho = np.empty((cfg.batch, cfg.nz, cfg.ny, cfg.nx), np.float64)
    u = np.empty((cfg.batch, cfg.D, cfg.nz, cfg.ny, cfg.nx), np.float64)
    diag = np.empty((cfg.batch, 4), np.float64)
    c = cfg._c()
    _check(_load().orc_moments(ctypes.byref(c), _ptr(g), _ptr(rho), _ptr(u), _ptr(diag)), "moments")
    return rho, u, diag


def step_adjoint(cfg: Config, g_n, lam_n1, theta=None):
    """(lam_n, dtheta) for one step: lam_n = J^T lam_n1, dtheta = (dC/dtheta)^T mu."""
    g_n = np.ascontiguousarray(g_n, dtype=np.float64)
    lam_n1 = np.ascontiguousarray(lam_n1, dtype=np.float64)
    lam_n = np.empty_like(g_n)
    dtheta = np.zeros(max(cfg.n_params, 1), np.float64)
    c = cfg._c()
    _check(_load().orc_step_adjoint(ctypes.byref(c), _ptr(_theta(cfg, theta)), _ptr(g_n),
                                    _ptr(lam_n1), _ptr(lam_n),
                                    _ptr(dtheta) if cfg.hidden else None), "step_adjoint")
    return lam_n, (dtheta if cfg.hidden else None)


def loss_velocity_mse(cfg: Config, g, u_target, want_grad: bool = True):
    g = np.ascontiguousarray(g, dtype=np.float64)
    ut = np.ascontiguousarray(u_target, dtype=np.float64)
    assert ut.shape == (cfg.batch, cfg.D, cfg.nz, cfg.ny, cfg.nx)
    loss = ctypes.c_double()
    grad = np.empty_like(g) if want_grad else None
    c = cfg._c()
    _check(_load().orc_loss_velocity_mse(ctypes.byref(c), _ptr(g), _ptr(ut), ctypes.byref(loss),
                                         _ptr(grad)), "loss")
    return loss.value, grad


def subsample(cfg: Config, g, factor: int):
    """Sub-sampling filter of the SI's training set on a canonical state of
    the fine configuration cfg."""
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == cfg.state_shape
    fz = factor if cfg.D == 3 else 1
    out = np.empty((cfg.batch, cfg.Q, cfg.nz // fz, cfg.ny // factor, cfg.nx // factor))
    c = cfg._c()
    _check(_load().orc_subsample(ctypes.byref(c), _ptr(g), factor, _ptr(out)), "subsample")
    return out


def loss_population_sse(cfg: Config, g_model, g_target, nodes, want_grad: bool = True):
    """eq. nn-loss on the node subset `nodes` (flat indices) for canonical
    pre-collision states; returns (loss, dL/dg_model or None)."""
    gm = np.ascontiguousarray(g_model, dtype=np.float64)
    gt = np.ascontiguousarray(g_target, dtype=np.float64)
    nd = np.ascontiguousarray(nodes, dtype=np.int32)
    loss = ctypes.c_double()
    grad = np.empty_like(gm) if want_grad else None
    c = cfg._c()
    _check(_load().orc_loss_population_sse(
        ctypes.byref(c), _ptr(gm), _ptr(gt), nd.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
        int(nd.size), ctypes.byref(loss), _ptr(grad)), "loss_population_sse")
    return loss.value, grad


def structure_functions(cfg: Config, u, lmax: int, pmax: int):
    """(S, S_abs), each [pmax][lmax]: the signed and absolute longitudinal
    structure functions of the canonical velocity field u [B][D][nz][ny][nx]."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert u.shape == (cfg.batch, cfg.D, cfg.nz, cfg.ny, cfg.nx)
    S = np.empty((pmax, lmax))
    Sa = np.empty((pmax, lmax))
    c = cfg._c()
    _check(_load().orc_structure_functions(ctypes.byref(c), _ptr(u), lmax, pmax, _ptr(S), _ptr(Sa)),
           "structure_functions")
    return S, Sa


def mrt_matrix():
    M = np.empty(19 * 19, np.int32)
    _load().orc_mrt_matrix(M.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return M.reshape(19, 19)


def mrt_moment_sums(cfg: Config, g_n, g_n1):
    """[19][5] sums of m_neq, m_diff, m_neq^2, m_neq m_diff, m_diff^2 over the
    nodes for consecutive canonical states g_n, g_n1 (D3Q19)."""
    a = np.ascontiguousarray(g_n, dtype=np.float64)
    b = np.ascontiguousarray(g_n1, dtype=np.float64)
    out = np.empty((19, 5))
    c = cfg._c()
    _check(_load().orc_mrt_moment_sums(ctypes.byref(c), _ptr(a), _ptr(b), _ptr(out)), "mrt_moment_sums")
    return out


def set_threads(n: int) -> int:
    """Host threads of the oracle's node loops (1 = serial, the default).
    Node results do not depend on it; the adjoint's parameter gradient is
    summed per thread and then in thread order.  Returns the count in use."""
    return int(_load().orc_set_threads(int(n)))


def default_threads() -> int:
    """A thread count for the tests' larger oracle runs: the CPUs this
    process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def adam(p, grad, m, v, lr, beta1, beta2, eps, weight_decay, t):
    """One Adam step with L2 weight decay, in float64, in place on p, m, v."""
    for a in (p, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = np.ascontiguousarray(grad, dtype=np.float64)
    assert p.shape == g.shape == m.shape == v.shape
    _check(_load().orc_adam(p.size, _ptr(p), _ptr(g), _ptr(m), _ptr(v), lr, beta1, beta2, eps,
                            weight_decay, int(t)), "adam")


def box_filter(src, factor: int):
    """Block mean of [batch][channels][nz][ny][nx] fields over factor^D fine
    nodes (nz untouched when it is 1)."""
    src = np.ascontiguousarray(src, dtype=np.float64)
    b, c, nz, ny, nx = src.shape
    fz = factor if nz > 1 else 1
    out = np.empty((b, c, nz // fz, ny // factor, nx // factor))
    _check(_load().orc_box_filter(b, c, nx, ny, nz, factor, _ptr(src), _ptr(out)), "box_filter")
    return out


def round_bf16(v: float) -> float:
    return _load().orc_round_bf16(float(v))


def round_fp16(v: float) -> float:
    return _load().orc_round_fp16(float(v))


def unrolled_loss_and_grad(cfg: Config, g0, theta, u_target, nsteps: int, ckpt: int = 0,
                           loss_fn=None):
    """Loss after `nsteps` steps from g0 and its gradient w.r.t. theta and g0.
    The loss is the velocity MSE against u_target, or loss_fn(g) -> (loss,
    dL/dg) when given.

    Reverse-mode through the whole trajectory (the unrolled training of the
    SI, "Unrolled training").  With ckpt > 0 only every ckpt-th state is kept
    and each segment is recomputed from its checkpoint before its adjoint
    steps, which must give the same numbers as keeping every state.
    """
    states = {}
    g = np.array(g0, dtype=np.float64, copy=True)
    for n in range(nsteps):
        if ckpt <= 0 or n % ckpt == 0:
            states[n] = g
        g = step(cfg, g, theta)
    loss, lam = loss_velocity_mse(cfg, g, u_target) if loss_fn is None else loss_fn(g)
    dtheta = np.zeros(cfg.n_params, np.float64)
    n = nsteps
    while n > 0:
        seg_start = (n - 1) if ckpt <= 0 else ((n - 1) // ckpt) * ckpt
        seg = [states[seg_start]]
        for m in range(seg_start, n - 1):
            seg.append(step(cfg, seg[-1], theta))
        for m in range(n - 1, seg_start - 1, -1):
            lam, dt = step_adjoint(cfg, seg[m - seg_start], lam, theta)
            dtheta += dt
        n = seg_start
    return loss, dtheta, lam
