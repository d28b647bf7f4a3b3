"""Shared helpers of the GPU parity tests: oracle configurations mirrored as
library configurations, conversion between the oracle's canonical state and
the library's pull-shifted state (pure data movement), and error norms."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2403_18466_amd import inputs

C9 = [[0, 0, 0], [-1, 0, 0], [0, -1, 0], [0, 1, 0], [1, 0, 0],
      [-1, -1, 0], [-1, 1, 0], [1, -1, 0], [1, 1, 0]]


def velocities(lattice):
    return oracle.tables(lattice)[0]


def to_shifted(g, lattice):
    """Canonical [B][Q][nz][ny][nx] -> pull-shifted A_q(y) = g_q(y + c_q)."""
    c = velocities(lattice)
    out = np.empty_like(g)
    for q in range(g.shape[1]):
        out[:, q] = np.roll(g[:, q], shift=(-c[q, 2], -c[q, 1], -c[q, 0]), axis=(1, 2, 3))
    return out


def to_canonical(A, lattice):
    c = velocities(lattice)
    out = np.empty_like(A)
    for q in range(A.shape[1]):
        out[:, q] = np.roll(A[:, q], shift=(c[q, 2], c[q, 1], c[q, 0]), axis=(1, 2, 3))
    return out


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def lib_config(ocfg, prec="fp32"):
    from paper_2403_18466_amd import lbm
    return lbm.Config(lattice=ocfg.lattice, nx=ocfg.nx, ny=ocfg.ny, nz=ocfg.nz,
                      batch=ocfg.batch, tau=ocfg.tau, rho0=ocfg.rho0,
                      force_kind=ocfg.force_kind, force_k=ocfg.force_k,
                      force_amp=ocfg.force_amp, hidden=ocfg.hidden, mlp_prec=prec,
                      out_scale=ocfg.out_scale, net=ocfg.net, collision=ocfg.collision,
                      smag_cs=ocfg.smag_cs)


def fourier_state(ocfg, umax=0.05, seed=0, kmax=4):
    """Canonical equilibrium state from the random-Fourier-mode recipe,
    rounded to float32 (the precision both sides start from)."""
    assert ocfg.lattice == "D2Q9"
    u = inputs.fourier_modes_velocity(ocfg.nx, ocfg.ny, kmax=kmax, umax=umax, seed=seed)
    us = np.stack([u] * ocfg.batch)[:, :, None]
    rho = np.ones((ocfg.batch, 1, ocfg.ny, ocfg.nx))
    g = oracle.init_equilibrium(ocfg, rho, us)
    return g.astype(np.float32).astype(np.float64)


def random_state(ocfg, seed, scale=0.02):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, ocfg.state_shape).astype(np.float32).astype(np.float64)


def params(Q, H, seed, kind="glorot"):
    p = inputs.glorot_params(Q, H, seed) if kind == "glorot" else inputs.random_params(Q, H, seed)
    return p.astype(np.float32)
