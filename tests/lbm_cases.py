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


# float32 value of c = 2 log2(e): the 16-bit tanh kernels evaluate
# tanh z = 1 - 2 / (1 + 2^(c z)) and carry c in the operands of the two tanh
# layers (a documented implementation choice of those kernels)
TANH_ARG_SCALE = np.float32(2.8853900817779268)


def _round16(a, prec):
    """float32 values rounded once to bf16 / fp16 (round to nearest even)."""
    import torch
    dt = torch.bfloat16 if prec == "bf16" else torch.float16
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32))
    return t.to(dt).to(torch.float64).numpy()


def kernel_operand_theta(theta, Q, H, prec, net="tanh"):
    """The parameters the 16-bit kernels compute with, in effect, as float64.

    Tanh network: the operands of layers 1 and 2 hold fl32(c w) rounded to
    the format and the layer-1 bias enters as one more operand column, so
    these layers compute c z with weights round(fl32(c w)) / c; b2 is held
    as fl32(c b2).  Layer 3 rounds its weights as they are; b3 stays float32.
    The SI's network (LeakyReLU) rounds every weight and, as an operand
    column, b1.  Passed to the oracle with quant_weights=False (activation
    rounding only), this reproduces the kernels' rounding, which the tight
    parity bars check; the plain-rounding emulation (every weight rounded as it is,
    biases exact) is the independent reference of the accuracy bars."""
    th = np.asarray(theta, np.float32)
    if prec not in ("bf16", "fp16"):
        return th.astype(np.float64)
    out = th.astype(np.float64).copy()
    if net == "tanh":
        c = TANH_ARG_SCALE
        cd = float(c)
        oW1, ob1 = 0, H * Q
        oW2, ob2 = ob1 + H, ob1 + H + H * H
        oW3 = ob2 + H
        out[oW1:ob1] = _round16(c * th[oW1:ob1], prec) / cd
        out[ob1:oW2] = _round16(c * th[ob1:oW2], prec) / cd
        out[oW2:ob2] = _round16(c * th[oW2:ob2], prec) / cd
        out[ob2:oW3] = (c * th[ob2:oW3]).astype(np.float64) / cd
        out[oW3:oW3 + Q * H] = _round16(th[oW3:oW3 + Q * H], prec)
        return out
    widths = [Q, 300, 300, 100, Q]
    o = 0
    for l in range(4):
        nw = widths[l + 1] * widths[l]
        out[o:o + nw] = _round16(th[o:o + nw], prec)
        if l == 0:
            out[o + nw:o + nw + widths[1]] = _round16(th[o + nw:o + nw + widths[1]], prec)
        o += nw + widths[l + 1]
    return out


def kernel_emulation(ocfg, theta, prec):
    """(oracle config, theta) reproducing the 16-bit kernels' rounding; see
    kernel_operand_theta."""
    import dataclasses
    cfg = dataclasses.replace(ocfg, quant=prec, quant_weights=False)
    return cfg, kernel_operand_theta(theta, ocfg.Q, ocfg.hidden, prec, ocfg.net)


def plain_rounding_config(ocfg, prec):
    """The oracle's emulation of the reduced-precision network at the
    rounding points of the precision plan: input, every weight and every
    hidden activation rounded; biases and sums exact."""
    import dataclasses
    return dataclasses.replace(ocfg, quant=prec, quant_weights=True)


def exact_config(ocfg):
    import dataclasses
    return dataclasses.replace(ocfg, quant="none", quant_weights=True)


def spectrum(u):
    """Shell-summed 1/2 |u_hat(k)|^2 of a (2, n, n) velocity field, float64."""
    n = u.shape[-1]
    uh = np.fft.fft2(u, axes=(-2, -1)) / (n * n)
    e = 0.5 * (np.abs(uh) ** 2).sum(0)
    k = np.fft.fftfreq(n, d=1.0 / n)
    kk = np.sqrt(k[:, None] ** 2 + k[None, :] ** 2)
    shell = np.rint(kk).astype(int)
    return np.bincount(shell.ravel(), weights=e.ravel())[: n // 2]


def spectral_errors(E, E_ref):
    """Energy-weighted relative error over k >= 1 and the largest relative
    error over the shells that hold at least 0.1% of the energy."""
    k = np.arange(1, len(E_ref))
    w = E_ref[k]
    sig = w > 1e-3 * w.sum()
    return float(np.abs(E[k] - w).sum() / w.sum()), float(np.abs(E[k][sig] / w[sig] - 1).max())
