"""Seeded synthetic inputs: initial velocity fields and network parameters.

This module holds no arithmetic of the lattice Boltzmann method itself (no
equilibrium, collision, streaming or network evaluation); it only draws the
seeded inputs that both the GPU path and the CPU oracle consume.  It imports
nothing from the rest of the package.

The paper's own DNS snapshots and trained weights are not available, so these
generators stand in for them (shapes and statistics of the workloads of the
SI, "Definition of the Training Dataset", and of the benchmark configurations).
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def fourier_mode_list(kmax: int = 4):
    """Half-plane integer modes (kx, ky) with 1 <= kx^2 + ky^2 <= kmax^2,
    kx > 0 or (kx == 0 and ky > 0), in lexicographic order of (kx, ky).
    For kmax = 4 there are 24 modes."""
    modes = []
    for kx in range(0, kmax + 1):
        for ky in range(-kmax, kmax + 1):
            k2 = kx * kx + ky * ky
            if k2 < 1 or k2 > kmax * kmax:
                continue
            if kx == 0 and ky <= 0:
                continue
            modes.append((kx, ky))
    return modes


def fourier_modes_velocity(nx: int, ny: int, kmax: int = 4, umax: float = 0.05,
                           seed: int = 0) -> np.ndarray:
    """Divergence-free 2-D velocity from a random streamfunction.

    psi = sum_k a_k cos(2 pi (kx x / nx + ky y / ny) + phi_k) over
    `fourier_mode_list(kmax)`; a_k ~ N(0, 1) for all modes, then
    phi_k ~ U[0, 2 pi) for all modes, from numpy default_rng(seed).
    u = (d psi/dy, -d psi/dx) analytically at integer nodes, scaled so that
    max |u| = umax.  Returns float64 (2, ny, nx).
    """
    modes = fourier_mode_list(kmax)
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(len(modes))
    phi = rng.uniform(0.0, TWO_PI, len(modes))
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    ux = np.zeros((ny, nx))
    uy = np.zeros((ny, nx))
    for (kx, ky), ak, pk in zip(modes, a, phi):
        th = TWO_PI * (kx * x / nx + ky * y / ny) + pk
        s = np.sin(th)
        ux += -ak * (TWO_PI * ky / ny) * s
        uy += ak * (TWO_PI * kx / nx) * s
    scale = umax / np.sqrt(ux * ux + uy * uy).max()
    return np.stack([ux * scale, uy * scale])


def _wavenumbers(n: int) -> np.ndarray:
    return np.fft.fftfreq(n, d=1.0 / n)


def solenoidal_spectrum_velocity(shape, k0: float, urms: float, seed: int) -> np.ndarray:
    """Random divergence-free velocity with energy spectrum E(k) ~ k^4 exp(-2 (k/k0)^2).

    shape = (ny, nx) or (nz, ny, nx), periodic, integer wavenumbers in units of
    2 pi / n.  D independent white-noise fields are drawn from numpy
    default_rng(seed) in component order (x, y[, z]); their Fourier transforms
    are shaped by sqrt(E(k) / S(k)) with S(k) the shell measure (2 pi k in 2-D,
    4 pi k^2 in 3-D), projected onto divergence-free modes with
    (I - k k^T / k^2), the k = 0 mode removed, and transformed back.  The
    result is scaled so that the per-component rms sqrt(<|u|^2> / D) = urms.
    Returns float64 (D, *shape).
    """
    shape = tuple(int(s) for s in shape)
    D = len(shape)
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal((D,) + shape)
    axes = tuple(range(1, D + 1))
    uh = np.fft.fftn(noise, axes=axes)
    ks = np.meshgrid(*[_wavenumbers(n) for n in shape], indexing="ij")
    # component order of u is (x, y[, z]); array axes are ([z,] y, x)
    kvec = ks[::-1]
    k2 = sum(k * k for k in kvec)
    k = np.sqrt(k2)
    E = k ** 4 * np.exp(-2.0 * (k / k0) ** 2)
    shell = TWO_PI * k if D == 2 else 4.0 * math.pi * k2
    with np.errstate(divide="ignore", invalid="ignore"):
        amp = np.where(k > 0, np.sqrt(E / np.where(shell > 0, shell, 1.0)), 0.0)
        inv_k2 = np.where(k2 > 0, 1.0 / np.where(k2 > 0, k2, 1.0), 0.0)
    uh = uh * amp
    kdotu = sum(kvec[a] * uh[a] for a in range(D))
    uh = np.stack([uh[a] - kvec[a] * kdotu * inv_k2 for a in range(D)])
    u = np.real(np.fft.ifftn(uh, axes=axes))
    u -= u.mean(axis=axes, keepdims=True)
    rms = math.sqrt(float(np.mean(np.sum(u * u, axis=0))) / D)
    return u * (urms / rms)


def taylor_green_velocity(nx: int, ny: int, U: float, kx: int = 1, ky: int = 1) -> np.ndarray:
    """2-D Taylor-Green vortex u = U(-cos(a x) sin(b y), (a/b) sin(a x) cos(b y))
    with a = 2 pi kx / nx, b = 2 pi ky / ny.  Returns (2, ny, nx)."""
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    a = TWO_PI * kx / nx
    b = TWO_PI * ky / ny
    ux = -U * np.cos(a * x) * np.sin(b * y)
    uy = U * (a / b) * np.sin(a * x) * np.cos(b * y)
    return np.stack([ux, uy])


def shear_wave_velocity(nx: int, ny: int, U: float, k: int = 1) -> np.ndarray:
    """u_x = U sin(2 pi k y / ny), u_y = 0.  Returns (2, ny, nx)."""
    y = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    return np.stack([U * np.sin(TWO_PI * k * y / ny), np.zeros((ny, nx))])


def param_count(Q: int, H: int) -> int:
    """Length of the packed parameter vector [W1 b1 W2 b2 W3 b3]."""
    return H * Q + H + H * H + H + Q * H + Q


def glorot_params(Q: int, H: int, seed: int) -> np.ndarray:
    """Packed MLP parameters Q -> H -> H -> Q, Glorot-uniform weights and zero
    biases.  Each W ~ U(-a, a), a = sqrt(6 / (fan_in + fan_out)), drawn from
    numpy default_rng(seed) in the order W1 (H x Q), W2 (H x H), W3 (Q x H),
    row-major [out][in], in float64 and then rounded to float32 (returned as
    float32).  Packing: [W1, b1, W2, b2, W3, b3]."""
    rng = np.random.default_rng(seed)

    def glorot(fo, fi):
        a = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, size=(fo, fi))

    W1 = glorot(H, Q)
    W2 = glorot(H, H)
    W3 = glorot(Q, H)
    parts = [W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), np.zeros(Q)]
    return np.concatenate(parts).astype(np.float32)


def random_params(Q: int, H: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """Packed parameters with every entry (weights and biases) ~ U(-scale, scale),
    for tests that must exercise nonzero biases."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, size=param_count(Q, H)).astype(np.float32)


# The network of the SI: hidden widths of the three LeakyReLU layers.
PAPER_WIDTHS = (300, 300, 100)


def net_widths(Q: int, H: int, net: str = "tanh") -> tuple:
    """Layer widths (input, hidden..., output) of a network kind."""
    if net == "tanh":
        return (Q, H, H, Q)
    if net == "paper":
        return (Q,) + PAPER_WIDTHS + (Q,)
    raise ValueError(f"unknown network kind {net!r}")


def net_param_count(widths) -> int:
    """Packed length: for each layer, W (out x in, row-major) then b."""
    return sum(widths[l + 1] * (widths[l] + 1) for l in range(len(widths) - 1))


def glorot_params_net(widths, seed: int) -> np.ndarray:
    """Glorot-uniform weights and zero biases for any layer list, drawn layer
    by layer from default_rng(seed), rounded to float32.  For (Q, H, H, Q)
    this equals glorot_params(Q, H, seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(len(widths) - 1):
        fi, fo = widths[l], widths[l + 1]
        a = math.sqrt(6.0 / (fi + fo))
        W = rng.uniform(-a, a, size=(fo, fi))
        parts += [W.ravel(), np.zeros(fo)]
    return np.concatenate(parts).astype(np.float32)


def random_params_net(widths, seed: int, scale: float = 0.3, bias: float | None = None) -> np.ndarray:
    """Every weight ~ U(-scale, scale), every bias ~ U(-bias, bias) (bias =
    scale by default), packed per layer, float32."""
    rng = np.random.default_rng(seed)
    b = scale if bias is None else bias
    parts = []
    for l in range(len(widths) - 1):
        fi, fo = widths[l], widths[l + 1]
        parts += [rng.uniform(-scale, scale, size=fo * fi), rng.uniform(-b, b, size=fo)]
    return np.concatenate(parts).astype(np.float32)
