"""Turbulence diagnostics of the SI, off the step's hot path.

* Structure functions S^p(l) (SI, eq. structure-fun-sm), signed and of the
  absolute increments, computed on the GPU by lbm_structure_functions from
  the velocity field of lbm_moments.
* Extended self-similarity: the exponents xi_p of S^p against S^3 over a
  fitting range of S^3, and the local slopes d log S^p / d log S^3 (SI,
  "Structure Functions and Extended Self Similarity").
* The energy spectrum E(k) of a velocity field: a float64 FFT on the host
  (main text, Fig. 3); the field comes from the GPU.
* The moment-space analysis of a collision (SI, section on the physical
  interpretation of the model's action): the effective relaxation time of
  each MRT moment from the regression of m_diff on m_neq, with the sums
  computed on the GPU by lbm_mrt_moment_sums.
"""
from __future__ import annotations

import numpy as np
import torch

from . import lbm

MRT_NAMES = ("rho", "e", "eps", "jx", "qx", "jy", "qy", "jz", "qz", "pxx", "pixx", "pww",
             "piww", "pxy", "pyz", "pxz", "mx", "my", "mz")


def structure_functions(L: "lbm.Lattice", A, lmax: int, pmax: int = 6):
    """(S, S_abs) as float64 numpy arrays [pmax][lmax] for the state A."""
    _, u, _ = L.moments(A)
    S = torch.empty((pmax, lmax), dtype=torch.float64, device=L.device)
    Sa = torch.empty_like(S)
    nws = lbm.lbm_structure_functions_workspace_bytes(L.ctx, lmax, pmax)
    ws = torch.empty(nws // 8 + 1, dtype=torch.float64, device=L.device)
    lbm.lbm_structure_functions(L.ctx, L.cfg, u, lmax, pmax, S, Sa, ws)
    return S.cpu().numpy(), Sa.cpu().numpy()


def ess_exponents(S_abs, s3_range, p_list=(1, 2, 4, 5, 6)):
    """Least-squares slopes xi_p of log S^p against log S^3 over the
    separations whose S^3 lies in s3_range (the absolute third moment, as
    ESS is usually carried out), plus the local slopes
    d log S^p / d log S^3 between neighbouring separations."""
    s3 = S_abs[2]
    sel = (s3 >= s3_range[0]) & (s3 <= s3_range[1])
    if sel.sum() < 2:
        raise ValueError("fewer than two separations in the fitting range")
    out, local = {}, {}
    x = np.log(s3)
    for p in p_list:
        y = np.log(S_abs[p - 1])
        out[p] = float(np.polyfit(x[sel], y[sel], 1)[0])
        local[p] = np.diff(y) / np.diff(x)
    return out, local


def energy_spectrum(u):
    """Shell-summed kinetic energy spectrum of a periodic velocity field
    u [D][...] (numpy, any float dtype), in float64:
    E(k) = sum over wavevectors with round(|k|) = k of |u_hat|^2 / 2, with
    u_hat the FFT normalised by the number of nodes, so that
    sum_k E(k) = <|u|^2> / 2 (Parseval)."""
    u = np.asarray(u, np.float64)
    D = u.shape[0]
    shape = u.shape[1:]
    N = int(np.prod(shape))
    e = np.zeros(shape)
    for a in range(D):
        uh = np.fft.fftn(u[a]) / N
        e += 0.5 * np.abs(uh) ** 2
    ks = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n) for n in shape], indexing="ij")
    kmag = np.rint(np.sqrt(sum(k * k for k in ks))).astype(int)
    return np.bincount(kmag.ravel(), weights=e.ravel())


def mrt_relaxation(L: "lbm.Lattice", A_n, A_n1):
    """Effective relaxation time of each MRT moment for the step A_n -> A_n1
    (D3Q19): tau_i = var(m_neq_i) / cov(m_neq_i, m_diff_i) over the nodes
    (centred, as in the SI), with the correlation coefficient of the pair;
    moments with no variance (the conserved ones) give nan."""
    stats = torch.empty((19, 5), dtype=torch.float64, device=L.device)
    lbm.lbm_mrt_moment_sums(L.ctx, A_n, A_n1, stats)
    return relaxation_from_sums(stats.cpu().numpy(), L.cfg.batch * L.cfg.nx * L.cfg.ny * L.cfg.nz)


def relaxation_from_sums(st, count):
    """tau_i and correlation from the [19][5] regression sums."""
    mn, md = st[:, 0] / count, st[:, 1] / count
    vn = st[:, 2] / count - mn * mn
    cov = st[:, 3] / count - mn * md
    vd = st[:, 4] / count - md * md
    # conserved moments have no non-equilibrium part: only rounding noise
    live = vn > 1e-10 * vn.max()
    with np.errstate(divide="ignore", invalid="ignore"):
        tau = np.where(live & (np.abs(cov) > 0), vn / cov, np.nan)
        corr = np.where(live & (vd > 0), cov / np.sqrt(vn * vd), np.nan)
    return {name: (float(t), float(c)) for name, t, c in zip(MRT_NAMES, tau, corr)}
