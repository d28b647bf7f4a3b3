"""Pins of the diagnostics: the oracle's structure functions and MRT
moment sums, and the host-side spectrum and ESS fit, against closed forms
and the matrix printed in the SI."""
import math
import os

import numpy as np
import pytest

import oracle
from paper_2403_18466_amd import diagnostics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_oracle_mrt_matrix_is_the_printed_one():
    M = np.loadtxt(os.path.join(GOLDEN, "mrt_matrix_M.txt")).astype(int)
    assert np.array_equal(oracle.mrt_matrix(), M)


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 8, 32)), ("D3Q19", (4, 5, 32))])
def test_structure_functions_single_mode(lat, shape):
    """u_x = A sin(2 pi k x / n), other components 0.  Along x the increment
    is d = 2 A sin(pi k l / n) cos(theta) with theta uniform over the n/k
    grid phases, so <d^p> = (2A sin)^p <cos^p> with <cos^p> = C(p, p/2) / 2^p
    for even p (n/k > p), 0 for odd p; the other axes give 0.  The mean over
    the D axes divides by D."""
    nz, ny, nx = shape
    cfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=1)
    D = cfg.D
    A, k = 0.03, 2
    u = np.zeros((1, D, nz, ny, nx))
    u[0, 0] = A * np.sin(2 * np.pi * k * np.arange(nx) / nx)[None, None, :]
    lmax, pmax = 6, 6
    S, Sa = oracle.structure_functions(cfg, u, lmax, pmax)
    for l in range(1, lmax + 1):
        amp = 2 * A * abs(math.sin(math.pi * k * l / nx))
        for p in range(1, pmax + 1):
            even = math.comb(p, p // 2) / 2 ** p if p % 2 == 0 else 0.0
            assert abs(S[p - 1, l - 1] - amp ** p * even / D) <= 1e-15 + 1e-12 * amp ** p
            if p % 2 == 0:
                assert abs(Sa[p - 1, l - 1] - amp ** p * even / D) <= 1e-12 * amp ** p + 1e-18
    # odd absolute moments are positive where the increment is not zero
    assert np.all(Sa[0] > 0)


def test_mrt_sums_of_bgk_give_tau():
    """BGK relaxes every moment at 1/tau: m_diff = m_neq / tau node by node,
    so the regression slope is 1/tau for the non-conserved moments, and the
    conserved ones (rho, j) have m_neq = m_diff = 0, also with a force
    (its f_ext is taken out of m_diff)."""
    for kw in ({}, dict(force_kind=2, force_amp=1e-3, force_k=1)):
        cfg = oracle.Config(lattice="D3Q19", nx=6, ny=5, nz=4, batch=2, tau=0.61, **kw)
        g = np.random.default_rng(90).normal(0, 0.02, cfg.state_shape)
        st = oracle.mrt_moment_sums(cfg, g, oracle.step(cfg, g))
        res = diagnostics.relaxation_from_sums(st, 2 * 6 * 5 * 4)
        for name, (tau, corr) in res.items():
            if name in ("rho", "jx", "jy", "jz"):
                assert math.isnan(tau)
                assert np.abs(st[diagnostics.MRT_NAMES.index(name)]).max() < 1e-12
            else:
                assert abs(tau - 0.61) < 1e-10 and abs(corr - 1.0) < 1e-10


def test_energy_spectrum_parseval_and_shell():
    n = 32
    x = np.arange(n)
    u = np.zeros((2, n, n))
    u[0] = 0.1 * np.sin(2 * np.pi * 3 * x / n)[None, :]   # |k| = 3
    u[1] = 0.05 * np.cos(2 * np.pi * 4 * x / n)[:, None]  # |k| = 4 (along the first axis)
    E = diagnostics.energy_spectrum(u)
    assert abs(E.sum() - 0.5 * np.mean(u[0] ** 2 + u[1] ** 2)) < 1e-15
    assert abs(E[3] - 0.5 * 0.1 ** 2 / 2) < 1e-15 and abs(E[4] - 0.5 * 0.05 ** 2 / 2) < 1e-15
    assert abs(E.sum() - E[3] - E[4]) < 1e-16


def test_ess_exponents_of_power_laws():
    l = np.arange(1, 17, dtype=float)
    zeta = {1: 0.37, 2: 0.70, 3: 1.0, 4: 1.28, 5: 1.54, 6: 1.78}
    Sa = np.array([2.0 * l ** zeta[p] for p in range(1, 7)])
    xi, local = diagnostics.ess_exponents(Sa, (Sa[2, 2], Sa[2, 12]))
    for p, v in xi.items():
        assert abs(v - zeta[p] / zeta[3]) < 1e-12
        assert np.allclose(local[p], zeta[p] / zeta[3])
