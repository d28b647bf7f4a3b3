"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself or with a retyped copy of its
own formulas: each test checks a property, a printed number, a closed form,
a library routine or a differently formulated brute-force computation.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import brute
import oracle
from paper_2403_18466_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rand_state(cfg, seed, scale=0.01):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, cfg.state_shape)


# --------------------------------------------------------------------------
# P1: stencils
# --------------------------------------------------------------------------

def test_d3q19_matches_table_s1():
    c, w = oracle.tables("D3Q19")
    rows = [l.split() for l in open(os.path.join(GOLDEN, "d3q19_table_s1.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 19
    for q, r in enumerate(rows):
        assert int(r[0]) == q
        assert tuple(int(v) for v in r[1:4]) == tuple(c[q])
        assert float(Fraction(r[4])) == w[q]


def test_d3q19_order_matches_moment_matrix_M():
    """The SI's MRT matrix M (an independent passage) has the momentum rows
    j_x, j_y, j_z equal to c_x, c_y, c_z in the velocity order of the oracle."""
    M = np.loadtxt(os.path.join(GOLDEN, "mrt_matrix_M.txt"))
    c, _ = oracle.tables("D3Q19")
    assert np.array_equal(M[3], c[:, 0])
    assert np.array_equal(M[5], c[:, 1])
    assert np.array_equal(M[7], c[:, 2])
    # e row: 19 |c|^2 - 30 (the energy moment)
    assert np.array_equal(M[1], 19 * (c * c).sum(1) - 30)


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_stencil_isotropy(lat):
    """Quadrature identities in exact rational arithmetic (weights are the
    doubles nearest to small fractions)."""
    c, w = oracle.tables(lat)
    D = 2 if lat == "D2Q9" else 3
    wf = [Fraction(x).limit_denominator(100) for x in w]
    assert all(float(a) == b for a, b in zip(wf, w))
    Q = len(w)
    assert sum(wf) == 1
    for a in range(D):
        assert sum(wf[q] * c[q, a] for q in range(Q)) == 0
        for b in range(D):
            s2 = sum(wf[q] * c[q, a] * c[q, b] for q in range(Q))
            assert s2 == (Fraction(1, 3) if a == b else 0)
            for e in range(D):
                assert sum(wf[q] * c[q, a] * c[q, b] * c[q, e] for q in range(Q)) == 0
                for f in range(D):
                    s4 = sum(wf[q] * c[q, a] * c[q, b] * c[q, e] * c[q, f] for q in range(Q))
                    iso = Fraction(int(a == b and e == f) + int(a == e and b == f)
                                   + int(a == f and b == e), 9)
                    assert s4 == iso
    # opposite velocities exist for every q
    for q in range(Q):
        assert any(np.array_equal(c[p], -c[q]) for p in range(Q))


def test_d2q9_reading_order():
    c, w = oracle.tables("D2Q9")
    assert np.array_equal(c[:, :2], brute.C9)
    assert np.array_equal(w, brute.W9)


def test_kappa_denominators():
    """The kappa constants of the SI: 19 and sum c_x^2 = 10 for D3Q19; the
    D2Q9 analogues 9 and 6."""
    c, _ = oracle.tables("D3Q19")
    assert len(c) == 19 and (c[:, 0] ** 2).sum() == 10
    c, _ = oracle.tables("D2Q9")
    assert len(c) == 9 and (c[:, 0] ** 2).sum() == 6


# --------------------------------------------------------------------------
# P2 / P3: equilibrium moments and BGK fixed point
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_equilibrium_moments(lat):
    cfg = oracle.Config(lattice=lat, nx=5, ny=4, nz=1 if lat == "D2Q9" else 3, batch=2)
    rng = np.random.default_rng(1)
    rho = 1.0 + rng.uniform(-0.05, 0.05, (cfg.batch, cfg.nz, cfg.ny, cfg.nx))
    u = rng.uniform(-0.1, 0.1, (cfg.batch, cfg.D, cfg.nz, cfg.ny, cfg.nx))
    g = oracle.init_equilibrium(cfg, rho, u)
    c, w = oracle.tables(lat)
    c = c[:, :cfg.D].astype(float)
    f = g + w[None, :, None, None, None] * cfg.rho0
    assert np.abs(g.sum(1) - (rho - 1.0)).max() < 1e-15
    j = np.einsum("bqzyx,qa->bazyx", f, c)
    assert np.abs(j - rho[:, None] * u).max() < 1e-15
    P = np.einsum("bqzyx,qa,qc->baczyx", f, c, c)
    want = (rho[:, None, None] * np.eye(cfg.D)[None, :, :, None, None, None] / 3.0
            + rho[:, None, None] * u[:, :, None] * u[:, None, :])
    assert np.abs(P - want).max() < 1e-15


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_bgk_fixed_point(lat):
    cfg = oracle.Config(lattice=lat, nx=6, ny=5, nz=1 if lat == "D2Q9" else 4, tau=0.55)
    rng = np.random.default_rng(2)
    rho = 1.0 + rng.uniform(-0.05, 0.05, (1, cfg.nz, cfg.ny, cfg.nx))
    u = rng.uniform(-0.1, 0.1, (1, cfg.D, cfg.nz, cfg.ny, cfg.nx))
    g = oracle.init_equilibrium(cfg, rho, u)
    post = oracle.collide(cfg, g)
    assert np.abs(post - g).max() < 1e-16
    # uniform equilibrium is invariant under a full step (collide + stream)
    rho_u = np.full((1, cfg.nz, cfg.ny, cfg.nx), 1.02)
    uu = np.zeros((1, cfg.D, cfg.nz, cfg.ny, cfg.nx))
    uu[:, 0] = 0.03
    g = oracle.init_equilibrium(cfg, rho_u, uu)
    assert np.abs(oracle.step(cfg, g) - g).max() < 1e-16


# --------------------------------------------------------------------------
# P4 / P5 / P6 / P7: conservation, EDM forcing, projection, reduction to BGK
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lat,H", [("D2Q9", 32), ("D3Q19", 16)])
def test_collision_conserves_mass_momentum(lat, H):
    cfg = oracle.Config(lattice=lat, nx=6, ny=5, nz=1 if lat == "D2Q9" else 3, tau=0.51,
                        hidden=H, out_scale=1.0)
    theta = inputs.random_params(cfg.Q, H, seed=3, scale=0.5)
    g = _rand_state(cfg, 4, scale=0.05)
    post = oracle.collide(cfg, g, theta)
    c, _ = oracle.tables(lat)
    d = post - g
    scale = np.abs(d).max()
    assert scale > 1e-3  # the network contributes a visible update
    assert np.abs(d.sum(1)).max() <= 1e-15 * 19 * scale
    assert np.abs(np.einsum("bqzyx,qa->bazyx", d, c.astype(float))).max() <= 1e-15 * 19 * scale


def test_edm_force_moments():
    """f^ext of eq. fext adds no mass and exactly the momentum F."""
    cfg = oracle.Config(nx=7, ny=16, tau=0.51, force_kind=1, force_amp=1e-3, force_k=2)
    cfg0 = oracle.Config(nx=7, ny=16, tau=0.51)
    g = _rand_state(cfg, 5, scale=0.02)
    fext = oracle.collide(cfg, g) - oracle.collide(cfg0, g)
    c, _ = oracle.tables("D2Q9")
    y = np.arange(16)[:, None] * np.ones((1, 7))
    Fx = 1e-3 * np.sin(2 * np.pi * 2 * y / 16)
    # fext is recovered as a difference of two post-collision states of size
    # |g| ~ 0.05, so each entry carries rounding of order eps |g|
    tol = 4 * 9 * np.finfo(float).eps * np.abs(g).max()
    assert np.abs(fext.sum(1)).max() < tol
    mom = np.einsum("bqzyx,qa->bazyx", fext, c.astype(float))
    assert np.abs(mom[0, 0, 0] - Fx).max() < tol
    assert np.abs(mom[0, 1, 0]).max() < tol


def test_three_component_forcing_momentum():
    cfg = oracle.Config(lattice="D3Q19", nx=8, ny=6, nz=5, tau=0.51, force_kind=2,
                        force_amp=5e-6, force_k=1)
    cfg0 = oracle.Config(lattice="D3Q19", nx=8, ny=6, nz=5, tau=0.51)
    g = _rand_state(cfg, 6, scale=0.02)
    fext = oracle.collide(cfg, g) - oracle.collide(cfg0, g)
    c, _ = oracle.tables("D3Q19")
    mom = np.einsum("bqzyx,qa->bazyx", fext, c.astype(float))[0]
    z, y, x = np.meshgrid(np.arange(5), np.arange(6), np.arange(8), indexing="ij")
    want = 5e-6 * np.stack([np.sin(2 * np.pi * y / 6), np.sin(2 * np.pi * z / 5),
                            np.sin(2 * np.pi * x / 8)])
    tol = 4 * 19 * np.finfo(float).eps * np.abs(g).max()
    assert np.abs(mom - want).max() < tol
    assert np.abs(fext.sum(1)).max() < tol
    assert np.abs(want).max() > 100 * tol


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_projection_is_orthogonal_projector(lat):
    """With W3 = 0 the network adds (s/tau) P b3.  P b3 must be orthogonal to
    1 and c_alpha, and b3 - P b3 must lie in their span."""
    H = 8
    cfg = oracle.Config(lattice=lat, nx=3, ny=2, nz=1 if lat == "D2Q9" else 2, tau=0.7,
                        hidden=H, out_scale=0.5)
    Q = cfg.Q
    theta = inputs.random_params(Q, H, seed=7).astype(np.float64)
    W3o = H * Q + H + H * H + H
    theta[W3o:W3o + Q * H] = 0.0
    b3 = theta[W3o + Q * H:].copy()
    g = _rand_state(cfg, 8)
    d = oracle.collide(cfg, g, theta) - oracle.collide(oracle.Config(lattice=lat, nx=3, ny=2, nz=cfg.nz, tau=0.7), g)
    Pb = d[0, :, 0, 0, 0] * cfg.tau / cfg.out_scale
    c, _ = oracle.tables(lat)
    B = np.concatenate([np.ones((Q, 1)), c[:, :cfg.D].astype(float)], axis=1)
    assert np.abs(B.T @ Pb).max() < 1e-15
    coef, res, *_ = np.linalg.lstsq(B, b3 - Pb, rcond=None)
    assert np.abs(B @ coef - (b3 - Pb)).max() < 1e-15
    # the printed kappa form (SI): k1 = -sum/Q, k_a = -sum c_a / sum c_a^2
    kap = b3 - b3.sum() / Q
    for a in range(cfg.D):
        kap = kap - (b3 @ c[:, a]) / (c[:, a] ** 2).sum() * c[:, a]
    assert np.abs(kap - Pb).max() < 1e-15


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_reduction_to_bgk(lat):
    H = 16
    kw = dict(lattice=lat, nx=5, ny=4, nz=1 if lat == "D2Q9" else 3, tau=0.6)
    cfg = oracle.Config(hidden=H, out_scale=1.0, **kw)
    cfg0 = oracle.Config(**kw)
    theta = inputs.random_params(cfg.Q, H, seed=9).astype(np.float64)
    W3o = H * cfg.Q + H + H * H + H
    theta[W3o:] = 0.0
    g = _rand_state(cfg, 10)
    assert np.array_equal(oracle.step(cfg, g, theta), oracle.step(cfg0, g))
    # b3 in span{1, c}: removed by the projection (up to rounding)
    c, _ = oracle.tables(lat)
    theta[W3o + cfg.Q * H:] = 0.3 + 0.2 * c[:, 0] - 0.1 * c[:, 1]
    tol = 4 * cfg.Q * np.finfo(float).eps * 0.6 / cfg.tau  # rounding of P b3, |b3| <= 0.6
    assert np.abs(oracle.step(cfg, g, theta) - oracle.step(cfg0, g)).max() < tol


# --------------------------------------------------------------------------
# P8: streaming is a permutation
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_streaming_permutation(lat):
    # tau = 1e300 makes the collision update vanish below the rounding of g
    n = 6
    cfg = oracle.Config(lattice=lat, nx=n, ny=n, nz=1 if lat == "D2Q9" else n, tau=1e300)
    g = _rand_state(cfg, 11) + 0.5  # no zeros
    g1 = oracle.step(cfg, g)
    c, _ = oracle.tables(lat)
    for q in range(cfg.Q):
        want = np.roll(g[0, q], shift=(c[q, 2], c[q, 1], c[q, 0]), axis=(0, 1, 2))
        assert np.array_equal(g1[0, q], want)
    assert np.array_equal(g1.sum(axis=(2, 3, 4)), g1.sum(axis=(2, 3, 4)))
    gn = oracle.run(cfg, g, nsteps=n)
    assert np.array_equal(gn, g)


# --------------------------------------------------------------------------
# P9: viscosity nu = c_s^2 (tau - 1/2)  (eq. tau)
# --------------------------------------------------------------------------

def _mode_amplitude(u, mode):
    return float((u * mode).sum() / (mode * mode).sum())


@pytest.mark.parametrize("kind,tau", [("tgv", 0.6), ("shear", 0.6), ("shear", 0.51)])
def test_viscous_decay_rate(kind, tau):
    L = 64
    U = 0.01
    cfg = oracle.Config(nx=L, ny=L, tau=tau)
    if kind == "tgv":
        u0 = inputs.taylor_green_velocity(L, L, U)
        rate_factor = 2.0  # u ~ exp(-2 nu k^2 t)
    else:
        u0 = inputs.shear_wave_velocity(L, L, U)
        rate_factor = 1.0
    g = oracle.init_equilibrium(cfg, np.ones((1, 1, L, L)), u0[None, :, None])
    mode = u0 / U
    t1, t2 = 200, 1000 if tau > 0.55 else 3000
    g = oracle.run(cfg, g, nsteps=t1)
    a1 = _mode_amplitude(oracle.moments(cfg, g)[1][0, :, 0], mode)
    g = oracle.run(cfg, g, nsteps=t2 - t1)
    a2 = _mode_amplitude(oracle.moments(cfg, g)[1][0, :, 0], mode)
    rate = math.log(a1 / a2) / (t2 - t1)
    nu = (tau - 0.5) / 3.0
    k = 2 * math.pi / L
    assert abs(rate / (rate_factor * nu * k * k) - 1.0) < 2e-3


# --------------------------------------------------------------------------
# P10: the paper's printed worked numbers
# --------------------------------------------------------------------------

def _paper_numbers():
    d = {}
    for line in open(os.path.join(GOLDEN, "paper_numbers.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()[:2]
            d[k] = float(v)
    return d


def test_paper_worked_numbers():
    p = _paper_numbers()
    nu = (p["dns_tau"] - 0.5) / 3.0  # eq. tau with c_s^2 = 1/3, dt = 1
    assert round(nu, 5) == p["dns_nu"]
    assert abs(p["dns_urms"] * p["dns_L"] / nu - p["dns_Re"]) / p["dns_Re"] < 1e-3
    assert abs(p["dns_L"] / p["dns_urms"] - p["dns_TL"]) < 1e-9
    tau4 = (p["dns_tau"] - 0.5) / 4 + 0.5  # eq. tau-rescaled, cg = 4
    assert round(tau4, 4) == p["cg4_tau_prime"]
    for t, re in [("gen_tau_lo", "gen_Re_lo"), ("gen_tau_hi", "gen_Re_hi")]:
        nu_t = (p[t] - 0.5) / 3.0
        assert abs(p["dns_urms"] * p["dns_L"] / nu_t - p[re]) / p[re] < 1e-3


# --------------------------------------------------------------------------
# P11: brute force on 8x8 (second formulation in tests/brute.py)
# --------------------------------------------------------------------------

def _flat(g):
    return g.reshape(-1)


@pytest.mark.parametrize("with_net,with_force", [(False, False), (True, False), (True, True)])
def test_brute_force_step_8x8(with_net, with_force):
    n = 8
    H = 32 if with_net else 0
    kw = dict(nx=n, ny=n, tau=0.6, hidden=H, out_scale=0.25)
    if with_force:
        kw.update(force_kind=1, force_amp=2e-3, force_k=1)
    cfg = oracle.Config(**kw)
    theta = inputs.random_params(9, 32, seed=12).astype(np.float64) if with_net else None
    g = _rand_state(cfg, 13, scale=0.03)
    got = _flat(oracle.step(cfg, g, theta))
    force = brute.kolmogorov_force(n, n, 2e-3, 1) if with_force else None
    want = brute.step(_flat(g), n, n, 0.6, theta=theta, H=H, out_scale=0.25, force=force)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


@pytest.mark.parametrize("with_force", [False, True])
def test_adjoint_is_transpose_of_jacobian_8x8(with_force):
    """Adjoint of one step vs the exact Jacobian from complex-step derivatives
    of the brute-force formulation (no finite-difference truncation)."""
    n, H, s = 8, 32, 0.25
    kw = dict(nx=n, ny=n, tau=0.6, hidden=H, out_scale=s)
    if with_force:
        kw.update(force_kind=1, force_amp=2e-3, force_k=1)
    cfg = oracle.Config(**kw)
    theta = inputs.random_params(9, H, seed=14).astype(np.float64)
    g = _flat(_rand_state(cfg, 15, scale=0.03))
    force = brute.kolmogorov_force(n, n, 2e-3, 1) if with_force else None
    N = g.size
    h = 1e-30
    J = np.empty((N, N))
    for i in range(N):
        gi = g.astype(complex)
        gi[i] += 1j * h
        J[:, i] = brute.step(gi, n, n, 0.6, theta=theta, H=H, out_scale=s, force=force).imag / h
    lam1 = np.random.default_rng(16).normal(size=N)
    lam0, dth = oracle.step_adjoint(cfg, g.reshape(cfg.state_shape), lam1.reshape(cfg.state_shape), theta)
    want = J.T @ lam1
    assert np.abs(_flat(lam0) - want).max() <= 1e-13 * np.abs(want).max()
    # parameter gradient of <lam1, step(g; theta)> for a spread of parameters
    idx = np.linspace(0, theta.size - 1, 40).astype(int)
    for i in idx:
        th = theta.astype(complex)
        th[i] += 1j * h
        d = (lam1 @ brute.step(g.astype(complex), n, n, 0.6, theta=th, H=H, out_scale=s,
                               force=force)).imag / h
        assert abs(dth[i] - d) <= 1e-12 * max(1.0, abs(d)), (i, dth[i], d)


# --------------------------------------------------------------------------
# P12: dot-product test of the adjoint on 16x16
# --------------------------------------------------------------------------

def test_dot_product_16x16():
    n, H, s = 16, 32, 0.25
    cfg = oracle.Config(nx=n, ny=n, tau=0.55, hidden=H, out_scale=s)
    theta = inputs.random_params(9, H, seed=17).astype(np.float64)
    rng = np.random.default_rng(18)
    g = rng.normal(0, 0.03, cfg.state_shape)
    v = rng.normal(size=cfg.state_shape)
    lam = rng.normal(size=cfg.state_shape)
    h = 1e-30
    Jv = brute.step(_flat(g) + 1j * h * _flat(v), n, n, 0.55, theta=theta, H=H, out_scale=s).imag / h
    JTlam, _ = oracle.step_adjoint(cfg, g, lam, theta)
    a = float(_flat(lam) @ Jv)
    b = float(_flat(JTlam) @ _flat(v))
    assert abs(a - b) <= 1e-13 * max(abs(a), abs(b))


# --------------------------------------------------------------------------
# P13: D3Q19 BGK in the moment space of the SI's matrix M
# --------------------------------------------------------------------------

def test_d3q19_moment_matrix_orthogonal_and_bgk_slope():
    M = np.loadtxt(os.path.join(GOLDEN, "mrt_matrix_M.txt"))
    G = M @ M.T
    assert np.abs(G - np.diag(np.diag(G))).max() == 0
    assert np.linalg.matrix_rank(M) == 19
    # conserved rows (rho, j) of the BGK update vanish; every other moment
    # relaxes with slope 1/tau: m_diff = M (post - pre) = (1/tau) m_neq
    cfg = oracle.Config(lattice="D3Q19", nx=4, ny=3, nz=2, tau=0.53)
    g = _rand_state(cfg, 19, scale=0.02)
    post = oracle.collide(cfg, g)
    rho, u, _ = oracle.moments(cfg, g)
    geq = oracle.init_equilibrium(cfg, rho, u)
    mdiff = np.einsum("mq,bqzyx->bmzyx", M, post - g)
    mneq = np.einsum("mq,bqzyx->bmzyx", M, geq - g)
    tol = 8 * np.finfo(float).eps * np.abs(M).sum(1).max() * np.abs(g).max() / cfg.tau
    for r in (0, 3, 5, 7):
        assert np.abs(mdiff[:, r]).max() < tol
    assert np.abs(mdiff - mneq / cfg.tau).max() < tol
    assert np.abs(mneq).max() > 1e5 * tol


# --------------------------------------------------------------------------
# P15: gradient through unrolled steps vs central finite differences
# --------------------------------------------------------------------------

@pytest.mark.slow
def test_unrolled_gradient_fd_32x32_16_steps():
    n, H, T = 32, 64, 16
    cfg = oracle.Config(nx=n, ny=n, tau=0.50125, hidden=H, out_scale=2.0 ** -4)
    theta = inputs.glorot_params(9, H, seed=1).astype(np.float64)
    rng = np.random.default_rng(20)
    theta[H * 9:H * 9 + H] = rng.uniform(-0.1, 0.1, H)  # nonzero b1 to exercise it
    u0 = inputs.fourier_modes_velocity(n, n, kmax=4, umax=0.05, seed=0)
    g0 = oracle.init_equilibrium(cfg, np.ones((1, 1, n, n)), u0[None, :, None])
    ut = 0.9 * inputs.fourier_modes_velocity(n, n, kmax=2, umax=0.04, seed=21)[None, :, None]
    loss, dtheta, _ = oracle.unrolled_loss_and_grad(cfg, g0, theta, ut, T, ckpt=0)
    loss_c, dtheta_c, _ = oracle.unrolled_loss_and_grad(cfg, g0, theta, ut, T, ckpt=8)
    assert loss_c == loss and np.array_equal(dtheta_c, dtheta)  # checkpointing is exact

    def L(th):
        g = oracle.run(cfg, g0, th, T)
        return oracle.loss_velocity_mse(cfg, g, ut, want_grad=False)[0]

    Q = 9
    offs = {"W1": 0, "b1": H * Q, "W2": H * Q + H, "b2": H * Q + H + H * H,
            "W3": H * Q + 2 * H + H * H, "b3": H * Q + 2 * H + H * H + Q * H}
    picks = [offs["W1"] + 5, offs["W1"] + 300, offs["b1"] + 7, offs["W2"] + 11,
             offs["W2"] + 2000, offs["b2"] + 3, offs["W3"] + 17, offs["W3"] + 500,
             offs["b3"] + 4, offs["b3"] + 8]
    for i in picks:
        hh = 1e-6 * max(1.0, abs(theta[i]))
        tp = theta.copy(); tp[i] += hh
        tm = theta.copy(); tm[i] -= hh
        fd = (L(tp) - L(tm)) / (2 * hh)
        assert abs(fd - dtheta[i]) <= 1e-6 * np.abs(dtheta).max() + 1e-6 * abs(fd), (i, fd, dtheta[i])
    d = rng.normal(size=theta.size)
    d /= np.linalg.norm(d)
    hh = 1e-6
    fd = (L(theta + hh * d) - L(theta - hh * d)) / (2 * hh)
    assert abs(fd - dtheta @ d) <= 1e-6 * abs(fd)


# --------------------------------------------------------------------------
# Emulated rounding against library conversions
# --------------------------------------------------------------------------

def test_round_fp16_matches_numpy():
    rng = np.random.default_rng(22)
    vals = np.concatenate([rng.normal(size=2000).astype(np.float32),
                           (rng.normal(size=500) * 1e-6).astype(np.float32),
                           np.array([65504, 65519.99, 65520, 1e-8, 6.1e-5, -2.5e-6],
                                    np.float32)]).astype(np.float64)
    # exact ties: midway between fp16 neighbours
    ties = (np.arange(1, 200, dtype=np.float64) * 2 + 1) * 2.0 ** -11
    for v in np.concatenate([vals, ties, -ties]):
        want = float(np.float16(v))
        assert oracle.round_fp16(v) == want, v


def test_round_bf16_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(23)
    vals = np.concatenate([rng.normal(size=3000), rng.normal(size=300) * 1e-30,
                           rng.normal(size=300) * 1e30]).astype(np.float32)
    ties = ((np.arange(1, 300) * 2 + 1) * 2.0 ** -8).astype(np.float32)  # 9-bit values
    vals = np.concatenate([vals, ties, -ties])
    want = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float64).numpy()
    for v, w in zip(vals.astype(np.float64), want):
        assert oracle.round_bf16(v) == w, v


# --------------------------------------------------------------------------
# A9 reading: stability of the untrained network is restored by s_out
# --------------------------------------------------------------------------

def _collision_jacobian(cfg, theta):
    g0 = np.zeros(cfg.state_shape)
    Q = cfg.Q
    J = np.empty((Q, Q))
    h = 1e-7
    for i in range(Q):
        gp = g0.copy(); gp[0, i] += h
        gm = g0.copy(); gm[0, i] -= h
        J[:, i] = (oracle.collide(cfg, gp, theta) - oracle.collide(cfg, gm, theta))[0, :, 0, 0, 0] / (2 * h)
    return J


def _max_amplification(J, c, nk=24):
    worst = 0.0
    for kx in np.linspace(0, 2 * np.pi, nk, endpoint=False):
        for ky in np.linspace(0, 2 * np.pi, nk, endpoint=False):
            ph = np.exp(-1j * (c[:, 0] * kx + c[:, 1] * ky))
            worst = max(worst, np.abs(np.linalg.eigvals(ph[:, None] * J)).max())
    return worst


def test_untrained_net_needs_output_scale():
    theta = inputs.glorot_params(9, 32, seed=1).astype(np.float64)
    c, _ = oracle.tables("D2Q9")
    big = _collision_jacobian(oracle.Config(nx=1, ny=1, tau=0.6, hidden=32, out_scale=1.0), theta)
    assert np.abs(np.linalg.eigvals(big)).max() > 1.0 + 1e-3
    small = _collision_jacobian(oracle.Config(nx=1, ny=1, tau=0.6, hidden=32, out_scale=2.0 ** -4), theta)
    assert _max_amplification(small, c) <= 1.0 + 1e-6


# --------------------------------------------------------------------------
# Moments, diagnostics and the velocity-MSE loss: an equilibrium built from a
# known (rho, u) must give back exactly those fields, and the diagnostics and
# loss must equal their plain definitions evaluated on them.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_moments_recover_equilibrium_fields(lat):
    cfg = oracle.Config(lattice=lat, nx=6, ny=5, nz=1 if lat == "D2Q9" else 4, batch=2)
    rng = np.random.default_rng(24)
    rho = 1.0 + rng.uniform(-0.05, 0.05, (cfg.batch, cfg.nz, cfg.ny, cfg.nx))
    u = rng.uniform(-0.08, 0.08, (cfg.batch, cfg.D, cfg.nz, cfg.ny, cfg.nx))
    g = oracle.init_equilibrium(cfg, rho, u)
    r2, u2, diag = oracle.moments(cfg, g)
    assert np.abs(r2 - rho).max() < 1e-15
    assert np.abs(u2 - u).max() < 1e-15
    for b in range(cfg.batch):
        assert abs(diag[b, 0] - rho[b].sum()) < 1e-12
        ke = 0.5 * (rho[b] * (u[b] ** 2).sum(0)).sum()
        assert abs(diag[b, 1] - ke) < 1e-14 * max(1.0, ke) * cfg.nx * cfg.ny * cfg.nz
        assert diag[b, 2] == 0
    # a non-finite population is counted and left out of the sums
    g_bad = g.copy()
    g_bad[1, 3, 0, 2, 1] = np.nan
    _, _, d2 = oracle.moments(cfg, g_bad)
    assert d2[1, 2] == 1 and d2[0, 2] == 0
    assert abs(d2[1, 0] - (rho[1].sum() - rho[1, 0, 2, 1])) < 1e-12


def test_moments_report_half_force_shift():
    """Under a body force the reported velocity is (j + F/2)/rho."""
    cfg = oracle.Config(nx=4, ny=8, force_kind=1, force_amp=1e-3, force_k=1)
    rho = np.full((1, 1, 8, 4), 1.0)
    u = np.zeros((1, 2, 1, 8, 4))
    g = oracle.init_equilibrium(cfg, rho, u)
    _, u2, _ = oracle.moments(cfg, g)
    y = np.arange(8)[:, None] * np.ones((1, 4))
    assert np.abs(u2[0, 0, 0] - 0.5e-3 * np.sin(2 * np.pi * y / 8)).max() < 1e-18
    assert np.abs(u2[0, 1]).max() == 0


def test_velocity_mse_loss_definition():
    cfg = oracle.Config(nx=7, ny=6, batch=3)
    rng = np.random.default_rng(25)
    rho = 1.0 + rng.uniform(-0.05, 0.05, (3, 1, 6, 7))
    u = rng.uniform(-0.05, 0.05, (3, 2, 1, 6, 7))
    ut = rng.uniform(-0.05, 0.05, (3, 2, 1, 6, 7))
    g = oracle.init_equilibrium(cfg, rho, u)
    loss, grad = oracle.loss_velocity_mse(cfg, g, ut)
    assert abs(loss - np.mean((u - ut) ** 2)) < 1e-16
    # the gradient against complex-step derivatives of the same definition,
    # with u computed from populations by the brute-force moment matrix
    M = brute.raw_moment_matrix()
    c, w = oracle.tables("D2Q9")
    h = 1e-30
    for (b, q, yy, xx) in [(0, 0, 0, 0), (1, 5, 3, 2), (2, 8, 5, 6), (0, 3, 2, 4)]:
        f = (g[b, :, 0, yy, xx] + w).astype(complex)
        f[q] += 1j * h
        m = M @ f
        uu = np.array([m[1] / m[0], m[2] / m[0]])
        e = ((uu - ut[b, :, 0, yy, xx]) ** 2).sum() / (3 * 2 * 6 * 7)
        assert abs(grad[b, q, 0, yy, xx] - e.imag / h) < 1e-15


# --------------------------------------------------------------------------
# P14: emulated reduced-precision network.  The same collision written as
# matrix products with torch's own float32 -> bfloat16 / float16 conversions
# at the stated rounding points: the input, both hidden activations and every
# weight; the biases and all sums stay exact.
# --------------------------------------------------------------------------

@pytest.mark.parametrize("quant", ["bf16", "fp16"])
def test_emulated_quantisation_points(quant):
    torch = pytest.importorskip("torch")
    dt = torch.bfloat16 if quant == "bf16" else torch.float16
    n, H, tau, s = 8, 32, 0.6, 0.25
    cfg_q = oracle.Config(nx=n, ny=n, tau=tau, hidden=H, out_scale=s, quant=quant)
    cfg_0 = oracle.Config(nx=n, ny=n, tau=tau)
    theta = inputs.random_params(9, H, seed=26).astype(np.float64)
    g = _rand_state(cfg_q, 27, scale=0.05)

    def rnd(a):
        # weights and biases are float32 numbers, which torch rounds
        # to the 16-bit format exactly once
        a = np.asarray(a, np.float64)
        assert np.array_equal(a.astype(np.float32).astype(np.float64), a)
        return torch.from_numpy(a).to(dt).to(torch.float64).numpy()

    def rnd_act(a):
        # the state and the activations are float64; torch would round them to float32 first
        # (a double rounding that can differ at ties), so they are rounded
        # directly: numpy's float64 -> float16 conversion, or the bfloat16
        # rounding pinned against torch above
        if quant == "fp16":
            return np.asarray(a, np.float64).astype(np.float16).astype(np.float64)
        return np.vectorize(oracle.round_bf16)(a)

    o = 0
    W1 = theta[o:o + H * 9].reshape(H, 9); o += H * 9
    b1 = theta[o:o + H]; o += H
    W2 = theta[o:o + H * H].reshape(H, H); o += H * H
    b2 = theta[o:o + H]; o += H
    W3 = theta[o:o + 9 * H].reshape(9, H); o += 9 * H
    b3 = theta[o:o + 9]
    x0 = rnd_act(g.reshape(9, -1))
    h1 = rnd_act(np.tanh(rnd(W1) @ x0 + b1[:, None]))
    h2 = rnd_act(np.tanh(rnd(W2) @ h1 + b2[:, None]))
    y = rnd(W3) @ h2 + b3[:, None]
    P = brute.projector()
    want = (oracle.collide(cfg_0, g).reshape(9, -1) + P @ ((s / tau) * y)).reshape(g.shape)
    got = oracle.collide(cfg_q, g, theta)
    assert np.abs(got - want).max() < 1e-14
    # with the weights taken as given, only the input and the activations round
    cfg_a = oracle.Config(nx=n, ny=n, tau=tau, hidden=H, out_scale=s, quant=quant,
                          quant_weights=False)
    h1 = rnd_act(np.tanh(W1 @ x0 + b1[:, None]))
    h2 = rnd_act(np.tanh(W2 @ h1 + b2[:, None]))
    y = W3 @ h2 + b3[:, None]
    want_a = (oracle.collide(cfg_0, g).reshape(9, -1) + P @ ((s / tau) * y)).reshape(g.shape)
    assert np.abs(oracle.collide(cfg_a, g, theta) - want_a).max() < 1e-14
    # passing the rounded weights in that mode is the full emulation
    th_r = np.concatenate([rnd(W1).ravel(), b1, rnd(W2).ravel(), b2, rnd(W3).ravel(), b3])
    assert np.abs(oracle.collide(cfg_a, g, th_r) - got).max() < 1e-15
    exact = oracle.collide(oracle.Config(nx=n, ny=n, tau=tau, hidden=H, out_scale=s), g, theta)
    assert np.abs(exact - got).max() > 1e-5
