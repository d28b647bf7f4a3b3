"""Pins of the oracle's Smagorinsky collision (SI, "Implementing the
Smagorinsky Turbulence Model in LBM"): BGK at the local relaxation time

    tau_eff = 3 (nu + C_s^2 |S|) + 1/2,  nu = (tau - 1/2) / 3,
    |S| = sqrt(2 S_ab S_ab),  S_ab = -3 / (2 tau) Pi^neq_ab,
    Pi^neq_ab = sum_q c_qa c_qb (f_q - f^eq_q).

The pins are closed forms for states whose non-equilibrium part is a pure
shear or a pure normal stress, derived by hand from those formulas, plus the
reduction to BGK and invariants.
"""
import numpy as np
import pytest

import oracle


def _one(lat, tau, cs, **kw):
    base = dict(lattice=lat, nx=1, ny=1, nz=1, tau=tau, collision="smagorinsky", smag_cs=cs)
    base.update(kw)
    return oracle.Config(**base)


def _eq_state(lat, rho, u):
    cfg = oracle.Config(lattice=lat, nx=1, ny=1, nz=1)
    D = cfg.D
    return oracle.init_equilibrium(cfg, np.full((1, 1, 1, 1), rho),
                                   np.array(u[:D], float).reshape(1, D, 1, 1, 1))


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
@pytest.mark.parametrize("a,b", [(0, 1), (1, 2), (0, 2)])
def test_shear_stress_closed_form(lat, a, b):
    """f = f^eq + eps (9/2) w_q c_qa c_qb leaves mass, momentum and f^eq
    unchanged and has Pi^neq_ab = Pi^neq_ba = eps / 2 (sum_q w c_a^2 c_b^2
    = 1/9 on both lattices), all other components 0.  Then |S| = 3|eps| /
    (2 tau) and tau_eff = tau + 9/2 C_s^2 |eps| / tau, and the collision maps
    the non-equilibrium part to (1 - 1/tau_eff) times itself."""
    if lat == "D2Q9" and 2 in (a, b):
        pytest.skip("no z axis")
    c, w = oracle.tables(lat)
    tau, cs, eps = 0.53, 0.17, 4e-3
    geq = _eq_state(lat, 1.02, [0.03, -0.02, 0.01])
    neq = eps * 4.5 * w * c[:, a] * c[:, b]
    g = geq + neq.reshape(geq.shape)
    tau_eff = tau + 4.5 * cs * cs * abs(eps) / tau
    post = oracle.collide(_one(lat, tau, cs), g)
    want = geq + (1.0 - 1.0 / tau_eff) * neq.reshape(geq.shape)
    assert np.abs(post - want).max() < 1e-15
    # and plain BGK relaxes at 1/tau, which differs
    bgk = oracle.collide(oracle.Config(lattice=lat, nx=1, ny=1, nz=1, tau=tau), g)
    assert np.abs(bgk - want).max() > 1e-6


@pytest.mark.parametrize("lat", ["D2Q9", "D3Q19"])
def test_normal_stress_closed_form(lat):
    """f^neq = eps (9/4) w_q (c_qx^2 - c_qy^2): no mass or momentum, and
    Pi^neq diagonal with Pi_xx = -Pi_yy (= eps / 2 on both lattices, from
    sum w c_x^4 = 1/3 and sum w c_x^2 c_y^2 = 1/9), checked from the tables;
    then |S| = sqrt(2 (S_xx^2 + S_yy^2)) by hand."""
    c, w = oracle.tables(lat)
    tau, cs, eps = 0.51, 0.3, -6e-3
    neq = eps * 2.25 * w * (c[:, 0] ** 2 - c[:, 1] ** 2)
    assert abs(neq.sum()) < 1e-18 and np.abs(c.T @ neq).max() < 1e-18
    pi = np.einsum("qa,qb,q->ab", c, c, neq)
    off = pi - np.diag(np.diag(pi))
    assert np.abs(off).max() < 1e-18 and abs(pi[0, 0] + pi[1, 1]) < 1e-18
    assert abs(pi[0, 0] - eps / 2) < 1e-18
    smag = np.sqrt(2 * ((1.5 / tau * pi[0, 0]) ** 2 + (1.5 / tau * pi[1, 1]) ** 2))
    tau_eff = tau + 3 * cs * cs * smag
    geq = _eq_state(lat, 0.97, [-0.01, 0.04, 0.02])
    g = geq + neq.reshape(geq.shape)
    post = oracle.collide(_one(lat, tau, cs), g)
    want = geq + (1.0 - 1.0 / tau_eff) * neq.reshape(geq.shape)
    assert np.abs(post - want).max() < 1e-15


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 9, 11)), ("D3Q19", (4, 5, 6))])
def test_reduces_to_bgk_and_conserves(lat, shape):
    nz, ny, nx = shape
    rng = np.random.default_rng(60)
    kw = dict(lattice=lat, nx=nx, ny=ny, nz=nz, tau=0.52)
    g = rng.normal(0, 0.02, oracle.Config(**kw).state_shape)
    bgk = oracle.step(oracle.Config(**kw), g)
    zero = oracle.step(oracle.Config(collision="smagorinsky", smag_cs=0.0, **kw), g)
    assert np.array_equal(bgk, zero)
    smag = oracle.collide(oracle.Config(collision="smagorinsky", smag_cs=0.2, **kw), g)
    plain = oracle.collide(oracle.Config(**kw), g)
    assert np.abs(smag - plain).max() > 1e-5  # the model acts ...
    c, _ = oracle.tables(lat)
    d = (smag - g)[0].reshape(c.shape[0], -1)
    assert np.abs(d.sum(axis=0)).max() < 1e-15  # ... and conserves mass
    assert np.abs(c.T @ d).max() < 1e-15        # and momentum at every node
    # the eddy viscosity only adds dissipation: the non-equilibrium part of
    # every node relaxes at least as fast as with BGK
    eq = oracle.collide(oracle.Config(tau=1.0, **{k: v for k, v in kw.items() if k != "tau"}), g)
    ne_s = np.abs(smag - eq).reshape(c.shape[0], -1)
    ne_b = np.abs(plain - eq).reshape(c.shape[0], -1)
    assert np.all(ne_s.sum(axis=0) <= ne_b.sum(axis=0) + 1e-15)


def test_invalid_combinations():
    with pytest.raises(RuntimeError):  # no network on top of the Smagorinsky collision
        oracle.step(oracle.Config(nx=4, ny=4, hidden=32, collision="smagorinsky", smag_cs=0.1),
                    np.zeros((1, 9, 1, 4, 4)), np.zeros(oracle.Config(nx=4, ny=4, hidden=32).n_params))
    with pytest.raises(RuntimeError):  # the adjoint covers the fixed-tau collision only
        cfg = oracle.Config(nx=4, ny=4, collision="smagorinsky", smag_cs=0.1)
        oracle.step_adjoint(cfg, np.zeros(cfg.state_shape), np.zeros(cfg.state_shape))
