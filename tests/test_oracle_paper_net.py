"""Pins of the oracle's second network kind: the network of the SI ("Neural
Network Architecture and Optimization"), Q -> 300 -> 300 -> 100 -> Q with
LeakyReLU after the hidden layers (negative slope 0.01, which the SI does not
state) and a linear output layer, inside the same collision.

As in test_oracle_pins.py the oracle is checked against a differently
written brute-force step (matrix products), exact complex-step Jacobians,
closed forms and invariants, never against a retyped copy of itself.
"""
import numpy as np
import pytest

import brute
import oracle
from paper_2403_18466_amd import inputs

SLOPE = 0.01


def _rand_state(cfg, seed, scale=0.03):
    return np.random.default_rng(seed).normal(0.0, scale, cfg.state_shape)


def _cfg(**kw):
    base = dict(nx=8, ny=8, tau=0.6, hidden=300, net="paper", out_scale=0.25)
    base.update(kw)
    return oracle.Config(**base)


def _flat(g):
    return g.reshape(-1)


def test_parameter_count_by_hand():
    # D3Q19: 19*300 + 300 | 300*300 + 300 | 300*100 + 100 | 100*19 + 19
    assert oracle.Config(lattice="D3Q19", hidden=300, net="paper").n_params == \
        6000 + 90300 + 30100 + 1919 == 128319
    # D2Q9: 9*300 + 300 | 90300 | 30100 | 100*9 + 9
    assert oracle.Config(hidden=300, net="paper").n_params == 3000 + 90300 + 30100 + 909
    # the width is fixed by the SI: any other hidden size is rejected
    bad = oracle.Config(hidden=64, net="paper")
    assert bad.n_params == 0
    with pytest.raises(ValueError):
        oracle.step(bad, np.zeros(bad.state_shape), np.zeros(10))


@pytest.mark.parametrize("with_force", [False, True])
def test_brute_force_step_8x8(with_force):
    kw = {}
    if with_force:
        kw.update(force_kind=1, force_amp=2e-3, force_k=1)
    cfg = _cfg(**kw)
    widths = inputs.net_widths(9, 0, "paper")
    theta = inputs.random_params_net(widths, seed=31, scale=0.1).astype(np.float64)
    g = _rand_state(cfg, 32)
    got = _flat(oracle.step(cfg, g, theta))
    force = brute.kolmogorov_force(8, 8, 2e-3, 1) if with_force else None
    want = brute.step(_flat(g), 8, 8, 0.6, theta=theta, out_scale=0.25, force=force, net="paper")
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    # the network really acts: without it the step differs
    plain = _flat(oracle.step(oracle.Config(nx=8, ny=8, tau=0.6, **kw), g))
    assert np.abs(got - plain).max() > 1e-4


def test_adjoint_is_transpose_of_jacobian_8x8():
    """lam^n = J^T lam^{n+1} and dtheta against complex-step derivatives of
    the brute-force step (exact away from the LeakyReLU kink, which random
    inputs do not hit)."""
    cfg = _cfg()
    widths = inputs.net_widths(9, 0, "paper")
    theta = inputs.random_params_net(widths, seed=33, scale=0.1).astype(np.float64)
    g = _flat(_rand_state(cfg, 34))
    N = g.size
    h = 1e-30
    J = np.empty((N, N))
    for i in range(N):
        gi = g.astype(complex)
        gi[i] += 1j * h
        J[:, i] = brute.step(gi, 8, 8, 0.6, theta=theta, out_scale=0.25, net="paper").imag / h
    lam1 = np.random.default_rng(35).normal(size=N)
    lam0, dth = oracle.step_adjoint(cfg, g.reshape(cfg.state_shape),
                                    lam1.reshape(cfg.state_shape), theta)
    want = J.T @ lam1
    assert np.abs(_flat(lam0) - want).max() <= 1e-12 * np.abs(want).max()
    # parameter gradient of <lam1, step(g; theta)>, spread over all four layers
    idx = np.unique(np.concatenate([np.linspace(0, theta.size - 1, 48).astype(int),
                                    [3000 - 1, 3000 + 90000, 124309 - 1]]))
    for i in idx:
        th = theta.astype(complex)
        th[i] += 1j * h
        d = (lam1 @ brute.step(g.astype(complex), 8, 8, 0.6, theta=th, out_scale=0.25,
                               net="paper")).imag / h
        assert abs(dth[i] - d) <= 1e-11 * max(1.0, abs(d)), (i, dth[i], d)


def _layers(theta, widths):
    out, o = [], 0
    for l in range(len(widths) - 1):
        nin, nout = widths[l], widths[l + 1]
        W = theta[o:o + nout * nin].reshape(nout, nin); o += nout * nin
        b = theta[o:o + nout]; o += nout
        out.append((W, b))
    return out


@pytest.mark.parametrize("regime", ["positive", "negative"])
def test_affine_regimes_closed_form(regime):
    """With every hidden pre-activation of one sign, LeakyReLU is the map
    a -> a (positive) or a -> 0.01 a (negative), and the network collapses to
    one affine map y = M x + c with
      M = s^3 W4 W3 W2 W1,
      c = s^3 W4 W3 W2 b1 + s^2 W4 W3 b2 + s W4 b3 + b4      (s = 1 or 0.01).
    The biases of +-1 and small weights fix the sign of every pre-activation;
    the test checks that they do."""
    widths = inputs.net_widths(9, 0, "paper")
    rng = np.random.default_rng(36)
    sign = 1.0 if regime == "positive" else -1.0
    parts = []
    for l in range(4):
        nin, nout = widths[l], widths[l + 1]
        scale = 0.1 if l == 0 else 1e-3
        parts += [rng.uniform(-scale, scale, nout * nin),
                  (sign * np.ones(nout)) if l < 3 else rng.uniform(-0.1, 0.1, nout)]
    theta = np.concatenate(parts).astype(np.float32).astype(np.float64)
    (W1, b1), (W2, b2), (W3, b3), (W4, b4) = _layers(theta, widths)
    cfg = _cfg()
    g = _rand_state(cfg, 37)
    x = g.reshape(9, -1)
    # the sign of every pre-activation, from the exact affine chain
    s = 1.0 if regime == "positive" else SLOPE
    a1 = W1 @ x + b1[:, None]
    a2 = W2 @ (s * a1) + b2[:, None]
    a3 = W3 @ (s * a2) + b3[:, None]
    for a in (a1, a2, a3):
        assert np.all(sign * a > 0)
    M = s ** 3 * (W4 @ W3 @ W2 @ W1)
    c = s ** 3 * (W4 @ W3 @ W2 @ b1) + s ** 2 * (W4 @ W3 @ b2) + s * (W4 @ b3) + b4
    y = M @ x + c[:, None]
    bgk = oracle.collide(oracle.Config(nx=8, ny=8, tau=0.6), g)
    want = bgk.reshape(9, -1) + brute.projector() @ ((0.25 / 0.6) * y)
    got = oracle.collide(cfg, g, theta).reshape(9, -1)
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_d3q19_collision_conserves_mass_and_momentum():
    """The kappa layer with the SI's D3Q19 denominators 19 and 10 makes the
    network term add no mass and no momentum, whatever the network."""
    cfg = oracle.Config(lattice="D3Q19", nx=4, ny=4, nz=4, tau=0.55, hidden=300, net="paper",
                        out_scale=1.0)
    widths = inputs.net_widths(19, 0, "paper")
    theta = inputs.random_params_net(widths, seed=38, scale=0.2).astype(np.float64)
    g = _rand_state(cfg, 39, scale=0.02)
    post = oracle.collide(cfg, g, theta)
    plain = oracle.collide(oracle.Config(lattice="D3Q19", nx=4, ny=4, nz=4, tau=0.55), g)
    c, _ = oracle.tables("D3Q19")
    d = (post - plain)[0].reshape(19, -1)
    assert np.abs(d).max() > 1e-3  # the network changes the populations ...
    assert np.abs(d.sum(axis=0)).max() < 1e-15  # ... but not the mass
    for a in range(3):
        assert np.abs((c[:, a, None] * d).sum(axis=0)).max() < 1e-15  # nor momentum


@pytest.mark.parametrize("quant", ["bf16", "fp16"])
def test_emulated_quantisation_points(quant):
    """Rounding at the input, every weight and the three hidden activations
    (biases exact), written as matrix products with library roundings."""
    torch = pytest.importorskip("torch")
    dt = torch.bfloat16 if quant == "bf16" else torch.float16
    cfg_q = _cfg(quant=quant)
    widths = inputs.net_widths(9, 0, "paper")
    theta = inputs.random_params_net(widths, seed=40, scale=0.1).astype(np.float64)
    g = _rand_state(cfg_q, 41, scale=0.05)

    def rnd(a):  # float32 values: one rounding by torch
        return torch.from_numpy(np.asarray(a, np.float64)).to(dt).to(torch.float64).numpy()

    def rnd_act(a):  # float64 values: rounded directly
        if quant == "fp16":
            return np.asarray(a, np.float64).astype(np.float16).astype(np.float64)
        return np.vectorize(oracle.round_bf16)(a)

    h = rnd_act(g.reshape(9, -1))
    layers = _layers(theta, widths)
    for l, (W, b) in enumerate(layers):
        a = rnd(W) @ h + b[:, None]
        h = rnd_act(brute.leaky(a)) if l < 3 else a
    bgk = oracle.collide(oracle.Config(nx=8, ny=8, tau=0.6), g)
    want = bgk.reshape(9, -1) + brute.projector() @ ((0.25 / 0.6) * h)
    got = oracle.collide(cfg_q, g, theta).reshape(9, -1)
    assert np.abs(got - want).max() < 1e-14
    exact = oracle.collide(_cfg(), g, theta).reshape(9, -1)
    assert np.abs(exact - got).max() > 1e-6
