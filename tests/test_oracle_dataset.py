"""Pins of the oracle's training-set pieces (SI, "Definition of the Training
Dataset" and "Unrolled training"): the sub-sampling filter and the
population loss of eq. nn-loss on a node subset, whose post-collision
values come from the inverse of the streaming."""
import numpy as np
import pytest

import oracle
from paper_2403_18466_amd import inputs


@pytest.mark.parametrize("lat,shape,f", [("D2Q9", (1, 12, 20), 2), ("D2Q9", (1, 16, 8), 4),
                                          ("D3Q19", (8, 4, 12), 2)])
def test_subsample_is_the_coarse_equilibrium(lat, shape, f):
    """The filter of an equilibrium state built from (rho, u) on the fine
    grid is the equilibrium of the same fields sampled at every f-th point."""
    nz, ny, nx = shape
    fine = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=2)
    fz = f if lat == "D3Q19" else 1
    coarse = oracle.Config(lattice=lat, nx=nx // f, ny=ny // f, nz=nz // fz, batch=2)
    rng = np.random.default_rng(70)
    rho = 1 + rng.uniform(-0.05, 0.05, (2, nz, ny, nx))
    u = rng.uniform(-0.05, 0.05, (2, fine.D, nz, ny, nx))
    g = oracle.init_equilibrium(fine, rho, u)
    got = oracle.subsample(fine, g, f)
    want = oracle.init_equilibrium(coarse, rho[:, ::fz, ::f, ::f], u[:, :, ::fz, ::f, ::f])
    assert np.array_equal(got, want)


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 10, 13)), ("D3Q19", (4, 5, 6))])
def test_population_loss_compares_post_collision_values(lat, shape):
    """With g_model = step(g0) and g_target = step(g1) the loss must be the
    sum over S of |collide(g0) - collide(g1)|^2 at the nodes themselves: the
    anti-streaming recovers each node's own post-collision vector."""
    nz, ny, nx = shape
    cfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=2, tau=0.6)
    rng = np.random.default_rng(71)
    g0 = rng.normal(0, 0.02, cfg.state_shape)
    g1 = rng.normal(0, 0.02, cfg.state_shape)
    N = nx * ny * nz
    nodes = rng.choice(2 * N, size=25, replace=False).astype(np.int32)
    loss, _ = oracle.loss_population_sse(cfg, oracle.step(cfg, g0), oracle.step(cfg, g1), nodes,
                                         want_grad=False)
    p0 = oracle.collide(cfg, g0).reshape(2, cfg.Q, N)
    p1 = oracle.collide(cfg, g1).reshape(2, cfg.Q, N)
    b, n = nodes // N, nodes % N
    want = float(((p0[b, :, n] - p1[b, :, n]) ** 2).sum())
    assert abs(loss - want) <= 1e-13 * want


def test_population_loss_gradient_and_range():
    """The loss is quadratic, so a central difference is exact up to
    rounding; components that feed no sampled node have zero gradient."""
    cfg = oracle.Config(nx=7, ny=6, batch=1)
    rng = np.random.default_rng(72)
    gm = rng.normal(0, 0.02, cfg.state_shape)
    gt = rng.normal(0, 0.02, cfg.state_shape)
    nodes = np.array([0, 5, 17, 41], np.int32)
    loss, grad = oracle.loss_population_sse(cfg, gm, gt, nodes)
    flat = gm.reshape(-1)
    h = 1e-3
    for e in list(rng.choice(flat.size, 30, replace=False)) + list(np.flatnonzero(grad)[:10]):
        gp = flat.copy(); gp[e] += h
        gn = flat.copy(); gn[e] -= h
        lp, _ = oracle.loss_population_sse(cfg, gp.reshape(gm.shape), gt, nodes, want_grad=False)
        ln, _ = oracle.loss_population_sse(cfg, gn.reshape(gm.shape), gt, nodes, want_grad=False)
        assert abs((lp - ln) / (2 * h) - grad.reshape(-1)[e]) < 1e-10
    assert np.count_nonzero(grad) == 4 * 9  # 9 sources per sampled node
    with pytest.raises(RuntimeError):
        oracle.loss_population_sse(cfg, gm, gt, np.array([42], np.int32))
