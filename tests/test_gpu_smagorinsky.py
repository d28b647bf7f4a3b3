"""GPU parity of the Smagorinsky collision (BGK at the local tau_eff of the
SI's Smagorinsky model, fused into the stream-collide pass) against the FP64
oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from lbm_cases import lib_config, random_state, rel_l2, to_canonical, to_shifted
from paper_2403_18466_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_18466_amd import lbm as m
    m.load_library()
    return m


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("lat,shape,batch,force", [
    ("D2Q9", (1, 45, 70), 2, 0),
    ("D2Q9", (1, 33, 300), 1, 1),
    ("D3Q19", (5, 6, 70), 2, 0),
    ("D3Q19", (6, 7, 9), 1, 2),
])
def test_smagorinsky_fp32_parity(lbm, lat, shape, batch, force):
    nz, ny, nx = shape
    kw = {}
    if force == 1:
        kw = dict(force_kind=1, force_amp=1e-4, force_k=1)
    elif force == 2:
        kw = dict(force_kind=2, force_amp=5e-5, force_k=1)
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=batch, tau=0.505,
                         collision="smagorinsky", smag_cs=0.17, **kw)
    g0 = random_state(ocfg, 61, scale=0.03)
    want = oracle.run(ocfg, g0, None, 10)
    L = lbm.Lattice(lib_config(ocfg))
    out = L.step(torch.from_numpy(to_shifted(g0, lat).astype(np.float32)).cuda(), None, 10)
    got = to_canonical(host(out), lat)
    L.close()
    bgk = oracle.run(oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=batch, tau=0.505, **kw),
                     g0, None, 10)
    err, effect = rel_l2(got, want), rel_l2(bgk, want)
    print(f"{lat} {shape} x{batch} force {force}: rel L2 {err:.2e} after 10 steps "
          f"(the eddy viscosity changes the state by {effect:.2e})")
    assert effect > 1e-3
    assert err < 1e-5


def test_smagorinsky_full_size_sampled(lbm):
    """D2Q9 4096^2 (the throughput size, Fourier-mode field, tau 0.505,
    C_s 0.17), one step in the launch configuration bench.py times, sampled
    nodes against the oracle's collision node by node, plus the field totals
    of mass and momentum."""
    n = 4096
    ocfg = oracle.Config(nx=n, ny=n, tau=0.505, collision="smagorinsky", smag_cs=0.17)
    u = inputs.fourier_modes_velocity(n, n, kmax=4, umax=0.05, seed=0)
    g = oracle.init_equilibrium(ocfg, np.ones((1, 1, n, n)), u[None, :, None])
    rng = np.random.default_rng(62)
    g += rng.normal(0, 1e-3, g.shape)  # a non-equilibrium part for the model to act on
    g32 = g.astype(np.float32)
    del g
    A = to_shifted(g32, "D2Q9")
    L = lbm.Lattice(lib_config(ocfg))
    out = L.step(torch.from_numpy(A).cuda(), None, 1)
    c = np.array(oracle.tables("D2Q9")[0], np.float64)
    tot_in = A.astype(np.float64).sum(axis=(0, 2, 3, 4))
    tot_out = out.double().sum(dim=(0, 2, 3, 4)).cpu().numpy()
    assert abs(tot_out.sum() - tot_in.sum()) < 1e-6 * np.abs(A).sum()
    assert np.abs(c.T @ (tot_out - tot_in)).max() < 1e-6 * np.abs(A).sum()
    pts = [(0, 0), (n - 1, n - 1), (0, n - 1), (255, 256)] + \
        [tuple(p) for p in rng.integers(0, n, size=(40, 2))]
    ys, xs = np.array([p[0] for p in pts]), np.array([p[1] for p in pts])
    got = out[0, :, 0].cpu().numpy()[:, ys, xs].astype(np.float64)
    one = oracle.Config(nx=1, ny=1, tau=0.505, collision="smagorinsky", smag_cs=0.17)
    want = np.stack([oracle.collide(one, g32[0, :, 0, y, x].astype(np.float64).reshape(1, 9, 1, 1, 1))
                     [0, :, 0, 0, 0] for y, x in pts], axis=1)
    pre = g32[0, :, 0][:, ys, xs].astype(np.float64)
    e_state = np.linalg.norm(got - want) / np.linalg.norm(want)
    e_upd = np.linalg.norm(got - want) / np.linalg.norm(want - pre)
    print(f"4096^2 Smagorinsky, {len(pts)} nodes: state rel L2 {e_state:.2e}, "
          f"|gpu - oracle| / |update| {e_upd:.2e}")
    assert e_state < 1e-6 and e_upd < 1e-4
    L.close()
