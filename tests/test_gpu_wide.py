"""GPU parity of the step with the SI's network (Q -> 300 -> 300 -> 100 -> Q,
LeakyReLU) against the FP64 oracle, through the C ABI: float32 over several
steps on small grids with ragged rows, bf16 / fp16 against the oracle's
emulated rounding, and one step at the 3-D throughput size (D3Q19 256^3) and
at a size where work items wrap over several rows per wavefront, on sampled
nodes the oracle computes one by one."""
import numpy as np
import pytest

import oracle
from lbm_cases import (plain_rounding_config, kernel_emulation, lib_config, random_state, rel_l2, to_canonical,
                       to_shifted)
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


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def wide_params(Q, seed, scale=0.05):
    return inputs.random_params_net(inputs.net_widths(Q, 0, "paper"), seed, scale=scale)


def run_gpu(lbm, ocfg, g0, theta, nsteps, prec="fp32"):
    L = lbm.Lattice(lib_config(ocfg, prec))
    assert L.n_param == ocfg.n_params
    A = dev(to_shifted(g0, ocfg.lattice))
    out = L.step(A, dev(theta), nsteps)
    res = to_canonical(host(out), ocfg.lattice)
    L.close()
    return res


@pytest.mark.parametrize("lat,shape,batch,force,nsteps", [
    ("D2Q9", (1, 20, 70), 2, 0, 4),
    ("D2Q9", (1, 9, 130), 1, 1, 4),
    ("D3Q19", (5, 6, 70), 2, 0, 2),
    ("D3Q19", (4, 5, 9), 1, 2, 3),
])
def test_wide_fp32_parity(lbm, lat, shape, batch, force, nsteps):
    nz, ny, nx = shape
    kw = {}
    if force == 1:
        kw = dict(force_kind=1, force_amp=1e-4, force_k=1)
    elif force == 2:
        kw = dict(force_kind=2, force_amp=5e-5, force_k=1)
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=batch, tau=0.55, hidden=300,
                         net="paper", out_scale=0.25, **kw)
    theta = wide_params(ocfg.Q, seed=50)
    g0 = random_state(ocfg, 51, scale=0.03)
    want = oracle.run(ocfg, g0, theta.astype(np.float64), nsteps)
    got = run_gpu(lbm, ocfg, g0, theta, nsteps)
    bgk = oracle.run(oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=batch, tau=0.55, **kw),
                     g0, None, nsteps)
    err = rel_l2(got, want)
    net_effect = rel_l2(bgk, want)
    print(f"{lat} {shape} x{batch} force {force}: rel L2 {err:.2e} after {nsteps} steps "
          f"(the network changes the state by {net_effect:.2e})")
    assert net_effect > 1e-3
    assert err < 1e-5
    # mass and momentum totals are conserved by the collision and by streaming
    c = np.array(oracle.tables(lat)[0], np.float64)
    one = run_gpu(lbm, ocfg, g0, theta, 1)
    d = one - g0
    assert abs(d.sum()) < 1e-6 * np.abs(g0).sum()
    if force == 0:
        assert np.abs(np.einsum("bqzyx,qa->a", d, c)).max() < 1e-6 * np.abs(g0).sum()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 40, 70)), ("D3Q19", (4, 6, 20))])
def test_wide_reduced_precision(lbm, prec, lat, shape):
    """One step with 16-bit operands against the oracle's emulated rounding;
    the same criterion as for the small network: the L2 gap is a small
    fraction of the rounding effect itself, and the largest deviation is
    bounded relative to the largest update."""
    nz, ny, nx = shape
    base = dict(lattice=lat, nx=nx, ny=ny, nz=nz, batch=1, tau=0.51, hidden=300, net="paper",
                out_scale=0.5)
    ocfg_x = oracle.Config(**base)
    theta = inputs.glorot_params_net(inputs.net_widths(ocfg_x.Q, 0, "paper"), seed=1)
    g0 = random_state(ocfg_x, 52, scale=0.05)
    got = run_gpu(lbm, ocfg_x, g0, theta, 1, prec=prec)
    kcfg, kth = kernel_emulation(ocfg_x, theta, prec)
    emu = oracle.step(kcfg, g0, kth)
    plain = oracle.step(plain_rounding_config(ocfg_x, prec), g0, theta.astype(np.float64))
    exact = oracle.step(ocfg_x, g0, theta.astype(np.float64))
    upd = np.abs(exact - g0).max()
    l2_emu = np.linalg.norm(got - emu)
    l2_round = np.linalg.norm(emu - exact)
    vs_exact = np.linalg.norm(got - exact) / np.linalg.norm(plain - exact)
    max_emu = np.abs(got - emu).max() / upd
    max_exact = np.abs(got - exact).max() / upd
    print(f"{prec} {lat}: L2 |gpu-emulated| / L2 |emulated-fp64| = {l2_emu / l2_round:.3f}; "
          f"L2 |gpu-fp64| / L2 |plain-fp64| = {vs_exact:.3f}; "
          f"max |gpu-emulated| {max_emu:.2e}, max |gpu-fp64| {max_exact:.2e} of max |update|")
    assert l2_emu < 0.25 * l2_round
    assert vs_exact < 1.5
    assert max_emu < (2e-3 if prec == "bf16" else 5e-4)
    assert max_exact < (1e-2 if prec == "bf16" else 2e-3)


def _sampled_case(lat, n):
    """(oracle config, canonical float32 state, pull-shifted state, points)."""
    if lat == "D3Q19":
        nx = ny = nz = n
        ocfg = oracle.Config(lattice="D3Q19", nx=n, ny=n, nz=n, tau=0.51, hidden=300, net="paper",
                             out_scale=2.0 ** -6)
        u = inputs.solenoidal_spectrum_velocity((n, n, n), 4.0, 0.04, seed=0)
        g = oracle.init_equilibrium(ocfg, np.ones((1, n, n, n)), u[None])
    else:
        nx, ny, nz = n, 96, 1
        ocfg = oracle.Config(nx=nx, ny=ny, tau=0.51, hidden=300, net="paper", out_scale=2.0 ** -6)
        u = inputs.fourier_modes_velocity(nx, ny, kmax=4, umax=0.05, seed=0)
        g = oracle.init_equilibrium(ocfg, np.ones((1, 1, ny, nx)), u[None, :, None])
    del u
    g32 = g.astype(np.float32)
    del g
    c = np.array(oracle.tables(lat)[0])
    A = np.empty_like(g32)
    for q in range(ocfg.Q):
        A[0, q] = np.roll(g32[0, q], shift=(-c[q, 2], -c[q, 1], -c[q, 0]), axis=(0, 1, 2))
    rng = np.random.default_rng(53)
    pts = [(0, 0, 0), (nz - 1, ny - 1, nx - 1), (0, ny - 1, 63), (nz - 1, 0, 64)]
    pts += [tuple(p) for p in rng.integers(0, [nz, ny, nx], size=(28, 3))]
    return ocfg, g32, A, pts


@pytest.mark.parametrize("lat,n", [("D3Q19", 256), ("D2Q9", 2048)])
def test_wide_one_step_sampled(lbm, lat, n):
    """D3Q19 256^3 is the 3-D throughput workload (solenoidal field with
    E(k) ~ k^4 exp(-2 (k/4)^2), u_rms 0.04, tau 0.51, s_out 2^-6, Glorot
    weights, bf16); D2Q9 2048 x 96 makes every wavefront walk two work items
    (the second one past the end for some), which small grids never do."""
    ocfg, g32, A, pts = _sampled_case(lat, n)
    Q = ocfg.Q
    theta = inputs.glorot_params_net(inputs.net_widths(Q, 0, "paper"), seed=1)
    L = lbm.Lattice(lib_config(ocfg, "bf16"))
    out = L.step(torch.from_numpy(A).cuda(), torch.from_numpy(theta).cuda(), 1)
    _, _, diag = L.moments(out, want_fields=False)
    torch.cuda.synchronize()
    assert int(diag[0, 2].item()) == 0
    c = np.array(oracle.tables(lat)[0], np.float64)
    tot_in = A.astype(np.float64).sum(axis=(0, 2, 3, 4))
    tot_out = out.double().sum(dim=(0, 2, 3, 4)).cpu().numpy()
    assert abs(tot_out.sum() - tot_in.sum()) < 1e-6 * np.abs(A).sum()
    assert np.abs(c.T @ (tot_out - tot_in)).max() < 1e-6 * np.abs(A).sum()
    del A
    zs, ys, xs = (np.array([p[i] for p in pts]) for i in range(3))
    got = out[0].cpu().numpy()[:, zs, ys, xs].astype(np.float64)
    kw = dict(lattice=lat, nx=1, ny=1, nz=1, tau=0.51, hidden=300, net="paper", out_scale=2.0 ** -6)
    one_x = oracle.Config(**kw)
    one_q, kth = kernel_emulation(one_x, theta, "bf16")
    th64 = theta.astype(np.float64)
    want, exact, pre = [], [], []
    for z, y, x in pts:
        gg = g32[0, :, z, y, x].astype(np.float64).reshape(1, Q, 1, 1, 1)
        want.append(oracle.collide(one_q, gg, kth)[0, :, 0, 0, 0])
        exact.append(oracle.collide(one_x, gg, th64)[0, :, 0, 0, 0])
        pre.append(gg[0, :, 0, 0, 0])
    want, exact, pre = np.array(want).T, np.array(exact).T, np.array(pre).T
    e_upd = np.linalg.norm(got - want) / np.linalg.norm(exact - pre)
    gap = np.linalg.norm(want - exact) / np.linalg.norm(exact - pre)
    e_state = np.linalg.norm(got - want) / np.linalg.norm(want)
    print(f"{lat} n={n} bf16: state rel L2 {e_state:.2e}; |gpu - emulated| / |update| {e_upd:.2e}; "
          f"emulated rounding / |update| {gap:.2e}")
    assert e_state < 1e-4 and e_upd < 0.5 * gap
    L.close()


def gpu_adjoint(lbm, ocfg, g, lam1, theta, prec="fp32"):
    L = lbm.Lattice(lib_config(ocfg, prec))
    lam0, dth = L.step_backward(dev(to_shifted(g, ocfg.lattice)), dev(theta),
                                dev(to_shifted(lam1, ocfg.lattice)))
    out = to_canonical(host(lam0), ocfg.lattice), host(dth)
    L.close()
    return out


def _blocks(Q):
    """Offsets of the eight parameter blocks [W1 b1 W2 b2 W3 b3 W4 b4]."""
    o, offs = 0, [0]
    for nin, nout in ((Q, 300), (300, 300), (300, 100), (100, Q)):
        o += nin * nout
        offs.append(o)
        o += nout
        offs.append(o)
    return offs


@pytest.mark.parametrize("lat,shape,batch,force", [
    ("D2Q9", (1, 9, 20), 2, 0),
    ("D2Q9", (1, 16, 70), 1, 1),
    ("D3Q19", (4, 5, 6), 2, 0),
    ("D3Q19", (5, 5, 5), 1, 2),
])
def test_wide_adjoint_fp32_parity(lbm, lat, shape, batch, force):
    """lam^n and dtheta of one step against the oracle's reverse pass, every
    parameter block separately (the node count is not a multiple of the
    64-row tiles, so padded rows are exercised too)."""
    nz, ny, nx = shape
    kw = {1: dict(force_kind=1, force_amp=1e-3, force_k=1),
          2: dict(force_kind=2, force_amp=1e-3, force_k=1)}.get(force, {})
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=batch, tau=0.55, hidden=300,
                         net="paper", out_scale=0.25, **kw)
    theta = wide_params(ocfg.Q, seed=54)
    g = random_state(ocfg, 55, scale=0.03)
    lam1 = random_state(ocfg, 56, scale=1.0)
    want, wdth = oracle.step_adjoint(ocfg, g, lam1, theta.astype(np.float64))
    got, gdth = gpu_adjoint(lbm, ocfg, g, lam1, theta)
    e_lam, e_th = rel_l2(got, want), rel_l2(gdth, wdth)
    print(f"{lat} {shape} x{batch} force {force}: lam rel L2 {e_lam:.2e}, dtheta rel L2 {e_th:.2e}")
    assert e_lam < 1e-5 and e_th < 1e-5
    offs = _blocks(ocfg.Q)
    for a, b in zip(offs[:-1], offs[1:]):
        assert np.abs(wdth[a:b]).max() > 0
        assert rel_l2(gdth[a:b], wdth[a:b]) < 1e-4, (a, b)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_wide_adjoint_reduced_precision(lbm, prec):
    """16-bit operands against the oracle's emulated-rounding adjoint; the
    GPU also rounds its backward operands (dY, dZ), so the bounds are
    stated, as for the small network."""
    ocfg = oracle.Config(lattice="D3Q19", nx=9, ny=6, nz=5, batch=1, tau=0.51, hidden=300,
                         net="paper", out_scale=0.25)
    theta = inputs.glorot_params_net(inputs.net_widths(19, 0, "paper"), seed=1)
    g = random_state(ocfg, 57, scale=0.03)
    lam1 = random_state(ocfg, 58, scale=1.0)
    kcfg, kth = kernel_emulation(ocfg, theta, prec)
    want, wdth = oracle.step_adjoint(kcfg, g, lam1, kth)
    got, gdth = gpu_adjoint(lbm, ocfg, g, lam1, theta, prec=prec)
    e_lam, e_th = rel_l2(got, want), rel_l2(gdth, wdth)
    print(f"{prec}: lam rel L2 {e_lam:.2e}, dtheta rel L2 {e_th:.2e}")
    assert e_lam < (2e-3 if prec == "bf16" else 3e-4)
    assert e_th < (2e-2 if prec == "bf16" else 3e-3)


def test_wide_adjoint_4335_nodes(lbm):
    """bf16 adjoint on 4335 nodes (68 node tiles of 64 in the products, the
    last one ragged) against the oracle's emulated-rounding adjoint, every
    parameter block on its own."""
    ocfg = oracle.Config(lattice="D3Q19", nx=17, ny=17, nz=15, batch=1, tau=0.51, hidden=300,
                         net="paper", out_scale=0.25)
    theta = inputs.glorot_params_net(inputs.net_widths(19, 0, "paper"), seed=1)
    g = random_state(ocfg, 57, scale=0.03)
    lam1 = random_state(ocfg, 58, scale=1.0)
    kcfg, kth = kernel_emulation(ocfg, theta, "bf16")
    want, wdth = oracle.step_adjoint(kcfg, g, lam1, kth)
    got, gdth = gpu_adjoint(lbm, ocfg, g, lam1, theta, prec="bf16")
    e_lam, e_th = rel_l2(got, want), rel_l2(gdth, wdth)
    offs = _blocks(ocfg.Q)
    errs = [rel_l2(gdth[a:b], wdth[a:b]) for a, b in zip(offs[:-1], offs[1:])]
    print(f"4335 nodes: lam rel L2 {e_lam:.2e}, dtheta rel L2 {e_th:.2e}, blocks " +
          " ".join(f"{e:.1e}" for e in errs))
    assert e_lam < 2e-3
    assert e_th < 2e-2
    for e in errs:
        assert e < 5e-2


def test_wide_unrolled_gradient(lbm):
    """6 unrolled steps of the SI's network on D3Q19 (forced), fp32, the
    population loss on a node subset: the parameter gradient against the
    oracle's reverse pass through all steps."""
    from paper_2403_18466_amd import training
    ocfg = oracle.Config(lattice="D3Q19", nx=7, ny=6, nz=5, batch=1, tau=0.55, hidden=300,
                         net="paper", out_scale=0.25, force_kind=2, force_amp=5e-5, force_k=1)
    theta = wide_params(19, seed=59)
    g0, gt = random_state(ocfg, 60, 0.02), random_state(ocfg, 61, 0.02)
    nodes = np.random.default_rng(62).choice(210, size=50, replace=False).astype(np.int32)
    wl, wth, _ = oracle.unrolled_loss_and_grad(
        ocfg, g0, theta.astype(np.float64), None, 6, 3,
        loss_fn=lambda g: oracle.loss_population_sse(ocfg, g, gt, nodes))
    L = lbm.Lattice(lib_config(ocfg))
    nd = torch.from_numpy(nodes).cuda()
    T = dev(to_shifted(gt, "D3Q19"))
    loss, dth, _ = training.unrolled_loss_and_grad(
        L, dev(to_shifted(g0, "D3Q19")), dev(theta), None, 6, 3,
        loss_fn=lambda A: L.loss_population_sse(A, T, nd))
    err = rel_l2(host(dth), wth)
    print(f"wide network, 6 unrolled steps: loss {loss.item():.6e} vs {wl:.6e}, dtheta rel L2 {err:.2e}")
    assert abs(loss.item() - wl) <= 1e-5 * wl
    assert err < 1e-5
    L.close()
