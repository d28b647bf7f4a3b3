"""GPU parity of the forward path (init, shift, moments, BGK step, learned
collision in fp32 / bf16 / fp16) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle
from lbm_cases import (plain_rounding_config, exact_config, fourier_state, kernel_emulation, lib_config,
                       params, random_state, rel_l2, to_canonical, to_shifted)

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


def run_gpu(lbm, ocfg, g0, theta, nsteps, prec="fp32"):
    L = lbm.Lattice(lib_config(ocfg, prec))
    A = dev(to_shifted(g0, ocfg.lattice))
    th = dev(theta) if theta is not None else None
    out = L.step(A, th, nsteps)
    res = to_canonical(host(out), ocfg.lattice)
    L.close()
    return res


# ------------------------------------------------------------------ plumbing
@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 8, 8)), ("D2Q9", (1, 45, 67)),
                                        ("D3Q19", (7, 9, 10))])
def test_init_and_moments(lbm, lat, shape):
    nz, ny, nx = shape
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=2)
    rng = np.random.default_rng(1)
    rho = (1 + rng.uniform(-0.05, 0.05, (2, nz, ny, nx))).astype(np.float32)
    u = rng.uniform(-0.08, 0.08, (2, ocfg.D, nz, ny, nx)).astype(np.float32)
    L = lbm.Lattice(lib_config(ocfg))
    A = L.init(dev(rho), dev(u))
    want = oracle.init_equilibrium(ocfg, rho.astype(np.float64), u.astype(np.float64))
    got = to_canonical(host(A), lat)
    assert np.abs(got - want).max() <= 2e-7 * np.abs(want).max()
    r2, u2, diag = L.moments(A)
    orho, ou, odiag = oracle.moments(ocfg, want)
    assert np.abs(host(r2) - orho).max() < 1e-6
    assert np.abs(host(u2) - ou).max() < 1e-6
    d = host(diag)
    assert np.abs(d[:, 0] - odiag[:, 0]).max() < 1e-6 * odiag[:, 0].max()
    assert np.abs(d[:, 1] - odiag[:, 1]).max() < 1e-5 * odiag[:, 1].max()
    assert (d[:, 2] == 0).all()


def test_moments_blocks_walk_several_chunks(lbm):
    """More 256-node row chunks per field than moments workgroups (2 chunks
    per row, the second ragged, 4200 chunks), two fields: every workgroup
    walks more than one chunk."""
    ocfg = oracle.Config(nx=300, ny=2100, batch=2)
    g = random_state(ocfg, 5, scale=0.03)
    L = lbm.Lattice(lib_config(ocfg))
    r2, u2, diag = L.moments(dev(to_shifted(g, "D2Q9")))
    orho, ou, odiag = oracle.moments(ocfg, g)
    assert np.abs(host(r2) - orho).max() < 1e-6
    assert np.abs(host(u2) - ou).max() < 1e-5
    d = host(diag)
    assert np.abs(d[:, 0] - odiag[:, 0]).max() < 1e-6 * odiag[:, 0].max()
    assert np.abs(d[:, 1] - odiag[:, 1]).max() < 1e-5 * odiag[:, 1].max()
    assert (d[:, 2] == 0).all()


def test_moments_count_nonfinite(lbm):
    ocfg = oracle.Config(nx=16, ny=8, batch=2)
    g = random_state(ocfg, 3)
    g[1, 4, 0, 3, 5] = np.nan
    g[1, 0, 0, 6, 1] = np.inf
    L = lbm.Lattice(lib_config(ocfg))
    _, _, diag = L.moments(dev(to_shifted(g, "D2Q9")))
    _, _, od = oracle.moments(ocfg, g)
    d = host(diag)
    assert d[0, 2] == 0 and d[1, 2] == 2 and od[1, 2] == 2
    assert abs(d[1, 0] - od[1, 0]) < 1e-6 * od[1, 0]


@pytest.mark.parametrize("lat,shape", [("D2Q9", (1, 13, 70)), ("D3Q19", (5, 6, 7))])
def test_shift_is_the_streaming_permutation(lbm, lat, shape):
    nz, ny, nx = shape
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=2)
    g = random_state(ocfg, 4)
    L = lbm.Lattice(lib_config(ocfg))
    A = L.shift(dev(g), -1)
    assert np.array_equal(host(A), to_shifted(g, lat))
    assert np.array_equal(host(L.shift(A, +1)), g)


def test_lattice_tables_match_oracle(lbm):
    for lat in ("D2Q9", "D3Q19"):
        c, w = lbm.lbm_lattice_tables(lat)
        oc, ow = oracle.tables(lat)
        assert np.array_equal(np.array(c), oc)
        assert np.array_equal(np.array(w), ow)


# ------------------------------------------------------------------ BGK
@pytest.mark.parametrize("lat,shape,force,nsteps", [
    ("D2Q9", (1, 8, 8), 0, 20),
    ("D2Q9", (1, 37, 70), 0, 50),
    ("D2Q9", (1, 64, 64), 1, 100),
    ("D3Q19", (6, 7, 9), 0, 20),
    ("D3Q19", (8, 8, 8), 2, 20),
])
def test_bgk_parity(lbm, lat, shape, force, nsteps):
    nz, ny, nx = shape
    kw = {}
    if force == 1:
        kw = dict(force_kind=1, force_amp=1e-4, force_k=2)
    elif force == 2:
        kw = dict(force_kind=2, force_amp=5e-5, force_k=1)
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=2, tau=0.56, **kw)
    g0 = random_state(ocfg, 5, scale=0.01)
    want = oracle.run(ocfg, g0, None, nsteps)
    got = run_gpu(lbm, ocfg, g0, None, nsteps)
    err = rel_l2(got, want)
    assert err < 1e-5, err
    # per-node mass conservation of every collision: total mass unchanged
    assert abs(got.sum() - g0.sum()) < 1e-6 * np.abs(g0).sum()


# -------------------------------------------------------- learned collision
def test_cfg1_fp32_500_steps(lbm):
    """D2Q9 64x64, tau 0.6, 9->32->32->9 tanh (Glorot, seed 1), s_out = 2^-4,
    Fourier-mode initial velocity (seed 0, max |u| 0.05), 500 steps: fp32
    GPU against the fp64 oracle, relative L2 <= 1e-5 on g and on u."""
    ocfg = oracle.Config(nx=64, ny=64, tau=0.6, hidden=32, out_scale=2.0 ** -4)
    g0 = fourier_state(ocfg)
    theta = params(9, 32, seed=1)
    want = oracle.run(ocfg, g0, theta.astype(np.float64), 500)
    got = run_gpu(lbm, ocfg, g0, theta, 500)
    assert rel_l2(got, want) <= 1e-5
    _, u_w, _ = oracle.moments(ocfg, want)
    _, u_g, _ = oracle.moments(ocfg, got)
    assert rel_l2(u_g, u_w) <= 1e-5
    assert np.abs(u_w).max() > 0.01  # the flow is still alive


@pytest.mark.parametrize("lat,shape,H,force", [
    ("D2Q9", (1, 8, 8), 32, 0),
    ("D2Q9", (1, 45, 70), 64, 0),
    ("D2Q9", (1, 32, 130), 64, 1),
    ("D3Q19", (5, 6, 70), 64, 0),
    ("D3Q19", (6, 6, 6), 32, 2),
])
def test_nlbm_fp32_parity(lbm, lat, shape, H, force):
    nz, ny, nx = shape
    kw = {}
    if force == 1:
        kw = dict(force_kind=1, force_amp=1e-4, force_k=1)
    elif force == 2:
        kw = dict(force_kind=2, force_amp=5e-5, force_k=1)
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=2, tau=0.55, hidden=H,
                         out_scale=0.25, **kw)
    theta = params(ocfg.Q, H, seed=7, kind="random")
    g0 = random_state(ocfg, 8, scale=0.03)
    want = oracle.run(ocfg, g0, theta.astype(np.float64), 10)
    got = run_gpu(lbm, ocfg, g0, theta, 10)
    err = rel_l2(got, want)
    assert err < 1e-5, err
    # every collision conserves mass and momentum to float32 rounding
    c = np.array(oracle.tables(lat)[0], np.float64)
    one = run_gpu(lbm, ocfg, g0, theta, 1)
    # streaming permutes populations: compare field totals of mass and momentum
    d = one - g0
    assert abs(d.sum()) < 1e-6 * np.abs(g0).sum()
    mom = np.einsum("bqzyx,qa->a", d, c)
    assert np.abs(mom).max() < 1e-6 * np.abs(g0).sum()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("lat,shape,H", [("D2Q9", (1, 64, 64), 64), ("D2Q9", (1, 20, 33), 32),
                                          ("D3Q19", (6, 7, 20), 64)])
def test_nlbm_reduced_precision(lbm, prec, lat, shape, H):
    """bf16/fp16 operands with fp32 accumulation, one step, three ways.

    Tight: against the oracle reproducing the kernel's own operand rounding
    (its exp2 argument scale carried in the tanh layers' weights; activation
    rounding emulated in the oracle, effective weights from the test).  The
    two then differ only where a float32 accumulation-order or tanh
    difference moves an activation across a rounding boundary: the L2 gap is
    a small fraction of the rounding effect.

    Accuracy (independent of the kernel's scheme): against the oracle's plain rounding
    emulation (input, weights, activations rounded as they are) and against
    plain fp64.  The kernel's error against fp64 must be of the size of the
    plain-rounding scheme's own error, and its distance from the plain rounding result within the
    bound stated here."""
    nz, ny, nx = shape
    base = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=1, tau=0.51, hidden=H,
                         out_scale=1.0)
    theta = params(base.Q, H, seed=1)
    g0 = random_state(base, 9, scale=0.05)
    got = run_gpu(lbm, base, g0, theta, 1, prec=prec)
    kcfg, kth = kernel_emulation(base, theta, prec)
    emu = oracle.step(kcfg, g0, kth)
    plain = oracle.step(plain_rounding_config(base, prec), g0, theta.astype(np.float64))
    exact = oracle.step(exact_config(base), g0, theta.astype(np.float64))
    upd = np.abs(exact - g0).max()
    r_plain = np.linalg.norm(plain - exact)
    tight = np.linalg.norm(got - emu) / np.linalg.norm(emu - exact)
    vs_plain = np.linalg.norm(got - plain) / r_plain
    vs_exact = np.linalg.norm(got - exact) / r_plain
    max_emu = np.abs(got - emu).max() / upd
    max_plain = np.abs(got - plain).max() / upd
    max_exact = np.abs(got - exact).max() / upd
    print(f"{prec} {lat} H={H}: L2 gap / L2 rounding effect: kernel scheme {tight:.3f}; "
          f"|gpu-plain| {vs_plain:.3f}, |gpu-fp64| {vs_exact:.3f} of |plain-fp64|; max of max|update|: "
          f"kernel scheme {max_emu:.2e}, plain rounding {max_plain:.2e}, fp64 {max_exact:.2e}")
    assert tight < 0.25
    assert max_emu < (2e-3 if prec == "bf16" else 5e-4)
    assert vs_exact < 1.5
    assert vs_plain < 2.0
    assert max_plain < (5e-3 if prec == "bf16" else 1e-3)
    assert max_exact < (5e-3 if prec == "bf16" else 1e-3)
