"""The float64 GPU reference step (lbm_step_f64): checked against the CPU
oracle on small grids, then used as the reference of the 1024^2 Kolmogorov
workload's full 10,000 steps (A = 1e-5, k = 4, tau 0.51, 9->64->64->9 tanh,
s_out 2^-6), which the oracle cannot run in a test: the float32 and bf16
runs' kinetic-energy series (every 500 steps) and final energy spectrum
against the float64 run's."""
import numpy as np
import pytest

import oracle
from lbm_cases import (lib_config, params, random_state, rel_l2, spectral_errors, spectrum,
                       to_canonical, to_shifted)
from paper_2403_18466_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_18466_amd import lbm as m
    m.load_library()
    n = oracle.set_threads(oracle.default_threads())
    yield m
    oracle.set_threads(1)


def run_f64(lbm, ocfg, g0, theta, nsteps, prec="fp32"):
    L = lbm.Lattice(lib_config(ocfg, prec))
    A = torch.from_numpy(to_shifted(g0, ocfg.lattice)).cuda()
    B = torch.empty_like(A)
    th = torch.from_numpy(np.asarray(theta, np.float64)).cuda() if theta is not None else None
    out = lbm.lbm_step_f64(L.ctx, L.cfg, A, B, th, nsteps)
    torch.cuda.synchronize()
    res = to_canonical(out.cpu().numpy(), ocfg.lattice)
    L.close()
    return res


@pytest.mark.parametrize("lat,shape,batch,H,force,nsteps,kind", [
    ("D2Q9", (1, 64, 64), 1, 32, 0, 500, "cfg1"),       # the 64^2 parity workload in full
    ("D2Q9", (1, 256, 256), 1, 64, 1, 100, "kolmogorov"),
    ("D2Q9", (1, 13, 70), 2, 64, 0, 10, "random"),       # biases nonzero, ragged rows
    ("D3Q19", (10, 12, 14), 1, 32, 2, 20, "random"),     # three-component force
    ("D3Q19", (6, 7, 9), 2, 0, 2, 30, "random"),         # plain BGK
])
def test_reference_f64_matches_oracle(lbm, lat, shape, batch, H, force, nsteps, kind):
    nz, ny, nx = shape
    kw = {1: dict(force_kind=1, force_amp=1e-5, force_k=4),
          2: dict(force_kind=2, force_amp=5e-5, force_k=1)}.get(force, {})
    if kind == "cfg1":
        ocfg = oracle.Config(nx=64, ny=64, tau=0.6, hidden=32, out_scale=2.0 ** -4)
        u = inputs.fourier_modes_velocity(64, 64, kmax=4, umax=0.05, seed=0)
        g0 = oracle.init_equilibrium(ocfg, np.ones((1, 1, 64, 64)), u[None, :, None])
        theta = inputs.glorot_params(9, 32, seed=1).astype(np.float64)
    elif kind == "kolmogorov":
        ocfg = oracle.Config(nx=nx, ny=ny, tau=0.51, hidden=H, out_scale=2.0 ** -6, **kw)
        u = inputs.fourier_modes_velocity(nx, ny, kmax=4, umax=0.01, seed=0)
        g0 = oracle.init_equilibrium(ocfg, np.ones((1, 1, ny, nx)), u[None, :, None])
        theta = inputs.glorot_params(9, H, seed=1).astype(np.float64)
    else:
        ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=batch, tau=0.55, hidden=H,
                             out_scale=0.25, **kw)
        g0 = np.random.default_rng(3).normal(0.0, 0.03, ocfg.state_shape)
        theta = (inputs.random_params(ocfg.Q, H, seed=4).astype(np.float64) if H else None)
    want = oracle.run(ocfg, g0, theta, nsteps)
    got = run_f64(lbm, ocfg, g0, theta, nsteps)
    e = rel_l2(got, want)
    upd = rel_l2(want, g0)
    print(f"{lat} {shape} x{batch} H={H} force {force}, {nsteps} steps: float64 GPU vs oracle "
          f"rel L2 {e:.2e} (the state changed by {upd:.2e})")
    assert e < 1e-12


def test_kolmogorov_1024_10k_against_f64_reference(lbm):
    """Kinetic energy every 500 steps and the final spectrum of the fp32 and
    bf16 runs against the float64 GPU run of the same 10,000 steps."""
    n, steps, every = 1024, 10000, 500
    ocfg = oracle.Config(nx=n, ny=n, tau=0.51, hidden=64, out_scale=2.0 ** -6, force_kind=1,
                         force_amp=1e-5, force_k=4)
    u0 = inputs.fourier_modes_velocity(n, n, kmax=4, umax=0.01, seed=0)
    g0 = oracle.init_equilibrium(ocfg, np.ones((1, 1, n, n)), u0[None, :, None])
    g0 = g0.astype(np.float32).astype(np.float64)
    theta = inputs.glorot_params(9, 64, seed=1)
    A0 = to_shifted(g0, "D2Q9")
    # float64 reference: canonical state to the host every 500 steps, moments in float64
    L = lbm.Lattice(lib_config(ocfg))
    a = torch.from_numpy(A0).cuda()
    b = torch.empty_like(a)
    th64 = torch.from_numpy(theta.astype(np.float64)).cuda()
    ke_ref, t = [], 0
    while t < steps:
        out = lbm.lbm_step_f64(L.ctx, L.cfg, a, b, th64, every)
        if out is b:
            a, b = b, a
        t += every
        g = to_canonical(a.cpu().numpy(), "D2Q9")
        _, u, d = oracle.moments(ocfg, g)
        ke_ref.append(d[0, 1])
    print(f"  float64 reference: {steps} steps done", flush=True)
    u_ref = u[0, :, 0]
    L.close()
    res = {}
    for prec in ("fp32", "bf16"):
        L = lbm.Lattice(lib_config(ocfg, prec))
        a = torch.from_numpy(A0.astype(np.float32)).cuda()
        b = torch.empty_like(a)
        th = torch.from_numpy(theta).cuda()
        ke, t = [], 0
        while t < steps:
            out = lbm.lbm_step(L.ctx, L.cfg, a, b, th, every)
            if out is b:
                a, b = b, a
            t += every
            _, uu, diag = L.moments(a)
            torch.cuda.synchronize()
            assert int(diag[0, 2].item()) == 0
            ke.append(diag[0, 1].item())
        res[prec] = (np.array(ke), uu.cpu().numpy()[0, :, 0].astype(np.float64))
        L.close()
    ke_ref = np.array(ke_ref)
    E_ref = spectrum(u_ref)
    errs = {}
    for prec, (ke, u) in res.items():
        weighted, energetic = spectral_errors(spectrum(u), E_ref)
        errs[prec] = (float(np.abs(ke / ke_ref - 1).max()), weighted, energetic, rel_l2(u, u_ref))
        print(f"1024^2 Kolmogorov, {steps} steps, {prec} vs float64 GPU reference: kinetic energy "
              f"max rel err over {len(ke)} samples {errs[prec][0]:.2e}; final spectrum weighted "
              f"{weighted:.2e}, max over energetic shells {energetic:.2e}; velocity rel L2 "
              f"{errs[prec][3]:.2e}")
    print(f"  kinetic energy {ke_ref[0]:.4e} at step {every} -> {ke_ref[-1]:.4e} at {steps}")
    assert errs["fp32"][0] < 1e-4 and errs["fp32"][1] < 1e-3 and errs["fp32"][3] < 1e-3
    assert errs["bf16"][0] < 1e-3 and errs["bf16"][1] < 1e-2 and errs["bf16"][2] < 5e-2
