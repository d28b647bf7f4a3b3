"""Kolmogorov-forced learned collision (F_x = A sin(2 pi k y / L), EDM
forcing, tau 0.51, 9->64->64->9 tanh): the float32 and bf16 networks
against the FP64 oracle on the velocity moments and the energy spectrum, on
a 128^2 field for 100 steps, and the bf16 run against the float32 run on the
1024^2 field for 10,000 steps (spectra in float64 on the host)."""
import numpy as np
import pytest

import oracle
from lbm_cases import lib_config, rel_l2, spectral_errors, spectrum, to_canonical, to_shifted
from paper_2403_18466_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def kolmogorov_cfg(n, prec_quant="none"):
    return oracle.Config(nx=n, ny=n, tau=0.51, hidden=64, out_scale=2.0 ** -6,
                         force_kind=1, force_amp=1e-5, force_k=4, quant=prec_quant)


def initial_state(ocfg):
    u = inputs.fourier_modes_velocity(ocfg.nx, ocfg.ny, kmax=4, umax=0.01, seed=0)
    g = oracle.init_equilibrium(ocfg, np.ones((1, 1, ocfg.ny, ocfg.nx)), u[None, :, None])
    return g.astype(np.float32).astype(np.float64)


@pytest.fixture(scope="module")
def lbm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_18466_amd import lbm as m
    return m


def test_kolmogorov_128_against_oracle(lbm):
    n, steps = 128, 100
    ocfg = kolmogorov_cfg(n)
    g0 = initial_state(ocfg)
    theta = inputs.glorot_params(9, 64, seed=1)
    want = oracle.run(ocfg, g0, theta.astype(np.float64), steps)
    _, u_w, d_w = oracle.moments(ocfg, want)
    E_w = spectrum(u_w[0, :, 0])
    errs = {}
    for prec in ("fp32", "bf16"):
        L = lbm.Lattice(lib_config(ocfg, prec))
        A = torch.from_numpy(to_shifted(g0, "D2Q9").astype(np.float32)).cuda()
        out = L.step(A, torch.from_numpy(theta).cuda(), steps)
        _, u_g, diag = L.moments(out)
        torch.cuda.synchronize()
        u_g = u_g.cpu().numpy().astype(np.float64)
        E_g = spectrum(u_g[0, :, 0])
        errs[prec] = (rel_l2(u_g, u_w), *spectral_errors(E_g, E_w),
                      abs(diag[0, 1].item() / d_w[0, 1] - 1))
        L.close()
    for prec, e in errs.items():
        print(f"{prec}: velocity rel L2 {e[0]:.2e}; spectrum: weighted rel err {e[1]:.2e}, "
              f"max over energetic shells {e[2]:.2e}; kinetic energy rel err {e[3]:.2e}")
    assert errs["fp32"][0] < 1e-5 and errs["fp32"][1] < 1e-5 and errs["fp32"][3] < 1e-5
    assert errs["bf16"][0] < 1e-3 and errs["bf16"][1] < 1e-3 and errs["bf16"][3] < 1e-3


def test_kolmogorov_1024_bf16_vs_fp32(lbm):
    n, steps = 1024, 10000
    ocfg = kolmogorov_cfg(n)
    g0 = initial_state(ocfg)
    theta = torch.from_numpy(inputs.glorot_params(9, 64, seed=1)).cuda()
    res = {}
    for prec in ("fp32", "bf16"):
        L = lbm.Lattice(lib_config(ocfg, prec))
        A = torch.from_numpy(to_shifted(g0, "D2Q9").astype(np.float32)).cuda()
        out = L.step(A, theta, steps)
        _, u, diag = L.moments(out)
        torch.cuda.synchronize()
        assert int(diag[0, 2].item()) == 0
        res[prec] = (u.cpu().numpy()[0, :, 0].astype(np.float64), diag[0, 1].item())
        L.close()
    E32, E16 = spectrum(res["fp32"][0]), spectrum(res["bf16"][0])
    weighted, energetic = spectral_errors(E16, E32)
    ke_err = abs(res["bf16"][1] / res["fp32"][1] - 1)
    print(f"1024^2, {steps} steps: bf16 vs fp32 velocity rel L2 "
          f"{rel_l2(res['bf16'][0], res['fp32'][0]):.2e}; spectrum weighted rel err "
          f"{weighted:.2e}, max over energetic shells {energetic:.2e}; kinetic energy rel err "
          f"{ke_err:.2e}")
    assert ke_err < 1e-3 and weighted < 1e-2 and energetic < 1e-2
