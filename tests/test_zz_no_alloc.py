"""lbm_step_backward_static, the adjoint entry point that allocates nothing
(its partial gradients live in a static device buffer of the library),
against lbm_step_backward with a caller workspace, through the C ABI: two
calls in a row, the second on a smaller grid (the static buffer keeps the
first call's contents), results bit-identical; configurations that need
more scratch than the buffer holds are refused before anything runs."""
import ctypes

import numpy as np
import pytest

import oracle
from lbm_cases import lib_config, params, random_state, to_shifted

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


def _case(lbm, lat, shape, H, prec, seed):
    nz, ny, nx = shape
    ocfg = oracle.Config(lattice=lat, nx=nx, ny=ny, nz=nz, batch=2, tau=0.51, hidden=H,
                         out_scale=0.25)
    L = lbm.Lattice(lib_config(ocfg, prec))
    A = dev(to_shifted(random_state(ocfg, seed, scale=0.03), lat))
    lam1 = dev(to_shifted(random_state(ocfg, seed + 1, scale=1.0), lat))
    th = dev(params(ocfg.Q, H, seed=seed + 2)) if H else None
    return L, A, lam1, th


@pytest.mark.parametrize("lat,prec,H,big,small", [
    ("D2Q9", "bf16", 64, (1, 96, 200), (1, 20, 33)),   # cooperative kernel
    ("D2Q9", "fp32", 64, (1, 40, 90), (1, 9, 17)),     # per-wave kernel
    ("D3Q19", "bf16", 64, (9, 10, 70), (3, 4, 5)),
    ("D2Q9", "bgk", 0, (1, 30, 70), (1, 8, 8)),        # no parameters, no scratch
])
def test_static_adjoint_matches_workspace_adjoint(lbm, lat, prec, H, big, small):
    lib = lbm.load_library()
    for k, shape in enumerate((big, small)):
        L, A, lam1, th = _case(lbm, lat, shape, H, "fp32" if prec == "bgk" else prec, 80 + 10 * k)
        lam_ref, dth_ref = L.step_backward(A, th, lam1)
        lam = torch.full_like(lam1, float("nan"))
        dth = torch.zeros(L.n_param, dtype=torch.float32, device="cuda") if H else None
        st = lib.lbm_step_backward_static(
            L.ctx, ctypes.c_void_p(A.data_ptr()),
            ctypes.c_void_p(th.data_ptr()) if H else None,
            ctypes.c_void_p(lam1.data_ptr()), ctypes.c_void_p(lam.data_ptr()),
            ctypes.c_void_p(dth.data_ptr()) if H else None,
            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == lbm.LBM_OK, lib.lbm_last_error()
        torch.cuda.synchronize()
        print(f"{lat} {prec} H={H} {shape}: lam equal {torch.equal(lam, lam_ref)}, "
              f"dtheta equal {torch.equal(dth, dth_ref) if H else None}")
        assert torch.equal(lam, lam_ref)
        if H:
            assert torch.equal(dth, dth_ref)
            # dtheta is accumulated, as by lbm_step_backward
            lbm.lbm_step_backward_static(L.ctx, L.cfg, A, th, lam1, lam, dth)
            torch.cuda.synchronize()
            assert torch.allclose(dth, 2 * dth_ref, rtol=1e-6, atol=0)
        L.close()


def test_static_adjoint_refuses_large_scratch(lbm):
    """The SI's network keeps every activation of every node in its
    workspace: at 16^3 that is far beyond the static buffer, so the call
    returns LBM_ERR_WORKSPACE and writes nothing."""
    ocfg = oracle.Config(lattice="D3Q19", nx=16, ny=16, nz=16, tau=0.51, hidden=300, net="paper",
                         out_scale=0.25)
    L = lbm.Lattice(lib_config(ocfg, "bf16"))
    assert lbm.lbm_workspace_bytes(L.ctx) > 8 << 20
    A = torch.zeros(ocfg.state_shape, dtype=torch.float32, device="cuda")
    lam1 = torch.ones_like(A)
    lam = torch.zeros_like(A)
    th = torch.zeros(L.n_param, dtype=torch.float32, device="cuda")
    dth = torch.zeros_like(th)
    with pytest.raises(lbm.LBMError) as e:
        lbm.lbm_step_backward_static(L.ctx, L.cfg, A, th, lam1, lam, dth)
    assert e.value.status == lbm.LBM_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert not torch.any(lam) and not torch.any(dth)
    L.close()
