"""Gradient parity of the unrolled training at the training workloads' own
shapes, in the launch configurations bench.py times.

* D2Q9, 8 fields of 256 x 256, tau' 0.50125, 9->64->64->9 tanh (s_out
  2^-10), 32 unrolled steps with a checkpoint every 8, velocity-MSE loss: the
  GPU gradient (cooperative 16-bit adjoint, segments through
  lbm_step_backward_seq) against the oracle's reverse pass over the whole
  batch.  fp32 against fp64; bf16 against the oracle reproducing the kernels'
  own operand rounding, and its error against fp64 as a multiple of the
  plain-rounding scheme's.

* D3Q19 256^3, tau 0.51, 19->64->64->19 tanh (s_out 2^-6), 8 forward and 8
  adjoint steps (one checkpoint segment) with the population loss of the
  SI's recipe on a few sampled nodes.  Eight steps move information at most
  eight nodes, so each sampled node's loss and gradient are those of a
  periodic crop of radius 12 around it: the oracle runs the crops, the sum of
  their parameter gradients is the full gradient, and the gradient with
  respect to the initial state must match inside each crop's light cone and
  vanish everywhere else.
"""
import numpy as np
import pytest

import oracle
from lbm_cases import exact_config, kernel_emulation, lib_config, plain_rounding_config, rel_l2
from paper_2403_18466_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def oracle_threads():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    n = oracle.set_threads(oracle.default_threads())
    yield n
    oracle.set_threads(1)


def shifted(g, c):
    A = np.empty(g.shape, np.float32)
    for q in range(g.shape[1]):
        A[:, q] = np.roll(g[:, q], shift=(-c[q, 2], -c[q, 1], -c[q, 0]), axis=(1, 2, 3))
    return A


def canonical(A, c):
    g = np.empty(A.shape, np.float64)
    for q in range(A.shape[1]):
        g[:, q] = np.roll(A[:, q], shift=(c[q, 2], c[q, 1], c[q, 0]), axis=(1, 2, 3))
    return g


def log(msg):
    print(msg, flush=True)


# ------------------------------------------------------ D2Q9 8 x 256^2, T = 32
@pytest.fixture(scope="module")
def train_case():
    n, B, T = 256, 8, 32
    ocfg = oracle.Config(nx=n, ny=n, batch=B, tau=0.50125, hidden=64, out_scale=2.0 ** -10)
    u = np.stack([inputs.solenoidal_spectrum_velocity((n, n), 16.0, 0.02, 100 + b)
                  for b in range(B)])
    g0 = oracle.init_equilibrium(ocfg, np.ones((B, 1, n, n)), u[:, :, None])
    g0 = g0.astype(np.float32).astype(np.float64)
    # target velocity: the fields' own velocities, damped and shifted by two
    # nodes, so that the loss gradient reaches every parameter block
    ut = (0.9 * np.roll(u, 2, axis=-1))[:, :, None].astype(np.float32).astype(np.float64)
    theta = inputs.glorot_params(9, 64, seed=1)
    theta[64 * 9:64 * 10] = np.random.default_rng(3).uniform(-0.1, 0.1, 64).astype(np.float32)
    log("  oracle: fp64 unrolled gradient, 8 x 256^2, 32 steps ...")
    exact = oracle.unrolled_loss_and_grad(ocfg, g0, theta.astype(np.float64), ut, T, ckpt=8)
    return ocfg, g0, ut, theta, T, exact


def gpu_unrolled(ocfg, prec, g0, ut, theta, T, ckpt, c):
    from paper_2403_18466_amd import lbm, training
    L = lbm.Lattice(lib_config(ocfg, prec))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    loss, dth, dA0 = training.unrolled_loss_and_grad(L, dev(shifted(g0, c)), dev(theta), dev(ut),
                                                     T, ckpt=ckpt, want_dA0=True)
    torch.cuda.synchronize()
    out = (float(loss.cpu()[0]), dth.cpu().numpy().astype(np.float64),
           canonical(dA0.cpu().numpy(), c))
    L.close()
    return out


BLOCKS9 = [0, 576, 640, 4736, 4800, 5376, 5385]  # W1 b1 W2 b2 W3 b3 at Q = 9, H = 64
BLOCKS19 = [0, 1216, 1280, 5376, 5440, 6656, 6675]  # the same at Q = 19


def block_errors(got, want, blocks):
    """Per parameter block: (norm of the block / norm of the whole gradient,
    error / max(norm of the block, 1e-3 norm of the whole gradient)).  The
    floor keeps blocks that are nearly zero by structure from being judged on
    their cancellation: the b3 gradient is the sum of the projected adjoint
    over all nodes, which conservation drives towards zero."""
    tot = np.linalg.norm(want)
    out = []
    for a, b in zip(blocks[:-1], blocks[1:]):
        nb = np.linalg.norm(want[a:b])
        out.append((nb / tot, np.linalg.norm(got[a:b] - want[a:b]) / max(nb, 1e-3 * tot)))
    return out


def fmt_blocks(be):
    return " ".join(f"[{n:.0e}: {e:.1e}]" for n, e in be)


# fp16 is not run here: at this loss scale the adjoint's network operands
# (dy = s_out / tau x the projected adjoint, about 1e-11) lie below the
# smallest fp16 subnormal (6e-8) and flush to zero, so the fp16 network's
# gradient vanishes; bf16 has the float32 exponent range.  fp16 adjoints are
# checked at unit-scale lam (test_gpu_backward.py).
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_cfg4_unrolled_gradient_8x256(train_case, prec):
    ocfg, g0, ut, theta, T, (xl, xdth, xlam) = train_case
    c9 = oracle.tables("D2Q9")[0]
    gl, gdth, glam = gpu_unrolled(ocfg, prec, g0, ut, theta, T, 8, c9)
    if prec == "fp32":
        e, el = rel_l2(gdth, xdth), rel_l2(glam, xlam)
        be = block_errors(gdth, xdth, BLOCKS9)
        log(f"8 x 256^2, 32 steps, fp32: loss rel {abs(gl / xl - 1):.1e}; dtheta rel L2 {e:.2e}, "
            f"blocks [size: error] {fmt_blocks(be)}; dL/dA0 rel L2 {el:.2e}")
        assert abs(gl / xl - 1) < 1e-5 and e < 1e-4 and el < 1e-4
        # per block, absolute error within 1e-4 of the block plus 1e-5 of the
        # whole gradient (b3 is 5e-6 of the whole: conservation makes the sum
        # of the projected adjoint nearly vanish, and float32 summation over
        # 16.8M node-steps leaves it at 1.7e-3 of its own size)
        tot = np.linalg.norm(xdth)
        for a, b in zip(BLOCKS9[:-1], BLOCKS9[1:]):
            assert (np.linalg.norm(gdth[a:b] - xdth[a:b])
                    <= 1e-4 * np.linalg.norm(xdth[a:b]) + 1e-5 * tot)
        return
    th64 = theta.astype(np.float64)
    kcfg, kth = kernel_emulation(ocfg, theta, prec)
    log("  oracle: kernel-scheme unrolled gradient ...")
    kl, kdth, klam = oracle.unrolled_loss_and_grad(kcfg, g0, kth, ut, T, ckpt=8)
    log("  oracle: plain-rounding unrolled gradient ...")
    pl, pdth, plam = oracle.unrolled_loss_and_grad(plain_rounding_config(ocfg, prec), g0, th64,
                                                   ut, T, ckpt=8)
    e_k = rel_l2(gdth, kdth)
    r_th = np.linalg.norm(gdth - xdth) / np.linalg.norm(pdth - xdth)
    r_lam = np.linalg.norm(glam - xlam) / np.linalg.norm(plam - xlam)
    log(f"  blocks vs kernel scheme {fmt_blocks(block_errors(gdth, kdth, BLOCKS9))}; plain "
        f"rounding vs fp64 {fmt_blocks(block_errors(pdth, xdth, BLOCKS9))}")
    log(f"8 x 256^2, 32 steps, {prec}: dtheta rel L2 vs kernel scheme {e_k:.2e}, vs fp64 "
        f"{rel_l2(gdth, xdth):.2e} (plain rounding {rel_l2(pdth, xdth):.2e}); |gpu-fp64| / "
        f"|plain-fp64|: dtheta {r_th:.2f}, dL/dA0 {r_lam:.2f}; loss rel vs fp64 "
        f"{abs(gl / xl - 1):.1e}")
    assert e_k < 3e-2
    assert r_th < 4.0 and r_lam < 4.0
    assert rel_l2(gdth, xdth) < 3e-2 and abs(gl / xl - 1) < 1e-3


# ------------------------------------------- D3Q19 256^3, 8 + 8 steps, sampled
N5, T5, R = 256, 8, 12


def _crop_index(z, y, x, n, r):
    ax = [np.arange(v - r, v + r + 1) % n for v in (z, y, x)]
    return np.ix_(ax[0], ax[1], ax[2])


@pytest.fixture(scope="module")
def cfg5_case():
    n = N5
    ocfg = oracle.Config(lattice="D3Q19", nx=n, ny=n, nz=n, tau=0.51, hidden=64,
                         out_scale=2.0 ** -6)
    u = inputs.solenoidal_spectrum_velocity((n, n, n), 4.0, 0.04, seed=0)
    g0 = oracle.init_equilibrium(ocfg, np.ones((1, n, n, n)), u[None]).astype(np.float32)
    del u
    ut = inputs.solenoidal_spectrum_velocity((n, n, n), 4.0, 0.04, seed=7)
    gt = oracle.init_equilibrium(ocfg, np.ones((1, n, n, n)), ut[None]).astype(np.float32)
    del ut
    theta = inputs.glorot_params(19, 64, seed=1)
    # sampled nodes more than 2 (R + 1) apart (periodic Chebyshev distance)
    rng = np.random.default_rng(42)
    pts = []
    while len(pts) < 6:
        p = rng.integers(0, n, 3)
        ok = True
        for q in pts:
            d = np.abs(p - q)
            d = np.minimum(d, n - d)
            ok &= d.max() > 2 * (R + 1)
        if ok:
            pts.append(p)
    pts[0] = np.array([0, 0, 0])  # a corner: every crop axis wraps
    return ocfg, g0, gt, theta, [tuple(int(v) for v in p) for p in pts]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_d3q19_256_unrolled_8_steps_sampled(cfg5_case, prec):
    from paper_2403_18466_amd import lbm, training
    ocfg, g0, gt, theta, pts = cfg5_case
    n = N5
    c19 = oracle.tables("D3Q19")[0]
    flat = np.array([(z * n + y) * n + x for z, y, x in pts], np.int32)
    L = lbm.Lattice(lib_config(ocfg, prec))
    A0 = torch.from_numpy(shifted(g0, c19)).cuda()
    Tt = torch.from_numpy(shifted(gt, c19)).cuda()
    nodes = torch.from_numpy(flat).cuda()
    loss, dth, dA0 = training.unrolled_loss_and_grad(
        L, A0, torch.from_numpy(theta).cuda(), None, T5, ckpt=8, want_dA0=True,
        loss_fn=lambda A: L.loss_population_sse(A, Tt, nodes))
    torch.cuda.synchronize()
    gl, gdth = float(loss.cpu()[0]), dth.cpu().numpy().astype(np.float64)
    del A0, Tt
    glam = canonical(dA0.cpu().numpy(), c19)
    L.close()
    del dA0
    torch.cuda.empty_cache()
    # the oracle on each node's crop, three ways for bf16
    m = 2 * R + 1
    ccfg = oracle.Config(lattice="D3Q19", nx=m, ny=m, nz=m, tau=0.51, hidden=64,
                         out_scale=2.0 ** -6)
    centre = np.array([((R * m + R) * m + R)], np.int32)
    th64 = theta.astype(np.float64)
    variants = {"exact": (exact_config(ccfg), th64)}
    if prec != "fp32":
        variants["kernel"] = kernel_emulation(ccfg, theta, prec)
        variants["plain"] = (plain_rounding_config(ccfg, prec), th64)
    res = {k: [0.0, np.zeros_like(gdth), []] for k in variants}
    inside = np.zeros((n, n, n), bool)
    for z, y, x in pts:
        idx = _crop_index(z, y, x, n, R)
        gc = g0[0][(slice(None),) + idx][None].astype(np.float64)
        tc = gt[0][(slice(None),) + idx][None].astype(np.float64)
        for k, (cf, th) in variants.items():
            l, d, lam = oracle.unrolled_loss_and_grad(
                cf, gc, th, None, T5, ckpt=8,
                loss_fn=lambda g, cf=cf, tc=tc: oracle.loss_population_sse(cf, g, tc, centre))
            res[k][0] += l
            res[k][1] += d
            res[k][2].append(lam)
        inside[idx] = True
    # dL/dA0: inside each crop it is the crop's (the light cone of 8 steps
    # stays 3 nodes inside the crop), outside every crop it is exactly 0
    got_in = [glam[0][(slice(None),) + _crop_index(z, y, x, n, R)] for z, y, x in pts]
    outside = float(np.abs(glam[0][:, ~inside]).max())
    xl, xdth = res["exact"][0], res["exact"][1]
    e_lam = rel_l2(np.concatenate([a.ravel() for a in got_in]),
                   np.concatenate([a[0].ravel() for a in res["exact"][2]]))
    msg = (f"D3Q19 256^3, 8 + 8 steps, {prec}, {len(pts)} sampled nodes: loss rel "
           f"{abs(gl / xl - 1):.1e}; dtheta rel L2 vs fp64 {rel_l2(gdth, xdth):.2e}; dL/dA0 in "
           f"the crops vs fp64 {e_lam:.2e}, max outside {outside:.1e}")
    assert outside == 0.0
    if prec == "fp32":
        log(msg + f"; blocks [size: error] {fmt_blocks(block_errors(gdth, xdth, BLOCKS19))}")
        assert abs(gl / xl - 1) < 1e-5 and rel_l2(gdth, xdth) < 1e-4 and e_lam < 1e-4
        return
    kdth, pdth = res["kernel"][1], res["plain"][1]
    e_k = rel_l2(gdth, kdth)
    r_th = np.linalg.norm(gdth - xdth) / np.linalg.norm(pdth - xdth)
    log(f"  blocks [size: error] gpu vs kernel scheme {fmt_blocks(block_errors(gdth, kdth, BLOCKS19))}"
        f"; gpu vs fp64 {fmt_blocks(block_errors(gdth, xdth, BLOCKS19))}; plain rounding vs "
        f"fp64 {fmt_blocks(block_errors(pdth, xdth, BLOCKS19))}")
    log(msg + f"; dtheta vs kernel scheme {e_k:.2e}; |gpu-fp64| / |plain-fp64| {r_th:.2f}")
    # The kernel rounds its backward operands (dy, d2, d1) to the format
    # before each product, and forms the bias gradients from those operands
    # (b1 through its constant input column, b2 and b3 as products with a
    # ones fragment); the emulation passes rounding straight through.  With
    # the loss on a handful of nodes the bias gradients are sums with heavy
    # cancellation (float32 already shows 5x the weight blocks' relative error
    # on them), which amplifies that per-node 2^-9 rounding: measured 0.14
    # (b1), 0.14 (b2) and 0.079 (b3) of the block, against 0.003 for the
    # plain-rounding scheme; the weight blocks 0.010-0.015, dL/dA0 3.3e-4.
    assert abs(gl / xl - 1) < 1e-3 and e_lam < 1e-3
    bias = (BLOCKS19[1], BLOCKS19[3], BLOCKS19[5])
    for (a, b), (_, err) in zip(zip(BLOCKS19[:-1], BLOCKS19[1:]),
                                block_errors(gdth, kdth, BLOCKS19)):
        assert err < (0.25 if a in bias else 0.03)
