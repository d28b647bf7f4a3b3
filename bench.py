"""Throughput of the learned-collision lattice Boltzmann step on one MI355X.

Workload: D2Q9 periodic 4096 x 4096, tau = 0.51, populations stored as
float32 deviations f - w rho0, collision = BGK + (s_out/tau) * MLP 9->64->64->9
(tanh; Glorot weights from seed 1, s_out = 2^-6) projected to conserve mass and
momentum; initial velocity from the random-Fourier-mode recipe (|k| <= 4,
max |u| = 0.05, seed 0).  One step = one stream-collide pass over the field
(one kernel launch).  The headline runs the network on bf16 matrix cores with
float32 accumulation; fp16, plain fp32 and plain BGK are timed at the same
size for comparison.

Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N = 4096
TAU = 0.51
S_OUT = 2.0 ** -6
HIDDEN = 64
BYTES_PER_LUP = 72            # 9 float32 read + 9 float32 written per node
TANH_PER_LUP = 2 * HIDDEN     # two hidden tanh layers
TRANS_PER_TANH = 2            # exp2 + reciprocal: no tanh instruction exists
HBM_PEAK = 8.0e12             # B/s, MI355X HBM3E
SIMD_CYCLES = 256 * 4 * 2.4e9  # 256 CUs x 4 SIMDs x 2.4 GHz
# per SIMD and clock: 16 FP32 VALU lanes (packed FP32 not used), 8 transcendental lanes
FP32_LANES, TRANS_LANES = 16, 8
TRANS_PEAK = SIMD_CYCLES * TRANS_LANES
# Minimal ALU work of the activation per LUP: 128 tanh, each one exp2 + one
# reciprocal (transcendental) and two FP32 ops (1 + e, 1 - 2r; the argument
# scale 2 log2 e rides in the bf16 weights), plus one packed conversion per
# two activations to the operand format.  In SIMD-cycles per LUP:
ACT_CYCLES_PER_LUP = (TANH_PER_LUP * (TRANS_PER_TANH / TRANS_LANES + 2 / FP32_LANES)
                      + TANH_PER_LUP / 2 / FP32_LANES)
ACT_PEAK_LUPS = SIMD_CYCLES / ACT_CYCLES_PER_LUP


# The adjoint step (H = 64, D2Q9): it reads A^n (pulled) and lam^{n+1} and
# writes lam^n (pushed), 3 x 36 B; its network work is the forward recompute
# (W1, W2), the data gradient (W3^T, W2^T, W1^T) and the weight gradients
# (dW3, dW2, dW1): 2 x (5 x 64 x 9 + 3 x 64 x 64) flops.  Its minimal ALU work
# adds to the forward's activation the tanh derivative 1 - t^2 times the
# incoming gradient (2 FP32 ops for each of the 128 hidden values) and the
# conversion of d1, d2 to the operand format (64 packed conversions).
ADJ_BYTES_PER_LUP = 108
ADJ_FLOP_PER_LUP = 2 * (5 * 64 * 9 + 3 * 64 * 64)
ADJ_ACT_CYCLES_PER_LUP = ACT_CYCLES_PER_LUP + TANH_PER_LUP * 2 / FP32_LANES + TANH_PER_LUP / 2 / FP32_LANES
ADJ_ACT_PEAK_LUPS = SIMD_CYCLES / ADJ_ACT_CYCLES_PER_LUP


# HBM bytes per launch of the bf16 step from rocprofv3 FETCH_SIZE / WRITE_SIZE,
# each scaled by the factor a plain copy of known size gives (2.000 / 1.000);
# None until taken for the current kernel (profiles/).
TRAFFIC_BYTES = 1.2294e9


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=200)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-train", action="store_true", help="skip the training-step timing")
    p.add_argument("--no-d3q19", action="store_true", help="skip the D3Q19 256^3 timing")
    p.add_argument("--no-wide", action="store_true",
                   help="skip the D3Q19 256^3 timing of the 19-300-300-100-19 network")
    p.add_argument("--no-si", action="store_true",
                   help="skip the timing of the SI's pipeline (DNS, wide-network training)")
    p.add_argument("--variants", default="bf16,fp16,fp32,bgk,smag")
    p.add_argument("--settle", type=float, default=2.0,
                   help="seconds of untimed steps before each D2Q9 leg's warm-up (clock settle)")
    return p.parse_args()


def make_state(torch, lbm, inputs, L):
    u = inputs.fourier_modes_velocity(N, N, kmax=4, umax=0.05, seed=0).astype("float32")
    ud = torch.from_numpy(u).reshape(1, 2, 1, N, N).cuda()
    rho = torch.ones((1, 1, N, N), dtype=torch.float32, device="cuda")
    return L.init(rho, ud)


SMAG_CS = 0.17  # Smagorinsky constant of the comparison collision


SETTLE_S = 2.0  # untimed running of each leg before its warm-up, so clocks are steady


def settle(torch, lbm, L, cfg, A, B, theta, seconds, stream):
    """Run the leg's own step untimed for `seconds` of wall time (chunks of
    20 steps): the GPU's clocks ramp over the first few hundred
    milliseconds of work.  Leaves the state in A."""
    t0 = time.perf_counter()
    steps = 0
    while time.perf_counter() - t0 < seconds:
        lbm.lbm_step(L.ctx, cfg, A, B, theta, 20, stream)
        torch.cuda.synchronize()
        steps += 20
    return steps


def time_variant(torch, lbm, inputs, prec, hidden, steps, warmup, A0, collision="bgk",
                 settle_s=SETTLE_S):
    cfg = lbm.Config(nx=N, ny=N, tau=TAU, hidden=hidden, mlp_prec=prec, out_scale=S_OUT,
                     collision=collision, smag_cs=SMAG_CS if collision == "smagorinsky" else 0.0)
    L = lbm.Lattice(cfg)
    theta = None
    if hidden:
        theta = torch.from_numpy(inputs.glorot_params(9, hidden, seed=1)).cuda()
    A = A0.clone()
    B = torch.empty_like(A)
    stream = torch.cuda.current_stream()
    settle_steps = settle(torch, lbm, L, cfg, A, B, theta, settle_s, stream)
    A.copy_(A0)
    if warmup > 0:
        lbm.lbm_step(L.ctx, cfg, A, B, theta, warmup, stream)
    torch.cuda.synchronize()
    # the timed steps run as up to 5 back-to-back chunks on one stream, with
    # an event between chunks: the total gives ms/step, the chunks the spread
    nchunk = min(5, steps)
    sizes = [steps // nchunk + (1 if i < steps % nchunk else 0) for i in range(nchunk)]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nchunk + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    src, other = A, B
    for i, k in enumerate(sizes):
        out = lbm.lbm_step(L.ctx, cfg, src, other, theta, k, stream)
        src, other = (out, B if out is A else A)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[0].elapsed_time(ev[-1]) / steps
    chunk = sorted(ev[i].elapsed_time(ev[i + 1]) / k for i, k in enumerate(sizes))
    _, _, diag = L.moments(out)
    torch.cuda.synchronize()
    d = diag.cpu().numpy()[0]
    L.close()
    return {"ms_per_step": ms, "mlups": N * N / (ms * 1e-3) / 1e6, "wall_s": wall,
            "settle_steps": settle_steps,
            "chunk_ms_per_step": {"median": chunk[len(chunk) // 2], "min": chunk[0],
                                  "max": chunk[-1], "chunks": nchunk},
            "mass": float(d[0]), "kinetic_energy": float(d[1]), "nonfinite": int(d[2])}


def time_kolmogorov(torch, lbm, inputs, steps):
    """The Kolmogorov workload's step: D2Q9 1024^2, F_x = 1e-5 sin(2 pi 4 y /
    1024) through the exact difference method, tau 0.51, 9->64->64->9 tanh
    (s_out 2^-6), bf16 and fp32 networks.  Its two state arrays (75 MB) stay
    in the 256 MB last-level cache, so this is not an HBM-roofline figure."""
    n = 1024
    u = inputs.fourier_modes_velocity(n, n, kmax=4, umax=0.01, seed=0).astype("float32")
    ud = torch.from_numpy(u).reshape(1, 2, 1, n, n).cuda()
    res = {}
    for prec in ("bf16", "fp32"):
        cfg = lbm.Config(nx=n, ny=n, tau=TAU, hidden=HIDDEN, mlp_prec=prec, out_scale=S_OUT,
                         force_kind=lbm.LBM_FORCE_KOLMOGOROV, force_k=4, force_amp=1e-5)
        L = lbm.Lattice(cfg)
        A = L.init(torch.ones((1, 1, n, n), device="cuda"), ud)
        B = torch.empty_like(A)
        theta = torch.from_numpy(inputs.glorot_params(9, HIDDEN, seed=1)).cuda()
        lbm.lbm_step(L.ctx, cfg, A, B, theta, 200)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        lbm.lbm_step(L.ctx, cfg, A, B, theta, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[prec] = {"ms_per_step": ms, "mlups": n * n / (ms * 1e-3) / 1e6}
        L.close()
    res["workload"] = ("D2Q9 1024^2 Kolmogorov forcing A 1e-5, k 4 (EDM), tau 0.51, 9-64-64-9 "
                       "tanh; cache-resident")
    print(f"# kolmogorov 1024^2: bf16 {res['bf16']['mlups']:.0f} MLUPS, fp32 "
          f"{res['fp32']['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    return res


def time_training(torch, lbm, inputs, prec, reps, ckpt=8):
    """One training step of the unrolled-training workload: 8 fields of
    256 x 256, 32 unrolled steps with a checkpoint every 8 (forward, segment
    recompute, 32 adjoint steps, loss gradient, Adam), tau' = 0.50125,
    network 9->64->64->9.  Inputs are synthetic (equilibria of random
    solenoidal fields); returns the median wall time of `reps` steps and the
    adjoint-kernel throughput.  ckpt = 32 keeps the whole trajectory (31
    states of 18.9 MB) and recomputes nothing."""
    from paper_2403_18466_amd import training
    import numpy as np
    n, B = 256, 8
    cfg = lbm.Config(nx=n, ny=n, batch=B, tau=0.50125, hidden=HIDDEN, mlp_prec=prec,
                     out_scale=2.0 ** -10)
    L = lbm.Lattice(cfg)
    u = np.stack([inputs.solenoidal_spectrum_velocity((n, n), 16.0, 0.02, 100 + b)
                  for b in range(B)]).astype("float32")
    ud = torch.from_numpy(u).reshape(B, 2, 1, n, n).cuda()
    A0 = L.init(torch.ones((B, 1, n, n), device="cuda"), ud)
    ut = torch.from_numpy(0.9 * u).reshape(B, 2, 1, n, n).cuda().contiguous()
    theta = torch.from_numpy(inputs.glorot_params(9, HIDDEN, seed=1)).cuda()
    opt = training.Adam(theta, lr=1e-4, weight_decay=1e-6)
    times = []
    for r in range(reps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss, dth, _ = training.unrolled_loss_and_grad(L, A0, theta, ut, 32, ckpt)
        opt.step(dth)
        torch.cuda.synchronize()
        if r >= 2:
            times.append(time.perf_counter() - t0)
    # adjoint kernel alone
    lam = torch.randn_like(A0)
    out = torch.empty_like(A0)
    dtheta = torch.zeros(L.n_param, device="cuda")
    ws = L.workspace()
    for _ in range(3):
        lbm.lbm_step_backward(L.ctx, cfg, A0, theta, lam, out, dtheta, ws)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(20):
        lbm.lbm_step_backward(L.ctx, cfg, A0, theta, lam, out, dtheta, ws)
    e1.record()
    torch.cuda.synchronize()
    ms_bwd = e0.elapsed_time(e1) / 20
    L.close()
    times.sort()
    return {"train_step_ms": 1e3 * times[len(times) // 2],
            "adjoint_ms": ms_bwd, "adjoint_mlups": n * n * B / (ms_bwd * 1e-3) / 1e6}


def time_d3q19(torch, lbm, inputs, steps):
    """The 3-D workload: D3Q19 256^3, tau 0.51, 19->64->64->19 tanh (s_out
    2^-6) on bf16 matrix cores, initial field with E(k) ~ k^4 exp(-2 (k/4)^2),
    u_rms 0.04 per component; plain BGK at the same size; the adjoint step."""
    import numpy as np
    n = 256
    u = inputs.solenoidal_spectrum_velocity((n, n, n), 4.0, 0.04, seed=0).astype("float32")
    ud = torch.from_numpy(u).reshape(1, 3, n, n, n).cuda()
    del u
    res = {}
    for name, hidden, coll in (("bf16", HIDDEN, "bgk"), ("bgk", 0, "bgk"),
                               ("smag", 0, "smagorinsky")):
        cfg = lbm.Config(lattice="D3Q19", nx=n, ny=n, nz=n, tau=TAU, hidden=hidden,
                         mlp_prec="bf16", out_scale=S_OUT, collision=coll,
                         smag_cs=SMAG_CS if coll == "smagorinsky" else 0.0)
        L = lbm.Lattice(cfg)
        A = L.init(torch.ones((1, n, n, n), device="cuda"), ud)
        B = torch.empty_like(A)
        theta = torch.from_numpy(inputs.glorot_params(19, HIDDEN, seed=1)).cuda() if hidden else None
        lbm.lbm_step(L.ctx, cfg, A, B, theta, 20)  # warm-up: clocks reach their steady state
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        out = lbm.lbm_step(L.ctx, cfg, A, B, theta, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        _, _, diag = L.moments(out, want_fields=False)
        r = {"ms_per_step": ms, "mlups": n ** 3 / (ms * 1e-3) / 1e6,
             "hbm_frac": 152 * n ** 3 / (ms * 1e-3) / HBM_PEAK, "nonfinite": int(diag[0, 2].item())}
        if hidden:
            lam = torch.randn_like(A)
            lam0 = torch.empty_like(A)
            dth = torch.zeros(L.n_param, device="cuda")
            ws = L.workspace()
            lbm.lbm_step_backward(L.ctx, cfg, A, theta, lam, lam0, dth, ws)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(8):
                lbm.lbm_step_backward(L.ctx, cfg, A, theta, lam, lam0, dth, ws)
            e1.record()
            torch.cuda.synchronize()
            r["adjoint_ms"] = e0.elapsed_time(e1) / 8
            r["adjoint_mlups"] = n ** 3 / (r["adjoint_ms"] * 1e-3) / 1e6
        if hidden:
            r["training_step"] = time_d3q19_training(torch, lbm, inputs, L, cfg, A, ud)
        del A, B
        L.close()
        res[name] = r
        print(f"# d3q19 256^3 {name}: {r['mlups']:.0f} MLUPS" +
              (f", adjoint {r['adjoint_mlups']:.0f} MLUPS" if hidden else ""), file=sys.stderr, flush=True)
    return res


def time_d3q19_training(torch, lbm, inputs, L, cfg, A0, ud, reps=5):
    """One training step of the 3-D workload: 8 forward steps of 256^3 kept as
    one checkpoint segment, the velocity-MSE loss against a target field, 8
    adjoint steps through lbm_step_backward_seq, and Adam; median wall time
    of `reps` steps after two untimed ones."""
    from paper_2403_18466_amd import training
    theta = torch.from_numpy(inputs.glorot_params(19, HIDDEN, seed=1)).cuda()
    ut = (0.9 * ud).contiguous()
    opt = training.Adam(theta.clone(), lr=1e-4, weight_decay=1e-6)
    times = []
    for r in range(reps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss, dth, _ = training.unrolled_loss_and_grad(L, A0, opt.p, ut, 8, 8)
        opt.step(dth)
        torch.cuda.synchronize()
        if r >= 2:
            times.append(time.perf_counter() - t0)
    times.sort()
    ms = 1e3 * times[len(times) // 2]
    return {"ms": ms, "workload": "D3Q19 256^3 bf16, 8 forward + 8 adjoint steps (one "
            "checkpoint segment), velocity-MSE loss, Adam", "nonfinite_loss": not bool(
                torch.isfinite(loss).all())}


# multiply-add flops of the 19 -> 300 -> 300 -> 100 -> 19 network per node
WIDE_FLOP_PER_LUP = 2 * (19 * 300 + 300 * 300 + 300 * 100 + 100 * 19)
MFMA_PEAK = {"bf16": 2.5e15, "fp16": 2.5e15}  # dense, MI355X


def time_wide(torch, lbm, inputs, steps):
    """The SI's collision network, 19 -> 300 -> 300 -> 100 -> 19 with
    LeakyReLU, on D3Q19 256^3 (tau 0.51, s_out 2^-6, Glorot weights from seed
    1, the same solenoidal initial field as the 3-D workload), bf16 and fp16
    matrix cores.  This path is bound by the matrix cores: the roofline is
    the network's algorithmic flops against the dense peak."""
    n = 256
    u = inputs.solenoidal_spectrum_velocity((n, n, n), 4.0, 0.04, seed=0).astype("float32")
    ud = torch.from_numpy(u).reshape(1, 3, n, n, n).cuda()
    del u
    theta = torch.from_numpy(inputs.glorot_params_net(inputs.net_widths(19, 0, "paper"), 1)).cuda()
    res = {}
    for prec in ("bf16", "fp16"):
        cfg = lbm.Config(lattice="D3Q19", nx=n, ny=n, nz=n, tau=TAU, hidden=300, net="paper",
                         mlp_prec=prec, out_scale=S_OUT)
        L = lbm.Lattice(cfg)
        A = L.init(torch.ones((1, n, n, n), device="cuda"), ud)
        B = torch.empty_like(A)
        lbm.lbm_step(L.ctx, cfg, A, B, theta, 2)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        out = lbm.lbm_step(L.ctx, cfg, A, B, theta, steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        _, _, diag = L.moments(out, want_fields=False)
        lups = n ** 3 / (ms * 1e-3)
        flops = WIDE_FLOP_PER_LUP * lups
        res[prec] = {"ms_per_step": ms, "mlups": lups / 1e6, "nonfinite": int(diag[0, 2].item()),
                     "roofline": {"bound": "mfma", "achieved": flops / 1e12,
                                  "peak": MFMA_PEAK[prec] / 1e12, "unit": "TFLOP/s",
                                  "frac": flops / MFMA_PEAK[prec],
                                  "hbm_frac": 152 * lups / HBM_PEAK}}
        del A, B
        L.close()
        print(f"# wide network D3Q19 256^3 {prec}: {lups / 1e6:.0f} MLUPS, "
              f"{flops / 1e12:.0f} TFLOP/s", file=sys.stderr, flush=True)
    res["workload"] = ("D3Q19 256^3, collision network 19-300-300-100-19 LeakyReLU (the SI's), "
                       "tau 0.51, s_out 2^-6, weights streamed through LDS, includes the "
                       "per-call weight packing")
    return res


# algorithmic flops per node of one adjoint step of the wide network: the
# hidden layers recomputed, the input gradients of all four layers, and the
# weight gradients
WIDE_ADJ_FLOP_PER_LUP = 2 * (19 * 300 + 300 * 300 + 300 * 100) + 2 * WIDE_FLOP_PER_LUP


def time_si_pipeline(torch, lbm, inputs):
    """The SI's training recipe at its sizes, timed on synthetic states: the
    forced D3Q19 128^3 DNS step (BGK, three-component sine force), and one
    training epoch of the 19-300-300-100-19 network on the 32^3 coarse grid
    (12 unrolled steps, checkpoint every 4, population loss on 512 nodes,
    Adam), with the adjoint step alone."""
    import numpy as np
    from paper_2403_18466_amd import training
    res = {}
    n = 128
    cfg = lbm.Config(lattice="D3Q19", nx=n, ny=n, nz=n, tau=0.5032,
                     force_kind=lbm.LBM_FORCE_SINE3, force_k=1, force_amp=5e-6)
    L = lbm.Lattice(cfg)
    u = inputs.solenoidal_spectrum_velocity((n, n, n), 4.0, 0.04, seed=0).astype("float32")
    A = L.init(torch.ones((1, n, n, n), device="cuda"), torch.from_numpy(u)[None].cuda())
    B = torch.empty_like(A)
    lbm.lbm_step(L.ctx, cfg, A, B, None, 10)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    lbm.lbm_step(L.ctx, cfg, A, B, None, 200)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 200
    res["dns_128_forced_bgk"] = {"ms_per_step": ms, "mlups": n ** 3 / (ms * 1e-3) / 1e6}
    L.close()
    del A, B
    m = 32
    cc = lbm.Config(lattice="D3Q19", nx=m, ny=m, nz=m, tau=0.5008, force_kind=lbm.LBM_FORCE_SINE3,
                    force_k=1, force_amp=2e-5, hidden=300, net="paper", mlp_prec="bf16")
    L = lbm.Lattice(cc)
    u = inputs.solenoidal_spectrum_velocity((m, m, m), 4.0, 0.04, seed=1).astype("float32")
    A0 = L.init(torch.ones((1, m, m, m), device="cuda"), torch.from_numpy(u)[None].cuda())
    T = L.step(A0, torch.zeros(L.n_param, device="cuda"), 12)
    theta = torch.from_numpy(inputs.glorot_params_net(inputs.net_widths(19, 0, "paper"), 1)).cuda()
    opt = training.Adam(theta, lr=1e-4, weight_decay=1e-6)
    rng = np.random.default_rng(0)
    nodes = torch.from_numpy(rng.choice(m ** 3, 512, replace=False).astype(np.int32)).cuda()

    def epoch():
        _, dth, _ = training.unrolled_loss_and_grad(
            L, A0, theta, None, 12, 4, loss_fn=lambda A: L.loss_population_sse(A, T, nodes))
        opt.step(dth)

    for _ in range(3):
        epoch()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        epoch()
    torch.cuda.synchronize()
    res["wide_training_epoch_ms"] = (time.perf_counter() - t0) / 20 * 1e3
    lam = torch.randn_like(A0)
    lam0 = torch.empty_like(A0)
    dth = torch.zeros(L.n_param, device="cuda")
    ws = L.workspace()
    lbm.lbm_step_backward(L.ctx, cc, A0, theta, lam, lam0, dth, ws)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(20):
        lbm.lbm_step_backward(L.ctx, cc, A0, theta, lam, lam0, dth, ws)
    e1.record()
    torch.cuda.synchronize()
    ams = e0.elapsed_time(e1) / 20
    res["wide_adjoint_32"] = {"ms": ams, "mlups": m ** 3 / (ams * 1e-3) / 1e6,
                              "tflops_algorithmic": WIDE_ADJ_FLOP_PER_LUP * m ** 3 / (ams * 1e-3) / 1e12}
    L.close()
    res["workload"] = ("SI recipe: forced D3Q19 128^3 DNS (tau 0.5032, F 5e-6); training epoch of "
                       "the 19-300-300-100-19 network on 32^3 (tau' 0.5008, L_T 12, checkpoint 4, "
                       "|S| 512, bf16, Adam) on synthetic states")
    print(f"# SI pipeline: DNS 128^3 {res['dns_128_forced_bgk']['mlups']:.0f} MLUPS, wide training "
          f"epoch {res['wide_training_epoch_ms']:.2f} ms, wide adjoint 32^3 {ams:.3f} ms",
          file=sys.stderr, flush=True)
    return res


def host_cpu():
    """CPU model and the number of CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return model, ncpu, os.cpu_count() or 1


def cpu_baseline():
    """The FP64 oracle (serial C) beside the GPU, on the machine's host CPU:

    * value: one host thread, 2 steps of a 4096 x 256 strip of the headline
      field (same network, tau, initial recipe, periodic in both directions):
      the per-node work of the headline workload, bounded to about 10 s;
    * the 64^2 parity workload in full (500 steps, 9->32->32->9);
    * context: 2 steps of the full 4096^2 headline field, and the first 20
      steps of the 1024^2 Kolmogorov workload, with the oracle's row-parallel
      loops on all host CPUs this process may use."""
    import numpy as np

    import oracle
    from paper_2403_18466_amd import inputs
    model, ncpu, total = host_cpu()
    theta = inputs.glorot_params(9, HIDDEN, seed=1).astype(np.float64)
    u = inputs.fourier_modes_velocity(N, N, kmax=4, umax=0.05, seed=0)
    full = oracle.Config(nx=N, ny=N, tau=TAU, hidden=HIDDEN, out_scale=S_OUT)
    g = oracle.init_equilibrium(full, np.ones((1, 1, N, N)), u[None, :, None])
    oracle.set_threads(1)
    rows = 256
    strip = oracle.Config(nx=N, ny=rows, tau=TAU, hidden=HIDDEN, out_scale=S_OUT)
    gs = np.ascontiguousarray(g[:, :, :, :rows])
    t0 = time.perf_counter()
    oracle.run(strip, gs, theta, 2)
    dt = time.perf_counter() - t0
    value = N * rows * 2 / dt / 1e6
    # the 64^2 parity workload in full
    c1 = oracle.Config(nx=64, ny=64, tau=0.6, hidden=32, out_scale=2.0 ** -4)
    u1 = inputs.fourier_modes_velocity(64, 64, kmax=4, umax=0.05, seed=0)
    g1 = oracle.init_equilibrium(c1, np.ones((1, 1, 64, 64)), u1[None, :, None])
    t1 = time.perf_counter()
    oracle.run(c1, g1, inputs.glorot_params(9, 32, seed=1).astype(np.float64), 500)
    d1 = time.perf_counter() - t1
    # all host threads on the full headline field
    nt = oracle.set_threads(min(ncpu, 64))
    t2 = time.perf_counter()
    oracle.run(full, g, theta, 2)
    d2 = time.perf_counter() - t2
    # all host threads: the first 20 steps of the 1024^2 Kolmogorov workload
    kc = oracle.Config(nx=1024, ny=1024, tau=TAU, hidden=HIDDEN, out_scale=S_OUT, force_kind=1,
                       force_amp=1e-5, force_k=4)
    uk = inputs.fourier_modes_velocity(1024, 1024, kmax=4, umax=0.01, seed=0)
    gk = oracle.init_equilibrium(kc, np.ones((1, 1, 1024, 1024)), uk[None, :, None])
    t3 = time.perf_counter()
    oracle.run(kc, gk, theta, 20)
    d3 = time.perf_counter() - t3
    oracle.set_threads(1)
    return {"value": value, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"2 steps of a {N}x{rows} strip of the headline field (same network, "
                      f"tau, initial recipe), fp64 oracle, serial C on one host thread "
                      f"({dt:.1f} s)",
            "host_cpu": model, "host_cpus_usable": ncpu, "host_cpus_total": total,
            "parity_workload_64_full": {"steps": 500, "s": d1,
                                        "mlups": 64 * 64 * 500 / d1 / 1e6, "threads": 1},
            "headline_4096_two_steps_all_threads": {"threads": nt, "s": d2,
                                                    "mlups": N * N * 2 / d2 / 1e6},
            "kolmogorov_1024_20_steps_all_threads": {"threads": nt, "s": d3,
                                                     "mlups": 1024 * 1024 * 20 / d3 / 1e6},
            "rows": oracle_rows()}


def oracle_rows():
    """The fp64 oracle on small samples of the other rows' workloads (one
    host thread, a fraction of a second to a few seconds each), in MLUPS,
    for context beside the GPU figures."""
    import numpy as np

    import oracle
    from paper_2403_18466_amd import inputs

    def rate(cfg, theta, adjoint=False, reps=1):
        g = np.random.default_rng(0).normal(0.0, 0.01, cfg.state_shape)
        t0 = time.perf_counter()
        for _ in range(reps):
            if adjoint:
                oracle.step_adjoint(cfg, g, g, theta)
            else:
                g = oracle.step(cfg, g, theta)
        nodes = cfg.nx * cfg.ny * cfg.nz * cfg.batch
        return nodes * reps / (time.perf_counter() - t0) / 1e6

    th9 = inputs.glorot_params(9, HIDDEN, seed=1).astype(np.float64)
    th19 = inputs.glorot_params(19, HIDDEN, seed=1).astype(np.float64)
    thw = inputs.glorot_params_net(inputs.net_widths(19, 0, "paper"), 1).astype(np.float64)
    rows = {
        "bgk_d2q9": (oracle.Config(nx=1024, ny=1024, tau=TAU), None, False),
        "smagorinsky_d2q9": (oracle.Config(nx=512, ny=512, tau=TAU, collision="smagorinsky",
                                           smag_cs=SMAG_CS), None, False),
        "adjoint_d2q9_h64": (oracle.Config(nx=256, ny=256, tau=0.50125, hidden=HIDDEN,
                                           out_scale=2.0 ** -10), th9, True),
        "nlbm_d3q19_h64": (oracle.Config(lattice="D3Q19", nx=48, ny=48, nz=48, tau=TAU,
                                         hidden=HIDDEN, out_scale=S_OUT), th19, False),
        "wide_d3q19": (oracle.Config(lattice="D3Q19", nx=16, ny=16, nz=16, tau=TAU, hidden=300,
                                     net="paper", out_scale=S_OUT), thw, False),
    }
    out = {}
    for name, (cfg, th, adj) in rows.items():
        shape = "x".join(str(v) for v in (cfg.nx, cfg.ny) + ((cfg.nz,) if cfg.nz > 1 else ()))
        out[name] = {"mlups": rate(cfg, th, adj), "sample": f"one {'adjoint ' if adj else ''}step "
                     f"on {shape}"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the library has no multi-GPU path)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2403_18466_amd import inputs, lbm
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    lbm.load_library()
    base = lbm.Lattice(lbm.Config(nx=N, ny=N, tau=TAU))
    A0 = make_state(torch, lbm, inputs, base)
    base.close()
    torch.cuda.synchronize()

    variants = {}
    wanted = args.variants.split(",")
    table = {"bf16": ("bf16", HIDDEN, "bgk"), "fp16": ("fp16", HIDDEN, "bgk"),
             "fp32": ("fp32", HIDDEN, "bgk"), "bgk": ("fp32", 0, "bgk"),
             "smag": ("fp32", 0, "smagorinsky")}
    # the headline leg runs last, after the other legs and its own settle
    for name in [v for v in wanted if v != "bf16"] + ["bf16"]:
        prec, hidden, coll = table[name]
        steps = args.steps if name != "fp32" else max(1, args.steps // 2)
        variants[name] = time_variant(torch, lbm, inputs, prec, hidden, steps, args.warmup, A0,
                                      coll, args.settle)
        print(f"# {name}: {variants[name]['ms_per_step']:.4f} ms/step, "
              f"{variants[name]['mlups']:.0f} MLUPS", file=sys.stderr, flush=True)

    head = variants["bf16"]
    t_launch = head["ms_per_step"] * 1e-3
    trans_rate = TANH_PER_LUP * TRANS_PER_TANH * N * N / t_launch
    hbm_rate = BYTES_PER_LUP * N * N / t_launch
    lups = N * N / t_launch
    roofline = {
        "bound": "alu",
        "achieved": lups / 1e9,
        "peak": ACT_PEAK_LUPS / 1e9,
        "unit": "GLUP/s (activation ALU ceiling: 128 tanh x (2 transcendental + 2 FP32) + "
                "64 conversions per LUP at 8 / 16 lanes per clock per SIMD)",
        "frac": lups / ACT_PEAK_LUPS,
        "traffic": TRAFFIC_BYTES,
        "trans_achieved_Tps": trans_rate / 1e12,
        "trans_peak_Tps": TRANS_PEAK / 1e12,
        "trans_frac": trans_rate / TRANS_PEAK,
        "hbm_achieved_GBps": hbm_rate / 1e9,
        "hbm_frac": hbm_rate / HBM_PEAK,
        "mfma_frac": 10496 * lups / 2.5e15,
        "kernel": "nlbm_step_kernel<D2Q9, 64, bf16>",
    }
    bgk = variants.get("bgk")
    result = {
        "metric": "MLUPS of learned-collision LBM step (BF16 vs FP32) + % HBM/MFMA roofline",
        "value": head["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "D2Q9 periodic 4096x4096 learned-collision throughput run, "
                               "MLP 9->64->64->9 tanh, bf16 MFMA / fp32 accumulate, "
                               "fp32 deviation populations, tau 0.51",
                   "grid": [N, N], "hidden": HIDDEN, "tau": TAU, "out_scale": S_OUT},
        "roofline": roofline,
        "timing": f"each leg: {args.settle:g} s of untimed steps (clock settle), then --warmup "
                  "steps from the initial state, then --steps timed with HIP events in up to 5 "
                  "chunks (chunk spread below); the headline leg runs after the others",
        "variants": {k: {"mlups": v["mlups"], "ms_per_step": v["ms_per_step"],
                         "hbm_frac": BYTES_PER_LUP * N * N / (v["ms_per_step"] * 1e-3) / HBM_PEAK,
                         "chunk_ms_per_step": v["chunk_ms_per_step"],
                         "nonfinite": v["nonfinite"]} for k, v in variants.items()},
    }
    if "fp32" in variants:
        result["bf16_over_fp32"] = head["mlups"] / variants["fp32"]["mlups"]
    if bgk:
        result["bgk_roofline"] = {"bound": "hbm", "achieved": BYTES_PER_LUP * N * N /
                                  (bgk["ms_per_step"] * 1e-3) / 1e9, "peak": HBM_PEAK / 1e9,
                                  "unit": "GB/s",
                                  "frac": BYTES_PER_LUP * N * N / (bgk["ms_per_step"] * 1e-3) /
                                  HBM_PEAK}
    smag = variants.get("smag")
    if smag:
        result["smagorinsky_roofline"] = {
            "bound": "hbm", "achieved": BYTES_PER_LUP * N * N / (smag["ms_per_step"] * 1e-3) / 1e9,
            "peak": HBM_PEAK / 1e9, "unit": "GB/s",
            "frac": BYTES_PER_LUP * N * N / (smag["ms_per_step"] * 1e-3) / HBM_PEAK,
            "collision": f"Smagorinsky LES, C_s = {SMAG_CS}, tau 0.51, same field"}
    # The secondary legs below are context for the headline: an exception in
    # one of them is recorded under its name (and printed), and the line is
    # still printed.
    def secondary(name, fn):
        try:
            result[name] = fn()
        except Exception as e:  # noqa: BLE001 -- recorded, not hidden
            print(f"# {name} failed: {type(e).__name__}: {e}", file=sys.stderr, flush=True)
            result[name] = {"error": f"{type(e).__name__}: {e}"}

    secondary("kolmogorov_1024", lambda: time_kolmogorov(torch, lbm, inputs, max(100, args.steps)))
    if not args.no_d3q19:
        secondary("d3q19_256", lambda: time_d3q19(torch, lbm, inputs, max(10, args.steps // 5)))
    if not args.no_wide:
        secondary("wide_d3q19_256", lambda: time_wide(torch, lbm, inputs, max(10, args.steps // 10)))
    if not args.no_si:
        secondary("si_pipeline", lambda: time_si_pipeline(torch, lbm, inputs))
    if not args.no_train:
        secondary("training", lambda: training_leg(torch, lbm, inputs))
    if not args.no_cpu:
        secondary("cpu_baseline", cpu_baseline)
    print(json.dumps(result), flush=True)


def training_leg(torch, lbm, inputs):
    """The unrolled-training workload in bf16 and fp32, with the adjoint's
    roofline."""
    tr = {p: time_training(torch, lbm, inputs, p, 5) for p in ("bf16", "fp32")}
    for p, v in tr.items():
        print(f"# training step {p}: {v['train_step_ms']:.2f} ms, adjoint "
              f"{v['adjoint_mlups']:.0f} MLUPS", file=sys.stderr, flush=True)
    # the same gradient with the whole trajectory kept in HBM (no recompute)
    keep = time_training(torch, lbm, inputs, "bf16", 5, ckpt=32)
    print(f"# training step bf16, whole trajectory kept: {keep['train_step_ms']:.2f} ms",
          file=sys.stderr, flush=True)
    lups = tr["bf16"]["adjoint_mlups"] * 1e6
    return {"workload": "8 x 256^2 D2Q9, 32 unrolled steps, checkpoint every 8, H=64, "
                        "forward + recompute + adjoint + Adam",
            **{p: v for p, v in tr.items()},
            "bf16_keep_all": {"train_step_ms": keep["train_step_ms"],
                              "workload": "the same 32 steps with every state kept (one segment "
                                          "of 32, 31 x 18.9 MB): no recompute, one gradient "
                                          "reduction"},
            "bf16_over_fp32_step_time": tr["fp32"]["train_step_ms"] / tr["bf16"]["train_step_ms"],
            "adjoint_roofline": {
                "kernel": "nlbm_backward_coop_kernel<D2Q9, 64, bf16> + grad_reduce_kernel",
                "bound": "alu", "achieved": lups / 1e9,
                "peak": ADJ_ACT_PEAK_LUPS / 1e9,
                "unit": "GLUP/s (activation ALU ceiling of the adjoint: the forward's 52 "
                        "SIMD-cycles per LUP plus 128 tanh derivatives x 2 FP32 and 64 "
                        "conversions)",
                "frac": lups / ADJ_ACT_PEAK_LUPS,
                "hbm_frac": ADJ_BYTES_PER_LUP * lups / HBM_PEAK,
                "mfma_frac": ADJ_FLOP_PER_LUP * lups / 2.5e15}}

if __name__ == "__main__":
    main()
