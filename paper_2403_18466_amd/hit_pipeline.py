"""The SI's training-data pipeline and training recipe on the GPU library.

SI, "Definition of the Training Dataset":
  * direct numerical simulation of forced homogeneous isotropic turbulence,
    D3Q19 on a periodic L^3 box (L = 128), BGK at tau = 0.5032, driven by the
    three-component sine force F_x(y), F_y(z), F_z(x) of amplitude F = 5e-6
    (Table S2) through the exact difference method;
  * an initial transient of T_0 steps, then samples every delta_T steps;
  * the sub-sampling filter: the coarse grid keeps one point in every cg
    along each axis;
  * pairs (pre-collision state at t, the state cg fine steps later): in the
    library's pull-shifted layout the coarse state one coarse step later holds
    the post-collision populations of step t, i.e. the anti-streaming of the
    SI's Fig. 2 is the layout itself.
SI, "Unrolled training": the model runs L_T coarse steps (12 for cg = 4, 24
for cg = 2) from a sampled state, the loss of eq. nn-loss compares the
post-collision populations on a random node subset S (|S| = 512) with the
filtered DNS, and Adam (lr 1e-4, weight decay 1e-6) updates the network after
backpropagation through all L_T steps.

Readings (stated where the SI is silent): the DNS starts from rest plus a
small solenoidal perturbation (seeded) that triggers the transition; the
coarse model keeps the force field with amplitude cg * F, one coarse step
standing for cg fine steps of momentum input, and uses tau' of
eq. tau-rescaled.

Every step, filter, loss, adjoint and Adam update runs in the HIP library;
this module only sequences calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import inputs, lbm, training


def rescaled_tau(tau: float, cg: int) -> float:
    """eq. tau-rescaled: tau' = (tau - 1/2) / cg + 1/2."""
    return (tau - 0.5) / cg + 0.5


@dataclass
class DNSSpec:
    L: int = 128
    tau: float = 0.5032
    F: float = 5e-6
    t0: int = 50000          # transient
    dT: int = 1000           # sampling interval
    n_samples: int = 8
    cg: int = 4
    LT: int = 12             # unrolled coarse steps
    init_urms: float = 1e-3  # seed perturbation, per component
    init_k0: float = 4.0
    seed: int = 0


@dataclass
class HITDataset:
    spec: DNSSpec
    coarse_cfg: lbm.Config
    starts: list = field(default_factory=list)    # coarse pull-shifted states at t_k
    targets: list = field(default_factory=list)   # coarse states cg * LT fine steps later
    ke: list = field(default_factory=list)        # DNS kinetic energy at each t_k
    wall_s: float = 0.0


def coarse_config(spec: DNSSpec, **net) -> lbm.Config:
    n = spec.L // spec.cg
    return lbm.Config(lattice="D3Q19", nx=n, ny=n, nz=n, tau=rescaled_tau(spec.tau, spec.cg),
                      force_kind=lbm.LBM_FORCE_SINE3, force_k=1, force_amp=spec.cg * spec.F,
                      **net)


def run_dns(spec: DNSSpec, device="cuda", log=None) -> HITDataset:
    """Run the forced DNS and collect the coarse (start, target) pairs."""
    L, cg = spec.L, spec.cg
    if L % cg:
        raise ValueError("L must be a multiple of cg")
    if cg * spec.LT > spec.dT:
        raise ValueError("the sampling interval must cover cg * LT fine steps")
    fcfg = lbm.Config(lattice="D3Q19", nx=L, ny=L, nz=L, tau=spec.tau,
                      force_kind=lbm.LBM_FORCE_SINE3, force_k=1, force_amp=spec.F)
    fine = lbm.Lattice(fcfg, device)
    u = inputs.solenoidal_spectrum_velocity((L, L, L), spec.init_k0, spec.init_urms, spec.seed)
    bufs = [fine.init(torch.ones((1, L, L, L), device=device),
                      torch.from_numpy(u.astype(np.float32))[None].to(device)), None]
    bufs[1] = torch.empty_like(bufs[0])
    del u
    ccfg = coarse_config(spec)
    n = L // cg

    def advance(k):
        if k > 0:
            res = lbm.lbm_step(fine.ctx, fcfg, bufs[0], bufs[1], None, k)
            if res is bufs[1]:
                bufs.reverse()

    def filtered():
        out = torch.empty((1, 19, n, n, n), dtype=torch.float32, device=device)
        lbm.lbm_subsample("D3Q19", bufs[0], out, 1, L, L, L, cg)
        return out

    t_start = time.perf_counter()
    advance(spec.t0)
    ds = HITDataset(spec, ccfg)
    for k in range(spec.n_samples):
        _, _, diag = fine.moments(bufs[0], want_fields=False)
        ds.ke.append(float(diag[0, 1].item()))
        if int(diag[0, 2].item()) != 0:
            raise RuntimeError("the DNS produced non-finite populations")
        ds.starts.append(filtered())
        advance(cg * spec.LT)
        ds.targets.append(filtered())
        advance(spec.dT - cg * spec.LT)
        if log:
            log(f"sample {k}: kinetic energy {ds.ke[-1]:.4e}")
    torch.cuda.synchronize()
    ds.wall_s = time.perf_counter() - t_start
    fine.close()
    return ds


@dataclass
class TrainSpec:
    hidden: int = 64
    net: str = "tanh"
    prec: str = "bf16"
    out_scale: float = 1.0
    epochs: int = 200
    lr: float = 1e-4
    weight_decay: float = 1e-6
    subset: int = 512
    ckpt: int = 4
    zero_output: bool = True  # start from exactly BGK at tau'
    seed: int = 1
    log_every: int = 50


def initial_params(ds: HITDataset, spec: TrainSpec, device="cuda"):
    widths = inputs.net_widths(19, spec.hidden, spec.net)
    th = torch.from_numpy(inputs.glorot_params_net(widths, spec.seed)).to(device)
    if spec.zero_output:
        th[th.numel() - widths[-1] * (widths[-2] + 1):] = 0.0
    return th


def population_loss(L: "lbm.Lattice", A, target, nodes):
    return L.loss_population_sse(A, target, nodes)


def train(ds: HITDataset, spec: TrainSpec, device="cuda", theta=None, log=print):
    """Unrolled training with the subset population loss; one epoch = one
    random sample and one random subset S.  Returns (theta, history)."""
    cfg = coarse_config(ds.spec, hidden=spec.hidden, net=spec.net, mlp_prec=spec.prec,
                        out_scale=spec.out_scale)
    L = lbm.Lattice(cfg, device)
    if theta is None:
        theta = initial_params(ds, spec, device)
    opt = training.Adam(theta, lr=spec.lr, weight_decay=spec.weight_decay)
    rng = np.random.default_rng(spec.seed)
    nnodes = cfg.nx * cfg.ny * cfg.nz
    hist = []
    t0 = time.perf_counter()
    for ep in range(spec.epochs):
        k = int(rng.integers(len(ds.starts)))
        nodes = torch.from_numpy(rng.choice(nnodes, size=min(spec.subset, nnodes),
                                            replace=False).astype(np.int32)).to(device)
        loss, dth, _ = training.unrolled_loss_and_grad(
            L, ds.starts[k], theta, None, ds.spec.LT, min(spec.ckpt, ds.spec.LT),
            loss_fn=lambda A: L.loss_population_sse(A, ds.targets[k], nodes))
        opt.step(dth)
        if ep % spec.log_every == 0 or ep == spec.epochs - 1:
            hist.append((ep, float(loss.item())))
            if log:
                log(f"epoch {ep}: subset loss {hist[-1][1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    L.close()
    return theta, hist


def evaluate(ds: HITDataset, theta, spec: TrainSpec, device="cuda"):
    """Mean over all samples of the population loss of eq. nn-loss on the
    whole coarse grid after LT coarse steps (theta None: BGK at tau'), and
    the number of non-finite nodes."""
    cfg = coarse_config(ds.spec, hidden=spec.hidden if theta is not None else 0, net=spec.net,
                        mlp_prec=spec.prec, out_scale=spec.out_scale)
    L = lbm.Lattice(cfg, device)
    nnodes = cfg.nx * cfg.ny * cfg.nz
    everything = torch.arange(nnodes, dtype=torch.int32, device=device)
    tot, bad = 0.0, 0
    for A0, T in zip(ds.starts, ds.targets):
        out = L.step(A0, theta, ds.spec.LT)
        loss, _ = L.loss_population_sse(out, T, everything, want_grad=False)
        _, _, diag = L.moments(out, want_fields=False)
        tot += float(loss.item())
        bad += int(diag[0, 2].item())
    L.close()
    return tot / len(ds.starts) / nnodes, bad


def rollout(ds: HITDataset, theta, spec: TrainSpec, steps: int, every: int = 50,
            device="cuda"):
    """Free run of the coarse model from the first sample (theta None: BGK at
    tau'): kinetic energy and non-finite node count every `every` steps.
    The SI notes that plain BGK at the coarse parameters is unstable."""
    cfg = coarse_config(ds.spec, hidden=spec.hidden if theta is not None else 0, net=spec.net,
                        mlp_prec=spec.prec, out_scale=spec.out_scale)
    L = lbm.Lattice(cfg, device)
    bufs = [ds.starts[0].clone(), torch.empty_like(ds.starts[0])]
    out = []
    done = 0
    while done < steps:
        k = min(every, steps - done)
        res = lbm.lbm_step(L.ctx, cfg, bufs[0], bufs[1], theta, k)
        if res is bufs[1]:
            bufs.reverse()
        done += k
        _, _, diag = L.moments(bufs[0], want_fields=False)
        out.append((done, float(diag[0, 1].item()), int(diag[0, 2].item())))
    L.close()
    return out


def diagnose(ds: HITDataset, theta, spec: TrainSpec, steps: int, device="cuda"):
    """The SI's evaluation quantities after `steps` coarse steps from the
    first sample, for BGK at tau' (theta None), the trained network, or the
    Smagorinsky collision (theta == "smagorinsky", C_s = 0.17): longitudinal
    structure functions (S, S_abs) up to p = 6 and l = L'/2, and the
    effective relaxation time of each MRT moment over the last step."""
    from . import diagnostics
    net = {}
    if isinstance(theta, str):
        net = dict(collision="smagorinsky", smag_cs=0.17)
        theta = None
    elif theta is not None:
        net = dict(hidden=spec.hidden, net=spec.net, mlp_prec=spec.prec, out_scale=spec.out_scale)
    cfg = coarse_config(ds.spec, **net)
    L = lbm.Lattice(cfg, device)
    A = L.step(ds.starts[0], theta, steps - 1) if steps > 1 else ds.starts[0].clone()
    A1 = L.step(A, theta, 1)
    S, Sa = diagnostics.structure_functions(L, A1, cfg.nx // 2, 6)
    tau = diagnostics.mrt_relaxation(L, A, A1)
    L.close()
    return S, Sa, tau


def main():
    """The SI's pipeline at its sizes: 128^3 DNS, cg = 4, L_T = 12, 8
    samples; --net paper trains the SI's own 19-300-300-100-19 LeakyReLU
    network, --net tanh the 19-64-64-19 tanh one."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--epochs", type=int, default=400)
    ap.add_argument("--samples", type=int, default=8)
    ap.add_argument("--t0", type=int, default=50000)
    ap.add_argument("--rollout", type=int, default=2000)
    ap.add_argument("--net", default="paper", choices=["paper", "tanh"])
    ap.add_argument("--prec", default="bf16")
    args = ap.parse_args()
    ds = run_dns(DNSSpec(n_samples=args.samples, t0=args.t0), log=print)
    print(f"DNS: {ds.wall_s:.1f} s")
    spec = TrainSpec(epochs=args.epochs, net=args.net, prec=args.prec,
                     hidden=300 if args.net == "paper" else 64)
    base = evaluate(ds, None, spec)
    theta, _ = train(ds, spec)
    trained = evaluate(ds, theta, spec)
    print(f"per-node population loss after {ds.spec.LT} coarse steps: BGK at tau' {base[0]:.4e} "
          f"({base[1]} non-finite), trained {trained[0]:.4e} ({trained[1]} non-finite)")
    for name, th in (("BGK at tau'", None), ("trained", theta)):
        traj = rollout(ds, th, spec, args.rollout, every=max(1, args.rollout // 8))
        print(f"free run, {name}: " + ", ".join(f"{t}: KE {e:.3e} ({b} non-finite)"
                                                for t, e, b in traj))
    from . import diagnostics
    cfg = coarse_config(ds.spec)
    Lc = lbm.Lattice(cfg)
    S_dns, Sa_dns = diagnostics.structure_functions(Lc, ds.targets[0], cfg.nx // 2, 6)
    Lc.close()
    print("structure functions S_abs^p(l), p = 2, 3, 6, l = 1, 2, 4, 8 "
          "(filtered DNS, then the models after 200 coarse steps):")
    print("  DNS:   " + " ".join(f"{Sa_dns[p - 1, l - 1]:.3e}" for p in (2, 3, 6) for l in (1, 2, 4, 8)))
    for name, th in (("trained", theta), ("Smag.", "smagorinsky")):
        S, Sa, tau = diagnose(ds, th, spec, 200)
        print(f"  {name}: " + " ".join(f"{Sa[p - 1, l - 1]:.3e}" for p in (2, 3, 6) for l in (1, 2, 4, 8)))
        print(f"  {name} effective relaxation times: " +
              ", ".join(f"{k} {v[0]:.4f}" for k, v in tau.items() if v[0] == v[0]))


if __name__ == "__main__":
    main()
