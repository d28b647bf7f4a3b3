"""Differentiable time stepping and unrolled training of the collision network
(SI, "Unrolled training": roll the model over L_T steps, evaluate the loss at
the end, backpropagate through every step, update with Adam).

Everything here orchestrates library calls; the arithmetic (steps, adjoint
steps, loss and its gradient, Adam, coarse-graining) runs in liblbm_hip.so.
PyTorch provides device memory, streams and the autograd interface.
"""
from __future__ import annotations

import torch

from . import lbm


class NLBMStep(torch.autograd.Function):
    """One stream-collide step A_{n+1} = step(A_n; theta) with the hand-written
    adjoint as its backward.  Usage: NLBMStep.apply(lattice, A, theta)."""

    @staticmethod
    def forward(ctx, lattice: "lbm.Lattice", A, theta):
        ctx.lattice = lattice
        ctx.save_for_backward(A, theta)
        out = lattice.empty_state()
        # a single step reads A and writes out; A is left untouched
        return lbm.lbm_step(lattice.ctx, lattice.cfg, A.detach(), out, theta.detach(), 1)

    @staticmethod
    def backward(ctx, grad_out):
        A, theta = ctx.saved_tensors
        L = ctx.lattice
        lam_n, dtheta = L.step_backward(A.detach(), theta.detach(),
                                        grad_out.contiguous())
        return None, lam_n, dtheta


def unrolled_loss_and_grad(L: "lbm.Lattice", A0, theta, u_target, nsteps: int, ckpt: int = 8,
                           want_dA0: bool = False, loss_fn=None):
    """Loss after `nsteps` steps from A0 and its gradient.

    The loss is the velocity MSE against u_target, or loss_fn(A) -> (loss,
    dL/dA) when given (e.g. the population loss on a node subset).  Forward
    keeps the state at every multiple of `ckpt` (plus A0); the backward pass
    walks the segments in reverse, recomputes each segment's states from its
    checkpoint, and runs the segment's adjoint steps (lbm_step_backward_seq:
    the per-workgroup gradient partials of a segment are reduced once).  The last
    segment's states are kept as the forward pass makes them (its backward
    pass comes next and would recompute the same values).  Memory:
    nsteps/ckpt checkpoints + ckpt segment states + 2 adjoint buffers.
    Returns (loss [1] float64 device tensor, dtheta, dA0 or None)."""
    assert nsteps >= 1 and ckpt >= 1
    last = ((nsteps - 1) // ckpt) * ckpt  # first step of the last segment
    a = A0.detach()  # read only: A0 is a checkpoint, never a free buffer
    ckpts = {0: a}
    kept = {}  # states last + 1 .. nsteps - 1
    spare = L.empty_state()
    for n in range(nsteps):
        keep = last < n + 1 < nsteps
        is_ckpt = (n + 1) % ckpt == 0 and n + 1 < nsteps
        # kept states and checkpoints are written to buffers of their own
        out = L.empty_state() if keep or is_ckpt else spare
        lbm.lbm_step(L.ctx, L.cfg, a, out, theta, 1)
        if not any(a is t for t in list(kept.values()) + list(ckpts.values())):
            spare = a  # a ping-pong buffer, free again
        elif out is spare:
            spare = L.empty_state()  # the input is still needed
        a = out
        if keep:
            kept[n + 1] = out
        if is_ckpt:
            ckpts[n + 1] = out
    if loss_fn is None:
        loss, lam = L.loss_velocity_mse(a, u_target, want_grad=True)
    else:
        loss, lam = loss_fn(a)
    dtheta = torch.zeros(L.n_param, dtype=torch.float32, device=L.device)
    lam_next = torch.empty_like(lam)
    ws = L.workspace()
    n = nsteps
    while n > 0:
        start = ((n - 1) // ckpt) * ckpt
        seg = [ckpts[start]]
        for m in range(start, n - 1):
            if m + 1 in kept:
                seg.append(kept.pop(m + 1))
                continue
            out = L.empty_state()
            lbm.lbm_step(L.ctx, L.cfg, seg[-1], out, theta, 1)
            seg.append(out)
        # the segment's adjoint steps, with one reduction of the gradient
        res = lbm.lbm_step_backward_seq(L.ctx, L.cfg, seg, theta, lam, lam_next, dtheta, ws)
        if res is lam_next:
            lam, lam_next = lam_next, lam
        n = start
    return loss, dtheta, (lam if want_dA0 else None)


class Adam:
    """Adam with L2 weight decay added to the gradient (Table S2 of the SI:
    learning rate 1e-4, weight decay 1e-6), on the library's adam kernel."""

    def __init__(self, param, lr=1e-4, betas=(0.9, 0.999), eps=1e-8, weight_decay=1e-6):
        self.p = param
        self.m = torch.zeros_like(param)
        self.v = torch.zeros_like(param)
        self.lr, self.betas, self.eps, self.wd = lr, betas, eps, weight_decay
        self.t = 0

    def step(self, grad):
        self.t += 1
        lbm.lbm_adam(self.p, grad, self.m, self.v, self.lr, self.betas[0], self.betas[1],
                     self.eps, self.wd, self.t)


def coarse_grain(fine: "lbm.Lattice", coarse: "lbm.Lattice", A_fine, factor: int):
    """Block-average the fine populations onto the coarse grid (4 x 4 blocks for
    factor 4): canonical fine -> box filter -> pull-shifted coarse.  The
    coarse velocity (j summed over the block over rho summed over the block)
    is then the coarse state's own moment."""
    cf = fine.cfg
    canon = fine.shift(A_fine, +1)
    cc = coarse.empty_state()
    lbm.lbm_box_filter(canon, cc, cf.batch, cf.Q, cf.nx, cf.ny, cf.nz, factor)
    return coarse.shift(cc, -1)
