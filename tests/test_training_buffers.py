"""Buffer handling of the checkpointed unrolled gradient (host logic, CPU).

The library calls are replaced by stand-ins on CPU tensors: a step adds 1
to every element, so state n holds n everywhere; the adjoint stand-in
records the states it is handed.  The checks: the caller's A0 is never
written, no step writes into its own input, the final state and every state
handed to the adjoint hold the right values, each state 0 .. nsteps-1
reaches the adjoint exactly once, and the number of forward steps is nsteps
plus the recomputation of every segment except the last."""
import types

import pytest

torch = pytest.importorskip("torch")


class FakeLattice:
    ctx = cfg = None
    n_param = 1
    device = "cpu"

    def empty_state(self):
        return torch.full((4,), float("nan"))

    def workspace(self):
        return None

    def loss_velocity_mse(self, a, u_target, want_grad=True):
        return a.sum(), torch.ones(4)


@pytest.mark.parametrize("nsteps,ckpt", [(32, 8), (12, 4), (9, 4), (8, 8), (5, 8), (1, 8)])
def test_unrolled_buffers(monkeypatch, nsteps, ckpt):
    from paper_2403_18466_amd import training
    seen, nfwd = [], [0]

    def lbm_step(ctx, cfg, a, out, theta, n):
        assert n == 1 and out.data_ptr() != a.data_ptr()
        out.copy_(a + 1)
        nfwd[0] += 1

    def lbm_step_backward_seq(ctx, cfg, seg, theta, lam, lam_next, dtheta, ws):
        vals = [int(s[0].item()) for s in seg]
        assert all(torch.all(s == v) for s, v in zip(seg, vals))
        assert vals == list(range(vals[0], vals[0] + len(seg)))
        seen.extend(vals)
        return lam_next if len(seg) % 2 else lam

    monkeypatch.setattr(training, "lbm", types.SimpleNamespace(
        lbm_step=lbm_step, lbm_step_backward_seq=lbm_step_backward_seq))
    A0 = torch.zeros(4)
    loss, _, _ = training.unrolled_loss_and_grad(FakeLattice(), A0, None, None, nsteps, ckpt)
    assert torch.equal(A0, torch.zeros(4))
    assert loss.item() == 4 * nsteps
    assert sorted(seen) == list(range(nsteps))
    last = ((nsteps - 1) // ckpt) * ckpt
    recompute = sum(ckpt - 1 for _ in range(0, last, ckpt))
    assert nfwd[0] == nsteps + recompute
