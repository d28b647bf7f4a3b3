"""The training loop on the GPU: fine BGK runs coarse-grained by block
averaging, loss through unrolled coarse steps at the rescaled tau
(eq. tau-rescaled), the library adjoint and Adam.  Checks that the library
gradient is a descent direction of the unrolled loss with the first-order
decrease it predicts, that training runs and moves the parameters, and
reports what the trained network gains over plain BGK on held-out fields
(the gain is measured, not pinned: the paper has no number for this 2-D
set-up)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def data():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_18466_amd import coarse_training as ct
    spec = dict(n_fine=256, cg=4, k0=16.0, urms=0.04, spinup=256, unroll=8)
    tr = ct.build_dataset(ct.DatasetSpec(n_snap=4, seeds=(100, 101, 102, 103), **spec))
    ho = ct.build_dataset(ct.DatasetSpec(n_snap=5, seeds=(200, 201), **spec))
    return ct, tr, ho


def test_gradient_is_descent_direction(data):
    from paper_2403_18466_amd import inputs, lbm, training
    ct, tr, _ = data
    c = tr.coarse_cfg
    assert abs(c.tau - 0.50125) < 1e-15
    cfg = lbm.Config(nx=c.nx, ny=c.ny, batch=c.batch, tau=c.tau, hidden=64, mlp_prec="fp32",
                     out_scale=2.0 ** -4)
    L = lbm.Lattice(cfg)
    th = torch.from_numpy(inputs.glorot_params(9, 64, seed=1)).cuda()
    loss0, g, _ = training.unrolled_loss_and_grad(L, tr.states[0], th, tr.velocities[1], 8, 4)
    l0 = loss0.item()
    alpha = 2e-3 / g.abs().max().item()
    loss1, _, _ = training.unrolled_loss_and_grad(L, tr.states[0], th - alpha * g,
                                                  tr.velocities[1], 8, 4)
    predicted = alpha * float((g.double() ** 2).sum())
    actual = l0 - loss1.item()
    print(f"loss {l0:.6e}; decrease along -grad {actual:.3e}, first-order prediction {predicted:.3e}")
    assert actual > 0
    assert abs(actual / predicted - 1) < 0.2
    L.close()


def test_training_runs_and_reports_gain(data):
    from paper_2403_18466_amd import inputs
    ct, tr, ho = data
    th0 = torch.from_numpy(inputs.glorot_params(9, 64, seed=1)).cuda()
    spec = ct.TrainSpec(prec="bf16", epochs=60, lr=1e-3, out_scale=2.0 ** -10, log_every=20)
    theta, hist = ct.train(tr, spec, theta=th0.clone(), log=None)
    assert all(np.isfinite(l) for _, l in hist)
    assert (theta - th0).abs().max().item() > 1e-3
    ks = [1, 2, 4]
    bgk = ct.rollout_mse(ho, None, 64, "bf16", 1.0, ks)
    untrained = ct.rollout_mse(ho, th0, 64, "bf16", 2.0 ** -10, ks)
    trained = ct.rollout_mse(ho, theta, 64, "bf16", 2.0 ** -10, ks)
    for k in ks:
        assert bgk[k][1] == 0 and trained[k][1] == 0
        print(f"held-out velocity MSE after {k * ho.spec.unroll} coarse steps: BGK {bgk[k][0]:.4e}, "
              f"untrained {untrained[k][0]:.4e}, trained {trained[k][0]:.4e}, "
              f"trained/BGK {trained[k][0] / bgk[k][0]:.4f}")
