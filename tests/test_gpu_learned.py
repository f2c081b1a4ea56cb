"""Learned coarse-grid correction: training on solver-generated systems
lowers the energy loss; flexible CG with the network converges to the same
answer as plain multigrid; a corrupted network falls back to the plain
V-cycle and still converges."""
import numpy as np
import pytest

import workloads as W
from tests.helpers import rel

pytestmark = pytest.mark.gpu


def _problem(seeds, shape=(16, 32, 32), **opts):
    import torch
    from paper_2502_18377_amd.api import Problem, pack
    pk = pack([W.reaction_diffusion_2d(s, shape=shape) for s in seeds], dtype=torch.float32, device="cuda")
    return Problem(pk["coeff"], pk["rhs"], pk["bc_values"], pk["shapes"], pk["steps"], pk["bc"], pk["mset"], **opts)


def test_training_lowers_loss_and_solve_agrees():
    from paper_2502_18377_amd.learned import Net, train
    probs = [_problem(range(100 + 8 * k, 108 + 8 * k)) for k in range(3)]
    net = Net(2 + 6, seed=3)
    hist = train(net, probs, 1, 240, lr=2e-3, lr_final=2e-4)
    loss = np.array([h[1] for h in hist]); plain = np.array([h[2] for h in hist])
    print("loss first/last", loss[:10].mean(), loss[-10:].mean(), "plain", plain[-10:].mean())
    assert np.isfinite(loss).all()
    assert loss[-10:].mean() < loss[:10].mean()
    # judged by the plain V-cycle on the same samples: the learned refinement
    # must not be worse in the energy norm at the end of training
    assert loss[-10:].mean() <= plain[-10:].mean() + 1e-6 * abs(plain[-10:].mean())
    evalp = _problem(range(500, 504), tol=1e-8)
    z0, i0 = evalp.solve()
    net.attach(evalp, 1)
    z1, i1 = evalp.solve()
    print("iters plain", i0["iters"], "learned", i1["iters"])
    assert i1["code"] == 0 and np.all(i1["relres"] <= 1e-8)
    assert rel(z1.double().cpu().numpy(), z0.double().cpu().numpy()) <= 1e-5


def test_corrupted_network_falls_back():
    from paper_2502_18377_amd.learned import Net
    net = Net(2 + 6, seed=5)
    w = net.get()
    w[:] = np.random.default_rng(0).standard_normal(w.size).astype(np.float32) * 50
    net.set(w)
    p = _problem([7, 8], tol=1e-8)
    z0, i0 = p.solve()
    net.attach(p, 1)
    z1, i1 = p.solve()
    assert i1["code"] == 0 and np.all(i1["relres"] <= 1e-8)
    assert rel(z1.double().cpu().numpy(), z0.double().cpu().numpy()) <= 1e-5
