"""Differentiable form: gradients of a per-edge mean travel-time loss with
respect to the 20 class parameters (4 classes x (v0_factor, T, a, b, s0)),
by the GPU reverse sweep with the forward's decisions frozen, against the
oracle's FP64 adjoint of the same frozen-decision problem (itself pinned to
central differences in tests/test_oracle_adjoint.py)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

STEPS = 7200   # 1 h at dt = 0.5 s


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03614_amd as M
    return M


@pytest.fixture(scope="module")
def calib(oracle_mod):
    """Config-1 network and demand with 4 classes; target means from hidden
    parameters theta* = base * (1 + U[-0.1, 0.1]) (clipped to the bounds)."""
    w = W.config1(n_classes=4, n_steps=STEPS)
    hidden = W.jitter_params(w.params, 0.1, seed=5)
    wt = W.Workload(w.name, w.net, w.route_off, w.route_edges, w.depart_step, w.vclass, w.alpha, hidden, STEPS)
    o = oracle_mod.OracleSim(wt)
    o.step(STEPS)
    s, c = o.edge_stats()
    target = np.where(c > 0, s / np.maximum(c, 1), 0.0)
    return w, target, c > 0


def gpu_grad(M, w, target, tcnt, record_every=120):
    w.params.record_every = record_every
    sim = M.Sim(w)
    sim.step(STEPS)
    mean, cnt = sim.mean_travel_times()
    use = (cnt > 0) & tcnt
    dl = np.where(use, 2.0 * (mean - target), 0.0)
    g = sim.backward(dl)
    w.params.record_every = 0
    return sim, mean, use, g


def test_backward_matches_fp64_adjoint(M, oracle_mod, calib):
    w, target, tcnt = calib
    sim, mean, use, g = gpu_grad(M, w, target, tcnt)
    o = oracle_mod.OracleSim(w)
    o.enable_record()
    o.step(STEPS)
    ouse = (o.edge_stats()[1] > 0) & tcnt        # the oracle's own mask, from its own run
    assert np.array_equal(ouse, use)
    loss, omean, og = o.replay(o.theta(w), target, ouse.astype(np.uint8), grad=True)
    og = og.reshape(-1, 5)
    rel = np.linalg.norm(g - og) / np.linalg.norm(og)
    big = np.abs(og) > 1e-3 * np.linalg.norm(og)
    comp = np.abs(g[big] - og[big]) / np.abs(og[big])
    print("relative gradient error vs FP64 adjoint:", rel, "largest per-component error:", comp.max())
    assert rel <= 1e-3
    # every component above 1e-3 of the gradient's norm within 1e-3 of itself
    assert np.all(comp <= 1e-3), comp


def test_checkpoint_interval_independent_and_reproducible(M, calib):
    """The reverse sweep adds every part in a fixed order (no floating-point
    atomics): the gradient is the same bit for bit whatever the checkpoint
    interval, and from run to run."""
    w, target, tcnt = calib
    g120 = gpu_grad(M, w, target, tcnt, 120)[3]
    assert np.array_equal(gpu_grad(M, w, target, tcnt, 120)[3], g120)
    for r in (45, STEPS):
        g = gpu_grad(M, w, target, tcnt, r)[3]
        assert np.array_equal(g, g120), r


def test_backward_leaves_state_and_needs_record(M, c1, calib):
    w, target, tcnt = calib
    sim, mean, use, g = gpu_grad(M, w, target, tcnt)
    st = sim.state()
    sim.backward(np.where(use, 1.0, 0.0))
    st2 = sim.state()
    for k in st:
        if k != "t":
            assert np.array_equal(np.asarray(st[k]), np.asarray(st2[k])), k
    plain = M.Sim(c1)
    plain.step(10)
    with pytest.raises(M.SimError) as ei:
        plain.backward(np.zeros(c1.net.n_edges))
    assert ei.value.name == "SIM_ESTATE"


def test_autograd_function(M, calib):
    import torch
    w, target, tcnt = calib
    theta = torch.tensor(np.stack([w.params.v0_factor, w.params.T, w.params.a, w.params.b, w.params.s0], 1),
                         dtype=torch.float64, requires_grad=True)
    mean = M.edge_mean_travel_time(theta, w, STEPS, 120)
    use = torch.from_numpy((mean.detach().numpy() > 0) & tcnt)
    loss = (((mean - torch.from_numpy(target)) ** 2) * use).sum()
    loss.backward()
    ref = gpu_grad(M, w, target, tcnt)[3]
    assert np.allclose(theta.grad.numpy(), ref, rtol=1e-9, atol=1e-12)
