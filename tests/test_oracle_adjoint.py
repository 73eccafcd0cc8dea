"""Pins for the differentiable form in the oracle: with the discrete decisions
of a recorded run frozen, the FP64 replay reproduces the run, and its reverse
sweep (adjoint of Eq. (1), the integration, the leader coupling and the
crossing-time interpolation) equals central finite differences of the replay."""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def recorded(oracle_mod):
    w = W.config1(n_classes=4, n_steps=3600)
    w.params = W.jitter_params(w.params, 0.1, seed=5)
    sim = oracle_mod.OracleSim(w)
    sim.enable_record()
    sim.step(3600)
    return w, sim


def test_replay_reproduces_the_run(recorded):
    w, sim = recorded
    s, c = sim.edge_stats()
    th = sim.theta(w)
    loss, mean, _ = sim.replay(th, target=np.zeros(w.net.n_edges))
    m = c > 0
    ref = s[m] / c[m]
    # FP64 replay of an FP32 run: same decisions, means within a few ms
    assert np.abs(mean[m] - ref).max() < 5e-3
    assert np.isfinite(loss)


def test_adjoint_equals_central_differences(recorded):
    w, sim = recorded
    th = sim.theta(w)
    _, mean, _ = sim.replay(th)
    rng = np.random.default_rng(3)
    target = mean * (1.0 + rng.uniform(-0.1, 0.1, mean.size))
    use = (mean > 0).astype(np.uint8)
    loss, _, g = sim.replay(th, target, use, grad=True)
    fd = np.empty_like(g)
    for k in range(th.size):
        h = 1e-6 * max(abs(th[k]), 1.0)
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (sim.replay(tp, target, use)[0] - sim.replay(tm, target, use)[0]) / (2 * h)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-5, (g, fd)
    big = np.abs(fd) > 1e-3 * np.linalg.norm(fd)
    assert np.all(np.abs(g[big] - fd[big]) / np.abs(fd[big]) < 1e-4)
    assert big.sum() >= 8


def test_loss_zero_at_own_means(recorded):
    w, sim = recorded
    th = sim.theta(w)
    _, mean, _ = sim.replay(th)
    loss, _, g = sim.replay(th, mean, (mean > 0).astype(np.uint8), grad=True)
    assert loss == 0.0 and np.all(g == 0.0)
