"""Pins for the per-driver free-flow speed (Sec. IV, model validation): each
driver's v0 on an edge is drawn around the edge's limit with standard
deviation 2 sigma_s, sigma_s = spread * limit (a synthetic stand-in for the
observed spread of speeds at that limit).  The draw is checked against
numpy's Philox, its moments against the normal it stands for, and the whole
step against the free-road closed form of Eq. (1) at the driver's own v0."""
import math

import numpy as np
import pytest

import workloads as W
from test_oracle_math import numpy_philox_block

SEED = 1234


def numpy_driver_limit(seed, edge, vid, lim, spread):
    """limit * max(1 + (2 spread) z, 0.1) in binary32, z the Irwin-Hall(12) - 6
    normal of stream 4 with the edge in the step's place (numpy's Philox)."""
    lim, spread = np.float32(lim), np.float32(spread)
    if spread == 0:
        return lim
    words = np.concatenate([numpy_philox_block([edge, vid, 4, b], [seed, 0]) for b in range(3)])
    S = sum(int(x) >> 40 for x in words)
    z = np.float32(np.int32(S - 6 * 2**24)) * np.float32(2.0 ** -24)
    f = np.float32(1.0) + (np.float32(2.0) * spread) * z
    f = max(f, np.float32(0.1))
    return np.float32(lim * f)


def test_driver_limit_from_numpy_words(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(60):
        e = int(rng.integers(0, 600_000))
        vid = int(rng.integers(0, 3_000_000))
        lim = float(np.float32(rng.uniform(8.0, 35.0)))
        for spread in (0.0, 0.03, 0.1, 0.25):
            ref = numpy_driver_limit(SEED, e, vid, lim, spread)
            assert oracle_mod.driver_limit(SEED, e, vid, lim, spread) == float(ref), (e, vid, lim, spread)
    # spread 0 leaves the limit untouched
    assert oracle_mod.driver_limit(SEED, 5, 7, 13.888889, 0.0) == float(np.float32(13.888889))


def test_driver_limit_floor(oracle_mod):
    """At spread 0.25 the factor 1 + z / 2 falls below 0.1 for z < -1.8
    (about 3.6 % of drivers): those drive at a tenth of the limit."""
    lim = float(np.float32(20.0))
    floored = 0
    for vid in range(3000):
        z = oracle_mod.normal(SEED, 11, vid, 4)
        got = oracle_mod.driver_limit(SEED, 11, vid, lim, 0.25)
        if z < -1.8:
            floored += 1
            assert got == float(np.float32(lim) * np.float32(0.1))
        else:
            assert got > 0.1 * lim
    assert 40 <= floored <= 180


def test_driver_limit_moments_and_keys(oracle_mod):
    """The factor has mean 1 and standard deviation 2 spread; it is fixed for a
    (driver, edge) pair and differs between edges and between drivers."""
    spread, lim = 0.05, 10.0
    n = 20_000
    f = np.array([oracle_mod.driver_limit(SEED, 3 + (i % 7), i, lim, spread, fp64=True) for i in range(n)]) / lim
    assert abs(f.mean() - 1.0) < 5 * 2 * spread / math.sqrt(n)
    assert abs(f.std() - 2 * spread) < 6 * 2 * spread / math.sqrt(2 * n)
    same = [oracle_mod.driver_limit(SEED, 42, 99, lim, spread) for _ in range(3)]
    assert len(set(same)) == 1
    per_edge = {oracle_mod.driver_limit(SEED, e, 99, lim, spread) for e in range(20)}
    per_driver = {oracle_mod.driver_limit(SEED, 42, v, lim, spread) for v in range(20)}
    assert len(per_edge) == 20 and len(per_driver) == 20


@pytest.mark.parametrize("vid_count", [3])
def test_lone_drivers_reach_their_own_v0(oracle_mod, vid_count):
    """Three drivers far apart on a 20 km edge: each settles at v0f * its own
    limit (the free-road equilibrium of Eq. (1)), not at the edge's limit."""
    p = W.base_params(1)
    p.v0_spread = 0.05
    w = W.single_edge_workload(length=20000.0, n_vehicles=vid_count, depart_step=[0, 150, 300], n_steps=0,
                               params=p)
    e01 = int(w.route_edges[0])
    lim = float(w.net.limit[e01])
    sim = oracle_mod.OracleSim(w, fp64=False)
    sim.step(700)
    st = sim.state()
    assert np.all(st["status"] == 1)
    x = st["x"]
    assert np.all(np.diff(np.sort(x)) > 500.0)        # no car follows another
    for i in range(vid_count):
        v0 = float(np.float32(p.v0_factor[0]) * numpy_driver_limit(p.seed, e01, i, lim, p.v0_spread))
        assert abs(v0 - lim) > 1e-3 * lim                # the spread acts
        # from rest, 1 - v/v0 falls below 1e-3 well within 400 steps (200 s)
        assert abs(float(st["v"][i]) - v0) < 1e-3 * v0, (i, float(st["v"][i]), v0)


def test_adjoint_with_spread_equals_central_differences(oracle_mod):
    """With a spread, v0 = v0f * (the driver's own limit): the reverse sweep's
    v0f gradient carries each driver's limit, and matches central differences
    of the FP64 replay like the rest of the gradient."""
    w = W.config1(n_classes=4, n_steps=1800)
    w.params = W.jitter_params(w.params, 0.1, seed=5)
    w.params.v0_spread = 0.05
    sim = oracle_mod.OracleSim(w)
    sim.enable_record()
    sim.step(1800)
    th = sim.theta(w)
    s, c = sim.edge_stats()
    _, mean, _ = sim.replay(th)
    m = c > 0
    assert np.abs(mean[m] - s[m] / c[m]).max() < 5e-3      # the replay reproduces the run
    rng = np.random.default_rng(4)
    target = mean * (1.0 + rng.uniform(-0.1, 0.1, mean.size))
    use = (mean > 0).astype(np.uint8)
    _, _, g = sim.replay(th, target, use, grad=True)
    fd = np.empty_like(g)
    for k in range(th.size):
        h = 1e-6 * max(abs(th[k]), 1.0)
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (sim.replay(tp, target, use)[0] - sim.replay(tm, target, use)[0]) / (2 * h)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-5, (g, fd)
    v0f = np.arange(0, th.size, 5)
    assert np.all(np.abs(g[v0f] - fd[v0f]) <= 1e-4 * np.abs(fd[v0f]) + 1e-9 * np.linalg.norm(fd))
