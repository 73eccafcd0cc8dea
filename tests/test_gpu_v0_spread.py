"""Per-driver free-flow speed (Sec. IV, model validation) on the GPU path:
with a spread, every driver's v0 on an edge comes from its own draw.  The
step matches the oracle bit for bit (events) and within the FP32 contract,
ensemble members keep the draws of their standalone runs (edges are keyed
within one scenario), and the reverse sweep matches the oracle's FP64 adjoint."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import compare_states, run_pair

pytestmark = pytest.mark.gpu

FIELDS = ("status", "lane", "cursor", "x", "v", "held_since", "mand", "ww", "tau_in", "t_arr")


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03614_amd as M
    return M


def spread_config1(spread, n_steps=3600):
    w = W.config1(n_classes=4, n_steps=n_steps)
    w.params = W.jitter_params(w.params, 0.1, seed=5)
    w.params.v0_spread = spread
    return w


@pytest.mark.parametrize("spread", [0.05, 0.25])
def test_parity_config1_with_spread(M, oracle_mod, spread):
    """10x10 grid, 4 classes; at 0.25 about 3.6 % of the (driver, edge) pairs
    sit on the 0.1 floor."""
    w = spread_config1(spread)
    g, o, bitwise = run_pair(M, oracle_mod, w, [10, 500, 1000, 2000, 3600])
    assert bitwise
    plain = M.Sim(spread_config1(0.0))
    plain.step(3600)
    # the spread changes the run
    assert not np.array_equal(plain.state()["t_arr"], g.state()["t_arr"])


def test_parity_scaled_config2_with_spread(M, oracle_mod):
    """Config 2's recipe on a 30x30 grid + ring, 15,000 vehicles, first 6,000 steps."""
    w = W.scaled_config2(n_vehicles=15000, rows=30, cols=30, n_steps=6000)
    w.params.v0_spread = 0.05
    _, _, bitwise = run_pair(M, oracle_mod, w, [1000, 3000, 6000])
    assert bitwise


def test_ensemble_members_keep_their_draws(M, oracle_mod):
    """The union network numbers member k's edges k * E + e; the draw keys the
    edge modulo E, so each member equals its standalone run and the oracle."""
    master, scen = W.config4(n_scen=3, base=2000, n_steps=1200)
    master.params.v0_spread = 0.05
    ens = M.Sim(master, scenarios=scen)
    ens.step(1200)
    es = ens.state()
    off = ens.offsets()
    E = master.net.n_edges
    for k, (n, red) in enumerate(scen):
        sw = W.scenario_workload(master, n, red)
        assert sw.params.v0_spread == 0.05
        solo = M.Sim(sw)
        solo.step(1200)
        ss = solo.state()
        sl = slice(int(off[k]), int(off[k + 1]))
        for f in FIELDS:
            assert np.array_equal(es[f][sl], ss[f]), (k, f)
        assert np.array_equal(es["edge"][sl] - k * E, ss["edge"]), k
    n, red = scen[1]
    o = oracle_mod.OracleSim(W.scenario_workload(master, n, red))
    o.step(1200)
    sl = slice(int(off[1]), int(off[2]))
    member = {f: es[f][sl] for f in FIELDS}
    member["edge"] = es["edge"][sl] - E
    assert compare_states(member, o.state(), "step 1200")


def test_backward_with_spread_matches_fp64_adjoint(M, oracle_mod):
    steps = 3600
    w = spread_config1(0.05, n_steps=steps)
    hidden = W.jitter_params(w.params, 0.1, seed=7)   # keeps the spread
    wt = W.Workload(w.name, w.net, w.route_off, w.route_edges, w.depart_step, w.vclass, w.alpha, hidden, steps)
    ot = oracle_mod.OracleSim(wt)
    ot.step(steps)
    s, c = ot.edge_stats()
    target = np.where(c > 0, s / np.maximum(c, 1), 0.0)
    w.params.record_every = 120
    sim = M.Sim(w)
    sim.step(steps)
    mean, cnt = sim.mean_travel_times()
    use = (cnt > 0) & (c > 0)
    g = sim.backward(np.where(use, 2.0 * (mean - target), 0.0))
    w.params.record_every = 0
    o = oracle_mod.OracleSim(w)
    o.enable_record()
    o.step(steps)
    ouse = (o.edge_stats()[1] > 0) & (c > 0)     # the oracle's own mask, from its own run
    assert np.array_equal(ouse, use)
    _, _, og = o.replay(o.theta(w), target, ouse.astype(np.uint8), grad=True)
    og = og.reshape(-1, 5)
    rel = np.linalg.norm(g - og) / np.linalg.norm(og)
    print("relative gradient error vs FP64 adjoint (v0 spread 0.05):", rel)
    assert rel <= 1e-3
