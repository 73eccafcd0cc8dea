"""Case 1 intersections (flashing red) on the GPU path: per-node crossing keys
by atomicMin in admission, the round-robin pointer advanced by the winner's
commit, departures held back from a lane the node's crossing enters.  The run
matches the oracle bit for bit, ensemble members keep their standalone runs,
and the reverse sweep matches the oracle's FP64 adjoint."""
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


def case1(w):
    w.params.intersection_mode = 1
    return w


def test_parity_config1_case1(M, oracle_mod):
    w = case1(W.config1())
    g, o, bitwise = run_pair(M, oracle_mod, w, list(range(1, 12)) + [100, 500, 1000, 2000, 3600])
    assert bitwise
    c = o.counters()
    assert c["arrived"] == 2000 and c["holds"] >= 4 * c["transfers"]


def test_parity_config1_case1_four_classes_and_spread(M, oracle_mod):
    w = case1(W.config1(n_classes=4))
    w.params = W.jitter_params(w.params, 0.1, seed=5)
    w.params.v0_spread = 0.05
    _, _, bitwise = run_pair(M, oracle_mod, w, [10, 700, 1800, 3600])
    assert bitwise


def test_parity_scaled_config2_case1(M, oracle_mod):
    """Config 2's recipe on a 30x30 grid + ring (ring nodes join ramps: up to
    3 x 3 pairs), 15,000 vehicles, first 6,000 steps."""
    w = case1(W.scaled_config2(n_vehicles=15000, rows=30, cols=30, n_steps=6000))
    _, _, bitwise = run_pair(M, oracle_mod, w, [500, 2000, 4000, 6000])
    assert bitwise


def test_parity_config2_case1_from_its_0800_state(M, oracle_mod):
    """Full-size config 2 with flashing red at every node, run on the GPU to
    08:00 (about 130,000 vehicles on the road); that state, written into a
    new handle and into the oracle (both restart the round-robin), then 200
    steps bit for bit, every vehicle and counter."""
    w = case1(W.config2())
    g = M.Sim(w)
    assert g.schedule()[2] > 1
    g.step(10_800)
    st = g.state()
    init = {k: st[k] for k in ("status", "edge", "lane", "cursor", "x", "v", "held_since", "mand", "ww",
                               "tau_in", "t_arr")}
    init.update(counters=np.zeros(len(M.COUNTERS), np.int64), t=int(st["t"]))
    g.close()
    oracle_mod.set_threads(0)
    try:
        g2, o, bitwise = run_pair(M, oracle_mod, w, [10_801, 10_850, 11_000], init=init)
    finally:
        oracle_mod.set_threads(1)
    assert bitwise
    assert o.counters()["transfers"] > 10_000


def test_case1_resume_from_written_state(M, oracle_mod):
    """sim_write_state restarts the round-robin on both sides.  The written
    state is the oracle's own at step 900."""
    w = case1(W.config1())
    a = oracle_mod.OracleSim(w)
    a.step(900)
    st = a.state()
    init = {k: st[k] for k in ("status", "edge", "lane", "cursor", "x", "v", "held_since", "mand", "ww",
                               "tau_in")}
    # the oracle's state input has no arrival times: both sides start without them
    init.update(t_arr=np.full(w.n_vehicles, -1.0), counters=None, t=int(st["t"]))
    _, _, bitwise = run_pair(M, oracle_mod, w, [901, 1200, 2400], init=init)
    assert bitwise


def test_ensemble_members_case1(M):
    master, scen = W.config4(n_scen=3, base=2000, n_steps=1200)
    master.params.intersection_mode = 1
    ens = M.Sim(master, scenarios=scen)
    ens.step(1200)
    es = ens.state()
    off = ens.offsets()
    E = master.net.n_edges
    for k, (n, red) in enumerate(scen):
        solo = M.Sim(W.scenario_workload(master, n, red))
        solo.step(1200)
        ss = solo.state()
        sl = slice(int(off[k]), int(off[k + 1]))
        for f in FIELDS:
            assert np.array_equal(es[f][sl], ss[f]), (k, f)
        assert np.array_equal(es["edge"][sl] - k * E, ss["edge"]), k


def test_backward_case1_matches_fp64_adjoint(M, oracle_mod):
    steps = 3600
    w = case1(W.config1(n_classes=4, n_steps=steps))
    hidden = W.jitter_params(w.params, 0.1, seed=7)
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
    print("relative gradient error vs FP64 adjoint (case 1):", rel)
    assert rel <= 1e-3
