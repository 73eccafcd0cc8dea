"""The paper's calibration loop (Sec. IV-A) on the GPU path: parameter sets
as scenarios of one ensemble handle.  Members with their own class
parameters equal standalone runs with those parameters (and the oracle); the
loop run on GPU ensembles takes the same decisions, with the same losses, as
the loop run on oracle evaluations."""
import copy

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("status", "lane", "cursor", "x", "v", "held_since", "mand", "ww", "tau_in", "t_arr")


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03614_amd as M
    return M


def with_class(w, cp):
    w2 = copy.copy(w)
    w2.params = copy.copy(w.params)
    cp = np.asarray(cp, np.float32).reshape(-1, 5)
    w2.params.v0_factor, w2.params.T, w2.params.a, w2.params.b, w2.params.s0 = (
        cp[:, 0].copy(), cp[:, 1].copy(), cp[:, 2].copy(), cp[:, 3].copy(), cp[:, 4].copy())
    return w2


def test_members_with_own_class_params(M, oracle_mod):
    w = W.config1(n_classes=2, n_vehicles=1200, n_steps=1200)
    rng = np.random.default_rng(2)
    base = np.stack([w.params.v0_factor, w.params.T, w.params.a, w.params.b, w.params.s0], 1)
    cps = [base * rng.uniform(0.8, 1.2, base.shape) for _ in range(3)]
    cps[1][:, 0] = 1.0                                    # v0_factor inside (0, 2]
    cps = [np.clip(c, [0.5, 0.1, 1.0, 1.0, 1.0], [2.0, 2.0, 10.0, 10.0, 5.0]).astype(np.float32) for c in cps]
    scen = [(1200, np.zeros(0, np.int32), cps[0]), (900, np.array([3, 40], np.int32), cps[1]),
            (1200, np.zeros(0, np.int32), None)]
    ens = M.Sim(w, scenarios=scen)
    assert ens.n_classes == 6
    ens.step(1200)
    es = ens.state()
    off = ens.offsets()
    E = w.net.n_edges
    esum, ecnt = ens.edge_stats()
    for k, (n, red, cp) in enumerate(scen):
        sw = W.scenario_workload(w, n, red)
        if cp is not None:
            sw = with_class(sw, cp)
        solo = M.Sim(sw)
        solo.step(1200)
        ss = solo.state()
        sl = slice(int(off[k]), int(off[k + 1]))
        for f in FIELDS:
            assert np.array_equal(es[f][sl], ss[f]), (k, f)
        s, c = solo.edge_stats()
        assert np.array_equal(esum[k * E:(k + 1) * E], s) and np.array_equal(ecnt[k * E:(k + 1) * E], c), k
    from test_gpu_parity import compare_states
    o = oracle_mod.OracleSim(with_class(W.scenario_workload(w, 900, np.array([3, 40])), cps[1]))
    o.step(1200)
    sl = slice(int(off[1]), int(off[2]))
    member = {f: es[f][sl] for f in FIELDS}
    member["edge"] = es["edge"][sl] - E
    assert compare_states(member, o.state(), "step 1200")


def test_random_search_same_decisions_as_on_oracle(M, oracle_mod):
    from paper_2007_03614_amd import calibrate as C
    steps = 900
    w = W.config1(n_vehicles=600, n_steps=steps)
    hidden = with_class(w, [[1.0, 1.2, 1.6, 2.6, 2.5]])
    oh = oracle_mod.OracleSim(hidden)
    oh.step(steps)
    s, c = oh.edge_stats()
    observed = C.edge_speeds(np.where(c > 0, s / np.maximum(c, 1), 0.0), c, w.net.length)
    deltas = np.random.default_rng(7).uniform(-1.0, 1.0, (3, 4, 4))

    def oracle_eval(sets):
        out = []
        for th in sets:
            o = oracle_mod.OracleSim(with_class(w, C.class_params(w, th)))
            o.step(steps)
            s, c = o.edge_stats()
            sp = C.edge_speeds(np.where(c > 0, s / np.maximum(c, 1), 0.0), c, w.net.length)
            out.append(C.l1_speed_loss(sp, observed))
        return out

    th_g, hg = C.random_search(w, observed, steps, deltas, tol=0.0)
    th_o, ho = C.random_search(w, observed, steps, deltas, tol=0.0, evaluate=oracle_eval)
    assert len(hg) == len(ho) == 3
    for a, b in zip(hg, ho):
        assert a["losses"] == b["losses"] and a["best"] == b["best"] and a["sets"] == b["sets"]
    assert np.array_equal(th_g, th_o)
    # the nominal set is always re-evaluated, so the best loss never rises
    best = [h["losses"][h["best"]] for h in hg]
    assert all(x >= y for x, y in zip(best, best[1:])) and best[-1] < hg[0]["losses"][0]


def test_gradient_descent_runs_within_bounds(M):
    from paper_2007_03614_amd import calibrate as C
    steps = 900
    w = W.config1(n_vehicles=600, n_steps=steps)
    hidden = with_class(w, [[1.0, 1.2, 1.6, 2.6, 2.5]])
    sim = M.Sim(hidden)
    sim.step(steps)
    mean, cnt = sim.mean_travel_times()
    observed = C.edge_speeds(mean, cnt, w.net.length)
    th, hist = C.gradient_descent(w, observed, steps, iterations=3)
    lo, hi = C._bounds_arrays()
    assert len(hist) == 3 and all(np.isfinite(h["loss"]) and np.all(np.isfinite(h["grad"])) for h in hist)
    assert np.all(th >= lo) and np.all(th <= hi)
    assert min(h["loss"] for h in hist[1:]) < hist[0]["loss"]
