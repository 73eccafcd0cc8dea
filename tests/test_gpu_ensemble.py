"""Ensemble form: one handle running several what-if scenarios (demand
subsets, edges cut to one lane) in the same launches.  Each member must be
bitwise identical to the same scenario run alone, and one member matches the
oracle; the autotuned schedule never changes results."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import compare_states

pytestmark = pytest.mark.gpu

FIELDS = ("status", "lane", "cursor", "x", "v", "held_since", "mand", "ww", "tau_in", "t_arr")


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03614_amd as M
    return M


@pytest.fixture(scope="module")
def small_ensemble():
    return W.config4(n_scen=5, base=2000, n_steps=1800)


def test_members_equal_standalone_runs(M, small_ensemble):
    master, scen = small_ensemble
    ens = M.Sim(master, scenarios=scen)
    ens.step(1800)
    es = ens.state()
    off = ens.offsets()
    E = master.net.n_edges
    esum, ecnt = ens.edge_stats()
    tot = np.zeros(len(M.COUNTERS), np.int64)
    for k, (n, red) in enumerate(scen):
        assert off[k + 1] - off[k] == n
        solo = M.Sim(W.scenario_workload(master, n, red))
        solo.step(1800)
        ss = solo.state()
        sl = slice(int(off[k]), int(off[k + 1]))
        for f in FIELDS:
            assert np.array_equal(es[f][sl], ss[f]), (k, f)
        assert np.array_equal(es["edge"][sl] - k * E, ss["edge"]), k
        s, c = solo.edge_stats()
        assert np.array_equal(esum[k * E:(k + 1) * E], s) and np.array_equal(ecnt[k * E:(k + 1) * E], c), k
        tot += ss["counters"]
    assert np.array_equal(tot, es["counters"])


def test_member_matches_oracle(M, oracle_mod, small_ensemble):
    master, scen = small_ensemble
    ens = M.Sim(master, scenarios=scen[:2])
    n, red = scen[1]
    o = oracle_mod.OracleSim(W.scenario_workload(master, n, red))
    for cp in (300, 900, 1800):
        ens.step(cp - o.t)
        o.step(cp - o.t)
        es = ens.state()
        off = ens.offsets()
        sl = slice(int(off[1]), int(off[2]))
        member = {f: es[f][sl] for f in FIELDS}
        member["edge"] = es["edge"][sl] - master.net.n_edges
        assert compare_states(member, o.state(), f"step {cp}")


def test_large_ensemble_members_equal_standalone_runs(M):
    """3,000 scenarios of the 10x10 grid make a union network of 1.08M edges
    (4,219 commit blocks); members still equal their standalone runs.  (The
    path above 8,192 blocks is checked against the oracle in
    test_gpu_metro.py.)"""
    master, scen = W.config4(n_scen=3000, base=20, n_steps=600)
    assert master.net.n_edges * len(scen) > 1_000_000
    ens = M.Sim(master, scenarios=scen)
    ens.step(600)
    es = ens.state()
    off = ens.offsets()
    E = master.net.n_edges
    for k in (0, 1500, 2999):
        n, red = scen[k]
        solo = M.Sim(W.scenario_workload(master, n, red))
        solo.step(600)
        ss = solo.state()
        sl = slice(int(off[k]), int(off[k + 1]))
        for f in FIELDS:
            assert np.array_equal(es[f][sl], ss[f]), (k, f)
        assert np.array_equal(es["edge"][sl] - k * E, ss["edge"]), k
    assert es["counters"][list(M.COUNTERS).index("arrived")] > 0


def test_autotune_keeps_results_and_caches(M, c1, tmp_path):
    ref = M.Sim(c1)
    ref.step(1500)
    a = M.Sim(c1)
    a.step(500)
    cache = str(tmp_path / "sched.txt")
    sched = a.autotune(cache, steps_per_trial=4)
    assert a.state()["t"] == 500
    a.step(1000)
    sa, sr = a.state(), ref.state()
    for k in sr:
        if k != "t":
            assert np.array_equal(np.asarray(sa[k]), np.asarray(sr[k])), k
    assert np.array_equal(a.edge_stats()[0], ref.edge_stats()[0])
    b = M.Sim(c1)
    assert b.autotune(cache, steps_per_trial=4) == sched   # read back from the cache
    assert open(cache).read().count("manta-schedule") == 1
    c = M.Sim(c1)                                          # the two-argument form reads the same line
    assert M._lib.sim_autotune(c._h, cache.encode()) == 0 and c.schedule() == sched
    assert open(cache).read().count("manta-schedule") == 1
