"""GPU parity on the metropolitan-scale workload (224k nodes, 549k directed
edges, 3.2M trips): the HIP path through the C ABI against the CPU oracle.

* Full size, from the 08:00 state built from the demand (about 465,000
  vehicles on the road), written into both sides: every vehicle's state and
  every counter after 1, 20 and 100 steps.
* The same recipe on a 40 x 41 lattice with 30,000 trips, the whole 7 h run
  from 05:00.
* The roofline probe's network (8 copies of the metropolitan network in one
  ensemble, 4.39M edges) at 5 % of jam density: the path for networks above
  8,192 commit blocks (2.1M edges), where the block offsets come from their
  own kernel and the scatter reads them from memory."""
import numpy as np
import pytest

import workloads as W
from test_gpu_parity import compare_states, run_pair

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    import paper_2007_03614_amd as M
    return M


@pytest.fixture(scope="module")
def metro():
    return W.config3()


def test_parity_metro_full_size_from_the_0800_state(M, oracle_mod, metro):
    w = metro
    assert w.net.n_edges == 549_008 and w.n_vehicles == 3_200_000
    s0, info = W.loaded_state(w, 21_600, speed_frac=0.4)
    assert info["active"] > 400_000
    init = dict(s0, counters=np.zeros(len(M.COUNTERS), np.int64))
    oracle_mod.set_threads(0)
    try:
        g, o, bitwise = run_pair(M, oracle_mod, w, [21_601, 21_620, 21_700], init=init)
    finally:
        oracle_mod.set_threads(1)
    c = o.counters()
    print("metro 08:00 window:", c, "bitwise x, v:", bitwise)
    # the window exercises what the step does: lane changes, transfers,
    # holds at full lanes, departures and arrivals
    assert c["lane_changes"] > 1000 and c["transfers"] > 10_000 and c["holds"] > 0
    assert c["departed"] > 0 and c["arrived"] > 0
    g.close()


def test_parity_metro_recipe_small_lattice_whole_run(M, oracle_mod):
    w = W.config3(n_vehicles=30_000, rows=40, cols=41, pool_size=400, cache=False)
    g, o, bitwise = run_pair(M, oracle_mod, w, [7_200, 18_000, 21_600, 30_000, 50_400])
    c = o.counters()
    print("metro 40x41 whole run:", c, "bitwise x, v:", bitwise)
    assert c["departed"] >= 0.99 * w.n_vehicles and c["arrived"] >= 0.95 * w.n_vehicles
    g.close()


FIELDS = ("status", "lane", "cursor", "x", "v", "held_since", "mand", "ww", "tau_in", "t_arr")


def test_parity_probe_network_above_the_lds_block_scan(M, oracle_mod):
    """Eight copies of the metropolitan network in one ensemble (4,392,064
    edges, 17,157 commit blocks), each lane at 5 % of jam density from the
    probe's recipe (469,530 vehicles per copy): members 0 and 7 equal the
    oracle's run of one copy vehicle for vehicle, and the ensemble's counters
    are 8 times the oracle's, after 1, 10 and 40 steps."""
    copies = 8
    w, st = W.probe_r(density=0.05)
    n, E = w.n_vehicles, w.net.n_edges
    assert copies * E > 8192 * 256             # more commit blocks than one workgroup scans in LDS
    ens = M.Sim(w, scenarios=[(n, np.zeros(0, np.int32))] * copies)
    ens.write_state(W.replicate_state(st, E, copies))
    o = oracle_mod.OracleSim(w)
    o.write_state(0, st)
    oracle_mod.set_threads(0)
    try:
        t = 0
        for cp in (1, 10, 40):
            ens.step(cp - t)
            o.step(cp - t)
            t = cp
            es, os_ = ens.state(), o.state()
            off = ens.offsets()
            for k in (0, copies - 1):
                sl = slice(int(off[k]), int(off[k + 1]))
                member = {f: es[f][sl] for f in FIELDS}
                member["edge"] = es["edge"][sl] - k * E    # every status reports an edge of its copy
                assert compare_states(member, os_, f"member {k}, step {cp}")
            oc = o.counters()
            assert dict(zip(M.COUNTERS, es["counters"].tolist())) == {c: copies * v for c, v in oc.items()}, cp
    finally:
        oracle_mod.set_threads(1)
    assert oc["transfers"] > 100_000 and oc["lane_changes"] > 10_000, oc
    ens.close()
