"""The HIP path against the stored oracle snapshots (tests/golden/): the same
seeded runs (10x10 grid in case 2; case 1 with 4 classes and a v0 spread;
the full-size perturbed grid with ring highway through its 08:00 peak),
stepped through the C ABI with the graph launches the bench uses.  Counters
and discrete state bit-exact; x and v bitwise (the binary32 contract, whole
state through its digest); entry and arrival times within 1e-9."""
import numpy as np
import pytest

from test_golden import load_snapshots, snapshot_module

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03614_amd as M
    return M


@pytest.mark.parametrize("case", ["grid10x10_case2", "grid10x10_case1_4classes_spread",
                                  "perturbed_grid_ring_peak"])
def test_gpu_matches_stored_oracle_snapshots(M, case):
    m = snapshot_module()
    rec = load_snapshots()["cases"][case]
    w = m.case_workload(case)
    ids = m.case_sample_ids(case, w.n_vehicles)
    sim = M.Sim(w)
    n_f = 1 + len(m.INT_FIELDS) + len(m.F32_FIELDS)
    t = 0
    for cp in rec["checkpoints"]:
        sim.step(cp["t"] - t)
        t = cp["t"]
        s = sim.state()
        assert s["t"] == t
        got = m.snapshot(s, sim.counters(), ids)
        assert got["counters"] == cp["counters"], t
        for g, o in zip(got["vehicles"], cp["vehicles"]):
            assert g[:n_f] == o[:n_f], (t, g, o)
            for a, b in zip(g[n_f:], o[n_f:]):
                assert abs(float.fromhex(a) - float.fromhex(b)) <= 1e-9 * max(1.0, abs(float.fromhex(b))), (t, g, o)
        assert got["digest"] == cp["digest"], t
    sim.close()
