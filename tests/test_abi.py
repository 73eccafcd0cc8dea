"""The C ABI library loads, exports every entry point the header declares,
and rejects invalid inputs at create time with the documented status codes.
Validation happens on the host before any device call, so these run on CPU."""
import copy
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def M():
    import paper_2007_03614_amd as M
    return M


def _declared():
    src = open(os.path.join(ROOT, "include", "manta.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z0-9_]+)\s*\(", src)))


def test_header_symbols_exported(M):
    names = _declared()
    assert "sim_create" in names and "sim_step" in names and "sim_read_state" in names
    lib = ctypes.CDLL(M.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert set(M.EXPORTED) == set(names)


def _expect(M, w, status):
    with pytest.raises(M.SimError) as ei:
        M.Sim(w, allocator="hip")
    assert ei.value.name == status, str(ei.value)
    return str(ei.value)


@pytest.fixture(scope="module")
def base():
    return W.config1(n_vehicles=50)


def test_bad_network(M, base):
    w = copy.deepcopy(base)
    w.net.lanes = w.net.lanes.copy()
    w.net.lanes[3] = 0
    _expect(M, w, "SIM_EINVAL")
    w = copy.deepcopy(base)
    w.net.length = w.net.length.copy()
    w.net.length[5] = 19.5
    assert "length" in _expect(M, w, "SIM_EINVAL")
    w = copy.deepcopy(base)
    w.net.limit = w.net.limit.copy()
    w.net.limit[0] = np.nan
    _expect(M, w, "SIM_EINVAL")
    w = copy.deepcopy(base)
    w.net.conn_mask = w.net.conn_mask.copy()
    w.net.conn_mask[0] = 0
    assert "mask" in _expect(M, w, "SIM_EINVAL")


def test_bad_routes(M, base):
    w = copy.deepcopy(base)
    re_ = w.route_edges.copy()
    # break continuity: replace the second edge of a route by an unrelated edge
    i = int(np.nonzero(np.diff(w.route_off) > 2)[0][0])
    a = int(w.route_off[i])
    e = int(re_[a])
    bad = [f for f in range(w.net.n_edges) if w.net.edge_from[f] != w.net.edge_to[e]][0]
    re_[a + 1] = bad
    w.route_edges = re_
    assert "continuous" in _expect(M, w, "SIM_EINVAL")
    w = copy.deepcopy(base)
    w.depart_step = w.depart_step.copy()
    w.depart_step[0] = -1
    _expect(M, w, "SIM_EINVAL")
    w = copy.deepcopy(base)
    w.alpha = w.alpha.copy()
    w.alpha[2] = 0.5
    _expect(M, w, "SIM_EINVAL")
    w = copy.deepcopy(base)
    w.vclass = w.vclass.copy()
    w.vclass[1] = 3
    _expect(M, w, "SIM_EINVAL")


@pytest.mark.parametrize("field,val", [("a", 0.5), ("a", 11.0), ("b", np.nan), ("T", 0.05), ("T", 2.5),
                                       ("s0", 0.5), ("s0", 6.0), ("v0_factor", 0.0), ("v0_factor", 2.5),
                                       ("veh_len", 0.0)])
def test_bad_params(M, base, field, val):
    w = copy.deepcopy(base)
    arr = getattr(w.params, field).copy()
    arr[0] = val
    setattr(w.params, field, arr)
    _expect(M, w, "SIM_EINVAL")


def test_unsupported_modes(M, base):
    w = copy.deepcopy(base)
    w.params.intersection_mode = 2
    _expect(M, w, "SIM_EINVAL")
    w = copy.deepcopy(base)
    w.params.record_every = -1
    _expect(M, w, "SIM_EINVAL")
    for spread in (-0.01, 0.3, float("nan")):
        w = copy.deepcopy(base)
        w.params.v0_spread = spread
        _expect(M, w, "SIM_EINVAL")


def test_flashing_red_needs_at_most_64_pairs_per_node(M):
    """Case 1 numbers a node's (in, out) pairs in 6 bits of its key: a star of
    nine two-way spokes (81 pairs at the hub) is refused by the library and by
    the oracle; eight spokes (64 pairs) pass the oracle."""
    import oracle
    for spokes in (9, 8):
        ang = np.arange(spokes) * 2 * np.pi / spokes
        nx = np.concatenate([[0.0], 300.0 * np.cos(ang)])
        ny = np.concatenate([[0.0], 300.0 * np.sin(ang)])
        net = W._finish_edges(nx, ny, np.zeros(spokes, np.int64), np.arange(1, spokes + 1),
                              np.full(spokes, 300.0, np.float32), np.full(spokes, 13.9, np.float32),
                              np.ones(spokes, np.int64))
        e_in = int(np.nonzero((net.edge_from == 1) & (net.edge_to == 0))[0][0])
        e_out = int(np.nonzero((net.edge_from == 0) & (net.edge_to == 2))[0][0])
        p = W.base_params(1)
        p.intersection_mode = 1
        w = W.Workload("star", net, np.array([0, 2], np.int64), np.array([e_in, e_out], np.int32),
                       np.zeros(1, np.int32), np.zeros(1, np.uint8), np.full(1, 0.2, np.float32), p, 10)
        if spokes == 9:
            _expect(M, w, "SIM_EUNSUPPORTED")
            with pytest.raises(ValueError):
                oracle.OracleSim(w)
        else:
            oracle.OracleSim(w)


def test_step_reach_bound(M, base):
    """An edge shorter than one step's reach could let an entering vehicle land
    past a vehicle already there; such networks are refused."""
    w = copy.deepcopy(base)
    w.params.v0_factor = np.array([2.0], np.float32)
    w.params.veh_len = np.array([20.0], np.float32)
    w.net.length = np.full_like(w.net.length, 25.0)
    assert "reach" in _expect(M, w, "SIM_EINVAL")


def test_allocator_callbacks_outlive_handles(M):
    """Handles keep the allocator function pointers they were created with;
    registering again must not free the callbacks an older handle will call."""
    M.use_torch_allocator()
    first = M._torch_cb
    M.use_torch_allocator()
    M.use_hip_allocator()
    M.use_torch_allocator()
    assert M._torch_cb is first


def test_ensemble_validation(M, base):
    with pytest.raises(M.SimError) as ei:
        M.Sim(base, allocator="hip", scenarios=[])
    assert ei.value.name == "SIM_EINVAL"
    with pytest.raises(M.SimError) as ei:
        M.Sim(base, allocator="hip", scenarios=[(base.n_vehicles + 1, np.array([], np.int32))])
    assert "n_vehicles" in str(ei.value)
    with pytest.raises(M.SimError) as ei:
        M.Sim(base, allocator="hip", scenarios=[(10, np.array([base.net.n_edges], np.int32))])
    assert "reduced edge" in str(ei.value)
