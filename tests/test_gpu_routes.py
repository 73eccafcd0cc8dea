"""Routes on travel times on the GPU (sim_shortest_routes): the same edge
lists as the oracle, on free-flow costs (many ties on the uniform grid), on
perturbed costs, and on the mean traversal times of a simulated run."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    assert torch.cuda.is_available()
    import paper_2007_03614_amd as M
    return M


def _check(M, oracle_mod, net, cost, o, d):
    off, edges = M.shortest_routes(net, cost, o, d)
    assert off[-1] == edges.size
    for q in range(o.size):
        ref = oracle_mod.route(net, cost, int(o[q]), int(d[q]))
        assert edges[off[q]:off[q + 1]].tolist() == ref, q


@pytest.mark.parametrize("kind", ["uniform", "free_flow", "perturbed"])
def test_grid_routes_equal_oracle(M, oracle_mod, kind):
    w = W.config1(n_vehicles=10, n_steps=10)
    net = w.net
    cost = {"uniform": np.full(net.n_edges, 10.0, np.float32),
            "free_flow": (net.length / net.limit).astype(np.float32),
            "perturbed": ((net.length / net.limit) * np.random.default_rng(5).uniform(0.5, 2.0, net.n_edges))
            .astype(np.float32)}[kind]
    rng = np.random.default_rng(6)
    o = rng.integers(0, net.n_nodes, 400).astype(np.int32)
    d = rng.integers(0, net.n_nodes, 400).astype(np.int32)
    d[o == d] = (d[o == d] + 1) % net.n_nodes
    _check(M, oracle_mod, net, cost, o, d)


def test_routes_on_simulated_travel_times(M, oracle_mod):
    """Config 2's recipe on a 30x30 grid + ring: costs = mean traversal times
    after 1 h (free-flow where no traversal), the O/D pairs of 150 vehicles."""
    w = W.scaled_config2(n_vehicles=15000, rows=30, cols=30, n_steps=7200)
    sim = M.Sim(w)
    sim.step(7200)
    mean, cnt = sim.mean_travel_times()
    ff = w.net.length / w.net.limit
    cost = np.where(cnt > 0, mean, ff).astype(np.float32)
    sel = np.random.default_rng(7).choice(w.n_vehicles, 150, replace=False)
    o = w.net.edge_from[w.route_edges[w.route_off[sel]]].astype(np.int32)
    d = w.net.edge_to[w.route_edges[w.route_off[sel + 1] - 1]].astype(np.int32)
    _check(M, oracle_mod, w.net, cost, o, d)


def test_errors(M):
    w = W.config1(n_vehicles=10, n_steps=10)
    net = w.net
    cost = np.full(net.n_edges, 10.0, np.float32)
    with pytest.raises(M.SimError):
        M.shortest_routes(net, cost, np.array([3], np.int32), np.array([3], np.int32))     # origin == destination
    bad = cost.copy()
    bad[5] = 0.0
    with pytest.raises(M.SimError):
        M.shortest_routes(net, bad, np.array([1], np.int32), np.array([7], np.int32))
    off, edges = M.shortest_routes(net, cost, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert off.tolist() == [0] and edges.size == 0


def test_reroute_future_departures_continues_like_the_oracle(M, oracle_mod):
    """Config 1 with departures over 30 min: at step 900 the vehicles not yet
    departed get routes on the mean traversal times so far (GPU routing);
    the run goes on from the same state on the GPU and in the oracle."""
    from paper_2007_03614_amd.reroute import reroute_future_departures
    from test_gpu_parity import run_pair
    w = W.config1(n_steps=3600)
    w.depart_step = (w.depart_step * 3).astype(np.int32)     # departures over 30 min
    sim = M.Sim(w)
    sim.step(900)
    mean, cnt = sim.mean_travel_times()
    cost = np.where(cnt > 0, mean, w.net.length / w.net.limit).astype(np.float32)
    w2, st = reroute_future_departures(w, sim.state(), cost)
    fut = np.nonzero(w.depart_step > 900)[0]
    assert fut.size > 500
    changed = sum(not np.array_equal(w.route_edges[w.route_off[i]:w.route_off[i + 1]],
                                     w2.route_edges[w2.route_off[i]:w2.route_off[i + 1]]) for i in fut)
    assert changed > 0
    _, o, bitwise = run_pair(M, oracle_mod, w2, [901, 1800, 3600], init=st)
    assert bitwise and o.counters()["arrived"] > 0


def test_routes_at_the_node_limit(M, oracle_mod):
    """A 125 x 128 grid has 16,000 nodes, the most whose labels one
    workgroup's LDS holds: routes on perturbed costs still equal the oracle's
    (corner to corner, about 250 edges).  One node more is refused."""
    net = W.grid_network(125, 128)
    assert net.n_nodes == 16000
    cost = ((net.length / net.limit) * np.random.default_rng(9).uniform(0.5, 2.0, net.n_edges)).astype(np.float32)
    o = np.array([0, 127, 8000, 15999, 15872, 64], np.int32)
    d = np.array([15999, 15872, 15999, 0, 127, 8000], np.int32)
    _check(M, oracle_mod, net, cost, o, d)
    big = W.grid_network(127, 127)
    assert big.n_nodes > 16000
    with pytest.raises(M.SimError):
        M.shortest_routes(big, np.full(big.n_edges, 1.0, np.float32), np.array([0], np.int32),
                          np.array([5], np.int32))
