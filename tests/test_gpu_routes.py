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


def _oracle_reroute(oracle_mod, w, ost):
    """The oracle's side of re-routing, from the oracle's own run: costs =
    its mean traversal times (free-flow where nothing traversed), new routes
    of the vehicles still waiting for a later departure from oracle.route,
    and the state to continue from (first route edge, cursor 0)."""
    t = int(ost["t"])
    s, c = ost["edge_stats"]
    mean = np.where(c > 0, s / np.maximum(c, 1), 0.0)
    cost = np.where(c > 0, mean, w.net.length / w.net.limit).astype(np.float32)
    net, roff, redges = w.net, w.route_off, w.route_edges
    routes = []
    for i in range(w.n_vehicles):
        r = redges[roff[i]:roff[i + 1]].tolist()
        if w.depart_step[i] > t and ost["status"][i] == 0:
            r = oracle_mod.route(net, cost, int(net.edge_from[r[0]]), int(net.edge_to[r[-1]]))
        routes.append(r)
    w2 = W.Workload(w.name, net, np.concatenate([[0], np.cumsum([len(r) for r in routes])]).astype(np.int64),
                    np.concatenate(routes).astype(np.int32), w.depart_step, w.vclass, w.alpha, w.params, w.n_steps)
    fut = np.nonzero((w.depart_step > t) & (ost["status"] == 0))[0]
    st = {k: np.array(ost[k], copy=True) for k in ("status", "edge", "lane", "cursor", "x", "v", "held_since",
                                                   "mand", "ww", "tau_in")}
    st["edge"][fut] = w2.route_edges[w2.route_off[fut]]
    st["cursor"][fut] = 0
    st.update(t_arr=np.full(w.n_vehicles, -1.0), counters=None, t=t)
    return w2, st, cost


def test_reroute_future_departures_continues_like_the_oracle(M, oracle_mod):
    """Config 1 with departures over 30 min: at step 900 the vehicles not yet
    departed get routes on the mean traversal times so far.  The GPU side
    re-routes from its own run with GPU routing, the oracle side from its own
    run with the oracle's routes; the costs, the new routes and the
    continued runs agree."""
    from paper_2007_03614_amd.reroute import reroute_future_departures
    from test_gpu_parity import compare_states
    w = W.config1(n_steps=3600)
    w.depart_step = (w.depart_step * 3).astype(np.int32)     # departures over 30 min
    sim = M.Sim(w)
    sim.step(900)
    mean, cnt = sim.mean_travel_times()
    cost = np.where(cnt > 0, mean, w.net.length / w.net.limit).astype(np.float32)
    w2, st = reroute_future_departures(w, sim.state(), cost)
    o0 = oracle_mod.OracleSim(w)
    o0.step(900)
    ost = o0.state()
    ost["edge_stats"] = o0.edge_stats()
    w2o, sto, costo = _oracle_reroute(oracle_mod, w, ost)
    assert np.array_equal(cost, costo)
    assert np.array_equal(w2.route_off, w2o.route_off) and np.array_equal(w2.route_edges, w2o.route_edges)
    fut = np.nonzero(w.depart_step > 900)[0]
    assert fut.size > 500
    changed = sum(not np.array_equal(w.route_edges[w.route_off[i]:w.route_off[i + 1]],
                                     w2.route_edges[w2.route_off[i]:w2.route_off[i + 1]]) for i in fut)
    assert changed > 0
    g = M.Sim(w2)
    g.write_state(st)
    o = oracle_mod.OracleSim(w2o)
    o.write_state(sto["t"], sto)
    t, bitwise = 900, True
    for cp in (901, 1800, 3600):
        g.step(cp - t)
        o.step(cp - t)
        t = cp
        bitwise &= compare_states(g.state(), o.state(), f"step {t}")
    assert bitwise and o.counters()["arrived"] > 0


def test_routes_at_the_node_limit(M, oracle_mod):
    """A 125 x 128 grid has 16,000 nodes, the most whose labels one
    workgroup's LDS holds: routes on perturbed costs still equal the oracle's
    (corner to corner, about 250 edges)."""
    net = W.grid_network(125, 128)
    assert net.n_nodes == 16000
    cost = ((net.length / net.limit) * np.random.default_rng(9).uniform(0.5, 2.0, net.n_edges)).astype(np.float32)
    o = np.array([0, 127, 8000, 15999, 15872, 64], np.int32)
    d = np.array([15999, 15872, 15999, 0, 127, 8000], np.int32)
    _check(M, oracle_mod, net, cost, o, d)


@pytest.mark.parametrize("which", ["grid", "metro"])
def test_routes_above_the_node_limit_equal_the_oracle(M, oracle_mod, which):
    """Above 16,000 nodes the labels live in device memory and are relaxed
    from a frontier: a 127 x 127 grid (16,129 nodes) and the metropolitan
    recipe on a 130 x 131 lattice (17,030 nodes), routes edge for edge equal
    to the oracle's on perturbed costs."""
    if which == "grid":
        net = W.grid_network(127, 127)
    else:
        net = W.metro_network(rows=130, cols=131, n_segments=int(round(274_504 * 130 * 131 / (473 * 474))), seed=4)
    assert net.n_nodes > 16000
    cost = ((net.length / net.limit) * np.random.default_rng(13).uniform(0.5, 2.0, net.n_edges)).astype(np.float32)
    rng = np.random.default_rng(14)
    V = net.n_nodes
    o = np.concatenate([[0, V - 1], rng.integers(0, V, 18)]).astype(np.int32)
    d = np.concatenate([[V - 1, 0], rng.integers(0, V, 18)]).astype(np.int32)
    d[o == d] = (d[o == d] + 1) % V
    _check(M, oracle_mod, net, cost, o, d)


def test_routes_for_the_metropolitan_demand(M):
    """The full metropolitan network (224,202 nodes): the GPU's routes for
    4,000 of its trips on free-flow costs are continuous, join origin to
    destination, and cost (binary32, summed from the destination back) no
    more than the generator's CPU route of the same trip -- they are the
    shortest in that arithmetic, so any other route costs at least as much."""
    w = W.config3()
    net = w.net
    cost = (net.length / net.limit).astype(np.float32)
    sel = np.random.default_rng(15).choice(w.n_vehicles, 4000, replace=False)
    o = net.edge_from[w.route_edges[w.route_off[sel]]].astype(np.int32)
    d = net.edge_to[w.route_edges[w.route_off[sel + 1] - 1]].astype(np.int32)
    off, edges = M.shortest_routes(net, cost, o, d)

    def c32(r):
        acc = np.float32(0.0)
        for e in r[::-1]:
            acc = np.float32(cost[e] + acc)
        return acc
    for q in range(sel.size):
        r = edges[off[q]:off[q + 1]]
        assert net.edge_from[r[0]] == o[q] and net.edge_to[r[-1]] == d[q]
        assert (net.edge_to[r[:-1]] == net.edge_from[r[1:]]).all()
        ref = w.route_edges[w.route_off[sel[q]]:w.route_off[sel[q] + 1]]
        assert c32(r) <= c32(ref), q


def _grid_with_hub(n_spokes):
    """10 x 10 grid plus a hub node joined both ways to n_spokes grid nodes:
    the hub's out-degree picks the label kernel (<= 4, <= 8 padded slots,
    above 8 the CSR form)."""
    g = W.grid_network(10, 10)
    spokes = np.linspace(0, 99, n_spokes).astype(int)
    seg_u = np.concatenate([g.edge_from[g.edge_from < g.edge_to], np.full(n_spokes, 100)])
    seg_v = np.concatenate([g.edge_to[g.edge_from < g.edge_to], spokes])
    nx = np.concatenate([g.node_x, [900.0]])
    ny = np.concatenate([g.node_y, [2300.0]])
    ln = np.hypot(nx[seg_u] - nx[seg_v], ny[seg_u] - ny[seg_v])
    n = seg_u.size
    return W._finish_edges(nx, ny, seg_u, seg_v, ln, np.full(n, np.float32(50 / 3.6)), np.full(n, 2))


@pytest.mark.parametrize("n_spokes", [3, 7, 12])
def test_label_kernels_by_out_degree(M, oracle_mod, n_spokes):
    net = _grid_with_hub(n_spokes)
    assert np.bincount(net.edge_from).max() == max(4, n_spokes)
    cost = ((net.length / net.limit) * np.random.default_rng(n_spokes).uniform(0.5, 2.0, net.n_edges)).astype(np.float32)
    rng = np.random.default_rng(11)
    o = np.concatenate([rng.integers(0, 101, 150), np.full(20, 100)]).astype(np.int32)
    d = np.concatenate([rng.integers(0, 101, 150), rng.integers(0, 100, 20)]).astype(np.int32)
    d[o == d] = (d[o == d] + 1) % 101
    _check(M, oracle_mod, net, cost, o, d)


@pytest.mark.parametrize("rows,cols", [(80, 128), (81, 127)])
def test_register_label_kernel_at_its_node_limit(M, oracle_mod, rows, cols):
    """The register-resident label kernel holds 10 nodes per thread of 1,024:
    10,240 nodes fill every slot (the last thread's last node is 10,239);
    10,287 nodes go to the padded kernel.  Routes equal the oracle's on both."""
    net = W.grid_network(rows, cols)
    cost = ((net.length / net.limit) * np.random.default_rng(rows).uniform(0.5, 2.0, net.n_edges)).astype(np.float32)
    V = net.n_nodes
    o = np.array([0, V - 1, cols - 1, V - cols], np.int32)
    d = np.array([V - 1, 0, V - cols, V - 2], np.int32)
    _check(M, oracle_mod, net, cost, o, d)
