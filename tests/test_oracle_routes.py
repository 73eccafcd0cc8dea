"""Pins for the routing on travel times (routes of Sec. II-C re-computed on
current edge costs): the oracle's distances against scipy's Dijkstra, its
routes against scipy's shortest-path tree where the costs make paths unique,
and the route invariants (connected, allowed moves, cost = distance)."""
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import dijkstra

import workloads as W


def _graph(net, cost):
    return csr_matrix((np.asarray(cost, np.float64), (net.edge_from, net.edge_to)), shape=(net.n_nodes, net.n_nodes))


def _allowed(net, e, f):
    return f in net.conn_to[net.conn_off[e]:net.conn_off[e + 1]]


@pytest.mark.parametrize("perturb", [False, True])
def test_distances_and_routes_against_scipy(oracle_mod, perturb):
    w = W.config1(n_vehicles=10, n_steps=10)
    net = w.net
    cost = (net.length / net.limit).astype(np.float32)
    if perturb:
        cost = (cost * np.random.default_rng(3).uniform(0.5, 2.0, cost.size)).astype(np.float32)
    g = _graph(net, cost)
    rng = np.random.default_rng(4)
    for d in rng.choice(net.n_nodes, 8, replace=False):
        ref, pred_rev = dijkstra(g.T.tocsr(), indices=int(d), return_predecessors=True)
        dist = oracle_mod.route_dist(net, cost, int(d))
        assert np.allclose(dist, ref, rtol=2e-6, atol=0.0)
        for o in rng.choice(net.n_nodes, 6, replace=False):
            if o == d:
                assert oracle_mod.route(net, cost, int(o), int(d)) is None
                continue
            r = oracle_mod.route(net, cost, int(o), int(d))
            assert r and net.edge_from[r[0]] == o and net.edge_to[r[-1]] == d
            for a, b in zip(r, r[1:]):
                assert net.edge_to[a] == net.edge_from[b] and _allowed(net, a, b)
            assert abs(float(np.sum(cost[r], dtype=np.float64)) - ref[o]) <= 1e-5 * ref[o]
            if perturb:   # continuous costs: the shortest path is unique, as scipy's tree has it
                v, nodes = int(o), [int(o)]
                while v != d:
                    v = int(pred_rev[v])
                    nodes.append(v)
                assert [int(net.edge_from[e]) for e in r] + [int(d)] == nodes


def test_ties_go_to_the_lower_edge_id(oracle_mod):
    """On the uniform grid many routes tie; the walk takes, at every node, the
    out-edge of smallest (cost + remaining distance, edge id)."""
    w = W.config1(n_vehicles=10, n_steps=10)
    net = w.net
    cost = np.full(net.n_edges, 10.0, np.float32)
    for o, d in [(0, 99), (9, 90), (45, 54), (99, 0)]:
        r = oracle_mod.route(net, cost, o, d)
        dist = oracle_mod.route_dist(net, cost, d)
        v = o
        for e in r:
            outs = np.nonzero(net.edge_from == v)[0]
            c = cost[outs] + dist[net.edge_to[outs]]
            assert e == outs[np.lexsort((outs, c))[0]]
            v = int(net.edge_to[e])
        assert v == d and len(r) == int(round(dist[o] / 10.0))
