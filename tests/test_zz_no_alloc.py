"""The entry point that allocates nothing (sim_shortest_routes_noalloc)
against sim_shortest_routes: the same routes, edge for edge, on two calls in
a row (the second smaller, so it runs on what the first left in the fixed
region), a call beyond the region refused with SIM_EINVAL, and a call after
that still right."""
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


def _queries(net, n, seed):
    rng = np.random.default_rng(seed)
    o = rng.integers(0, net.n_nodes, n).astype(np.int32)
    d = rng.integers(0, net.n_nodes, n).astype(np.int32)
    d[o == d] = (d[o == d] + 1) % net.n_nodes
    return o, d


def _same(M, net, cost, o, d):
    a_off, a_edges = M.shortest_routes(net, cost, o, d)
    b_off, b_edges = M.shortest_routes_noalloc(net, cost, o, d)
    assert np.array_equal(a_off, b_off)
    assert np.array_equal(a_edges, b_edges)
    return b_off, b_edges


def test_noalloc_routes_equal_the_allocating_entry_point(M):
    w = W.scaled_config2(n_vehicles=10, rows=30, cols=30, n_steps=10)
    net = w.net
    cost = ((net.length / net.limit) * np.random.default_rng(3).uniform(0.5, 2.0, net.n_edges)).astype(np.float32)
    o, d = _queries(net, 3000, 1)                      # about 900 destinations
    off1, e1 = _same(M, net, cost, o, d)
    assert e1.size > 10 * o.size
    # a second, smaller call on a smaller network
    g = W.config1(n_vehicles=10, n_steps=10).net
    gcost = (g.length / g.limit).astype(np.float32)
    o2, d2 = _queries(g, 100, 2)
    _same(M, g, gcost, o2, d2)


def test_noalloc_refuses_more_than_its_region(M):
    w = W.config2(n_vehicles=10, n_steps=10)           # 10,040 nodes
    net = w.net
    cost = (net.length / net.limit).astype(np.float32)
    o, d = _queries(net, 4000, 4)                      # labels alone: about 4 x 10,040 x 3,300 bytes > 64 MiB
    with pytest.raises(M.SimError) as ei:
        M.shortest_routes_noalloc(net, cost, o, d)
    assert ei.value.name == "SIM_EINVAL" and "scratch" in str(ei.value)
    # the region is still usable afterwards
    g = W.config1(n_vehicles=10, n_steps=10).net
    o2, d2 = _queries(g, 50, 5)
    _same(M, g, (g.length / g.limit).astype(np.float32), o2, d2)
