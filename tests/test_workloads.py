"""The seeded input generators: the metropolitan-scale network and demand,
routing by destination, the turn-lane rule, and the mid-run states built from
the demand.  Each is checked against a plain restatement of what it must
produce (brute force on small sizes), not against itself."""
import math

import numpy as np
import pytest

import workloads as W


def _turn_masks_loop(net):
    """The turn-lane rule written out one edge at a time."""
    E = net.n_edges
    fr, to = net.edge_from, net.edge_to
    out_start = np.searchsorted(fr, np.arange(net.n_nodes + 1))
    off, cto, cmask = [0], [], []
    for e in range(E):
        u, v = int(fr[e]), int(to[e])
        outs = list(range(out_start[v], out_start[v + 1]))
        cand = [f for f in outs if int(to[f]) != u] or outs
        dxi, dyi = net.node_x[v] - net.node_x[u], net.node_y[v] - net.node_y[u]
        ang = []
        for f in cand:
            w = int(to[f])
            dx, dy = net.node_x[w] - net.node_x[v], net.node_y[w] - net.node_y[v]
            ang.append((math.atan2(dxi * dy - dyi * dx, dxi * dx + dyi * dy), f))
        ang.sort()
        m, L = len(ang), int(net.lanes[e])
        row = []
        for k, (_, f) in enumerate(ang):
            lo = (k * L) // m
            hi = max(lo, -((-(k + 1) * L) // m) - 1)
            row.append((f, sum(1 << q for q in range(lo, hi + 1))))
        row.sort()
        cto += [f for f, _ in row]
        cmask += [mk for _, mk in row]
        off.append(len(cto))
    return np.array(off), np.array(cto), np.array(cmask)


@pytest.fixture(scope="module")
def small_metro():
    return W.metro_network(rows=40, cols=41, n_segments=int(round(274_504 * 40 * 41 / (473 * 474))), seed=3)


@pytest.mark.parametrize("which", ["grid", "perturbed", "metro"])
def test_turn_lane_rule_matches_the_plain_loop(which, small_metro):
    net = {"grid": lambda: W.grid_network(), "perturbed": lambda: W.perturbed_grid_ring(rows=20, cols=20),
           "metro": lambda: small_metro}[which]()
    off, cto, cmask = _turn_masks_loop(net)
    assert np.array_equal(net.conn_off, off)
    assert np.array_equal(net.conn_to, cto)
    assert np.array_equal(net.conn_mask, cmask)


def test_metro_network_shape(small_metro):
    net = small_metro
    n = 40 * 41
    n_seg = int(round(274_504 * n / (473 * 474)))
    assert net.n_nodes == n and net.n_edges == 2 * n_seg
    # every segment is two-way and no segment repeats
    key = set(zip(net.edge_from.tolist(), net.edge_to.tolist()))
    assert len(key) == net.n_edges and all((b, a) in key for a, b in key)
    # connected: a breadth-first search from node 0 reaches every node
    adj = [[] for _ in range(n)]
    for a, b in key:
        adj[a].append(b)
    seen, todo = {0}, [0]
    while todo:
        u = todo.pop()
        for v in adj[u]:
            if v not in seen:
                seen.add(v)
                todo.append(v)
    assert len(seen) == n
    # lattice neighbours only: 4-neighbours or one diagonal per cell
    r, c = np.divmod(np.arange(n), 41)
    dr = np.abs(r[net.edge_from] - r[net.edge_to])
    dc = np.abs(c[net.edge_from] - c[net.edge_to])
    assert ((dr <= 1) & (dc <= 1) & (dr + dc >= 1)).all()
    diag = set()
    for a, b in key:
        if abs(r[a] - r[b]) == 1 and abs(c[a] - c[b]) == 1:
            diag.add((min(r[a], r[b]), min(c[a], c[b]), min(a, b), max(a, b)))
    cells = {}
    for rr, cc, a, b in diag:
        cells.setdefault((rr, cc), set()).add((a, b))
    assert all(len(s) == 1 for s in cells.values())      # planar: never both diagonals of a cell
    # lanes 1..5, limit 30..110 km/h within 10 km/h of 30 + 20 (lanes - 1), lengths clamped
    assert net.lanes.min() >= 1 and net.lanes.max() <= 5
    kmh = net.limit.astype(np.float64) * 3.6
    assert (kmh >= 30 - 1e-4).all() and (kmh <= 110 + 1e-4).all()
    assert (np.abs(kmh - np.clip(30 + 20 * (net.lanes - 1.0), 30, 110)) <= 10 + 1e-4).all()
    assert net.length.min() >= 25.0 and net.length.max() <= 2000.0


def test_metro_network_full_size_statistics():
    """The full-size network: the paper's 549,008 directed edges, the lane
    shares and the 120 m median length."""
    net = W.metro_network()
    assert net.n_nodes == 473 * 474 and net.n_edges == 549_008
    share = np.bincount(net.lanes, minlength=6)[1:] / net.n_edges
    assert np.allclose(share, W.METRO_LANE_P, atol=0.005)
    assert abs(np.median(net.length) - 120.0) < 1.5


def test_routing_by_destination_equals_routing_by_origin(small_metro):
    net = small_metro
    r = np.random.default_rng(0)
    o = r.integers(0, net.n_nodes, 3000).astype(np.int32)
    d = r.integers(0, net.n_nodes, 3000).astype(np.int32)
    a = W.shortest_routes(net, o, d)
    b = W.shortest_routes_to(net, o, d)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[2], o != d)
    w = net.length.astype(np.float64) / net.limit.astype(np.float64)
    for q in range(0, 3000, 7):
        if not a[2][q]:
            continue
        ra, rb = a[1][a[0][q]:a[0][q + 1]], b[1][b[0][q]:b[0][q + 1]]
        assert net.edge_from[rb[0]] == o[q] and net.edge_to[rb[-1]] == d[q]
        assert (net.edge_to[rb[:-1]] == net.edge_from[rb[1:]]).all()
        assert math.isclose(w[ra].sum(), w[rb].sum(), rel_tol=1e-12)


def test_routing_by_destination_is_shortest_brute_force():
    """Bellman-Ford by hand on a tiny network: every route's free-flow time
    equals the shortest one."""
    net = W.metro_network(rows=8, cols=9, n_segments=90, seed=1)
    w = net.length.astype(np.float64) / net.limit.astype(np.float64)
    n = net.n_nodes
    o = np.repeat(np.arange(n), n).astype(np.int32)
    d = np.tile(np.arange(n), n).astype(np.int32)
    ro, re_, ok = W.shortest_routes_to(net, o, d)
    for dst in range(n):
        dist = np.full(n, np.inf)
        dist[dst] = 0.0
        for _ in range(n):
            dist = np.minimum(dist, np.array([min([w[e] + dist[net.edge_to[e]]
                                                   for e in np.nonzero(net.edge_from == u)[0]] + [np.inf])
                                              if u != dst else 0.0 for u in range(n)]))
        for src in range(n):
            q = src * n + dst
            if src == dst:
                assert not ok[q]
                continue
            assert ok[q]
            assert math.isclose(w[re_[ro[q]:ro[q + 1]]].sum(), dist[src], rel_tol=1e-12)


def test_metro_demand(small_metro):
    net = small_metro
    o, d = W.metro_demand(net, 20_000, seed=0, pool_size=200, median_m=1500.0)
    pool = set(np.unique(d).tolist())
    assert len(pool) <= 200 and (o != d).all()
    assert o.min() >= 0 and o.max() < net.n_nodes
    # straight-line trip lengths: the drawn log-normal distance, up to the
    # snapping to the nearest pool node and the redraw of points outside
    dist = np.hypot(net.node_x[o] - net.node_x[d], net.node_y[o] - net.node_y[d])
    assert 800.0 < np.median(dist) < 2000.0


def test_config3_small_demand_and_classes():
    w = W.config3(n_vehicles=5000, rows=30, cols=31, pool_size=300, cache=False)
    assert w.n_vehicles == 5000 and w.n_steps == 50_400
    assert w.depart_step.min() >= 0 and w.depart_step.max() < 36_000          # 05:00-10:00
    # departures peak at 08:00 (step 21,600) with sd 45 min (5,400 steps)
    assert abs(np.median(w.depart_step) - 21_600) < 400
    assert 4500 < np.std(w.depart_step) < 6000
    assert set(np.unique(w.vclass).tolist()) == {0, 1, 2, 3}
    base = W.base_params(4)
    for k in ("v0_factor", "T", "b", "s0"):
        rel = getattr(w.params, k) / getattr(base, k) - 1.0
        assert (np.abs(rel) <= 0.1 + 1e-6).all() and np.abs(rel).max() > 0.0
    assert (w.params.a >= 1.0).all()          # a = 1 sits on its lower bound
    ro, re_ = w.route_off, w.route_edges
    inner = np.ones(re_.size - 1, bool)
    inner[ro[1:-1] - 1] = False
    assert (w.net.edge_to[re_[:-1]] == w.net.edge_from[re_[1:]])[inner].all()


def _check_state(w, s, t0, gap_m):
    """What a written state must satisfy, and what loaded_state promises."""
    st = s["status"]
    dep = w.depart_step
    assert ((st == 0) == (dep >= t0)).all()            # every vehicle due before t0 has left
    rl = np.diff(w.route_off)
    assert (s["cursor"] >= 0).all() and (s["cursor"] < rl).all()
    act = np.nonzero(st == 1)[0]
    e = s["edge"][act]
    assert (w.route_edges[w.route_off[act] + s["cursor"][act]] == e).all()
    assert (s["lane"][act] >= 0).all() and (s["lane"][act] < w.net.lanes[e]).all()
    x = s["x"][act]
    assert (x >= 0).all() and (x <= w.net.length[e]).all()
    assert (s["v"][act] >= 0).all() and (s["v"][act] <= w.net.limit[e]).all()
    order = np.lexsort((-act, -x, s["lane"][act], e))
    ge = e[order].astype(np.int64) * 8 + s["lane"][act][order]
    same = ge[1:] == ge[:-1]
    gaps = (x[order][:-1] - w.params.veh_len.max()) - x[order][1:]
    assert (gaps[same] >= gap_m - 1e-3).all()
    # most vehicles sit in a lane that may take their next move (the rest
    # were moved to another lane of their edge to find room)
    a2 = act[s["cursor"][act] + 1 < rl[act]]
    good = 0
    for i in a2:
        ee, ll = s["edge"][i], s["lane"][i]
        ff = w.route_edges[w.route_off[i] + s["cursor"][i] + 1]
        c0, c1 = w.net.conn_off[ee], w.net.conn_off[ee + 1]
        k = c0 + int(np.nonzero(w.net.conn_to[c0:c1] == ff)[0][0])
        good += (int(w.net.conn_mask[k]) >> int(ll)) & 1
    assert good >= 0.9 * a2.size


def test_loaded_state_is_valid_and_accepted_by_the_oracle(oracle_mod):
    w = W.config3(n_vehicles=20_000, rows=30, cols=31, pool_size=300, cache=False)
    t0 = 21_600
    s, info = W.loaded_state(w, t0, speed_frac=0.6, gap_m=2.5)
    assert info["active"] > 500 and info["arrived"] > 0 and info["waiting"] > 0
    assert info["active"] + info["arrived"] + info["waiting"] == w.n_vehicles
    _check_state(w, s, t0, 2.5)
    # the drive along the route: the time of entry into the current edge is
    # the departure plus the drive over the route's earlier edges
    act = np.nonzero(s["status"] == 1)[0][:300]
    tt = w.net.length.astype(np.float64) / (0.6 * w.net.limit.astype(np.float64))
    for i in act:
        k = s["cursor"][i]
        prev = w.route_edges[w.route_off[i]:w.route_off[i] + k]
        assert s["tau_in"][i] <= t0 * 0.5 + 1e-9
        assert s["tau_in"][i] >= w.depart_step[i] * 0.5 + tt[prev].sum() - tt[w.route_edges[w.route_off[i] + k]] - 1e-6
    o = oracle_mod.OracleSim(w)
    o.write_state(t0, s)
    o.step(20)
    c = o.counters()
    after = o.state()
    # conservation: vehicles only move between the three states in order
    assert c["departed"] == int(((s["status"] == 0) & (after["status"] != 0)).sum())
    assert c["arrived"] == int(((s["status"] != 2) & (after["status"] == 2)).sum())
    assert c["active_sum"] > 20 * info["active"] * 0.9


def test_oracle_threads_give_identical_results(oracle_mod):
    """Phases 1-2 run over vehicles in parallel; any thread count gives the
    same state, counters and per-edge sums bit for bit."""
    w = W.config3(n_vehicles=20_000, rows=30, cols=31, pool_size=300, cache=False)
    s, _ = W.loaded_state(w, 21_600)
    out = []
    for th in (1, 3):
        oracle_mod.set_threads(th)
        o = oracle_mod.OracleSim(w)
        o.write_state(21_600, s)
        o.step(60)
        out.append((o.state(), o.counters(), o.edge_stats()))
    oracle_mod.set_threads(1)
    (s1, c1, e1), (s3, c3, e3) = out
    assert c1 == c3
    for k in s1:
        assert np.array_equal(np.asarray(s1[k]), np.asarray(s3[k])), k
    assert np.array_equal(e1[0], e3[0]) and np.array_equal(e1[1], e3[1])
