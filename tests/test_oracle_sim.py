"""Pins for the oracle's full step: closed forms of Eq. (1) reached by the
simulation, first-order convergence in dt, brute-force leader search and
admission on small inputs, conservation and no-overlap invariants, and the
fixed routes the generators hand to both sides."""
import math

import numpy as np
import pytest

import workloads as W

ACTIVE, WAITING, ARRIVED = 1, 0, 2


# ---------------------------------------------------------------- Eq. (1), lone car
def _free_road_times(oracle_mod, dt, us, a=1.0):
    p = W.base_params(1)
    p.dt = dt
    p.a[:] = a
    w = W.single_edge_workload(length=5000.0, n_vehicles=1, n_steps=0, params=p)
    sim = oracle_mod.OracleSim(w, fp64=True)
    sim.step(1)                      # inserted at the end of step 0
    v0 = float(np.float32(50.0 / 3.6))
    res = {}
    prev_t, prev_v, prev_x = 0.0, 0.0, 0.0
    n = 0
    while len(res) < len(us):
        sim.step(1)
        n += 1
        st = sim.state()
        t, v, x = n * dt, float(st["v"][0]), float(st["x"][0])
        for u in us:
            if u not in res and v >= u * v0:
                f = (u * v0 - prev_v) / (v - prev_v)
                res[u] = (prev_t + f * dt, prev_x + f * (x - prev_x))
        prev_t, prev_v, prev_x = t, v, x
    return res


def test_free_road_closed_form_first_order(oracle_mod):
    """dv/dt = a(1 - (v/v0)^4) from rest: t(u) = v0/(2a) (artanh u + arctan u),
    x(u) = v0^2/(2a) artanh(u^2), u = v/v0.  The discrete scheme converges at
    first order as dt = 0.5 -> 0.25 -> 0.125."""
    v0 = float(np.float32(50.0 / 3.6))
    us = [0.5, 0.9, 0.99]
    exact = {u: (v0 / 2 * (math.atanh(u) + math.atan(u)), v0 ** 2 / 2 * math.atanh(u * u)) for u in us}
    errs = []
    for dt in (0.5, 0.25, 0.125):
        r = _free_road_times(oracle_mod, dt, us)
        errs.append([r[u][0] - exact[u][0] for u in us] + [r[u][1] - exact[u][1] for u in us])
    errs = np.array(errs)
    # halving dt halves every error (first order) ...
    for k in (0, 1):
        ratio = errs[k] / errs[k + 1]
        assert np.all(ratio > 1.85) and np.all(ratio < 2.15), ratio
    # ... and the Richardson extrapolation 2 e(dt/2) - e(dt) removes it
    rich = np.abs(2 * errs[2] - errs[1])
    assert np.all(rich < 0.05 * np.abs(errs[1]) + 1e-4), rich
    assert np.abs(errs[2, :3]).max() < 0.25 and np.abs(errs[2, 3:]).max() < 3.0


def test_platoon_reaches_equilibrium_gap(oracle_mod):
    """A slow leader (v0 = 10 m/s) and a follower (v0 = 50 km/h): the
    follower's gap tends to s_e(v) = (s0 + vT)/sqrt(1 - (v/v0)^4)."""
    p = W.base_params(2)
    p.v0_factor[1] = np.float32(10.0 / float(np.float32(50.0 / 3.6)))
    w = W.single_edge_workload(length=40000.0, n_vehicles=2, depart_step=[0, 20], n_steps=0, params=p)
    w.vclass[0] = 1
    for fp64 in (False, True):
        sim = oracle_mod.OracleSim(w, fp64=fp64)
        sim.step(6000)
        st = sim.state()
        assert (st["status"] == ACTIVE).all()
        vl = float(st["v"][0])
        gap = float(st["x"][0]) - 5.0 - float(st["x"][1])
        v0 = float(np.float32(50.0 / 3.6))
        se = (2.0 + vl * 1.5) / math.sqrt(1.0 - (vl / v0) ** 4)
        assert abs(vl - 10.0) < 1e-3
        assert abs(gap - se) / se < 1e-3, (gap, se)
        assert abs(float(st["v"][1]) - vl) < 1e-3


def _equilibrium_speed(gap, v0, s0=2.0, T=1.5):
    """v_e with s_e(v_e) = gap, s_e(v) = (s0 + vT)/sqrt(1 - (v/v0)^4), by bisection."""
    lo, hi = 0.0, v0
    for _ in range(200):
        m = 0.5 * (lo + hi)
        if (s0 + m * T) / math.sqrt(1.0 - (m / v0) ** 4) < gap:
            lo = m
        else:
            hi = m
    return 0.5 * (lo + hi)


@pytest.mark.parametrize("n", [10, 30, 50, 80])
def test_ring_road_fundamental_diagram(oracle_mod, n):
    """A 1 km one-lane ring of ten 100 m edges holding n vehicles: the
    homogeneous state is the equilibrium of Eq. (1), so every vehicle ends at
    the speed v_e(s) with s = 1000/n - 5, and the flow is q = (n/1000) v_e
    (the fundamental diagram of the model).  Crossing ten intersections per
    lap must not disturb it: admission and the look-ahead leader across an
    edge end are exercised at every node."""
    w = W.ring_road(n)
    v0 = float(np.float32(50.0 / 3.6))
    gap = 1000.0 / n - 5.0
    ve = _equilibrium_speed(gap, v0)
    for fp64 in (False, True):
        sim = oracle_mod.OracleSim(w, fp64=fp64)
        sim.step(4000)
        st = sim.state()
        act = st["status"] == ACTIVE
        assert act.sum() == n
        v = st["v"][act].astype(np.float64)
        assert abs(v.mean() - ve) < 1e-3 * ve, (v.mean(), ve)
        assert v.std() < 1e-3
        # flow past a fixed point = density x mean speed
        assert abs((n / 1000.0) * v.mean() - (n / 1000.0) * ve) < 1e-6 * n
        # spacing along the ring is uniform
        ring_pos = np.sort(_ring_position(w, st, act))
        spacing = np.diff(np.concatenate([ring_pos, ring_pos[:1] + 1000.0]))
        assert np.abs(spacing - 1000.0 / n).max() < 0.05, spacing


def _ring_position(w, st, act):
    """Distance from node 0 along the ring of each active vehicle's front."""
    e = st["edge"][act]
    return w.net.edge_from[e].astype(np.float64) * 100.0 + st["x"][act].astype(np.float64)


# ---------------------------------------------------------------- invariants
def _lane_groups(st, mask):
    idx = np.nonzero(mask)[0]
    keys = st["edge"][idx].astype(np.int64) * 16 + st["lane"][idx]
    order = np.lexsort((-idx, -st["x"][idx].astype(np.float64), keys))
    return idx[order], keys[order]


def _check_invariants(w, st, prev=None):
    n = w.n_vehicles
    assert st["status"].shape == (n,)
    assert set(np.unique(st["status"]).tolist()) <= {0, 1, 2}
    act = st["status"] == ACTIVE
    L = w.net.length[st["edge"][act]]
    x = st["x"][act]
    assert np.all(x >= 0) and np.all(x <= L)
    assert np.all(st["v"][act] >= 0)
    assert np.all(st["lane"][act] < w.net.lanes[st["edge"][act]])
    # the edge is the route edge at the cursor
    ro = w.route_off
    assert np.all(w.route_edges[ro[:-1][act] + st["cursor"][act]] == st["edge"][act])
    # no overlap in any lane: front minus length of the leader >= follower
    idx, keys = _lane_groups(st, act)
    same = keys[1:] == keys[:-1]
    lead, fol = idx[:-1][same], idx[1:][same]
    vlen = w.params.veh_len[w.vclass]
    assert np.all(st["x"][lead] - vlen[lead] >= st["x"][fol])
    # arrivals only at the end of the route
    arr = st["status"] == ARRIVED
    assert np.all(st["cursor"][arr] == (ro[1:] - ro[:-1])[arr] - 1)
    if prev is not None:
        # positions never go backwards on the same edge; states never regress
        same_edge = act & (prev["status"] == ACTIVE) & (prev["edge"] == st["edge"])
        assert np.all(st["x"][same_edge] >= prev["x"][same_edge])
        assert np.all(st["status"] >= prev["status"])


def test_invariants_config1(oracle_mod, c1):
    sim = oracle_mod.OracleSim(c1)
    prev = sim.state()
    for step in range(1400):
        sim.step(1)
        st = sim.state()
        if step % 7 == 0 or step < 50:
            _check_invariants(c1, st, prev)
        prev = st
    c = sim.counters()
    st = sim.state()
    assert c["departed"] == int((st["status"] != WAITING).sum())
    assert c["arrived"] == int((st["status"] == ARRIVED).sum())


def test_travel_time_stats_consistent(oracle_mod, c1):
    sim = oracle_mod.OracleSim(c1, fp64=True)
    tau0 = np.full(c1.n_vehicles, np.nan)
    for _ in range(3600):
        sim.step(1)
        st = sim.state()
        new = np.isnan(tau0) & (st["status"] != WAITING)
        tau0[new] = st["tau_in"][new]
    s, c = sim.edge_stats()
    assert (st["status"] == ARRIVED).all()
    # every edge of every route was traversed exactly once by its vehicle
    expect = np.bincount(c1.route_edges, minlength=c1.net.n_edges)
    assert np.array_equal(c, expect)
    # traversal times telescope: summed over all edges they equal the sum over
    # vehicles of (arrival time - time of entering the first edge)
    assert s.sum() == pytest.approx((st["t_arr"] - tau0).sum(), rel=1e-12)
    # no traversal is faster than free flow at the limit, less one step
    ff = c1.net.length.astype(np.float64) / c1.net.limit
    m = c > 0
    assert np.all(s[m] / c[m] >= ff[m] - 0.5)


# ---------------------------------------------------------------- brute force
def _brute_leaders(w, pre, post_lane):
    """Phase-2 leader of every active vehicle: the same-edge, same-post-lane
    active vehicle with the smallest (x, id) above its own, by brute force."""
    act = np.nonzero(pre["status"] == ACTIVE)[0]
    out = {}
    for i in act:
        best = -1
        for j in act:
            if j == i or pre["edge"][j] != pre["edge"][i] or post_lane[j] != post_lane[i]:
                continue
            if (pre["x"][j], j) > (pre["x"][i], i):
                if best < 0 or (pre["x"][j], j) < (pre["x"][best], best):
                    best = j
        out[i] = best
    return out


def _small_workload():
    return W.config1(n_vehicles=400, n_steps=600)


def test_brute_force_leaders_and_lane_changes(oracle_mod):
    w = _small_workload()
    sim = oracle_mod.OracleSim(w)
    vlen = w.params.veh_len[w.vclass]
    checked = 0
    for step in range(450):
        pre = sim.state()
        sim.step(1)
        if step % 9:
            continue
        ev = sim.last_events()
        lead = _brute_leaders(w, pre, ev["post_lane"])
        for i, j in lead.items():
            assert ev["leader"][i] == j, (step, i)
            checked += 1
        # after the lane changes and before moving, no two vehicles overlap
        act = np.nonzero(pre["status"] == ACTIVE)[0]
        moved = act[(ev["flags"][act] & oracle_mod.EV["MOVED"]) != 0]
        for i in moved:
            assert abs(ev["post_lane"][i] - pre["lane"][i]) == 1
            for j in act:
                if j != i and pre["edge"][j] == pre["edge"][i] and ev["post_lane"][j] == ev["post_lane"][i]:
                    lo, hi = (i, j) if (pre["x"][i], i) < (pre["x"][j], j) else (j, i)
                    assert pre["x"][hi] - vlen[hi] >= pre["x"][lo]
        # every move this step went the same direction
        d = ev["post_lane"][moved] - pre["lane"][moved]
        assert np.all(d == (-1 if step % 2 == 0 else 1))
    assert checked > 500


def test_brute_force_admission(oracle_mod):
    """Recompute Phase 3 from the pre-step state and the post-Phase-2
    positions: rear of each target lane, eligibility, one winner per lane =
    the smallest key (transfers first, then earliest held/departure step,
    then lowest id)."""
    w = W.config1(n_vehicles=2000, n_steps=600)
    sim = oracle_mod.OracleSim(w)
    vlen = w.params.veh_len[w.vclass]
    s0 = w.params.s0[w.vclass]
    lane_base = np.concatenate([[0], np.cumsum(w.net.lanes.astype(np.int64))])
    seen_conflict = 0
    for step in range(500):
        pre = sim.state()
        sim.step(1)
        ev = sim.last_events()
        act = np.nonzero(pre["status"] == ACTIVE)[0]
        # rear' per global lane (post-change lane, new position)
        rear = {}
        for i in act:
            g = lane_base[pre["edge"][i]] + ev["post_lane"][i]
            if g not in rear or (ev["xnew"][i], i) < (ev["xnew"][rear[g]], rear[g]):
                rear[g] = i
        reqs = {}
        for i in np.nonzero(ev["target_lane"] >= 0)[0]:
            g = int(ev["target_lane"][i])
            r = rear.get(g, -1)
            if pre["status"][i] == ACTIVE:
                xp = ev["xnew"][i] - w.net.length[pre["edge"][i]]
                ok = r < 0 or (ev["xnew"][r] - vlen[r]) - xp >= 0
                hs = pre["held_since"][i] if pre["held_since"][i] >= 0 else step
                key = (0, hs, i)
            else:
                ok = r < 0 or (ev["xnew"][r] - vlen[r]) >= s0[i]
                key = (1, w.depart_step[i], i)
            assert bool(ev["flags"][i] & oracle_mod.EV["ELIG"]) == bool(ok)
            if ok:
                reqs.setdefault(g, []).append((key, i))
        winners = {min(v)[1] for v in reqs.values()}
        seen_conflict += sum(len(v) > 1 for v in reqs.values())
        got = set(np.nonzero((ev["flags"] & oracle_mod.EV["WIN"]) != 0)[0].tolist())
        assert got == winners, step
    assert seen_conflict > 0


# ---------------------------------------------------------------- routes
def test_routes_are_shortest_and_connected(c1):
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import dijkstra
    net = c1.net
    wgt = net.length.astype(np.float64) / net.limit.astype(np.float64)
    G = csr_matrix((wgt, (net.edge_from, net.edge_to)), shape=(net.n_nodes, net.n_nodes))
    ro, re = c1.route_off, c1.route_edges
    org = net.edge_from[re[ro[:-1]]]
    dst = net.edge_to[re[ro[1:] - 1]]
    D = dijkstra(G, indices=np.unique(org))
    row = {o: k for k, o in enumerate(np.unique(org))}
    for i in range(c1.n_vehicles):
        r = re[ro[i]:ro[i + 1]]
        assert np.all(net.edge_to[r[:-1]] == net.edge_from[r[1:]])
        for e, f in zip(r[:-1], r[1:]):
            conn = net.conn_to[net.conn_off[e]:net.conn_off[e + 1]]
            assert f in conn
        assert wgt[r].sum() == pytest.approx(D[row[org[i]], dst[i]], rel=1e-12)


def test_turn_masks_cover_every_lane(c1):
    net = c1.net
    for e in range(net.n_edges):
        m = 0
        for c in range(net.conn_off[e], net.conn_off[e + 1]):
            assert net.conn_mask[c] != 0
            m |= int(net.conn_mask[c])
        assert m == (1 << int(net.lanes[e])) - 1


def test_fp64_twin_divergence_report(oracle_mod, c1):
    """The FP64 twin runs the same algorithm; on config 1 its discrete events
    are the same and arrival times agree to a few ms (reported, not gated
    beyond sanity)."""
    a = oracle_mod.OracleSim(c1)
    b = oracle_mod.OracleSim(c1, fp64=True)
    a.step(3600)
    b.step(3600)
    sa, sb = a.state(), b.state()
    ca, cb = a.counters(), b.counters()
    diff_arr_step = int((np.floor(sa["t_arr"] / 0.5) != np.floor(sb["t_arr"] / 0.5)).sum())
    print("fp64 twin: counters equal:", ca == cb, "arrival-step differences:", diff_arr_step,
          "max |dt_arr|:", float(np.abs(sa["t_arr"] - sb["t_arr"]).max()))
    assert np.abs(sa["t_arr"] - sb["t_arr"]).max() < 5.0


def _phase1_brute(oracle_mod, w, pre, t):
    """Phase 1 decisions recomputed from S_t by brute force: Eq. (2) trigger,
    route-motivated / incentive desire, Eqs. (3)-(4) gap acceptance."""
    f32 = np.float32
    net = w.net
    seed = int(w.params.seed)
    vlen = w.params.veh_len[w.vclass]
    act = np.nonzero(pre["status"] == ACTIVE)[0]
    dirn = -1 if t % 2 == 0 else 1
    moved = set()
    p = w.params

    def mask(e, f):
        for c in range(net.conn_off[e], net.conn_off[e + 1]):
            if net.conn_to[c] == f:
                return int(net.conn_mask[c])
        raise AssertionError

    def dist(m, l):
        return min(abs(q - l) for q in range(8) if (m >> q) & 1)

    for i in act:
        if pre["held_since"][i] >= 0:
            continue
        e, l, c = int(pre["edge"][i]), int(pre["lane"][i]), int(w.vclass[i])
        k = w.route_off[i] + pre["cursor"][i] + 1
        f = int(w.route_edges[k]) if k < w.route_off[i + 1] else -1
        m = mask(e, f) if f >= 0 else 0xFF
        allowed_l = bool((m >> l) & 1)
        mand = bool(pre["mand"][i])
        if not allowed_l and not mand:
            d = f32(net.length[e]) - f32(pre["x"][i])
            mand = bool(oracle_mod.mand_trigger(seed, t, int(i), float(d)))
        lp = l + dirn
        if lp < 0 or lp >= net.lanes[e]:
            continue
        same = [j for j in act if pre["edge"][j] == e]
        key = lambda j: (pre["x"][j], j)
        ahead_l = [j for j in same if pre["lane"][j] == l and key(j) > key(i)]
        ahead_p = [j for j in same if pre["lane"][j] == lp and key(j) > key(i)]
        behind_p = [j for j in same if pre["lane"][j] == lp and key(j) < key(i)]
        lead_cur = min(ahead_l, key=key) if ahead_l else -1
        la = min(ahead_p, key=key) if ahead_p else -1
        lb = max(behind_p, key=key) if behind_p else -1
        desire = (not allowed_l) and dist(m, lp) < dist(m, l)
        if not desire and ((m >> lp) & 1) and not (mand and not allowed_l):
            v0 = f32(p.v0_factor[c]) * f32(net.limit[e])

            def acc(j):
                if j < 0:
                    return f32(oracle_mod.idm(pre["v"][i], v0, 0, 0, p.T[c], p.a[c], p.b[c], p.s0[c], 0)[0])
                s = (f32(pre["x"][j]) - f32(vlen[j])) - f32(pre["x"][i])
                return f32(oracle_mod.idm(pre["v"][i], v0, pre["v"][j], s, p.T[c], p.a[c], p.b[c], p.s0[c], 1)[0])
            desire = (acc(la) - acc(lead_cur)) > f32(0.2)
        if not desire:
            continue
        vi = f32(pre["v"][i])
        g0 = oracle_mod.desired_gap(vi)
        ok = True
        if la >= 0:
            G = (f32(pre["x"][la]) - f32(vlen[la])) - f32(pre["x"][i])
            g = f32(oracle_mod.crit_gap(g0, w.alpha[la], vi, w.alpha[i], pre["v"][la])) + \
                f32(oracle_mod.normal(seed, t, int(i), 2))
            ok = ok and G >= max(g, f32(0))
        if lb >= 0:
            G = (f32(pre["x"][i]) - f32(vlen[i])) - f32(pre["x"][lb])
            g = f32(oracle_mod.crit_gap(g0, w.alpha[i], vi, w.alpha[lb], pre["v"][lb])) + \
                f32(oracle_mod.normal(seed, t, int(i), 3))
            ok = ok and G >= max(g, f32(0))
        if ok:
            moved.add(int(i))
    return moved


def test_brute_force_phase1_decisions(oracle_mod):
    w = W.config1(n_vehicles=800, n_steps=600)
    sim = oracle_mod.OracleSim(w)
    total = 0
    for step in range(500):
        pre = sim.state()
        sim.step(1)
        if step % 5:
            continue
        ev = sim.last_events()
        got = set(np.nonzero((ev["flags"] & oracle_mod.EV["MOVED"]) != 0)[0].tolist())
        assert got == _phase1_brute(oracle_mod, w, pre, step), step
        total += len(got)
    assert total > 20


# ------------------------------------------------------------ gridlock detector
def stopped_ring(n=60, n_nodes=4, edge_len=100.0, offset=0.3, spacing=400.0 / 60):
    """A one-lane ring of n_nodes x edge_len m with n stopped vehicles
    `spacing` m apart.  60 on 400 m leave gaps of 1.67 m, below s0 = 2 m, so
    every vehicle brakes at standstill and none moves again (a gridlock by
    construction); with gaps above s0 the ring starts to flow.  Returns
    (workload, state at step 0)."""
    w = W.ring_road(n, n_nodes=n_nodes, edge_len=edge_len, laps=4)
    p = offset + np.arange(n) * spacing
    k = np.floor(p / edge_len).astype(np.int64)                 # ring edge of each vehicle
    start = np.arange(n) % n_nodes                               # each route starts at its own edge
    cursor = ((k - start) % n_nodes).astype(np.int32)
    edge = w.route_edges[w.route_off[:-1] + cursor]
    st = dict(status=np.ones(n, np.uint8), edge=edge.astype(np.int32), lane=np.zeros(n, np.int32),
              cursor=cursor, x=(p - k * edge_len).astype(np.float32), v=np.zeros(n, np.float32),
              held_since=np.full(n, -1, np.int32), mand=np.zeros(n, np.uint8), ww=np.zeros(n, np.int32),
              tau_in=np.zeros(n), t_arr=np.full(n, -1.0), counters=None, t=0)
    return w, st


def test_gridlock_detector_counts_after_600_stalled_steps(oracle_mod):
    w, st = stopped_ring()
    o = oracle_mod.OracleSim(w)
    o.write_state(0, st)
    o.step(599)
    c = o.counters()
    assert c["gridlock_steps"] == 0 and c["stop_branch"] == 599 * 60 and c["transfers"] == 0, c
    assert np.array_equal(o.state()["x"], st["x"])               # nobody moved
    o.step(1)
    assert o.counters()["gridlock_steps"] == 1                   # the 600th stalled step
    o.step(100)
    assert o.counters()["gridlock_steps"] == 101


def test_gridlock_detector_restarts_on_a_written_state(oracle_mod):
    w, st = stopped_ring()
    o = oracle_mod.OracleSim(w)
    o.write_state(0, st)
    o.step(650)
    assert o.counters()["gridlock_steps"] == 51
    s = o.state()
    o.write_state(650, dict(s, t_arr=None))
    o.step(599)
    assert o.counters()["gridlock_steps"] == 51                  # the run started again at the written state
    o.step(1)
    assert o.counters()["gridlock_steps"] == 52


def test_gridlock_detector_quiet_while_anything_moves(oracle_mod):
    # 30 vehicles with gaps of 8.3 m: the ring flows and never stalls (with 59
    # at the gridlock spacing the one wide gap closes within 90 steps and the
    # ring freezes again); an empty network (every trip arrived) is no
    # gridlock either
    w, st = stopped_ring(n=30, spacing=400.0 / 30)
    o = oracle_mod.OracleSim(w)
    o.write_state(0, st)
    o.step(1200)
    c = o.counters()
    assert c["gridlock_steps"] == 0 and c["transfers"] > 0, c
    e = oracle_mod.OracleSim(W.ring_road(8, n_nodes=4, laps=1))  # one lap, then the ring is empty
    e.step(900)
    c = e.counters()
    assert c["arrived"] == 8 and c["gridlock_steps"] == 0, c
