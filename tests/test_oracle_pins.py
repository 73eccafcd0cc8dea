"""Pins for the parts of the oracle whose mistakes the whole-run tests would
not show: the crossing time inside a step (the per-edge traversal times of
Sec. IV-A, the calibration target), Phase 2's choice of leader kind (same-lane
vehicle, free road, stop line, look-ahead into the next edge's start-of-step
table), and the wrong-lane hold with its patience waiver.

Each test compares the oracle with something it does not compute itself:
closed forms of Eq. (1), exact kinematics at constant speed, or a plain
Python re-derivation from the start-of-step state S_t."""
import math

import numpy as np
import pytest

import workloads as W

ACTIVE, WAITING, ARRIVED = 1, 0, 2
f32 = np.float32


# ---------------------------------------------------------------- helpers
def _chain(lengths, lanes=1, limit=50.0 / 3.6):
    """Straight road of consecutive edges (node k at the sum of the first k
    lengths); the only move at an inner node is straight on."""
    xs = np.concatenate([[0.0], np.cumsum(lengths)])
    n = len(lengths)
    net = W._finish_edges(xs, np.zeros_like(xs), np.arange(n), np.arange(1, n + 1),
                          np.asarray(lengths, np.float32), np.full(n, limit, np.float32), np.full(n, lanes))
    fwd = [int(np.nonzero((net.edge_from == k) & (net.edge_to == k + 1))[0][0]) for k in range(n)]
    return net, fwd


def _workload(net, routes, params=None, depart=None):
    route_off = np.concatenate([[0], np.cumsum([len(r) for r in routes])]).astype(np.int64)
    route_edges = np.concatenate([np.asarray(r, np.int32) for r in routes])
    n = len(routes)
    dep = np.zeros(n, np.int32) if depart is None else np.asarray(depart, np.int32)
    return W.Workload("pin", net, route_off, route_edges, dep, np.zeros(n, np.uint8),
                      np.full(n, 0.2, np.float32), params or W.base_params(1), 0)


def _place(sim, t, vehicles):
    """Write an explicit state at step t: vehicles = list of dicts with edge,
    lane, cursor, x, v (and optionally mand, ww, held_since, tau_in); every
    other vehicle waits."""
    st = sim.state()
    n = sim.n
    s = {k: np.array(st[k]) for k in ("status", "edge", "lane", "cursor", "x", "v", "held_since", "mand", "ww",
                                       "tau_in")}
    s["status"][:] = WAITING
    for i, q in enumerate(vehicles):
        s["status"][i] = ACTIVE
        s["edge"][i] = q["edge"]
        s["lane"][i] = q["lane"]
        s["cursor"][i] = q.get("cursor", 0)
        s["x"][i] = q["x"]
        s["v"][i] = q["v"]
        s["held_since"][i] = q.get("held_since", -1)
        s["mand"][i] = q.get("mand", 0)
        s["ww"][i] = q.get("ww", 0)
        s["tau_in"][i] = q.get("tau_in", t * 0.5)
    sim.write_state(t, s)


# ---------------------------------------------------------------- crossing time
@pytest.mark.parametrize("fp64", [False, True])
def test_cruise_traversal_times_are_length_over_speed(oracle_mod, fp64):
    """A lone vehicle at exactly v0 keeps v0 (Eq. (1) on a free road gives
    acc = a(1 - 1) = 0), so it crosses every edge end at the exact time
    x/v0 and each recorded traversal lasts L/v0.  The lengths are chosen so
    the stop lines fall at different fractions of a step: a crossing time
    rounded to the step start or end, or interpolated from the wrong
    positions, is off by up to dt on some edge."""
    lengths = [200.0, 317.0, 451.25, 263.7, 389.9]
    net, fwd = _chain(lengths)
    w = _workload(net, [fwd])
    w.depart_step[:] = 10 ** 6             # never departs by itself: the state is written
    sim = oracle_mod.OracleSim(w, fp64=fp64)
    v0 = float(f32(50.0 / 3.6))
    t0 = 3
    _place(sim, t0, [dict(edge=fwd[0], lane=0, x=0.0, v=v0, tau_in=t0 * 0.5)])
    total = sum(lengths)
    sim.step(int(total / (v0 * 0.5)) + 3)
    st = sim.state()
    assert st["status"][0] == ARRIVED
    s, c = sim.edge_stats()
    got = np.array([s[e] for e in fwd])
    assert np.array_equal(np.array([c[e] for e in fwd]), np.ones(len(fwd)))
    expect = np.asarray([float(f32(L)) for L in lengths]) / v0
    tol = 1e-9 if fp64 else 2e-3           # positions accumulate binary32 rounding of x + v dt
    assert np.abs(got - expect).max() < tol, (got - expect)
    assert st["t_arr"][0] == pytest.approx(t0 * 0.5 + sum(float(f32(L)) for L in lengths) / v0, abs=5 * tol)


def _first_edge_time(oracle_mod, L, dt, fp64=True):
    p = W.base_params(1)
    p.dt = dt
    w = W.single_edge_workload(length=L, n_vehicles=1, n_steps=0, params=p)
    sim = oracle_mod.OracleSim(w, fp64=fp64)
    n = 0
    while sim.state()["status"][0] != ARRIVED:
        sim.step(1)
        n += 1
        assert n < 100000
    s, c = sim.edge_stats()
    assert c.sum() == 1
    return float(s.sum())


def test_first_edge_from_rest_converges_to_closed_form(oracle_mod):
    """From rest on a free road, dv/dt = a(1 - (v/v0)^4) reaches x = L at
    t(L) = v0/(2a) (artanh u + arctan u) with u = sqrt(tanh(2aL/v0^2)).  The
    recorded traversal (entry at x = 0 at the end of the departure step,
    exit interpolated inside the step) converges to it at first order: the
    error halves with dt, and the Richardson combination removes it.  A
    crossing time taken at a step boundary has an error that jumps with the
    phase of the stop line instead, and fails the ratio."""
    v0 = float(np.float32(50.0 / 3.6))
    for L in (150.0, 333.0, 1000.0):
        u = math.sqrt(math.tanh(2.0 * float(f32(L)) / v0 ** 2))
        exact = v0 / 2.0 * (math.atanh(u) + math.atan(u))
        dts = (0.5, 0.25, 0.125, 0.0625)
        err = np.array([_first_edge_time(oracle_mod, L, dt) - exact for dt in dts])
        ratio = err[:-1] / err[1:]
        assert np.all(ratio > 1.8) and np.all(ratio < 2.2), (L, err, ratio)
        rich = 2 * err[1:] - err[:-1]
        assert np.all(np.abs(rich) < 0.1 * np.abs(err[:-1])), (L, rich, err)
        assert abs(err[-1]) < 0.2


def _merge():
    """Two one-lane approaches (from nodes 0 and 1) merge at node 2 into one
    one-lane edge to node 3."""
    nx = np.array([-200.0, -200.0, 0.0, 200.0])
    ny = np.array([100.0, -100.0, 0.0, 0.0])
    net = W._finish_edges(nx, ny, np.array([0, 1, 2]), np.array([2, 2, 3]),
                          np.full(3, 300.0, np.float32), np.full(3, f32(50.0 / 3.6), np.float32), np.ones(3))
    e = lambda a, b: int(np.nonzero((net.edge_from == a) & (net.edge_to == b))[0][0])
    return net, e(0, 2), e(1, 2), e(2, 3)


def test_released_hold_crosses_at_the_step_start(oracle_mod):
    """Two fronts reach the merge in the same step; one lane takes one
    vehicle per step, so the higher id is refused and waits at x = L, v = 0
    until the winner has cleared the entry.  When it is admitted it has not
    moved before the line, so its crossing fraction is 0 and its traversal
    ends exactly at that step's start."""
    net, ea, eb, ec = _merge()
    w = _workload(net, [[ea, ec], [eb, ec]])
    w.depart_step[:] = 10 ** 6
    sim = oracle_mod.OracleSim(w)
    L = float(f32(300.0))
    _place(sim, 0, [dict(edge=ea, lane=0, x=L - 1.0, v=3.0, tau_in=0.0),
                    dict(edge=eb, lane=0, x=L - 1.0, v=3.0, tau_in=0.0)])
    sim.step(1)
    st = sim.state()
    assert st["edge"][0] == ec and st["edge"][1] == eb          # the lower id wins the lane
    assert st["held_since"][1] == 0 and st["x"][1] == L and st["v"][1] == 0.0
    held, exit_step = 1, None
    for t in range(1, 200):
        sim.step(1)
        st = sim.state()
        if st["edge"][1] == ec:
            exit_step = t
            break
        assert st["x"][1] == L and st["v"][1] == 0.0 and st["held_since"][1] == 0
        held += 1
    assert held >= 2 and exit_step is not None
    s, c = sim.edge_stats()
    assert c[eb] == 1 and c[ea] == 1
    assert s[eb] == exit_step * 0.5                  # crossed at the start of the winning step
    assert sim.state()["tau_in"][1] == exit_step * 0.5
    assert s[ea] != round(2 * s[ea]) / 2             # the winner crossed inside step 0


# ---------------------------------------------------------------- Phase 2 kinds
def _mask(net, e, f):
    for c in range(net.conn_off[e], net.conn_off[e + 1]):
        if net.conn_to[c] == f:
            return int(net.conn_mask[c])
    raise AssertionError((e, f))


def _phase2_brute(oracle_mod, w, pre, ev, t):
    """Phase 2 of every active vehicle re-derived from S_t and the post-change
    lanes: kind, partner, gap and leader speed, Eq. (1), the ballistic step,
    the clamp to the leader's start-of-step rear and the wrong-lane hold.
    Returns per-vehicle (kind, partner, xnew, vnew, flag bits) and how often
    the start-of-step rear of the look-ahead lane differs from its post-change
    rear (the cases that tell the two tables apart).  The mandatory flag and
    the wrong-lane wait after Phase 2 are returned as well: a move into an
    allowed lane clears both, a wrong-lane hold sets the flag and counts."""
    net, p = w.net, w.params
    vlen = p.veh_len[w.vclass].astype(np.float32)
    dt = f32(p.dt)
    act = np.nonzero(pre["status"] == ACTIVE)[0]
    x = pre["x"].astype(np.float32)
    v = pre["v"].astype(np.float32)
    # lane lists in (x, id) order: post-change lanes for leaders, start-of-step
    # lanes for the look-ahead table M_t
    post, start = {}, {}
    for i in act:
        post.setdefault((int(pre["edge"][i]), int(ev["post_lane"][i])), []).append(int(i))
        start.setdefault((int(pre["edge"][i]), int(pre["lane"][i])), []).append(int(i))
    keyf = lambda j: (x[j], j)
    rear_start = {k: min(vs, key=keyf) for k, vs in start.items()}
    rear_post = {k: min(vs, key=keyf) for k, vs in post.items()}
    out, differ = {}, 0
    for i in act:
        i = int(i)
        e, lp, c = int(pre["edge"][i]), int(ev["post_lane"][i]), int(w.vclass[i])
        k = w.route_off[i] + pre["cursor"][i] + 1
        f = int(w.route_edges[k]) if k < w.route_off[i + 1] else -1
        allowed = f < 0 or bool((_mask(net, e, f) >> lp) & 1)
        moved = lp != int(pre["lane"][i])
        mand = bool(pre["mand"][i]) or bool(ev["flags"][i] & oracle_mod.EV["MAND_TRIG"])
        ww = int(pre["ww"][i])
        if moved and allowed:
            mand, ww = False, 0
        ahead = [j for j in post[(e, lp)] if keyf(j) > keyf(i)]
        j = min(ahead, key=keyf) if ahead else -1
        L = f32(net.length[e])
        s = vl = f32(0)
        partner = -1
        if j >= 0:
            kind, partner = 1, j
            s = f32(f32(x[j] - vlen[j]) - x[i])
            vl = v[j]
        elif f < 0:
            kind = 0
        elif mand and not allowed and ww < 60:
            kind = 2
            s = f32(L - x[i])
        else:
            lam = min(lp, int(net.lanes[f]) - 1)
            r = rear_start.get((f, lam), -1)
            if rear_post.get((f, lam), -1) != r:
                differ += 1
            if r >= 0:
                kind, partner = 3, r
                s = f32(f32(L - x[i]) + f32(x[r] - vlen[r]))
                vl = v[r]
            else:
                kind = 0
        v0 = f32(f32(p.v0_factor[c]) * f32(net.limit[e]))
        acc = f32(oracle_mod.idm(float(v[i]), float(v0), float(vl), float(s), float(p.T[c]), float(p.a[c]),
                                 float(p.b[c]), float(p.s0[c]), kind)[0])
        bits = 0
        vn = f32(v[i] + f32(acc * dt))
        if vn >= 0:
            xn = f32(f32(x[i] + f32(v[i] * dt)) + f32(f32(f32(0.5) * acc) * f32(dt * dt)))
        else:
            xn = f32(x[i] - f32(f32(v[i] * v[i]) / f32(f32(2.0) * acc)))
            vn = f32(0)
            bits |= oracle_mod.EV["STOPB"]
        if kind == 1 and xn > f32(x[j] - vlen[j]):
            xn = f32(x[j] - vlen[j])
            bits |= oracle_mod.EV["CLAMP"]
        if f >= 0 and not allowed and ww < 60 and xn >= L:
            xn, vn = L, f32(0)
            bits |= oracle_mod.EV["WHOLD"]
        if bits & oracle_mod.EV["WHOLD"]:
            mand, ww = True, ww + 1
        out[i] = (kind, partner, xn, vn, bits, mand, ww)
    return out, differ


def test_brute_force_phase2_kinds_and_integration(oracle_mod):
    """Multi-lane config-1 steps: for every active vehicle the oracle's kind,
    partner, new position, new speed and clamp / stop / hold flags equal the
    re-derivation, bit for bit.  Every kind occurs, wrong-lane holds occur,
    and look-ahead lanes whose start-of-step rear differs from the
    post-change rear occur, so a look-ahead read from the wrong table
    would be caught."""
    w = W.config1(n_vehicles=2000, n_steps=900)
    sim = oracle_mod.OracleSim(w)
    flags = oracle_mod.EV["STOPB"] | oracle_mod.EV["CLAMP"] | oracle_mod.EV["WHOLD"]
    seen = np.zeros(4, int)
    holds = clamps = stops = differ = waits = 0
    for step in range(700):
        pre = sim.state()
        sim.step(1)
        if step < 60 or step % 4:
            continue
        ev = sim.last_events()
        post = sim.state()
        got, dif = _phase2_brute(oracle_mod, w, pre, ev, step)
        differ += dif
        for i, (kind, partner, xn, vn, bits, mand, ww) in got.items():
            if post["status"][i] == ACTIVE and post["edge"][i] == pre["edge"][i]:
                assert (bool(post["mand"][i]), int(post["ww"][i])) == (mand, ww), (step, i)
                waits += ww > 0
            assert ev["kind"][i] == kind, (step, i)
            assert ev["partner"][i] == partner, (step, i)
            assert f32(ev["xnew"][i]) == xn and f32(ev["vnew"][i]) == vn, (step, i, ev["xnew"][i], xn)
            assert (ev["flags"][i] & flags) == bits, (step, i)
            seen[kind] += 1
            holds += bool(bits & oracle_mod.EV["WHOLD"])
            clamps += bool(bits & oracle_mod.EV["CLAMP"])
            stops += bool(bits & oracle_mod.EV["STOPB"])
    assert np.all(seen > 0), seen
    assert holds > 0 and stops > 0 and differ > 0 and waits > 0, (holds, stops, differ, waits)


def test_same_lane_leader_comes_before_the_stop_line(oracle_mod):
    """A vehicle flagged for a mandatory change, in a lane that cannot take
    its turn, follows a same-lane leader (kind VEH) rather than stopping at
    the line: the leader is the nearer obstacle.  (A three-lane approach: the
    left turn takes lanes 1-2, the right turn lanes 0-1.)  On step 0 changes
    go right, so the left turner in lane 0 stays there."""
    net, e01, e12, e13 = _t_junction(lanes=3)
    assert _mask(net, e01, e12) == 3 and _mask(net, e01, e13) == 6
    w = _workload(net, [[e01, e13], [e01, e12]])
    w.depart_step[:] = 10 ** 6
    sim = oracle_mod.OracleSim(w)
    _place(sim, 0, [dict(edge=e01, lane=0, x=150.0, v=10.0, mand=1),
                    dict(edge=e01, lane=0, x=170.0, v=0.0)])
    pre = sim.state()
    sim.step(1)
    ev = sim.last_events()
    got, _ = _phase2_brute(oracle_mod, w, pre, ev, 0)
    assert got[0][0] == oracle_mod.KIND["VEH"] and got[0][1] == 1
    for i in (0, 1):
        kind, partner, xn, vn, bits, mand, ww = got[i]
        assert (ev["kind"][i], ev["partner"][i]) == (kind, partner)
        assert f32(ev["xnew"][i]) == xn and f32(ev["vnew"][i]) == vn


# ---------------------------------------------------------------- patience
def _t_junction(lanes=2):
    """Edge 0 -> 1 ends at a junction with a right turn (to node 2) and a
    left turn (to node 3); with two lanes the right turn takes lane 0 only,
    the left turn lane 1 only."""
    nx = np.array([0.0, 200.0, 200.0, 200.0])
    ny = np.array([0.0, 0.0, -200.0, 200.0])
    net = W._finish_edges(nx, ny, np.array([0, 1, 1]), np.array([1, 2, 3]),
                          np.full(3, 200.0, np.float32), np.full(3, f32(50.0 / 3.6), np.float32),
                          np.full(3, lanes))
    e = lambda a, b: int(np.nonzero((net.edge_from == a) & (net.edge_to == b))[0][0])
    return net, e(0, 1), e(1, 2), e(1, 3)


def test_wrong_lane_deadlock_waived_after_60_held_steps(oracle_mod):
    """Two vehicles side by side at the stop line, each in the lane the
    other needs (a right turner in the left lane, a left turner in the right
    lane): neither can change lanes (each overlaps the other), so each is held
    at the line, one held step after another, exactly 60 times.  The next step
    waives the lane restriction and both leave from their wrong lanes,
    counted as waived exits."""
    net, e01, e12, e13 = _t_junction()
    assert _mask(net, e01, e12) == 1 and _mask(net, e01, e13) == 2
    w = _workload(net, [[e01, e13], [e01, e12]])
    w.depart_step[:] = 10 ** 6
    sim = oracle_mod.OracleSim(w)
    L = float(f32(200.0))
    _place(sim, 0, [dict(edge=e01, lane=0, x=L, v=0.0, mand=1),
                    dict(edge=e01, lane=1, x=L, v=0.0, mand=1)])
    for t in range(60):
        sim.step(1)
        st = sim.state()
        assert np.all(st["edge"][:2] == e01), t
        assert np.all(st["ww"][:2] == t + 1) and np.all(st["x"][:2] == L) and np.all(st["v"][:2] == 0.0)
        ev = sim.last_events()
        assert np.all(ev["kind"][:2] == oracle_mod.KIND["STOP"])
        assert np.all(ev["flags"][:2] & oracle_mod.EV["WHOLD"])
    c = sim.counters()
    assert c["wrong_lane_holds"] == 120 and c["lane_changes"] == 0 and c["transfers"] == 0
    sim.step(1)                                     # step 60: patience exhausted
    st = sim.state()
    assert st["edge"][0] == e13 and st["edge"][1] == e12
    c = sim.counters()
    assert c["wrong_lane_holds"] == 120 and c["waived_exits"] == 2 and c["transfers"] == 2
    s, cnt = sim.edge_stats()
    assert cnt[e01] == 2 and s[e01] == 2 * 60 * 0.5   # both stood at x = L: crossed at the step start


def test_wrong_lane_vehicle_with_room_changes_lanes_instead(oracle_mod):
    """The same junction with the left lane empty: the left turner in the
    right lane moves over on the first step whose lane-change direction is
    to the left, is never held, and leaves from an allowed lane."""
    net, e01, e12, e13 = _t_junction()
    w = _workload(net, [[e01, e13]])
    w.depart_step[:] = 10 ** 6
    sim = oracle_mod.OracleSim(w)
    _place(sim, 0, [dict(edge=e01, lane=0, x=150.0, v=5.0)])
    for t in range(60):
        sim.step(1)
        if sim.state()["edge"][0] == e13:
            break
    c = sim.counters()
    assert sim.state()["edge"][0] == e13
    assert c["lane_changes"] == 1 and c["waived_exits"] == 0 and c["wrong_lane_holds"] == 0
