"""Pins for case 1 intersections (flashing red, Sec. II-D and the red/green
light runs): a vehicle passes only after stopping 2 s at the line, one vehicle
crosses a node at a time, and the node serves its n x m (in, out) pairs
round-robin, the vehicles of a pair in the order they reached the line.
Admission is re-derived step by step in plain Python from the pre-step state
and the post-Phase-2 positions, with its own round-robin pointers."""
import math

import numpy as np
import pytest

import workloads as W

ACTIVE, WAITING = 1, 0


def case1(w):
    w.params.intersection_mode = 1
    return w


def _pairs(net):
    """(in, out) pair numbering: in-edge major, both in edge-id order."""
    V = int(max(net.edge_from.max(), net.edge_to.max())) + 1
    indeg, outdeg = np.zeros(V, int), np.zeros(V, int)
    in_idx, out_idx = np.zeros(net.n_edges, int), np.zeros(net.n_edges, int)
    for e in range(net.n_edges):
        in_idx[e] = indeg[net.edge_to[e]]
        indeg[net.edge_to[e]] += 1
        out_idx[e] = outdeg[net.edge_from[e]]
        outdeg[net.edge_from[e]] += 1
    return in_idx, out_idx, indeg * outdeg, outdeg


def test_brute_force_case1_admission(oracle_mod):
    w = case1(W.config1(n_vehicles=2000, n_steps=900))
    net = w.net
    sim = oracle_mod.OracleSim(w)
    vlen = w.params.veh_len[w.vclass]
    s0 = w.params.s0[w.vclass]
    lane_base = np.concatenate([[0], np.cumsum(net.lanes.astype(np.int64))])
    in_idx, out_idx, nm, outdeg = _pairs(net)
    rr = {}
    stop = math.ceil(2.0 / w.params.dt - 1e-6)
    served_multi = 0
    transfers = 0
    for step in range(800):
        pre = sim.state()
        sim.step(1)
        ev = sim.last_events()
        post = sim.state()
        act = np.nonzero(pre["status"] == ACTIVE)[0]
        rear = {}
        for i in act:
            g = lane_base[pre["edge"][i]] + ev["post_lane"][i]
            if g not in rear or (ev["xnew"][i], i) < (ev["xnew"][rear[g]], rear[g]):
                rear[g] = i
        node_reqs, lane_reqs = {}, {}
        for i in np.nonzero(ev["target_lane"] >= 0)[0]:
            g = int(ev["target_lane"][i])
            r = rear.get(g, -1)
            if pre["status"][i] == ACTIVE:
                e = int(pre["edge"][i])
                f = int(w.route_edges[w.route_off[i] + pre["cursor"][i] + 1])
                xp = ev["xnew"][i] - net.length[e]
                hs = int(pre["held_since"][i])
                room = r < 0 or (ev["xnew"][r] - vlen[r]) - xp >= 0
                ok = room and hs >= 0 and step - hs >= stop
                node = int(net.edge_from[f])
                pr = in_idx[e] * outdeg[node] + out_idx[f]
                dist = (pr - rr.get(node, -1) - 1) % nm[node]
                src = lane_base[e] + ev["post_lane"][i]
                if ok:
                    node_reqs.setdefault(node, []).append(((dist, hs, src), i, pr))
            else:
                ok = r < 0 or (ev["xnew"][r] - vlen[r]) >= s0[i]
                if ok:
                    lane_reqs.setdefault(g, []).append(((w.depart_step[i], i), i))
            assert bool(ev["flags"][i] & oracle_mod.EV["ELIG"]) == bool(ok), (step, i)
        winners, entered = set(), set()
        for node, rs in node_reqs.items():
            _, i, pr = min(rs)
            winners.add(i)
            entered.add(int(ev["target_lane"][i]))
            rr[node] = pr
            served_multi += len({x[2] for x in rs}) > 1
        for g, rs in lane_reqs.items():
            if g not in entered:
                winners.add(min(rs)[1])
        got = set(np.nonzero((ev["flags"] & oracle_mod.EV["WIN"]) != 0)[0].tolist())
        assert got == winners, step
        # one crossing per node per step, each after a stop of 2 s at the line
        crossed = [i for i in act if post["status"][i] == ACTIVE and post["edge"][i] != pre["edge"][i]]
        nodes = [int(net.edge_from[post["edge"][i]]) for i in crossed]
        assert len(nodes) == len(set(nodes)), step
        for i in crossed:
            assert pre["held_since"][i] >= 0 and step - pre["held_since"][i] >= stop
            assert pre["x"][i] == net.length[pre["edge"][i]] and pre["v"][i] == 0.0
        transfers += len(crossed)
    assert served_multi > 20 and transfers > 500


def test_case1_slower_than_case2_and_conserves(oracle_mod):
    """Config 1 under both controls: every vehicle still arrives; the stops
    make trips longer, and every transfer of case 1 is preceded by holds."""
    res = {}
    for mode in (0, 1):
        w = W.config1()
        w.params.intersection_mode = mode
        sim = oracle_mod.OracleSim(w)
        sim.step(3600)
        st = sim.state()
        c = sim.counters()
        assert c["departed"] == c["arrived"] == 2000
        res[mode] = (float(np.mean(st["t_arr"])), c)
    assert res[1][0] > res[0][0] + 30.0
    assert res[1][1]["holds"] >= 4 * res[1][1]["transfers"]


def test_lone_vehicle_waits_two_seconds_per_node(oracle_mod):
    """One vehicle on an empty 10x10 grid: at each node on its route it is held
    at the line for exactly ceil(2 s / dt) steps, then passes (nothing blocks it)."""
    for dt in (0.5, 0.3):
        w = case1(W.config1(n_vehicles=1, n_steps=0))
        w.params.dt = dt
        w.depart_step[:] = 0
        sim = oracle_mod.OracleSim(w)
        hops = int(w.route_off[1] - w.route_off[0]) - 1
        holds, t = 0, 0
        while sim.state()["status"][0] != 2 and t < 20000:
            sim.step(1)
            t += 1
        c = sim.counters()
        assert c["arrived"] == 1 and c["transfers"] == hops
        stop = math.ceil(2.0 / dt - 1e-6)
        # the first request is refused (not yet stopped), then stop - 1 more
        assert c["holds"] == hops * stop, (dt, c["holds"], hops, stop)
