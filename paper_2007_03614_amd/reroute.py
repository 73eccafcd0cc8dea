"""Dynamic re-routing on current travel times (routes of Sec. II-C, which the
paper computes once, re-computed during a run): the vehicles that have not
yet reached their departure step get the shortest route from their origin to
their destination on the given edge costs (``shortest_routes`` on the GPU);
the run continues on a new handle from the current state."""
from __future__ import annotations

import copy

import numpy as np

from . import shortest_routes


def reroute_future_departures(workload, state: dict, cost: np.ndarray):
    """Returns (workload with the new routes, the state to write into a handle
    created from it).  Vehicles whose departure step is after state["t"] and
    that are still waiting are re-routed; every other route is kept.  The
    returned state carries no arrival times (the oracle's state input has
    none) and no counters."""
    t = int(state["t"])
    net = workload.net
    roff, redges = workload.route_off, workload.route_edges
    fut = np.nonzero((workload.depart_step > t) & (np.asarray(state["status"]) == 0))[0]
    o = net.edge_from[redges[roff[fut]]].astype(np.int32)
    d = net.edge_to[redges[roff[fut + 1] - 1]].astype(np.int32)
    off, edges = shortest_routes(net, cost, o, d)
    lens = np.diff(roff).astype(np.int64)
    lens[fut] = np.diff(off)
    new_off = np.zeros(roff.size, np.int64)
    new_off[1:] = np.cumsum(lens)
    new_edges = np.empty(int(new_off[-1]), np.int32)
    keep = np.ones(workload.n_vehicles, bool)
    keep[fut] = False
    for i in np.nonzero(keep)[0]:
        new_edges[new_off[i]:new_off[i + 1]] = redges[roff[i]:roff[i + 1]]
    for k, i in enumerate(fut):
        new_edges[new_off[i]:new_off[i + 1]] = edges[off[k]:off[k + 1]]
    w2 = copy.copy(workload)
    w2.route_off, w2.route_edges = new_off, new_edges
    st = {k: np.array(v, copy=True) for k, v in state.items() if k not in ("counters", "t")}
    st["edge"][fut] = new_edges[new_off[fut]]
    st["cursor"][fut] = 0
    st["t_arr"] = np.full(workload.n_vehicles, -1.0)
    st.update(counters=None, t=t)
    return w2, st
