"""Seeded synthetic inputs for the per-timestep vehicle update.

This module is the only code shared by the CPU oracle (``oracle/``) and the
HIP path (``paper_2007_03614_amd/``).  It produces *inputs* only — road
networks, turn-lane masks, origin/destination demand, departure steps and
fixed routes — and holds none of the simulation arithmetic.

The paper's workloads (Sec. II-A network, II-B demand, II-C routing, II-D
departures) rely on OpenStreetMap and MTC data that are not available, so the
generators below build stand-ins with the shapes and distributions the paper
states: grid/planar road graphs with lanes, lengths and speed limits, origins
and destinations on nodes, departures drawn from a stated distribution, and
shortest routes on free-flow time computed before the simulation starts.

Every draw uses numpy ``PCG64`` seeded by ``SeedSequence(seed, spawn_key=(purpose,))``
so a workload is a pure function of (config, seed, overrides).
"""
from __future__ import annotations

import ctypes
import functools
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_DIJ_SRC = os.path.join(_HERE, "dijkstra.c")
_DIJ_SO = os.path.join(_HERE, "libdijkstra.so")

KMH = 1.0 / 3.6

# purposes for SeedSequence spawn keys
_P_NET, _P_DEL, _P_SEG, _P_OD, _P_DEP, _P_ALPHA, _P_CLASS, _P_SCEN, _P_HIDDEN = range(9)


def _rng(seed: int, purpose: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed, spawn_key=(purpose,))))


# --------------------------------------------------------------------------- build
def build_dijkstra(force: bool = False) -> str:
    """Compile the route generator's C Dijkstra (plain gcc, -O2)."""
    if force or not os.path.exists(_DIJ_SO) or os.path.getmtime(_DIJ_SO) < os.path.getmtime(_DIJ_SRC):
        tmp = _DIJ_SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread",
                               _DIJ_SRC, "-o", tmp])
        os.replace(tmp, _DIJ_SO)
    return _DIJ_SO


@functools.lru_cache(maxsize=1)
def _dij_lib():
    lib = ctypes.CDLL(build_dijkstra())
    P = ctypes.c_void_p
    lib.dij_solve.restype = P
    lib.dij_solve.argtypes = [ctypes.c_int32, P, P, P, P, P, ctypes.c_int32, P,
                              ctypes.c_int32, P, P, P, ctypes.c_int32]
    lib.dij_lengths.argtypes = [P, P]
    lib.dij_copy.argtypes = [P, P, P]
    lib.dij_free.argtypes = [P]
    return lib


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


# --------------------------------------------------------------------------- data
@dataclass
class Network:
    """Directed road network, edges sorted by (from, to).

    lanes: 1..8 per edge (lane 0 is the rightmost); length in metres;
    limit in m/s; conn_* is the CSR of allowed (e -> f) moves with a lane mask
    (bit l set: lane l of e may proceed to f)."""
    node_x: np.ndarray
    node_y: np.ndarray
    edge_from: np.ndarray
    edge_to: np.ndarray
    length: np.ndarray
    limit: np.ndarray
    lanes: np.ndarray
    conn_off: np.ndarray = None
    conn_to: np.ndarray = None
    conn_mask: np.ndarray = None

    @property
    def n_nodes(self) -> int:
        return int(self.node_x.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edge_from.shape[0])


@dataclass
class Params:
    """Per-class car-following parameters and run constants."""
    v0_factor: np.ndarray
    T: np.ndarray
    a: np.ndarray
    b: np.ndarray
    s0: np.ndarray
    veh_len: np.ndarray
    dt: float = 0.5
    seed: int = 0
    intersection_mode: int = 0
    record_every: int = 0
    v0_spread: float = 0.0     # per-driver v0: sigma_s = v0_spread * limit, drawn at 2 sigma_s

    @property
    def n_classes(self) -> int:
        return int(self.T.shape[0])


@dataclass
class Workload:
    name: str
    net: Network
    route_off: np.ndarray      # int64 [n_veh+1]
    route_edges: np.ndarray    # int32
    depart_step: np.ndarray    # int32 [n_veh]
    vclass: np.ndarray         # uint8 [n_veh]
    alpha: np.ndarray          # float32 [n_veh]
    params: Params
    n_steps: int
    info: dict = field(default_factory=dict)

    @property
    def n_vehicles(self) -> int:
        return int(self.depart_step.shape[0])


def base_params(n_classes: int = 1, seed: int = 0) -> Params:
    """The config-1 car-following parameters: v0 = limit, T = 1.5 s,
    a = 1.0, b = 2.0 m/s^2, s0 = 2 m, vehicle length 5 m."""
    f = lambda v: np.full(n_classes, v, dtype=np.float32)
    return Params(v0_factor=f(1.0), T=f(1.5), a=f(1.0), b=f(2.0), s0=f(2.0),
                  veh_len=f(5.0), seed=seed)


# calibration bounds of the car-following parameters (Sec. IV-A)
BOUNDS = dict(v0_factor=(0.05, 2.0), T=(0.1, 2.0), a=(1.0, 10.0), b=(1.0, 10.0), s0=(1.0, 5.0))


def jitter_params(p: Params, rel: float, seed: int, purpose: int = _P_CLASS) -> Params:
    """Each (class, parameter) scaled by (1 + U[-rel, rel]), then clipped to
    the calibration bounds (a = 1 sits on its lower bound)."""
    r = _rng(seed, purpose)
    k = p.n_classes

    def g(arr, name):
        lo, hi = BOUNDS[name]
        return np.clip(arr.astype(np.float64) * (1.0 + r.uniform(-rel, rel, size=k)), lo, hi).astype(np.float32)
    return Params(v0_factor=g(p.v0_factor, "v0_factor"), T=g(p.T, "T"), a=g(p.a, "a"), b=g(p.b, "b"),
                  s0=g(p.s0, "s0"),
                  veh_len=p.veh_len.copy(), dt=p.dt, seed=p.seed,
                  intersection_mode=p.intersection_mode, record_every=p.record_every, v0_spread=p.v0_spread)


# --------------------------------------------------------------------------- networks
def _finish_edges(nx, ny, seg_u, seg_v, seg_len, seg_lim, seg_lanes) -> Network:
    """Turn undirected segments into directed edges sorted by (from, to)."""
    fr = np.concatenate([seg_u, seg_v]).astype(np.int32)
    to = np.concatenate([seg_v, seg_u]).astype(np.int32)
    ln = np.concatenate([seg_len, seg_len]).astype(np.float32)
    li = np.concatenate([seg_lim, seg_lim]).astype(np.float32)
    la = np.concatenate([seg_lanes, seg_lanes]).astype(np.uint8)
    order = np.lexsort((to, fr))
    net = Network(node_x=np.asarray(nx, np.float64), node_y=np.asarray(ny, np.float64),
                  edge_from=fr[order], edge_to=to[order], length=ln[order],
                  limit=li[order], lanes=la[order])
    turn_lane_masks(net)
    return net


def turn_lane_masks(net: Network) -> None:
    """Connections and which lanes may take them (geometric rule).

    At node v, the moves out of incoming edge e = (u -> v) are all out-edges
    (v -> w) with w != u; a U-turn is allowed only at a dead end.  The moves
    are ranked by turn angle from rightmost to leftmost; with m moves and L
    lanes on e, rank k may use lanes floor(kL/m) .. max(floor(kL/m), ceil((k+1)L/m) - 1).
    """
    E = net.n_edges
    fr, to = net.edge_from, net.edge_to
    out_start = np.searchsorted(fr, np.arange(net.n_nodes + 1))
    conn_off = np.zeros(E + 1, np.int32)
    conn_to, conn_mask = [], []
    for e in range(E):
        u, v = int(fr[e]), int(to[e])
        outs = list(range(out_start[v], out_start[v + 1]))
        cand = [f for f in outs if int(to[f]) != u]
        if not cand:
            cand = outs  # dead end: U-turn
        dx_in = net.node_x[v] - net.node_x[u]
        dy_in = net.node_y[v] - net.node_y[u]
        angs = []
        for f in cand:
            w = int(to[f])
            dx = net.node_x[w] - net.node_x[v]
            dy = net.node_y[w] - net.node_y[v]
            cross = dx_in * dy - dy_in * dx
            dot = dx_in * dx + dy_in * dy
            angs.append((math.atan2(cross, dot), f))
        angs.sort()  # most negative (sharpest right) first; ties by edge id
        m = len(angs)
        L = int(net.lanes[e])
        row = []
        for k, (_, f) in enumerate(angs):
            lo = (k * L) // m
            hi = max(lo, -((-(k + 1) * L) // m) - 1)
            mask = 0
            for l in range(lo, hi + 1):
                mask |= 1 << l
            row.append((f, mask))
        row.sort()
        for f, mask in row:
            conn_to.append(f)
            conn_mask.append(mask)
        conn_off[e + 1] = len(conn_to)
    net.conn_off = conn_off
    net.conn_to = np.asarray(conn_to, np.int32)
    net.conn_mask = np.asarray(conn_mask, np.uint8)


def grid_network(rows: int = 10, cols: int = 10, spacing: float = 200.0, lanes: int = 2,
                 limit_kmh: float = 50.0) -> Network:
    """Regular grid, node id = cols*row + col, uniform segments."""
    ids = np.arange(rows * cols).reshape(rows, cols)
    nx = (np.arange(rows * cols) % cols) * spacing
    ny = (np.arange(rows * cols) // cols) * spacing
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    n = u.shape[0]
    lim = np.float32(np.float64(limit_kmh) / 3.6)
    return _finish_edges(nx, ny, u, v, np.full(n, spacing), np.full(n, lim), np.full(n, lanes))


def _largest_component(n_nodes, u, v):
    parent = np.arange(n_nodes)

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a
    for a, b in zip(u.tolist(), v.tolist()):
        ra, rb = find(a), find(b)
        if ra != rb:
            parent[max(ra, rb)] = min(ra, rb)
    roots = np.array([find(i) for i in range(n_nodes)])
    vals, counts = np.unique(roots, return_counts=True)
    return roots == vals[np.argmax(counts)]


def perturbed_grid_ring(rows: int = 100, cols: int = 100, spacing: float = 250.0,
                        delete_frac: float = 0.10, ring_nodes: int = 40, ring_offset: float = 1000.0,
                        seed: int = 0) -> Network:
    """Grid with a fraction of segments deleted (largest connected part kept;
    segments are two-way so it is strongly connected), 1-3 lanes,
    40-60 km/h, lengths U[100, 400] m, plus a 4-lane 100 km/h ring highway
    outside the grid joined to the nearest boundary node by 1-lane 60 km/h ramps."""
    rd = _rng(seed, _P_DEL)
    rs = _rng(seed, _P_SEG)
    ids = np.arange(rows * cols).reshape(rows, cols)
    gx = (np.arange(rows * cols) % cols) * spacing
    gy = (np.arange(rows * cols) // cols) * spacing
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    keep = np.ones(u.shape[0], bool)
    keep[rd.choice(u.shape[0], size=int(round(delete_frac * u.shape[0])), replace=False)] = False
    u, v = u[keep], v[keep]
    alive = _largest_component(rows * cols, u, v)
    m = alive[u] & alive[v]
    u, v = u[m], v[m]
    nseg = u.shape[0]
    lanes = rs.integers(1, 4, size=nseg)
    lim = (rs.uniform(40.0, 60.0, size=nseg) * KMH).astype(np.float32)
    length = rs.uniform(100.0, 400.0, size=nseg).astype(np.float32)
    # renumber kept grid nodes
    old = np.nonzero(alive)[0]
    newid = -np.ones(rows * cols, np.int64)
    newid[old] = np.arange(old.shape[0])
    u, v = newid[u], newid[v]
    nx, ny = list(gx[old]), list(gy[old])
    n_grid = old.shape[0]
    # ring: square loop ring_offset outside the grid, ring_nodes evenly spaced
    lo, hi = -ring_offset, (cols - 1) * spacing + ring_offset
    side = hi - lo
    per = 4 * side
    ring_xy = []
    for k in range(ring_nodes):
        s = per * k / ring_nodes
        if s < side:
            ring_xy.append((lo + s, lo))
        elif s < 2 * side:
            ring_xy.append((hi, lo + s - side))
        elif s < 3 * side:
            ring_xy.append((hi - (s - 2 * side), hi))
        else:
            ring_xy.append((lo, hi - (s - 3 * side)))
    ring_ids = list(range(n_grid, n_grid + ring_nodes))
    for (x, y) in ring_xy:
        nx.append(x)
        ny.append(y)
    nxa, nya = np.asarray(nx), np.asarray(ny)
    seg_u, seg_v = list(u), list(v)
    seg_len, seg_lim, seg_lanes = list(length), list(lim), list(lanes)
    for k in range(ring_nodes):
        a, b = ring_ids[k], ring_ids[(k + 1) % ring_nodes]
        seg_u.append(a); seg_v.append(b)
        seg_len.append(np.float32(math.hypot(nxa[a] - nxa[b], nya[a] - nya[b])))
        seg_lim.append(np.float32(100.0 * KMH)); seg_lanes.append(4)
    # ramps: each ring node to the nearest kept boundary grid node
    gxo, gyo = gx[old], gy[old]
    bnd = (gxo == 0) | (gyo == 0) | (gxo == (cols - 1) * spacing) | (gyo == (rows - 1) * spacing)
    bidx = np.nonzero(bnd)[0]
    for k in range(ring_nodes):
        r = ring_ids[k]
        d2 = (gxo[bidx] - nxa[r]) ** 2 + (gyo[bidx] - nya[r]) ** 2
        g = int(bidx[np.argmin(d2)])
        seg_u.append(r); seg_v.append(g)
        seg_len.append(np.float32(math.sqrt(float(np.min(d2)))))
        seg_lim.append(np.float32(60.0 * KMH)); seg_lanes.append(1)
    return _finish_edges(nxa, nya, np.asarray(seg_u), np.asarray(seg_v), np.asarray(seg_len, np.float32),
                         np.asarray(seg_lim, np.float32), np.asarray(seg_lanes))


# --------------------------------------------------------------------------- routing
def shortest_routes(net: Network, orig: np.ndarray, dst: np.ndarray, n_threads: int = 0):
    """Fixed routes on free-flow time (length / limit), one per OD row.

    Returns (route_off int64[n+1], route_edges int32, ok bool[n]); rows with
    O == D or no path get an empty route and ok = False."""
    lib = _dij_lib()
    E, N = net.n_edges, net.n_nodes
    out_off = np.searchsorted(net.edge_from, np.arange(N + 1)).astype(np.int32)
    out_edge = np.arange(E, dtype=np.int32)  # edges are sorted by from, ids ascending
    w = net.length.astype(np.float64) / net.limit.astype(np.float64)
    orig = np.asarray(orig, np.int32)
    dst = np.asarray(dst, np.int32)
    order = np.argsort(orig, kind="stable").astype(np.int32)
    uo, starts = np.unique(orig[order], return_index=True)
    grp_off = np.append(starts, order.shape[0]).astype(np.int32)
    grp_origin = uo.astype(np.int32)
    if n_threads <= 0:
        n_threads = min(16, os.cpu_count() or 1)
    edge_from = np.ascontiguousarray(net.edge_from, np.int32)
    edge_to = np.ascontiguousarray(net.edge_to, np.int32)
    res = lib.dij_solve(N, _ptr(out_off), _ptr(out_edge), _ptr(edge_from), _ptr(edge_to), _ptr(w),
                        int(orig.shape[0]), _ptr(dst), int(grp_origin.shape[0]), _ptr(grp_origin),
                        _ptr(grp_off), _ptr(order), int(n_threads))
    if not res:
        raise MemoryError("route generation failed")
    try:
        plen = np.empty(orig.shape[0], np.int32)
        lib.dij_lengths(res, _ptr(plen))
        ok = plen > 0
        route_off = np.zeros(orig.shape[0] + 1, np.int64)
        route_off[1:] = np.cumsum(np.maximum(plen, 0))
        route_edges = np.empty(int(route_off[-1]), np.int32)
        lib.dij_copy(res, _ptr(route_off), _ptr(route_edges))
    finally:
        lib.dij_free(res)
    return route_off, route_edges, ok


def _od_routes(net, n_veh, seed, nodes=None):
    """Uniform origin and destination nodes (O != D), routed."""
    r = _rng(seed, _P_OD)
    pool = np.arange(net.n_nodes) if nodes is None else np.asarray(nodes)
    o = pool[r.integers(0, pool.shape[0], size=n_veh)]
    d = pool[r.integers(0, pool.shape[0], size=n_veh)]
    same = o == d
    while same.any():
        d[same] = pool[r.integers(0, pool.shape[0], size=int(same.sum()))]
        same = o == d
    route_off, route_edges, ok = shortest_routes(net, o, d)
    if not ok.all():
        raise RuntimeError("network is not strongly connected")
    return route_off, route_edges, o, d


# --------------------------------------------------------------------------- configs
def config1(seed: int = 0, n_vehicles: int = 2000, n_steps: int = 3600, n_classes: int = 1) -> Workload:
    """10x10 grid of signal-free intersections, two-way 2-lane 200 m edges at
    50 km/h; uniform-random O/D nodes; departures U[0, 10 min); routes on
    free-flow time; base car-following parameters; dt = 0.5 s; 30 min."""
    net = grid_network()
    route_off, route_edges, _, _ = _od_routes(net, n_vehicles, seed)
    rdp = _rng(seed, _P_DEP)
    dep = np.floor(rdp.uniform(0.0, 600.0, size=n_vehicles) / 0.5).astype(np.int32)
    alpha = _rng(seed, _P_ALPHA).uniform(0.05, 0.40, size=n_vehicles).astype(np.float32)
    if n_classes == 1:
        vclass = np.zeros(n_vehicles, np.uint8)
    else:
        vclass = _rng(seed, _P_CLASS).integers(0, n_classes, size=n_vehicles).astype(np.uint8)
    p = base_params(n_classes, seed)
    return Workload("grid10x10", net, route_off, route_edges, dep, vclass, alpha, p, n_steps,
                    info={"departures": "U[0,600) s", "horizon_min": n_steps * 0.5 / 60})


@functools.lru_cache(maxsize=4)
def _c2_network(rows, cols, seed):
    return perturbed_grid_ring(rows=rows, cols=cols, seed=seed)


def config2(seed: int = 0, n_vehicles: int = 200_000, n_steps: int = 21_600, rows: int = 100,
            cols: int = 100) -> Workload:
    """Perturbed 100x100 grid (10% of segments deleted, largest connected part
    kept; 1-3 lanes, 40-60 km/h, 100-400 m) plus a 4-lane 100 km/h ring
    highway; departures N(08:00, 40 min) truncated to [06:30, 09:30); the run
    starts at 06:30 and lasts 3 h at dt = 0.5 s."""
    net = _c2_network(rows, cols, seed)
    route_off, route_edges, _, _ = _od_routes(net, n_vehicles, seed)
    r = _rng(seed, _P_DEP)
    t = r.normal(90.0 * 60.0, 40.0 * 60.0, size=n_vehicles)  # seconds after 06:30
    bad = (t < 0.0) | (t >= 3 * 3600.0)
    while bad.any():
        t[bad] = r.normal(90.0 * 60.0, 40.0 * 60.0, size=int(bad.sum()))
        bad = (t < 0.0) | (t >= 3 * 3600.0)
    dep = np.floor(t / 0.5).astype(np.int32)
    alpha = _rng(seed, _P_ALPHA).uniform(0.05, 0.40, size=n_vehicles).astype(np.float32)
    vclass = np.zeros(n_vehicles, np.uint8)
    return Workload(f"perturbed_grid{rows}x{cols}_ring", net, route_off, route_edges, dep, vclass, alpha,
                    base_params(1, seed), n_steps,
                    info={"departures": "N(08:00, 40 min) in [06:30, 09:30)", "start": "06:30"})


def single_edge_workload(length: float = 5000.0, limit: float = 50.0 / 3.6, lanes: int = 1,
                         n_vehicles: int = 1, depart_step=None, n_steps: int = 100,
                         params: Params = None) -> Workload:
    """A two-node network with one long edge each way; every vehicle drives
    the single edge 0 -> 1 and arrives at its end.  Used by closed-form tests."""
    nx = np.array([0.0, length])
    ny = np.array([0.0, 0.0])
    net = _finish_edges(nx, ny, np.array([0]), np.array([1]), np.array([length], np.float32),
                        np.array([limit], np.float32), np.array([lanes]))
    e01 = int(np.nonzero((net.edge_from == 0) & (net.edge_to == 1))[0][0])
    route_off = np.arange(n_vehicles + 1, dtype=np.int64)
    route_edges = np.full(n_vehicles, e01, np.int32)
    dep = np.zeros(n_vehicles, np.int32) if depart_step is None else np.asarray(depart_step, np.int32)
    alpha = np.full(n_vehicles, 0.2, np.float32)
    vclass = np.zeros(n_vehicles, np.uint8)
    return Workload("single_edge", net, route_off, route_edges, dep, vclass, alpha,
                    params or base_params(1), n_steps)


def ring_road(n_vehicles: int, n_nodes: int = 10, edge_len: float = 100.0, limit: float = 50.0 / 3.6,
              laps: int = 60, n_steps: int = 0, params: Params = None) -> Workload:
    """A one-lane ring road of n_nodes edges of edge_len metres (both
    directions exist; vehicles use the forward one).  Vehicle j enters at the
    start of edge j mod n_nodes at step 2 * (j // n_nodes) and drives `laps`
    laps.  For the fundamental diagram of the car-following model."""
    ang = 2.0 * math.pi * np.arange(n_nodes) / n_nodes
    rad = n_nodes * edge_len / (2.0 * math.pi)
    u = np.arange(n_nodes)
    net = _finish_edges(rad * np.cos(ang), rad * np.sin(ang), u, (u + 1) % n_nodes,
                        np.full(n_nodes, edge_len, np.float32), np.full(n_nodes, limit, np.float32),
                        np.ones(n_nodes, np.int64))
    fwd = np.empty(n_nodes, np.int32)
    for i in range(n_nodes):
        fwd[i] = int(np.nonzero((net.edge_from == i) & (net.edge_to == (i + 1) % n_nodes))[0][0])
    j = np.arange(n_vehicles)
    start = j % n_nodes
    route_edges = fwd[(start[:, None] + np.arange(laps * n_nodes)[None, :]) % n_nodes].astype(np.int32).ravel()
    route_off = np.arange(n_vehicles + 1, dtype=np.int64) * laps * n_nodes
    dep = (2 * (j // n_nodes)).astype(np.int32)
    return Workload(f"ring{n_nodes}x{int(edge_len)}_n{n_vehicles}", net, route_off, route_edges, dep,
                    np.zeros(n_vehicles, np.uint8), np.full(n_vehicles, 0.2, np.float32),
                    params or base_params(1), n_steps)


def scaled_config2(n_vehicles: int, rows: int, cols: int, n_steps: int, seed: int = 0) -> Workload:
    """Config 2's recipe on a smaller grid (for oracle-sized parity cases)."""
    w = config2(seed=seed, n_vehicles=n_vehicles, n_steps=n_steps, rows=rows, cols=cols)
    w.name = f"perturbed_grid{rows}x{cols}_ring_n{n_vehicles}"
    return w


def scenario_workload(master: Workload, n_vehicles: int, reduced_edges) -> Workload:
    """One what-if scenario on its own: the first n_vehicles of the master
    demand on the master network with `reduced_edges` cut to one lane (every
    move out of a reduced edge then leaves from lane 0)."""
    net = master.net
    lanes = net.lanes.copy()
    mask = net.conn_mask.copy()
    for e in np.asarray(reduced_edges, np.int64):
        lanes[e] = 1
        mask[net.conn_off[e]:net.conn_off[e + 1]] = 1
    n2 = Network(node_x=net.node_x, node_y=net.node_y, edge_from=net.edge_from, edge_to=net.edge_to,
                 length=net.length, limit=net.limit, lanes=lanes, conn_off=net.conn_off, conn_to=net.conn_to,
                 conn_mask=mask)
    ro = master.route_off[:n_vehicles + 1].copy()
    return Workload(f"{master.name}_scenario", n2, ro, master.route_edges[:int(ro[-1])].copy(),
                    master.depart_step[:n_vehicles].copy(), master.vclass[:n_vehicles].copy(),
                    master.alpha[:n_vehicles].copy(), master.params, master.n_steps)


def ensemble_scenarios(n_scen: int, base: int, n_edges: int, seed: int = 0, scale=(0.8, 1.2),
                       reduced_frac: float = 0.01):
    """Scenario list: demand round(U[scale] * base) vehicles of the master
    list and ceil(reduced_frac * n_edges) random edges cut to one lane."""
    r = _rng(seed, _P_SCEN)
    k = int(math.ceil(reduced_frac * n_edges))
    out = []
    for _ in range(n_scen):
        n = int(round(r.uniform(*scale) * base))
        red = np.sort(r.choice(n_edges, size=k, replace=False)).astype(np.int32)
        out.append((n, red))
    return out


def config4(seed: int = 0, n_scen: int = 64, base: int = 200_000, n_steps: int = 14_400):
    """Ensemble on the 10x10 grid: a master demand of 1.2 * base vehicles
    (uniform O/D, departures U[0, 2 h)), n_scen scenarios taking the first
    round(U[0.8, 1.2] * base) of them, 1 % of the edges cut to one lane in
    each; 2 h at dt = 0.5 s."""
    net = grid_network()
    n_master = int(round(1.2 * base))
    route_off, route_edges, _, _ = _od_routes(net, n_master, seed)
    dep = np.floor(_rng(seed, _P_DEP).uniform(0.0, n_steps * 0.5, size=n_master) / 0.5).astype(np.int32)
    alpha = _rng(seed, _P_ALPHA).uniform(0.05, 0.40, size=n_master).astype(np.float32)
    master = Workload("grid10x10_master", net, route_off, route_edges, dep, np.zeros(n_master, np.uint8), alpha,
                      base_params(1, seed), n_steps, info={"departures": "U[0, 2 h)"})
    return master, ensemble_scenarios(n_scen, base, net.n_edges, seed)


CONFIGS = {"grid10x10": config1, "perturbed_grid_ring": config2}
